"""MI355X (gfx950) piecewise flat embeddings: the split-Bregman / PCG hot path
of Meinhold, Hayes and Cahill (arXiv 1612.06496) as a HIP library (libpfe.so,
C ABI in include/pfe.h) with a thin Python binding.

    from paper_1612_06496_amd import Graph, Solver

Graph and Solver load libpfe.so on first use and raise ImportError if it has
not been built (there is no fallback implementation).
"""

__all__ = ["Graph", "Solver", "Mpnn", "kmeans", "le_init", "use_torch_allocator", "live_allocations", "close_all"]


def __getattr__(name):
    if name in __all__:
        from . import solver
        return getattr(solver, name)
    raise AttributeError(name)
