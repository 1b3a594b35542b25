"""FP64 CPU oracle for the piecewise-flat-embedding hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import it; only
``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
call into it.  It shares no code with the HIP library: it builds its own graph,
weights, operators and solves, with numpy/scipy in float64, following the paper
(Meinhold, Hayes, Cahill, "Efficiently Computing Piecewise Flat Embeddings for
Data Clustering and Image Segmentation") step by step.

Parity status per function is listed in the module docstrings; every function
here is pinned by a ``-m "not gpu"`` test in ``tests/test_oracle_*.py``.
"""
from .pfe import *  # noqa: F401,F403
from . import classical  # noqa: F401,E402
from . import kmeans  # noqa: F401,E402
