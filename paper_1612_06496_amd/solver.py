"""Python face of libpfe: the C entry points with torch tensors for device
memory and streams.  Argument marshalling only — every step of the
piecewise-flat-embedding iteration runs in the HIP library.
"""
from __future__ import annotations

import atexit
import ctypes as C
import sys
import weakref
from typing import Optional

import numpy as np
import torch

from . import _lib as L

_WHICH = {"Y": L.PFE_Y, "P": L.PFE_P, "B": L.PFE_B, "Yhat": L.PFE_YHAT,
          "b": L.PFE_BSPLIT, "d": L.PFE_DSPLIT, "rhs": L.PFE_RHS, "resid": L.PFE_RESID}


def _stream_handle(stream: Optional[torch.cuda.Stream]) -> C.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev(x, dtype) -> torch.Tensor:
    """Contiguous CUDA tensor of the given dtype (copies host arrays in)."""
    if isinstance(x, np.ndarray):
        x = torch.from_numpy(np.ascontiguousarray(x))
    return x.to(device="cuda", dtype=dtype).contiguous()


def kmeans(Y, C0, max_iter: int = 100, stream: Optional[torch.cuda.Stream] = None):
    """Lloyd k-means on the rows of Y (n x d, float32 or float64; host arrays
    are copied in as float64) from the initial centroids C0 (K x d) through
    pfe_kmeans.  Returns (labels int32 tensor, centroids float64 tensor,
    iterations run)."""
    if isinstance(Y, torch.Tensor) and Y.is_cuda and Y.dtype in (torch.float32, torch.float64):
        Yd = Y.contiguous()
    else:
        Yd = _dev(Y, torch.float64)
    n, d = Yd.shape
    cen0 = _dev(C0, torch.float64)
    K = cen0.shape[0]
    labels = torch.empty(n, dtype=torch.int32, device="cuda")
    cen = torch.empty((K, d), dtype=torch.float64, device="cuda")
    iters = C.c_int32()
    dt = L.PFE_FP64 if Yd.dtype == torch.float64 else L.PFE_FP32
    L.check(L.lib.pfe_kmeans(Yd.data_ptr(), n, d, dt, cen0.data_ptr(), K, int(max_iter), labels.data_ptr(),
                             cen.data_ptr(), C.byref(iters), _stream_handle(stream)), "pfe_kmeans")
    return labels, cen, iters.value


def le_init(graph: "Graph", d: int, X0, tol: float = 1e-10, max_iter: int = 200,
            stream: Optional[torch.cuda.Stream] = None):
    """Laplacian-eigenmap embedding of a graph (pfe_le_init): the d smallest
    nontrivial solutions of (D - W) y = mu D y from the starting block X0
    (n x k, k >= d, the caller's random draw).  Returns (Y float64 n x d on the
    device, mu numpy array, info dict); raises on failure (PFE_E_NOCONV too)."""
    x0 = _dev(X0, torch.float64)
    n, k = x0.shape
    Y = torch.empty((n, d), dtype=torch.float64, device="cuda")
    mu = np.empty(d, dtype=np.float64)
    inf = L.pfe_le_info()
    L.check(L.lib.pfe_le_init(graph._h, int(d), x0.data_ptr(), int(k), float(tol), int(max_iter), Y.data_ptr(),
                              mu.ctypes.data, C.byref(inf), _stream_handle(stream)), "pfe_le_init")
    return Y, mu, dict(iterations=inf.iterations, degree=inf.degree, residual=inf.residual,
                       converged=inf.converged)


_TORCH_ALLOC = None

# Library objects still open.  Teardown is explicit: close() destroys an
# object at once, close_all() (also run at interpreter exit, while the HIP
# runtime is still up) destroys what is left, contexts and networks before the
# graphs they use.  A destructor that runs during interpreter finalisation
# makes no library call.
_LIVE = weakref.WeakSet()


def close_all() -> None:
    """Destroy every solver, network and graph of the library still open."""
    objs = list(_LIVE)
    for kind in (Solver, Mpnn, Graph):
        for o in objs:
            if isinstance(o, kind):
                o.close()


atexit.register(close_all)


def _finalizing() -> bool:
    return sys.is_finalizing()


def use_torch_allocator(enable: bool = True) -> None:
    """Route the library's device memory through PyTorch's caching allocator
    (pfe_set_allocator), or back to hipMalloc.  Only while no graph, solver or
    network of the library is alive."""
    global _TORCH_ALLOC
    if not enable:
        L.check(L.lib.pfe_set_allocator(None, None, None), "pfe_set_allocator")
        _TORCH_ALLOC = None
        return
    alloc_t = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_int, C.c_void_p)
    free_t = C.CFUNCTYPE(None, C.c_void_p, C.c_int, C.c_void_p)

    def _alloc(nbytes, device, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device)
        except Exception:      # out of memory: the library reports the failure
            return None

    def _free(ptr, device, user):
        torch.cuda.caching_allocator_delete(ptr)

    fns = (alloc_t(_alloc), free_t(_free))       # kept alive while installed
    L.check(L.lib.pfe_set_allocator(C.cast(fns[0], C.c_void_p), C.cast(fns[1], C.c_void_p), None),
            "pfe_set_allocator")
    _TORCH_ALLOC = fns


def live_allocations() -> int:
    """Device allocations of the library currently live."""
    return int(L.lib.pfe_live_allocations())


class Graph:
    """A graph built by pfe_build_graph (CSR adjacency, heat-kernel weights)."""

    def __init__(self, handle: C.c_void_p, stream):
        self._h = handle
        self._stream = stream
        _LIVE.add(self)
        n, e, nnz = C.c_int64(), C.c_int64(), C.c_int64()
        L.check(L.lib.pfe_graph_info(self._h, C.byref(n), C.byref(e), C.byref(nnz)), "pfe_graph_info")
        self.n, self.n_edges, self.nnz_A = n.value, e.value, nnz.value

    @classmethod
    def grid(cls, feat, H: int, W: int, stencil: int, sigma: float, stream=None) -> "Graph":
        f = _dev(feat, torch.float32).reshape(H * W, -1)
        desc = L.pfe_graph_desc(kind=L.PFE_GRID, H=H, W=W, m=f.shape[1], feat=f.data_ptr(),
                                stencil=stencil, sigma=sigma, on_device=1)
        h = C.c_void_p()
        L.check(L.lib.pfe_build_graph(C.byref(desc), _stream_handle(stream), C.byref(h)), "pfe_build_graph")
        return cls(h, stream)

    @classmethod
    def edges(cls, n: int, src, dst, dist2, sigma: float, stream=None) -> "Graph":
        s = _dev(src, torch.int32)
        t = _dev(dst, torch.int32)
        q = _dev(dist2, torch.float64)
        desc = L.pfe_graph_desc(kind=L.PFE_EDGES, n=n, n_edges=s.numel(), src=s.data_ptr(),
                                dst=t.data_ptr(), dist2=q.data_ptr(), sigma=sigma, on_device=1)
        h = C.c_void_p()
        L.check(L.lib.pfe_build_graph(C.byref(desc), _stream_handle(stream), C.byref(h)), "pfe_build_graph")
        return cls(h, stream)

    @classmethod
    def union(cls, parts, stream=None) -> "Graph":
        """Block-diagonal union (one segment per part) of already built graphs."""
        arr = (C.c_void_p * len(parts))(*[g._h for g in parts])
        h = C.c_void_p()
        L.check(L.lib.pfe_graph_union(arr, len(parts), _stream_handle(stream), C.byref(h)), "pfe_graph_union")
        return cls(h, stream)

    @property
    def segments(self):
        """(row0, edge0): first vertex and first edge of each segment, with the
        totals appended."""
        k = C.c_int()
        L.check(L.lib.pfe_graph_segments(self._h, C.byref(k), None, None), "pfe_graph_segments")
        row0 = np.empty(k.value + 1, dtype=np.int64)
        edge0 = np.empty(k.value + 1, dtype=np.int64)
        L.check(L.lib.pfe_graph_segments(self._h, C.byref(k), row0.ctypes.data, edge0.ctypes.data),
                "pfe_graph_segments")
        return row0, edge0

    def csr(self):
        rowptr = torch.empty(self.n + 1, dtype=torch.int32, device="cuda")
        col = torch.empty(2 * self.n_edges, dtype=torch.int32, device="cuda")
        w = torch.empty(2 * self.n_edges, dtype=torch.float32, device="cuda")
        deg = torch.empty(self.n, dtype=torch.float64, device="cuda")
        L.check(L.lib.pfe_graph_csr(self._h, rowptr.data_ptr(), col.data_ptr(), w.data_ptr(),
                                    deg.data_ptr()), "pfe_graph_csr")
        return dict(rowptr=rowptr, col=col, w=w, degree=deg)

    def close(self):
        if self._h:
            L.lib.pfe_destroy_graph(self._h)
            self._h = None
        _LIVE.discard(self)

    def __del__(self):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """A pfe_ctx: the SOC / Split-Bregman iteration on one graph."""

    def __init__(self, graph: Graph, Y0, *, lam: float, r: float, n_inner: int, tol: float = 1e-6,
                 maxit: int = 1000, ortho: str = "polar", fp64: bool = False, init_ortho: bool = True,
                 keep_split: bool = False, persistent: bool = True, graphs: bool = False,
                 warm_start: bool = True, stream=None):
        self.graph = graph
        self.dtype = torch.float64 if fp64 else torch.float32
        y0 = _dev(Y0, self.dtype)
        self.n, self.d = y0.shape
        self.params = L.pfe_params(
            d=self.d, lambda_=lam, r=r, n_inner=n_inner, tol=tol, maxit=maxit,
            precond=L.PFE_JACOBI, ortho=L.PFE_POLAR if ortho == "polar" else L.PFE_CHOL,
            dtype=L.PFE_FP64 if fp64 else L.PFE_FP32, init_ortho=int(init_ortho),
            keep_split=int(keep_split), persistent=int(persistent), graphs=int(graphs),
            cold_start=int(not warm_start))
        self._stream = stream
        h = C.c_void_p()
        L.check(L.lib.pfe_init(graph._h, C.byref(self.params), y0.data_ptr(), _stream_handle(stream),
                               C.byref(h)), "pfe_init")
        self._h = h
        _LIVE.add(self)

    # -- iteration -----------------------------------------------------------
    @staticmethod
    def _info_dict(info: L.pfe_step_info):
        return dict(solves=info.solves, cg_iters_total=info.cg_iters_total,
                    cg_iters_max=info.cg_iters_max, cg_iters_last=info.cg_iters_last,
                    rel_res_max=info.rel_res_max, status=info.status, fallbacks=info.fallbacks,
                    workgroups=info.workgroups, flags=info.flags)

    def step(self, granularity: str = "outer", info: bool = False, allow_noconv: bool = False):
        g = L.PFE_INNER if granularity == "inner" else L.PFE_OUTER
        inf = L.pfe_step_info() if info else None
        st = L.lib.pfe_step(self._h, g, C.byref(inf) if info else None)
        L.check(st, "pfe_step", allow=(L.PFE_E_NOCONV,) if allow_noconv else ())
        return self._info_dict(inf) if info else None

    def solve(self, n_outer: int, info: bool = False, allow_noconv: bool = False):
        inf = L.pfe_step_info() if info else None
        st = L.lib.pfe_solve(self._h, n_outer, C.byref(inf) if info else None)
        L.check(st, "pfe_solve", allow=(L.PFE_E_NOCONV,) if allow_noconv else ())
        return self._info_dict(inf) if info else None

    def split_bregman(self, n_iter: int, info: bool = False, allow_noconv: bool = False):
        """Stage II: n_iter Split-Bregman iterations with P and B held fixed (pfe_split_bregman)."""
        inf = L.pfe_step_info() if info else None
        st = L.lib.pfe_split_bregman(self._h, int(n_iter), C.byref(inf) if info else None)
        L.check(st, "pfe_split_bregman", allow=(L.PFE_E_NOCONV,) if allow_noconv else ())
        return self._info_dict(inf) if info else None

    def stats(self, reset: bool = False, allow_noconv: bool = False) -> dict:
        """Statistics accumulated since the last reset."""
        inf = L.pfe_step_info()
        st = L.lib.pfe_stats(self._h, C.byref(inf), int(reset))
        L.check(st, "pfe_stats", allow=(L.PFE_E_NOCONV,) if allow_noconv else ())
        return self._info_dict(inf)

    def autotune(self, trials: int = 2) -> list:
        """Time the candidate launch shapes on this graph and keep the fastest."""
        res = (L.pfe_tune_result * 32)()
        n = C.c_int()
        L.check(L.lib.pfe_autotune(self._h, int(trials), res, 32, C.byref(n)), "pfe_autotune",
                allow=(L.PFE_E_NOCONV,))
        return [dict(persistent=r.persistent, team=r.team, row_cache=r.row_cache, strips=r.strips,
                     second_weight=r.second_weight, one_pass=r.one_pass, pixel=r.pixel, workgroups=r.workgroups,
                     ms=r.ms, chosen=r.chosen)
                for r in res[:n.value]]

    def set_launch_shape(self, persistent: bool = False, strips: int = 0, team: int = 1, row_cache: bool = False,
                         second_weight: float = 1.0, one_pass: bool = False, pixel: int = 0) -> None:
        """Run later iterations in the given launch shape (the fields of an
        autotune() result): persistent with teams / row cache / second-workgroup
        share, or one launch per phase on row chunks (strips = 0) or on image
        strips sized for 1 or 2 waves (factor preconditioners: one or two passes
        per CG iteration), with Jacobi PCG by per-row (pixel) launches on pixel
        (1 or 2) workgroups per CU."""
        sh = L.pfe_tune_result(persistent=int(persistent), team=int(team), row_cache=int(row_cache),
                               strips=int(strips), second_weight=float(second_weight), one_pass=int(one_pass),
                               pixel=int(pixel))
        L.check(L.lib.pfe_set_launch_shape(self._h, C.byref(sh)), "pfe_set_launch_shape")

    # -- state ---------------------------------------------------------------
    def get(self, which: str) -> torch.Tensor:
        rows = self.graph.n_edges if which in ("b", "d") else self.n
        out = torch.empty(rows, self.d, dtype=self.dtype, device="cuda")
        L.check(L.lib.pfe_get(self._h, _WHICH[which], out.data_ptr()), f"pfe_get({which})")
        return out

    def set(self, which: str, value) -> None:
        v = _dev(value, self.dtype)
        L.check(L.lib.pfe_set(self._h, _WHICH[which], v.data_ptr()), f"pfe_set({which})")

    @property
    def inner_index(self) -> int:
        k = C.c_int()
        L.check(L.lib.pfe_get_inner_index(self._h, C.byref(k)), "pfe_get_inner_index")
        return k.value

    @inner_index.setter
    def inner_index(self, k: int) -> None:
        L.check(L.lib.pfe_set_inner_index(self._h, int(k)), "pfe_set_inner_index")

    def set_penalties(self, lam: float, r: float) -> None:
        L.check(L.lib.pfe_set_penalties(self._h, lam, r), "pfe_set_penalties")

    def monitor(self) -> dict:
        m = L.pfe_monitors()
        L.check(L.lib.pfe_monitor(self._h, C.byref(m)), "pfe_monitor")
        return dict(objective=m.objective, constraint=m.constraint, split=m.split,
                    orthogonality=m.orthogonality, split_nonzero=m.split_nonzero)

    # -- operator and solver entry points ------------------------------------
    def apply_A(self, X) -> torch.Tensor:
        x = _dev(X, self.dtype)
        q = torch.empty_like(x)
        L.check(L.lib.pfe_apply_A(self._h, x.data_ptr(), q.data_ptr()), "pfe_apply_A")
        return q

    def pcg(self, rhs, x0, allow_noconv: bool = False):
        b = _dev(rhs, self.dtype)
        x = _dev(x0, self.dtype).clone()
        iters = (C.c_int32 * self.d)()
        inf = L.pfe_step_info()
        st = L.lib.pfe_pcg(self._h, b.data_ptr(), x.data_ptr(), iters, C.byref(inf))
        L.check(st, "pfe_pcg", allow=(L.PFE_E_NOCONV,) if allow_noconv else ())
        return x, np.array(list(iters)), self._info_dict(inf)

    # -- learned preconditioner ------------------------------------------------
    def set_learned(self, net: "Mpnn") -> None:
        """Evaluate the network on this system and precondition with G^T G."""
        L.check(L.lib.pfe_set_learned(self._h, net._h), "pfe_set_learned")

    def set_fsai(self) -> None:
        """Compute the FSAI factor of this system on the device and precondition with it."""
        L.check(L.lib.pfe_set_fsai(self._h), "pfe_set_fsai")

    def set_preconditioner(self, which: str) -> None:
        code = {"jacobi": L.PFE_JACOBI, "learned": L.PFE_LEARNED, "fsai": L.PFE_FSAI}[which]
        L.check(L.lib.pfe_set_preconditioner(self._h, code), "pfe_set_preconditioner")

    def get_factor(self):
        """(Gt_ji per undirected edge (i < j, lexicographic), diag(Gt))."""
        ev = torch.empty(self.graph.n_edges, dtype=self.dtype, device="cuda")
        dg = torch.empty(self.n, dtype=self.dtype, device="cuda")
        L.check(L.lib.pfe_get_factor(self._h, ev.data_ptr(), dg.data_ptr()), "pfe_get_factor")
        return ev, dg

    def edge_quantile(self, q: float) -> float:
        out = C.c_double()
        L.check(L.lib.pfe_edge_quantile(self._h, q, C.byref(out)), "pfe_edge_quantile")
        return out.value

    def close(self):
        if getattr(self, "_h", None):
            L.lib.pfe_destroy_ctx(self._h)
            self._h = None
        _LIVE.discard(self)

    def __del__(self):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Mpnn:
    """The learned-preconditioner network (weights + Adam state on the device)."""

    NPARAMS = L.PFE_MPNN_NPARAMS

    def __init__(self, params=None):
        h = C.c_void_p()
        if params is None:
            L.check(L.lib.pfe_mpnn_create(None, C.byref(h)), "pfe_mpnn_create")
        else:
            p = np.ascontiguousarray(params, dtype=np.float32)
            assert p.size == self.NPARAMS
            L.check(L.lib.pfe_mpnn_create(p.ctypes.data, C.byref(h)), "pfe_mpnn_create")
        self._h = h
        _LIVE.add(self)

    @property
    def params(self) -> np.ndarray:
        out = np.empty(self.NPARAMS, dtype=np.float32)
        L.check(L.lib.pfe_mpnn_get_params(self._h, out.ctypes.data, None), "pfe_mpnn_get_params")
        return out

    @property
    def grad(self) -> np.ndarray:
        out = np.empty(self.NPARAMS, dtype=np.float32)
        L.check(L.lib.pfe_mpnn_get_params(self._h, None, out.ctypes.data), "pfe_mpnn_get_params")
        return out

    def set_params(self, params) -> None:
        p = np.ascontiguousarray(params, dtype=np.float32)
        L.check(L.lib.pfe_mpnn_set_params(self._h, p.ctypes.data), "pfe_mpnn_set_params")

    def save(self, path: str) -> None:
        """Write the parameters to a network file (pfe_mpnn_save)."""
        L.check(L.lib.pfe_mpnn_save(self._h, str(path).encode()), "pfe_mpnn_save")

    @classmethod
    def load(cls, path: str) -> "Mpnn":
        """A network from a file written by save (pfe_mpnn_load)."""
        h = C.c_void_p()
        L.check(L.lib.pfe_mpnn_load(str(path).encode(), C.byref(h)), "pfe_mpnn_load")
        net = cls.__new__(cls)
        net._h = h
        _LIVE.add(net)
        return net

    def train_step(self, solver: Solver, samples, lr: float) -> float:
        """One Adam step (lr = 0: gradient only) on residual samples (n x k)."""
        x = _dev(samples, solver.dtype)
        loss = C.c_double()
        L.check(L.lib.pfe_mpnn_train_step(self._h, solver._h, x.data_ptr(), x.shape[1], float(lr),
                                          C.byref(loss)), "pfe_mpnn_train_step")
        return loss.value

    def close(self):
        if getattr(self, "_h", None):
            L.lib.pfe_mpnn_destroy(self._h)
            self._h = None
        _LIVE.discard(self)

    def __del__(self):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass
