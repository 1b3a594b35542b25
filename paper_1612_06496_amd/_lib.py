"""ctypes declarations of the libpfe C ABI (include/pfe.h).

Argument marshalling only: every computation happens inside libpfe.so.  The
library must have been built (``python -m paper_1612_06496_amd.build`` or
``__graft_entry__.build()``); importing this module without it raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("PFE_LIB_PATH") or os.path.join(HERE, "libpfe.so")

# pfe_status
PFE_OK = 0
PFE_E_ARG = -1
PFE_E_GRAPH = -2
PFE_E_HIP = -3
PFE_E_NOMEM = -4
PFE_E_NOT_SPD = -5
PFE_E_RANK = -6
PFE_E_NOCONV = -7
PFE_E_STATE = -8
# enums
PFE_GRID, PFE_EDGES = 0, 1
PFE_JACOBI, PFE_LEARNED, PFE_FSAI = 0, 1, 2
PFE_POLAR, PFE_CHOL = 0, 1
PFE_FP32, PFE_FP64 = 0, 1
PFE_INNER, PFE_OUTER = 0, 1
PFE_Y, PFE_P, PFE_B, PFE_YHAT, PFE_BSPLIT, PFE_DSPLIT, PFE_RHS, PFE_RESID = range(8)
PFE_MPNN_NPARAMS = 722


class pfe_graph_desc(C.Structure):
    _fields_ = [
        ("kind", C.c_int), ("H", C.c_int), ("W", C.c_int), ("m", C.c_int),
        ("feat", C.c_void_p), ("stencil", C.c_int),
        ("n", C.c_int64), ("n_edges", C.c_int64),
        ("src", C.c_void_p), ("dst", C.c_void_p), ("dist2", C.c_void_p),
        ("sigma", C.c_double), ("on_device", C.c_int),
    ]


class pfe_params(C.Structure):
    _fields_ = [
        ("d", C.c_int), ("lambda_", C.c_double), ("r", C.c_double),
        ("n_inner", C.c_int), ("tol", C.c_double), ("maxit", C.c_int),
        ("precond", C.c_int), ("ortho", C.c_int), ("dtype", C.c_int),
        ("init_ortho", C.c_int), ("keep_split", C.c_int), ("persistent", C.c_int),
        ("graphs", C.c_int), ("cold_start", C.c_int),
    ]


class pfe_step_info(C.Structure):
    _fields_ = [
        ("solves", C.c_int64), ("cg_iters_total", C.c_int64),
        ("cg_iters_max", C.c_int32), ("cg_iters_last", C.c_int32),
        ("rel_res_max", C.c_double), ("status", C.c_int32), ("fallbacks", C.c_int32),
        ("workgroups", C.c_int32), ("flags", C.c_int32),
    ]


class pfe_monitors(C.Structure):
    _fields_ = [("objective", C.c_double), ("constraint", C.c_double),
                ("split", C.c_double), ("orthogonality", C.c_double), ("split_nonzero", C.c_double)]


class pfe_le_info(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("degree", C.c_int32), ("residual", C.c_double),
                ("converged", C.c_int32)]


class pfe_tune_result(C.Structure):
    _fields_ = [("persistent", C.c_int32), ("team", C.c_int32), ("row_cache", C.c_int32),
                ("workgroups", C.c_int32), ("ms", C.c_double), ("chosen", C.c_int32),
                ("strips", C.c_int32), ("second_weight", C.c_double), ("one_pass", C.c_int32),
                ("pixel", C.c_int32)]


_P = C.c_void_p
_S = C.c_int  # pfe_status

SIGNATURES = {
    "pfe_build_graph": (_S, [C.POINTER(pfe_graph_desc), _P, C.POINTER(_P)]),
    "pfe_graph_info": (_S, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "pfe_graph_csr": (_S, [_P, _P, _P, _P, _P]),
    "pfe_graph_union": (_S, [_P, C.c_int, _P, C.POINTER(_P)]),
    "pfe_graph_segments": (_S, [_P, C.POINTER(C.c_int), _P, _P]),
    "pfe_destroy_graph": (None, [_P]),
    "pfe_init": (_S, [_P, C.POINTER(pfe_params), _P, _P, C.POINTER(_P)]),
    "pfe_set_penalties": (_S, [_P, C.c_double, C.c_double]),
    "pfe_step": (_S, [_P, C.c_int, C.POINTER(pfe_step_info)]),
    "pfe_solve": (_S, [_P, C.c_int, C.POINTER(pfe_step_info)]),
    "pfe_split_bregman": (_S, [_P, C.c_int, C.POINTER(pfe_step_info)]),
    "pfe_stats": (_S, [_P, C.POINTER(pfe_step_info), C.c_int]),
    "pfe_autotune": (_S, [_P, C.c_int, C.POINTER(pfe_tune_result), C.c_int, C.POINTER(C.c_int)]),
    "pfe_set_launch_shape": (_S, [_P, C.POINTER(pfe_tune_result)]),
    "pfe_get": (_S, [_P, C.c_int, _P]),
    "pfe_set": (_S, [_P, C.c_int, _P]),
    "pfe_get_inner_index": (_S, [_P, C.POINTER(C.c_int)]),
    "pfe_set_inner_index": (_S, [_P, C.c_int]),
    "pfe_monitor": (_S, [_P, C.POINTER(pfe_monitors)]),
    "pfe_apply_A": (_S, [_P, _P, _P]),
    "pfe_pcg": (_S, [_P, _P, _P, C.POINTER(C.c_int32), C.POINTER(pfe_step_info)]),
    "pfe_edge_quantile": (_S, [_P, C.c_double, C.POINTER(C.c_double)]),
    "pfe_mpnn_create": (_S, [_P, C.POINTER(_P)]),
    "pfe_mpnn_get_params": (_S, [_P, _P, _P]),
    "pfe_mpnn_set_params": (_S, [_P, _P]),
    "pfe_mpnn_destroy": (None, [_P]),
    "pfe_mpnn_save": (_S, [_P, C.c_char_p]),
    "pfe_mpnn_load": (_S, [C.c_char_p, C.POINTER(_P)]),
    "pfe_mpnn_train_step": (_S, [_P, _P, _P, C.c_int, C.c_float, C.POINTER(C.c_double)]),
    "pfe_set_learned": (_S, [_P, _P]),
    "pfe_set_preconditioner": (_S, [_P, C.c_int]),
    "pfe_set_fsai": (_S, [_P]),
    "pfe_get_factor": (_S, [_P, _P, _P]),
    "pfe_destroy_ctx": (None, [_P]),
    "pfe_stream_copy": (_S, [_P, _P, C.c_size_t, _P]),
    "pfe_set_allocator": (_S, [_P, _P, _P]),
    "pfe_live_allocations": (C.c_int64, []),
    "pfe_kmeans": (_S, [_P, C.c_int64, C.c_int, C.c_int, _P, C.c_int, C.c_int, _P, _P, C.POINTER(C.c_int32), _P]),
    "pfe_le_init": (_S, [_P, C.c_int, _P, C.c_int, C.c_double, C.c_int, _P, _P, C.POINTER(pfe_le_info), _P]),
    "pfe_kmeans_noalloc": (_S, [_P, C.c_int64, C.c_int, C.c_int, _P, C.c_int, C.c_int, _P, _P, C.POINTER(C.c_int32),
                                _P]),
    "pfe_status_string": (C.c_char_p, [C.c_int]),
    "pfe_last_error": (C.c_char_p, []),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"libpfe.so not found at {LIB_PATH}; build it with "
            "`python -m paper_1612_06496_amd.build` (the HIP library is required, "
            "there is no fallback)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


class PFEError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = lib.pfe_last_error().decode(errors="replace")
        text = lib.pfe_status_string(status).decode()
        super().__init__(f"{where}: {text} ({status}): {msg}")
        self.status = status


def check(status: int, where: str, allow=()):
    if status != PFE_OK and status not in allow:
        raise PFEError(status, where)
    return status
