"""Shared set-up for the GPU parity tests: the same seeded inputs go to the HIP
library (through its C ABI) and to the FP64 oracle."""
from __future__ import annotations

import sys

import numpy as np

import oracle as O
import synth


def banner(msg: str) -> None:
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def rel(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def maxrel(a, b) -> float:
    """Element-wise error: the largest |a - b| of each column over that
    column's largest |b|, maximised over the columns (an error confined to a
    few rows, e.g. one band of image strips, is not averaged away)."""
    a = np.asarray(a, dtype=np.float64).reshape(len(a), -1)
    b = np.asarray(b, dtype=np.float64).reshape(len(b), -1)
    scale = np.abs(b).max(axis=0)
    scale[scale == 0] = 1.0
    return float((np.abs(a - b).max(axis=0) / scale).max())


def oracle_graph(wl):
    if wl.kind == "grid":
        return O.build_grid_graph(wl.feat, wl.H, wl.W, wl.stencil, wl.sigma)
    return O.build_edge_graph(wl.n, wl.src, wl.dst, wl.dist2, wl.sigma)


def gpu_graph(wl):
    from paper_1612_06496_amd import Graph
    if wl.kind == "grid":
        return Graph.grid(wl.feat, wl.H, wl.W, wl.stencil, wl.sigma)
    return Graph.edges(wl.n, wl.src, wl.dst, wl.dist2, wl.sigma)


def penalties(wl, g, Y):
    """lambda = r as given by the workload, else the shrink-active scale
    computed by the oracle from the initial embedding."""
    if wl.lam is not None:
        return wl.lam, wl.r
    c = O.shrink_active_scale(g, Y, 0.99)
    return c, c


def mid_run_state(g, wl, lam, r, n_outer_before=2, inner_before=2):
    """An oracle state part-way through a run: (Y, P, B) after some SOC
    iterations, then (Y, b, dd) after some Split-Bregman iterations of the
    next one."""
    Y = O.orthonormalize_init(g, wl.y0)
    P = np.sqrt(g.D)[:, None] * Y
    B = np.zeros_like(Y)
    solve = O.DirectSolver(O.system_matrix(g, lam, r))
    for _ in range(n_outer_before):
        Y, P, B = O.soc_outer_step(g, solve, Y, P, B, lam, r, wl.n_inner)
    b = np.zeros((g.n_edges, wl.d))
    dd = np.zeros((g.n_edges, wl.d))
    for _ in range(inner_before):
        Y, b, dd = O.sb_inner_step(g, solve, Y, P, B, b, dd, lam, r)
    return solve, Y, P, B, b, dd
