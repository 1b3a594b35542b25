"""Write preconditioner_counts_voronoi1024_r2.json: PCG iteration counts of
the oracle (FP64) on the 1024x1024 5x5-window image with three preconditioners
— Jacobi, FSAI, and IC(0), the incomplete Cholesky the paper uses (Sec. III) —
at lambda/r = 1, 10, 100, 1000.

The system is the first inner solve of the first SOC iteration (Algorithm 1,
Algorithm 2, Eq. 13): Y0 D-orthonormalised, P = D^{1/2} Y0, B = 0, so
rhs = r/2 D Y0; warm start x0 = Y0; stop when ||r_c|| <= 1e-6 ||rhs_c|| per
column.  lambda = ratio c, r = c with 1/c the 0.99-quantile of |M Y0| (the
counts do not depend on c: A and rhs scale together).

Calls only the oracle and the seeded input generators.  Run from the
repository root: python tests/golden/make_preconditioner_counts.py (CPU, about
15 minutes)."""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
import synth  # noqa: E402
from oracle import classical as C  # noqa: E402
from oracle.learned import pcg_preconditioned  # noqa: E402

WORKLOAD = "voronoi1024_r2"
RATIOS = (1.0, 10.0, 100.0, 1000.0)
TOL = 1e-6


def main():
    wl = synth.make_workload(WORKLOAD, 0)
    g = O.build_grid_graph(wl.feat, wl.H, wl.W, wl.stencil, wl.sigma)
    Y = O.orthonormalize_init(g, wl.y0)
    c = O.shrink_active_scale(g, Y)
    out = {"workload": WORKLOAD, "seed": 0, "n": int(g.n), "d": int(wl.d), "c": c, "tol": TOL,
           "system": "first inner solve of the first SOC iteration: rhs = r/2 D Y0, x0 = Y0, Y0 D-orthonormalised",
           "ratios": {}}
    for ratio in RATIOS:
        lam, r = ratio * c, c
        A = O.system_matrix(g, lam, r).tocsr()
        rhs = 0.5 * r * g.D[:, None] * Y
        res = {}
        t = time.time()
        _, it, _ = O.pcg(A, rhs, Y, 1.0 / A.diagonal(), TOL, 20000)
        res["jacobi"] = it.tolist()
        t1 = time.time()
        _, it = pcg_preconditioned(A, rhs, Y, C.fsai_apply(C.fsai(A)), TOL, 20000)
        res["fsai"] = it.tolist()
        t2 = time.time()
        _, it = pcg_preconditioned(A, rhs, Y, C.ic0_apply(C.ic0(A)), TOL, 20000)
        res["ic0"] = it.tolist()
        t3 = time.time()
        out["ratios"][str(ratio)] = res
        print(f"lambda/r = {ratio:g}: max iterations jacobi {max(res['jacobi'])}, fsai {max(res['fsai'])}, "
              f"ic0 {max(res['ic0'])} ({t1 - t:.0f} s, {t2 - t1:.0f} s, {t3 - t2:.0f} s)", flush=True)
    with open(os.path.join(HERE, f"preconditioner_counts_{WORKLOAD}.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
