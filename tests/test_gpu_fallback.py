"""Jacobi-PCG as the fallback of the factor preconditioners (learned, FSAI).

A factor-preconditioned solve that breaks down (a non-positive or non-finite
CG scalar) or reaches maxit is redone with Jacobi-PCG from the same starting
point; `fallbacks` counts such solves.  Both failures are produced from the
host with networks of finite weights on an ordinary numeric path:
  - a zero factor: every output weight 0 and the diagonal bias -200, so the
    softplus diagonal underflows to exactly 0 in FP32 and G = 0: r^T z = 0 at
    the first step (breakdown);
  - a badly conditioned factor: output constant c = 2 on every off-diagonal
    entry (G_ij = 2 At_ij), for which the oracle's factor PCG needs about 390
    iterations on this system where Jacobi needs 34, run with maxit = 100.
In both cases the result must equal the Jacobi solve from the same start in
the same launch shape, bit for bit."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_helpers import banner, rel
from oracle import learned as LN

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

OUT = slice(672, 722)            # output heads u, v, q and the constants c, bd


def zero_factor_params():
    th = np.zeros(LN.NPARAM, dtype=np.float32)
    th[721] = -200.0             # softplus(-200) == 0 in FP32
    return th


def slow_factor_params():
    th = np.zeros(LN.NPARAM, dtype=np.float32)
    th[720] = 2.0                # G_ij = 2 At_ij on every lower slot
    th[721] = LN.SOFTPLUS_ONE    # unit diagonal
    return th


def make(wl, maxit, pre):
    from paper_1612_06496_amd import Graph, Mpnn, Solver
    G = Graph.grid(wl.feat, wl.H, wl.W, wl.stencil, wl.sigma)
    S = Solver(G, wl.y0, lam=20.0, r=1.0, n_inner=2, tol=1e-6, maxit=maxit, persistent=False)
    if pre is not None:
        S.set_learned(Mpnn(pre))
    return G, S


@pytest.mark.parametrize("case", ["breakdown", "maxit"])
def test_failed_factor_solve_is_redone_with_jacobi(case):
    banner(f"Jacobi fallback: {case}")
    wl = synth.grid_workload("t", 40, 48, 6, 0.05, 3, stencil=8, d=4)
    th = zero_factor_params() if case == "breakdown" else slow_factor_params()
    maxit = 100
    _, S_l = make(wl, maxit, th)
    _, S_j = make(wl, maxit, None)
    # two inner iterations (two solves) in each context from the same start
    info_l = S_l.step("inner", info=True)
    info_l2 = S_l.step("inner", info=True)
    info_j = S_j.step("inner", info=True)
    info_j2 = S_j.step("inner", info=True)
    print(f"learned ({case}): fallbacks {info_l['fallbacks']}, {info_l2['fallbacks']}; "
          f"status {info_l['status']}, {info_l2['status']}; jacobi iterations {info_j['cg_iters_last']}, "
          f"{info_j2['cg_iters_last']}")
    assert info_l["fallbacks"] == 1 and info_l2["fallbacks"] == 1
    assert info_l["status"] == 0 and info_l2["status"] == 0
    assert info_j["fallbacks"] == 0
    for which in ("Y", "rhs", "b"):
        a = S_l.get(which).cpu().numpy()
        b = S_j.get(which).cpu().numpy()
        assert np.array_equal(a, b), (which, rel(a, b))


def test_factor_solve_after_fused_residual_is_redone_with_jacobi():
    """An SOC iteration in one call, so that the second solve starts from the
    residual the first edge update formed (which then also stores the
    right-hand side): with a factor whose PCG breaks down, both solves are redone
    with Jacobi (the second from the stored right-hand side), and the state
    follows the Jacobi context's (FP32; that context's second solve starts from
    the fused kernel's residual, which rounds differently)."""
    banner("Jacobi fallback after a fused edge update and residual")
    wl = synth.grid_workload("t", 40, 48, 6, 0.05, 3, stencil=8, d=4)
    _, S_l = make(wl, 100, zero_factor_params())
    _, S_j = make(wl, 100, None)
    info_l = S_l.solve(1, info=True)
    info_j = S_j.solve(1, info=True)
    print(f"fallbacks {info_l['fallbacks']}, status {info_l['status']}, flags {info_l['flags']} / {info_j['flags']}")
    assert info_l["flags"] & 8 and info_j["flags"] & 8
    assert info_l["fallbacks"] == 2 and info_l["status"] == 0 and info_j["fallbacks"] == 0
    for which in ("Y", "P"):
        a = S_l.get(which).cpu().numpy()
        b = S_j.get(which).cpu().numpy()
        assert rel(a, b) <= 1e-5, (which, rel(a, b))


def test_pcg_entry_point_falls_back_and_reports_jacobi_counts():
    banner("Jacobi fallback: pfe_pcg")
    wl = synth.grid_workload("t", 40, 48, 6, 0.05, 3, stencil=8, d=4)
    g = O.build_grid_graph(wl.feat, wl.H, wl.W, wl.stencil, wl.sigma)
    SS = LN.ScaledSystem(g, 20.0, 1.0)
    rhs = np.random.default_rng(5).normal(size=(g.n, 4))
    _, S_l = make(wl, 100, slow_factor_params())
    _, S_j = make(wl, 100, None)
    x_l, it_l, info_l = S_l.pcg(rhs, np.zeros_like(rhs))
    x_j, it_j, info_j = S_j.pcg(rhs, np.zeros_like(rhs))
    _, it_o = LN.pcg_preconditioned(SS.A, rhs, np.zeros_like(rhs), lambda q: q / SS.dA[:, None], 1e-6, 5000)
    print(f"fallbacks {info_l['fallbacks']}; iterations after the fallback {it_l}, jacobi {it_j}, "
          f"oracle jacobi {it_o}")
    assert info_l["fallbacks"] == 1 and info_l["status"] == 0
    assert np.array_equal(it_l, it_j)
    assert np.array_equal(x_l.cpu().numpy(), x_j.cpu().numpy())
    assert np.all(np.abs(it_l - it_o) <= 1)
    exact = O.DirectSolver(SS.A)(rhs)
    assert rel(x_l.cpu().numpy(), exact) <= 1e-4


def test_healthy_factor_takes_no_fallback():
    banner("Jacobi fallback: none for a working factor")
    wl = synth.grid_workload("t", 40, 48, 6, 0.05, 3, stencil=8, d=4)
    th = np.random.default_rng(4).normal(0.0, 0.2, size=LN.NPARAM).astype(np.float32)
    th[721] = LN.SOFTPLUS_ONE
    _, S_l = make(wl, 5000, th)
    info = S_l.step("outer", info=True)
    assert info["fallbacks"] == 0 and info["status"] == 0
    assert info["solves"] == 2
