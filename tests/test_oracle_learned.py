"""Pins for the learned-preconditioner oracle (CPU, float64): identity start is
exactly Jacobi, G^T G is SPD for any weights, autograd gradients agree with
central finite differences, bf16 emulation stays within its rounding, and
training lowers both the loss and the PCG iteration count on held-out data."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
import synth
from oracle import learned as LN


def small_system(lam=5.0, r=1.0, H=10, W=12, seed=4):
    wl = synth.grid_workload("t", H, W, 3, 0.05, seed, stencil=8, d=3)
    g = O.build_grid_graph(wl.feat, wl.H, wl.W, wl.stencil, wl.sigma)
    return g, LN.ScaledSystem(g, lam, r)


def random_params(seed):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, 0.3, size=LN.NPARAM)


def test_parameter_count_and_identity_start():
    assert LN.NPARAM == 722
    g, S = small_system()
    gv, dg = LN.factor(LN.identity_params(0), S)
    assert np.all(gv.numpy() == 0.0)
    assert np.abs(dg.numpy() - 1.0).max() < 1e-15
    # preconditioner == Jacobi
    r = np.random.default_rng(1).normal(size=(g.n, 3))
    z = LN.apply_preconditioner(gv, dg, S, r)
    assert np.abs(z - r / S.dA[:, None]).max() <= 1e-15 * np.abs(z).max()


def test_identity_start_reproduces_jacobi_pcg_iterates():
    g, S = small_system(lam=20.0)
    gv, dg = LN.factor(LN.identity_params(3), S)
    rhs = np.random.default_rng(2).normal(size=(g.n, 3))
    x1, it1 = LN.pcg_preconditioned(S.A, rhs, np.zeros_like(rhs),
                                    lambda rr: LN.apply_preconditioner(gv, dg, S, rr), 1e-10, 1000)
    x2, it2, _ = O.pcg(S.A, rhs, np.zeros_like(rhs), 1.0 / S.dA, 1e-10, 1000)
    assert np.array_equal(it1, it2)
    assert np.abs(x1 - x2).max() <= 1e-12 * np.abs(x2).max()


def test_factor_is_lower_triangular_with_positive_diagonal_and_spd():
    g, S = small_system()
    for seed in range(3):
        gv, dg = LN.factor(random_params(seed), S)
        Gt = LN.factor_matrix(gv, dg, S).toarray()
        assert np.all(np.triu(Gt, 1) == 0.0)
        assert np.all(np.diag(Gt) > 0.0)
        s = 1.0 / np.sqrt(S.dA)
        Minv = (s[:, None] * Gt.T) @ (Gt * s[None, :])
        assert np.abs(Minv - Minv.T).max() <= 1e-12 * np.abs(Minv).max()
        assert np.linalg.eigvalsh(Minv).min() > 0.0
        # pattern: off-diagonal entries only on edges of the graph
        off = (Gt != 0) & ~np.eye(g.n, dtype=bool)
        Adense = S.A.toarray()
        assert np.all(Adense[off] != 0.0)


def test_gradient_matches_central_differences():
    g, S = small_system(H=5, W=6)
    rho = np.random.default_rng(5).normal(size=(g.n, 2))
    rho /= np.linalg.norm(rho, axis=0)
    th = random_params(7)
    L0, gr = LN.loss_and_grad(th, S, rho, bf16=False)
    h = 1e-6
    rng = np.random.default_rng(8)
    idx = rng.choice(LN.NPARAM, 60, replace=False)
    fd = np.empty(len(idx))
    for k, i in enumerate(idx):
        e = np.zeros(LN.NPARAM)
        e[i] = h
        lp = float(LN.loss(th + e, S, rho, bf16=False))
        lm = float(LN.loss(th - e, S, rho, bf16=False))
        fd[k] = (lp - lm) / (2 * h)
    err = np.abs(fd - gr[idx]).max() / np.abs(gr).max()
    print("max relative FD error", err)
    assert err < 1e-6


def test_bf16_emulation_within_rounding():
    g, S = small_system()
    th = random_params(11) * 0.5
    g1, d1 = LN.factor(th, S, bf16=True)
    g2, d2 = LN.factor(th, S, bf16=False)
    scale = max(np.abs(g2.numpy()).max(), 1e-30)
    assert np.abs(g1.numpy() - g2.numpy()).max() <= 2e-2 * scale
    assert np.abs(d1.numpy() - d2.numpy()).max() <= 2e-2 * np.abs(d2.numpy()).max()


@pytest.mark.slow
def test_training_gains_on_held_out_graph():
    """Train on one image's system, evaluate on another image (held out)."""
    lam, r = 50.0, 1.0
    wl_a = synth.grid_workload("a", 24, 28, 5, 0.05, 21, stencil=8, d=3)
    wl_b = synth.grid_workload("b", 24, 28, 5, 0.05, 22, stencil=8, d=3)
    ga = O.build_grid_graph(wl_a.feat, wl_a.H, wl_a.W, 8, 0.1)
    gb = O.build_grid_graph(wl_b.feat, wl_b.H, wl_b.W, 8, 0.1)
    Sa, Sb = LN.ScaledSystem(ga, lam, r), LN.ScaledSystem(gb, lam, r)
    rng = np.random.default_rng(0)
    rho = rng.normal(size=(ga.n, 24)) / np.sqrt(Sa.dA)[:, None]
    rho /= np.linalg.norm(rho, axis=0)
    th = LN.identity_params(0)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    L0, _ = LN.loss_and_grad(th, Sa, rho)
    for t in range(1, 151):
        L, gr = LN.loss_and_grad(th, Sa, rho)
        th, m, v = LN.adam_step(th, gr, m, v, t, 3e-3)
    assert L < 0.7 * L0
    gv, dg = LN.factor(th, Sb)
    rhs = rng.normal(size=(gb.n, 3))
    _, itj = LN.pcg_preconditioned(Sb.A, rhs, np.zeros_like(rhs), lambda q: q / Sb.dA[:, None], 1e-6, 5000)
    _, itl = LN.pcg_preconditioned(Sb.A, rhs, np.zeros_like(rhs),
                                   lambda q: LN.apply_preconditioner(gv, dg, Sb, q), 1e-6, 5000)
    print("held-out iterations: jacobi", itj, "learned", itl)
    assert itl.max() < itj.max()
    # and the learned PCG still reaches the exact solution
    x, _ = LN.pcg_preconditioned(Sb.A, rhs, np.zeros_like(rhs),
                                 lambda q: LN.apply_preconditioner(gv, dg, Sb, q), 1e-10, 5000)
    exact = spla.splu(Sb.A.tocsc()).solve(rhs)
    assert np.abs(x - exact).max() <= 1e-6 * np.abs(exact).max()


def test_adam_matches_its_definition_on_a_quadratic():
    # minimise 0.5 ||x - a||^2: Adam reaches a
    a = np.array([1.0, -2.0, 3.0])
    x = np.zeros(3)
    m = np.zeros(3)
    v = np.zeros(3)
    for t in range(1, 3001):
        x, m, v = LN.adam_step(x, x - a, m, v, t, 1e-2)
    assert np.abs(x - a).max() < 1e-3
