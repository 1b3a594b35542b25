"""Pins for the learned-preconditioner oracle (CPU, float64): identity start is
exactly Jacobi, G^T G is SPD for any weights, autograd gradients agree with
central finite differences, bf16 emulation stays within its rounding, and
training lowers both the loss and the PCG iteration count on held-out data."""
import math

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


# --- the network and its loss against a plain, loop-by-loop reading of the
# definitions in the module docstring (dense matrices, no index scatter) ------

def _tiny_five(seed=3):
    """5 vertices, 7 edges with uneven weights (so rows differ in degree)."""
    rng = np.random.default_rng(seed)
    pairs = [(0, 1), (0, 3), (1, 2), (1, 4), (2, 3), (2, 4), (3, 4)]
    ei = np.array([p[0] for p in pairs])
    ej = np.array([p[1] for p in pairs])
    w = rng.uniform(0.3, 1.0, size=len(pairs))
    return O.Graph(5, ei, ej, w)


def _loop_reference(theta, g, lam, r, slip=None):
    """Gt (dense, lower triangular) and At (dense, unit diagonal) computed entry
    by entry.  A is written from Eq. (13) entrywise: A_ij = -lam/2 w_ij^2 for an
    edge, A_ii = lam/2 sum_j w_ij^2 + r/2 sum_j w_ij.  `slip` plants one of the
    plausible mistakes the oracle must not make, to show this reference tells
    them apart."""
    n = g.n
    W = np.zeros((n, n))
    for i, j, w in zip(g.ei, g.ej, g.w):
        W[i, j] = W[j, i] = w
    A = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j and W[i, j] > 0:
                A[i, j] = -0.5 * lam * W[i, j] ** 2
        A[i, i] = 0.5 * lam * sum(W[i, j] ** 2 for j in range(n)) + 0.5 * r * sum(W[i, :])
    At = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            At[i, j] = A[i, j] / math.sqrt(A[i, i] * A[j, j])
    nb = [[j for j in range(n) if j != i and W[i, j] > 0] for i in range(n)]
    degmax = max(len(v) for v in nb)
    p = LN.unpack(np.asarray(theta, dtype=np.float64))
    x = [np.array([1.0, sum(abs(At[i, j]) for j in nb[i]), max(abs(At[i, j]) for j in nb[i]),
                   len(nb[i]) / degmax]) for i in range(n)]
    sgn = 1.0 if slip == "agg_sign" else -1.0

    def layer(h, Ws, Wm, b):
        out = []
        for i in range(n):
            agg = sum(sgn * At[i, j] * h[j] for j in nb[i])
            pre = [sum(Ws[k, f] * h[i][f] for f in range(len(h[i])))
                   + sum(Wm[k, f] * agg[f] for f in range(len(h[i]))) + b[k]
                   for k in range(LN.HIDDEN)]
            out.append(np.array([max(0.0, v) for v in pre]))
        return out

    h1 = layer(x, p["W1s"], p["W1m"], p["b1"])
    h2 = layer(h1, p["W2s"], p["W2m"], p["b2"])
    U = [float(np.dot(p["u"], h)) for h in h2]
    V = [float(np.dot(p["v"], h)) for h in h2]
    Z = [float(np.dot(p["q"], h)) + p["bd"][0] for h in h2]
    Gt = np.zeros((n, n))
    for i in range(n):
        for j in nb[i]:
            if j < i:
                a, b = (j, i) if slip == "uv_swap" else (i, j)
                Gt[i, j] = At[i, j] * (U[a] + V[b] + p["c"][0])
        Gt[i, i] = math.log1p(math.exp(Z[i]))
    return Gt, At


def _loop_loss(Gt, At, rho, slip=None):
    tot = 0.0
    M = Gt @ Gt.T if slip == "gt_order" else Gt.T @ Gt
    for k in range(rho.shape[1]):
        e = At @ (M @ rho[:, k]) - rho[:, k]
        tot += float(e @ e)
    return tot / rho.shape[1]


def _active_params(seed):
    """Random weights with positive biases so most hidden units are active
    (a relu that is zero everywhere would hide a mistake behind it)."""
    th = random_params(seed)
    p = LN.unpack(th)
    p["b1"][...] = np.abs(p["b1"]) + 0.5
    p["b2"][...] = np.abs(p["b2"]) + 0.5
    return th


def test_factor_matches_loop_reading_of_its_definition():
    g = _tiny_five()
    lam, r = 3.0, 1.0
    S = LN.ScaledSystem(g, lam, r)
    for seed in (0, 1, 2):
        th = _active_params(seed)
        Gt_ref, At_ref = _loop_reference(th, g, lam, r)
        # the scaled system itself
        assert np.abs(S.At.toarray() - At_ref).max() <= 1e-14
        gv, dg = LN.factor(th, S, bf16=False)
        Gt = LN.factor_matrix(gv, dg, S).toarray()
        err = np.abs(Gt - Gt_ref).max() / np.abs(Gt_ref).max()
        print(f"seed {seed}: factor vs loop reference, max rel err {err:.1e}")
        assert err <= 1e-13
        # both slots of an edge carry the edge's lower entry Gt_{max(i,j), min(i,j)}
        gvn = gv.numpy()
        for s, (i, j) in enumerate(zip(S.si, S.sj)):
            assert gvn[s] == pytest.approx(Gt_ref[max(i, j), min(i, j)], rel=1e-13, abs=1e-300)
        # the mistakes named below change the factor by far more than the bound
        for slip in ("uv_swap", "agg_sign"):
            Gs, _ = _loop_reference(th, g, lam, r, slip=slip)
            assert np.abs(Gs - Gt_ref).max() / np.abs(Gt_ref).max() > 1e-3, slip


def test_loss_matches_dense_reading_and_the_pcg_preconditioner():
    g = _tiny_five(seed=5)
    lam, r = 4.0, 1.0
    S = LN.ScaledSystem(g, lam, r)
    rho = np.random.default_rng(9).normal(size=(g.n, 3))
    rho /= np.linalg.norm(rho, axis=0)
    for seed in (3, 4):
        th = _active_params(seed)
        Gt_ref, At_ref = _loop_reference(th, g, lam, r)
        L_ref = _loop_loss(Gt_ref, At_ref, rho)
        L = float(LN.loss(th, S, rho, bf16=False))
        print(f"seed {seed}: loss {L:.15e} loop reference {L_ref:.15e}")
        assert abs(L - L_ref) <= 1e-13 * L_ref
        assert abs(_loop_loss(Gt_ref, At_ref, rho, slip="gt_order") - L_ref) > 1e-3 * L_ref
        # the same loss through the preconditioner the PCG applies:
        # z = D_A^{-1/2} Gt^T Gt D_A^{-1/2} r with r = D_A^{1/2} rho gives
        # At Gt^T Gt rho = D_A^{-1/2} A z
        gv, dg = LN.factor(th, S, bf16=False)
        z = LN.apply_preconditioner(gv, dg, S, np.sqrt(S.dA)[:, None] * rho)
        e = (S.A @ z) / np.sqrt(S.dA)[:, None] - rho
        assert abs((e ** 2).sum() / rho.shape[1] - L_ref) <= 1e-13 * L_ref
