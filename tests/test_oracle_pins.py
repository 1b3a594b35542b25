"""Pins for the FP64 oracle: each test checks the oracle against something other
than itself (the paper's printed numbers, closed forms, optimality conditions,
brute force on tiny inputs, invariances, independent library routines)."""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.optimize as sopt
import scipy.sparse as sp

import oracle as O
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def tiny_graph(n=9, seed=0, extra=4):
    """A small connected graph: a path plus random chords, random weights."""
    rng = np.random.default_rng(seed)
    pairs = {(i, i + 1) for i in range(n - 1)}
    while len(pairs) < n - 1 + extra:
        a, b = sorted(rng.choice(n, 2, replace=False))
        pairs.add((int(a), int(b)))
    pairs = sorted(pairs)
    ei = np.array([p[0] for p in pairs])
    ej = np.array([p[1] for p in pairs])
    w = rng.uniform(0.2, 1.0, size=len(pairs))
    return O.Graph(n, ei, ej, w)


def random_state(g, d, seed):
    rng = np.random.default_rng(seed)
    Y = rng.normal(size=(g.n, d))
    P = rng.normal(size=(g.n, d))
    B = 0.1 * rng.normal(size=(g.n, d))
    b = 0.1 * rng.normal(size=(g.n_edges, d))
    dd = 0.1 * rng.normal(size=(g.n_edges, d))
    return Y, P, B, b, dd


# --- P1: structure of A ---------------------------------------------------

def test_p1_laplacian_of_squared_weights_annihilates_ones():
    wl = synth.make_workload("voronoi64_4nbr", 0)
    g = O.build_grid_graph(wl.feat, wl.H, wl.W, wl.stencil, wl.sigma)
    LtL = g.M.T @ g.M
    err = np.abs(LtL @ np.ones(g.n)).max()
    print("P1 |M^T M 1|_max =", err, "bound", 1e-13 * g.D.max())
    assert err <= 1e-13 * g.D.max()
    # off-diagonal entries are -w^2, diagonal entries sum of w^2 (M carries w)
    W2 = g.adjacency().multiply(g.adjacency())
    assert abs(LtL - (sp.diags(np.asarray(W2.sum(1)).ravel()) - W2)).max() < 1e-15
    # D = diag(W 1) from the symmetric adjacency
    assert np.abs(np.asarray(g.adjacency().sum(1)).ravel() - g.D).max() < 1e-15
    A = O.system_matrix(g, 1.0, 3.0)
    assert np.allclose(A @ np.ones(g.n), 1.5 * g.D, rtol=0, atol=1e-13)


def test_grid_edges_counts_and_order():
    # open grids: 4-nbr has H(W-1) + W(H-1) edges; 8-nbr adds 2(H-1)(W-1);
    # a 5x5 window adds the remaining offsets.
    H, W = 7, 5
    i, j = O.grid_edges(H, W, 4)
    assert len(i) == H * (W - 1) + W * (H - 1)
    i8, j8 = O.grid_edges(H, W, 8)
    assert len(i8) == H * (W - 1) + W * (H - 1) + 2 * (H - 1) * (W - 1)
    i2, j2 = O.grid_edges(H, W, -2)
    # brute force: every pair within Chebyshev distance 2
    brute = {(a, b) for a in range(H * W) for b in range(a + 1, H * W)
             if max(abs(a // W - b // W), abs(a % W - b % W)) <= 2}
    assert set(zip(i2.tolist(), j2.tolist())) == brute
    assert np.all(i2 < j2)
    assert np.all(np.diff(i2 * H * W + j2) > 0)        # lexicographic order


def test_heat_kernel_limits():
    # identical features -> weight 1; weight halves at ||dx||^2 = 2 sigma^2 ln 2
    s = 0.1
    assert O.heat_kernel(0.0, s) == 1.0
    assert abs(O.heat_kernel(2 * s * s * math.log(2), s) - 0.5) < 1e-15


# --- P2/P3: compact forms equal the Kronecker forms ---------------------------

def test_p2_compact_operators_match_kronecker():
    g = tiny_graph(12, seed=1, extra=6)
    d = 3
    Y, P, B, b, dd = random_state(g, d, 2)
    L = O.kron_L(g, d)
    Dt = O.kron_Dt(g, d)
    Yv = O.vec(Y)
    assert np.abs(L @ Yv - O.vec(g.M @ Y)).max() < 1e-14                      # Eq. 7
    assert np.abs(np.sqrt(Dt.diagonal()) * Yv - O.vec(np.sqrt(g.D)[:, None] * Y)).max() < 1e-14  # Eq. 8
    assert np.abs(L.T @ (L @ Yv) - O.vec(g.M.T @ (g.M @ Y))).max() < 1e-14     # Eq. 11
    assert np.abs(Dt @ Yv - O.vec(g.D[:, None] * Y)).max() < 1e-14             # Eq. 12
    # Eqs. 9-10: shrink and Bregman on vec(M Y) equal the compact |E| x d forms
    lam = 2.0
    t_kron = L @ Yv + O.vec(b)
    assert np.abs(O.shrink(t_kron, 1 / lam) - O.vec(O.shrink(g.M @ Y + b, 1 / lam))).max() == 0.0


def test_p3_compact_system_matches_kronecker_normal_equations():
    g = tiny_graph(10, seed=3, extra=5)
    d, lam, r = 3, 1.7, 0.6
    Y, P, B, b, dd = random_state(g, d, 4)
    L = O.kron_L(g, d)
    Dt = O.kron_Dt(g, d)
    # Eq. 6 with q1 = d - b and (sign reading) q2 = P - B, solved densely
    K = (0.5 * lam * (L.T @ L) + 0.5 * r * Dt).toarray()
    rhs = 0.5 * lam * (L.T @ O.vec(dd - b)) + 0.5 * r * np.sqrt(Dt.diagonal()) * O.vec(P - B)
    y_kron = np.linalg.solve(K, rhs)
    solve = O.DirectSolver(O.system_matrix(g, lam, r))
    Y1, _, _ = O.sb_inner_step(g, solve, Y, P, B, b, dd, lam, r)
    assert np.abs(O.unvec(y_kron, g.n) - Y1).max() < 1e-12


# --- P4/P5: the least-squares step is the argmin of Algorithm 2's objective ---

def test_p4_y_update_is_argmin_of_split_bregman_subproblem():
    g = tiny_graph(11, seed=5, extra=5)
    d, lam, r = 2, 3.0, 0.8
    Y, P, B, b, dd = random_state(g, d, 6)
    L = O.kron_L(g, d).toarray()
    Dth = np.sqrt(O.kron_Dt(g, d).diagonal())
    # Stacked least squares straight from Algorithm 2's Y-update:
    #   lambda/2 ||L y + b - d||^2 + r/2 ||D~^{1/2} y - P + B||^2
    Amat = np.vstack([math.sqrt(lam / 2) * L, math.sqrt(r / 2) * np.diag(Dth)])
    rhs = np.concatenate([math.sqrt(lam / 2) * O.vec(dd - b), math.sqrt(r / 2) * O.vec(P - B)])
    y_ls = np.linalg.lstsq(Amat, rhs, rcond=None)[0]
    solve = O.DirectSolver(O.system_matrix(g, lam, r))
    Y1, _, _ = O.sb_inner_step(g, solve, Y, P, B, b, dd, lam, r)
    err = np.abs(O.unvec(y_ls, g.n) - Y1).max()
    print("P4 argmin error", err)
    assert err < 1e-10

    def f(y):
        return (lam / 2 * np.sum((L @ y + O.vec(b) - O.vec(dd)) ** 2)
                + r / 2 * np.sum((Dth * y - O.vec(P) + O.vec(B)) ** 2))
    # the printed right-hand side sign (B - P) gives a strictly worse value
    wrong = 0.5 * lam * (L.T @ O.vec(dd - b)) + 0.5 * r * Dth * O.vec(B - P)
    y_wrong = np.linalg.solve(0.5 * lam * L.T @ L + 0.5 * r * np.diag(Dth ** 2), wrong)
    assert f(O.vec(Y1)) < f(y_wrong)


def test_p5_lambda_zero_reduces_to_scaled_split_target():
    g = tiny_graph(8, seed=7)
    d = 3
    Y, P, B, b, dd = random_state(g, d, 8)
    solve = O.DirectSolver(O.system_matrix(g, 0.0, 1.3))
    Y1, b1, dd1 = O.sb_inner_step(g, solve, Y, P, B, b, dd, 0.0, 1.3)
    expect = (P - B) / np.sqrt(g.D)[:, None]
    assert np.abs(Y1 - expect).max() <= 1e-14 * np.abs(expect).max()
    assert np.all(dd1 == 0.0)                        # infinite threshold


# --- P6: shrink ------------------------------------------------------------------

def test_p6_shrink_is_the_l1_proximal_map():
    gam = 0.37
    eps = np.finfo(np.float64).eps
    y = np.array([0.0, -0.0, gam, -gam, gam * (1 + eps), -gam * (1 + eps), gam * (1 - eps),
                  5.0, -5.0, 1e300, -1e300, 0.1, -0.1, 0.5, -0.5])
    z = O.shrink(y, gam)
    # closed-form soft threshold
    assert np.all(z[np.abs(y) <= gam] == 0.0)
    big = np.abs(y) > gam
    assert np.all(np.sign(z[big]) == np.sign(y[big]))
    # optimality of argmin_z 1/2 (z - y)^2 + gam |z|: y - z in gam * subdiff|z|
    g_ = y - z
    nz = z != 0
    assert np.all(np.abs(g_[nz] - gam * np.sign(z[nz])) <= 1e-15 * np.maximum(1, np.abs(y[nz])))
    assert np.all(np.abs(g_[~nz]) <= gam)
    # brute force on a fine grid for moderate values
    grid = np.linspace(-2, 2, 400001)
    for yy in [0.05, -0.2, 0.37, 0.9, -1.3]:
        zb = grid[np.argmin(0.5 * (grid - yy) ** 2 + gam * np.abs(grid))]
        assert abs(zb - O.shrink(yy, gam)) <= 1e-5
    # Bregman residual t - shrink(t) is the clamp of t to [-gam, gam]
    t = np.linspace(-3, 3, 1001)
    assert np.allclose(t - O.shrink(t, gam), np.clip(t, -gam, gam), atol=4e-16)


# --- Split Bregman reaches the minimiser of the Y-subproblem (Eq. 5) ------------

def test_split_bregman_converges_to_eq5_minimiser():
    g = tiny_graph(6, seed=11, extra=2)
    d, lam, r = 1, 2.0, 1.5
    rng = np.random.default_rng(12)
    P = rng.normal(size=(g.n, d))
    B = 0.2 * rng.normal(size=(g.n, d))
    solve = O.DirectSolver(O.system_matrix(g, lam, r))
    Y = np.zeros((g.n, d))
    b = np.zeros((g.n_edges, d))
    dd = np.zeros((g.n_edges, d))
    for _ in range(3000):
        Y, b, dd = O.sb_inner_step(g, solve, Y, P, B, b, dd, lam, r)
    # independent minimiser of ||M y||_1 + r/2 ||D^{1/2} y - P + B||^2 (Eq. 5) as a
    # smooth QP with slacks s >= |M y|
    M = g.M.toarray()
    E = g.n_edges
    sD = np.sqrt(g.D)
    tgt = (P - B)[:, 0]

    def fun(v):
        y, s = v[:g.n], v[g.n:]
        return s.sum() + r / 2 * np.sum((sD * y - tgt) ** 2)

    def jac(v):
        y = v[:g.n]
        return np.concatenate([r * sD * (sD * y - tgt), np.ones(E)])

    cons = [{"type": "ineq", "fun": lambda v: v[g.n:] - M @ v[:g.n],
             "jac": lambda v: np.hstack([-M, np.eye(E)])},
            {"type": "ineq", "fun": lambda v: v[g.n:] + M @ v[:g.n],
             "jac": lambda v: np.hstack([M, np.eye(E)])}]
    v0 = np.concatenate([tgt / sD, np.abs(M @ (tgt / sD)) + 1.0])
    res = sopt.minimize(fun, v0, jac=jac, constraints=cons, method="SLSQP",
                        options=dict(ftol=1e-15, maxiter=1000))
    err = np.abs(res.x[:g.n] - Y[:, 0]).max()
    print("SB vs QP minimiser", err)
    assert err < 1e-6
    # KKT certificate from the Bregman variable: g = lambda b is a subgradient of |.|
    gsub = lam * b[:, 0]
    assert np.all(np.abs(gsub) <= 1 + 1e-9)
    stat = M.T @ gsub + r * sD * (sD * Y[:, 0] - tgt)
    assert np.abs(stat).max() < 1e-8


def test_stage2_split_bregman_reaches_dual_certified_minimiser():
    """Stage II (Algorithm 2 alone, P and B frozen) converges, for any split
    penalty lambda, to the minimiser of ||M Y||_1 + r/2 ||D^{1/2} Y - P + B||^2,
    column by column.  The minimiser comes from the dual problem, a box-constrained
    QP over |z| <= 1 (||M y||_1 = max z^T M y) solved by L-BFGS-B, with
    y = D^{-1/2} (q - D^{-1/2} M^T z / r); the primal-dual gap certifies it."""
    g = tiny_graph(12, seed=21, extra=6)
    d, r = 3, 1.2
    rng = np.random.default_rng(22)
    P = rng.normal(size=(g.n, d))
    B = 0.3 * rng.normal(size=(g.n, d))
    M = g.M.toarray()
    sD = np.sqrt(g.D)
    K = M / sD[None, :]
    H = K @ K.T / r
    Ystar = np.zeros((g.n, d))
    for k in range(d):
        q = (P - B)[:, k]
        c = K @ q
        res = sopt.minimize(lambda z: (0.5 * z @ H @ z - z @ c, H @ z - c), np.zeros(g.n_edges), jac=True,
                            method="L-BFGS-B", bounds=[(-1.0, 1.0)] * g.n_edges,
                            options=dict(ftol=1e-16, gtol=1e-13, maxiter=20000, maxcor=50))
        z = res.x
        y = (q - K.T @ z / r) / sD
        primal = np.abs(M @ y).sum() + r / 2 * np.sum((sD * y - q) ** 2)
        dual = c @ z - 0.5 * z @ H @ z
        print(f"column {k}: primal {primal:.12f}, duality gap {primal - dual:.2e}")
        assert primal - dual <= 1e-7 * primal
        Ystar[:, k] = y
    for lam in (0.7, 2.0, 5.0):
        solve = O.DirectSolver(O.system_matrix(g, lam, r))
        Y, b, dd = O.split_bregman(g, solve, np.zeros((g.n, d)), P, B, lam, r, 1000)
        err = np.abs(Y - Ystar).max()
        print(f"lambda {lam}: Stage II after 1000 iterations vs dual minimiser {err:.2e}")
        assert err <= 1e-7
        # the split variables are consistent with the edge differences at the limit
        assert np.abs(dd - g.M @ Y).max() <= 1e-6


# --- P7/P8: P-update ---------------------------------------------------------------

def test_p7_polar_update_properties():
    rng = np.random.default_rng(13)
    Z = rng.normal(size=(40, 5))
    P = O.p_update(Z, "polar")
    assert np.abs(P.T @ P - np.eye(5)).max() < 1e-13
    S = P.T @ Z
    assert np.abs(S - S.T).max() < 1e-12                 # P^T Z symmetric ...
    assert np.linalg.eigvalsh(0.5 * (S + S.T)).min() > 0  # ... positive definite
    # minimiser: no random orthonormal Q is closer to Z
    best = np.linalg.norm(P - Z)
    for k in range(200):
        Q, _ = np.linalg.qr(rng.normal(size=(40, 5)))
        assert np.linalg.norm(Q - Z) >= best
        Qp = sla.expm(1e-3 * (lambda X: X - X.T)(rng.normal(size=(5, 5))))
        assert np.linalg.norm(P @ Qp - Z) >= best       # nearby feasible points too
    # already orthonormal Z is returned unchanged
    Q, _ = np.linalg.qr(rng.normal(size=(40, 5)))
    assert np.abs(O.p_update(Q, "polar") - Q).max() < 1e-13
    # Cholesky mode: orthonormal, same column space, upper-triangular map
    Pc = O.p_update(Z, "chol")
    assert np.abs(Pc.T @ Pc - np.eye(5)).max() < 1e-12
    Rm = np.linalg.lstsq(Pc, Z, rcond=None)[0]
    assert np.abs(np.tril(Rm, -1)).max() < 1e-12 and np.all(np.diag(Rm) > 0)
    assert np.abs(Pc @ Rm - Z).max() < 1e-12


def test_p8_constraint_after_every_outer_step():
    wl = synth.make_workload("voronoi64_4nbr", 0)
    g = O.build_grid_graph(wl.feat, wl.H, wl.W, wl.stencil, wl.sigma)
    for mode in ("polar", "chol"):
        st = O.pfe_run(g, wl.y0, 1.0, 1.0, 4, 3, mode=mode, monitor=True)
        for h in st.history:
            assert h["constraint"] < 1e-10


# --- P9: disconnected cliques --------------------------------------------------------

def clique_graph(sizes, seed=0):
    rng = np.random.default_rng(seed)
    ei, ej, base = [], [], 0
    for s in sizes:
        for a in range(s):
            for b in range(a + 1, s):
                ei.append(base + a)
                ej.append(base + b)
        base += s
    w = rng.uniform(0.3, 1.0, size=len(ei))
    return O.Graph(base, np.array(ei), np.array(ej), w)


@pytest.mark.parametrize("mode", ["polar", "chol"])
def test_p9_clique_indicators_are_a_zero_objective_fixed_point(mode):
    sizes = [5, 7, 4, 6]
    g = clique_graph(sizes, seed=1)
    d = len(sizes)
    Y0 = np.zeros((g.n, d))
    base = 0
    for k, s in enumerate(sizes):
        Y0[base:base + s, k] = 1.0
        base += s
    Y0 = Y0 / np.sqrt(np.einsum("ij,i,ij->j", Y0, g.D, Y0))[None, :]
    assert O.objective(g, Y0) == 0.0
    solve = O.DirectSolver(O.system_matrix(g, 2.0, 1.0))
    P0 = np.sqrt(g.D)[:, None] * Y0
    B0 = np.zeros_like(Y0)
    Y1, P1, B1, b, dd = O.soc_outer_step(g, solve, Y0, P0, B0, 2.0, 1.0, 4, mode,
                                         return_split=True)
    assert np.abs(Y1 - Y0).max() <= 1e-13
    assert np.abs(P1 - P0).max() <= 1e-13
    assert np.abs(B1).max() <= 1e-13
    assert np.abs(b).max() <= 1e-13 and np.abs(dd).max() <= 1e-13
    assert O.objective(g, P1 / np.sqrt(g.D)[:, None]) <= 1e-13


# --- P10: Laplacian eigenmaps ---------------------------------------------------------

def test_p10_le_init_dense_and_sparse_agree_with_generalised_eigenproblem():
    wl = synth.grid_workload("t", 30, 34, 4, 0.05, 3, stencil=4, d=3)
    g = O.build_grid_graph(wl.feat, wl.H, wl.W, wl.stencil, wl.sigma)
    Yd, mud = O.le_init(g, 3, dense_max=10**9)
    Ys, mus = O.le_init(g, 3, dense_max=0)
    Lap = (sp.diags(g.D) - g.adjacency()).toarray()
    for Y, mu in ((Yd, mud), (Ys, mus)):
        res = Lap @ Y - (g.D[:, None] * Y) * mu[None, :]
        assert np.abs(res).max() < 1e-9
        assert np.abs(Y.T @ (g.D[:, None] * Y) - np.eye(3)).max() < 1e-10
    # same eigenvalues; same subspace (projector Y Y^T D)
    ev = sla.eigh(Lap, np.diag(g.D), eigvals_only=True)
    assert np.allclose(mud, ev[1:4], rtol=0, atol=1e-10)
    assert np.allclose(mus, ev[1:4], rtol=0, atol=1e-10)
    Pd = Yd @ (Yd.T * g.D[None, :])
    Ps = Ys @ (Ys.T * g.D[None, :])
    assert np.abs(Pd - Ps).max() < 1e-8


# --- P11: invariances ----------------------------------------------------------------

def test_p11_permutation_orientation_and_zero_weight_edges():
    g = tiny_graph(14, seed=21, extra=8)
    d, lam, r = 3, 2.0, 1.0
    rng = np.random.default_rng(22)
    Y0 = rng.normal(size=(g.n, d))
    ref = O.pfe_run(g, Y0, lam, r, 3, 3)
    # vertex permutation
    perm = rng.permutation(g.n)
    inv = np.argsort(perm)                       # new index of old vertex
    a, b = inv[g.ei], inv[g.ej]
    gp = O.Graph(g.n, np.minimum(a, b), np.maximum(a, b), g.w)
    Y0p = np.empty_like(Y0)
    Y0p[inv] = Y0
    st = O.pfe_run(gp, Y0p, lam, r, 3, 3)
    assert np.abs(st.Y[inv] - ref.Y).max() < 1e-12
    assert np.abs(st.P[inv] - ref.P).max() < 1e-12
    # flipping the orientation of every row of M (i.e. using -M)
    gf = O.Graph(g.n, g.ei, g.ej, g.w)
    gf.M = -gf.M
    st = O.pfe_run(gf, Y0, lam, r, 3, 3)
    assert np.abs(st.Y - ref.Y).max() < 1e-12
    # extra edges of zero weight
    ei = np.concatenate([g.ei, [0, 2]])
    ej = np.concatenate([g.ej, [13, 9]])
    w = np.concatenate([g.w, [0.0, 0.0]])
    o = np.lexsort((ej, ei))
    gz = O.Graph(g.n, ei[o], ej[o], w[o])
    st = O.pfe_run(gz, Y0, lam, r, 3, 3)
    assert np.abs(st.Y - ref.Y).max() < 1e-12
    assert np.abs(st.B - ref.B).max() < 1e-12


# --- P12: the memory example of Sec. III ---------------------------------------------

def test_p12_memory_example_matches_paper():
    with open(os.path.join(HERE, "golden", "memory_example.json")) as f:
        gold = json.load(f)
    m = O.kronecker_memory(gold["n"], gold["d"], gold["edges_per_vertex"])
    assert m["M_shape"] == (gold["M_rows"], gold["M_cols"])
    assert m["M_nnz"] == gold["M_nnz"]
    assert m["L_shape"] == (gold["L_rows"], gold["L_cols"])
    assert m["L_nnz"] == gold["L_nnz"]
    assert m["Dt_shape"] == (gold["Dt_rows"], gold["Dt_cols"])
    MiB = 2 ** 20
    assert m["W_bytes"] == 0.5 * MiB
    assert m["Y_bytes"] == 8 * MiB
    assert m["M_bytes"] == 1 * MiB
    assert m["L_bytes"] == 64 * MiB
    assert m["Dt_bytes"] == 8 * MiB
    assert m["inverse_bytes"] == 8 * 2 ** 40
    # the paper's count differs from an open 128x128 grid's true edge count
    i, j = O.grid_edges(128, 128, 4)
    assert len(i) == 32512


# --- P13: PCG -------------------------------------------------------------------------

def test_p13_pcg_error_and_iteration_bound():
    wl = synth.grid_workload("t", 24, 20, 4, 0.05, 5, stencil=8, d=3)
    g = O.build_grid_graph(wl.feat, wl.H, wl.W, wl.stencil, wl.sigma)
    rng = np.random.default_rng(1)
    for lam, r in ((1.0, 1.0), (10.0, 1.0), (100.0, 1.0)):
        A = O.system_matrix(g, lam, r)
        kappa = O.jacobi_condition_number(A)
        rhs = rng.normal(size=(g.n, 3))
        exact = np.linalg.solve(A.toarray(), rhs)
        tol = 1e-8
        x, it, rel = O.pcg(A, rhs, np.zeros_like(rhs), 1.0 / A.diagonal(), tol, 5000)
        assert np.all(rel <= tol)
        # ||x - x*||_A <= 2 ((sqrt k - 1)/(sqrt k + 1))^k ||x*||_A -> iterations bound
        bound = math.ceil(0.5 * math.sqrt(kappa) * math.log(2 * math.sqrt(kappa) / tol)) + 1
        print(f"lam/r={lam/r} kappa={kappa:.2f} iters={it.max()} bound={bound}")
        assert it.max() <= bound
        err = np.linalg.norm(x - exact, axis=0) / np.linalg.norm(exact, axis=0)
        assert np.all(err <= kappa * tol * 2)
    # zero right-hand side column gives x = 0 without iterating
    x, it, _ = O.pcg(A, np.zeros((g.n, 1)), np.ones((g.n, 1)), 1.0 / A.diagonal(), 1e-8, 10)
    assert np.all(x == 0) and it[0] == 0


def test_cg_solver_matches_direct():
    wl = synth.make_workload("voronoi64_4nbr", 0)
    g = O.build_grid_graph(wl.feat, wl.H, wl.W, wl.stencil, wl.sigma)
    A = O.system_matrix(g, 5.0, 1.0)
    rhs = np.random.default_rng(3).normal(size=(g.n, 4))
    xd = O.DirectSolver(A)(rhs)
    xc = O.CGSolver(A, tol=1e-13)(rhs)
    assert np.abs(xd - xc).max() <= 1e-11 * np.abs(xd).max()


def test_shrink_active_scale_sets_threshold_at_quantile():
    wl = synth.make_workload("voronoi96x80_8nbr", 0)
    g = O.build_grid_graph(wl.feat, wl.H, wl.W, wl.stencil, wl.sigma)
    Y = O.orthonormalize_init(g, wl.y0)
    c = O.shrink_active_scale(g, Y, 0.99)
    v = np.abs(g.M @ Y)
    frac = np.mean(v > 1.0 / c)
    assert 0.005 < frac <= 0.0101


def test_kmeans_agreement_is_one_for_identical_embeddings():
    rng = np.random.default_rng(0)
    Y = np.concatenate([rng.normal(k * 5, 0.1, size=(50, 2)) for k in range(3)])
    frac, _ = O.kmeans_agreement(Y, Y, 3)
    assert frac == 1.0
    # label permutation invariance: relabelled but same partition
    frac2, _ = O.kmeans_agreement(Y, Y[:, ::-1].copy(), 3)
    assert frac2 == 1.0


# --- objective: Eq. (5)'s l1 term, once per undirected edge ------------------

def test_objective_hand_computed_once_per_edge():
    """4 vertices, 4 edges, values chosen so every term is exact in binary:
      (0,1) w=0.5 : |0-2| + |1-1|  = 2 -> 1.0
      (0,2) w=0.25: |0-1| + |1+1|  = 3 -> 0.75
      (1,3) w=1   : |2-2| + |1-3|  = 2 -> 2.0
      (2,3) w=2   : |1-2| + |-1-3| = 5 -> 10.0
    ||M Y||_1 = 13.75 (each undirected edge once, Eq. 5); Eq. (1)'s sum over
    ordered pairs (i, j) counts every edge from both ends: 27.5."""
    g = O.Graph(4, np.array([0, 0, 1, 2]), np.array([1, 2, 3, 3]),
                np.array([0.5, 0.25, 1.0, 2.0]))
    Y = np.array([[0.0, 1.0], [2.0, 1.0], [1.0, -1.0], [2.0, 3.0]])
    assert O.objective(g, Y) == 13.75
    # Eq. (1): sum over all ordered pairs with the symmetric W
    Wd = g.adjacency().toarray()
    eq1 = sum(Wd[i, j] * np.abs(Y[i] - Y[j]).sum() for i in range(4) for j in range(4))
    assert eq1 == 27.5
    assert O.objective(g, Y) == 0.5 * eq1
    # a constant shift of Y and a sign flip of a column leave it unchanged
    assert O.objective(g, Y + 3.0) == 13.75
    assert O.objective(g, Y * np.array([1.0, -1.0])) == 13.75
