"""Pins for the oracle's classical preconditioners (IC(0), the paper's
preconditioner, and FSAI), each against something other than its own
recurrence: the exact Cholesky factor where IC(0) drops no fill, the exact
inverse factor where FSAI's pattern holds it, the defining equations checked by
sparse products, and preconditioned PCG against a direct solve."""
import numpy as np
import scipy.sparse as sp

import oracle as O
from oracle import classical as C
from oracle.learned import pcg_preconditioned


def path_system(n=40, seed=0):
    rng = np.random.default_rng(seed)
    ei = np.arange(n - 1)
    g = O.Graph(n, ei, ei + 1, rng.uniform(0.2, 1.0, n - 1))
    return O.system_matrix(g, 30.0, 1.0).tocsr()


def grid_system(H=9, W=11, stencil=8, lam=50.0, r=1.0, seed=0):
    rng = np.random.default_rng(seed)
    feat = rng.uniform(0, 1, size=(H * W, 3))
    g = O.build_grid_graph(feat, H, W, stencil, 0.3)
    return O.system_matrix(g, lam, r).tocsr()


def test_ic0_is_exact_cholesky_when_no_fill_is_dropped():
    # a path (tridiagonal A) and a star with its hub numbered last (arrow
    # matrix): Cholesky creates no fill, so IC(0) must be the exact factor
    A1 = path_system()
    n = 12
    rng = np.random.default_rng(3)
    g = O.Graph(n, np.arange(n - 1), np.full(n - 1, n - 1), rng.uniform(0.2, 1.0, n - 1))
    A2 = O.system_matrix(g, 10.0, 1.0).tocsr()
    for A in (A1, A2):
        L = C.ic0(A).toarray()
        Lx = np.linalg.cholesky(A.toarray())
        err = np.abs(L - Lx).max() / np.abs(Lx).max()
        print(f"IC(0) vs Cholesky {err:.2e}")
        assert err <= 1e-14


def test_ic0_defining_equations_on_grid_system():
    A = grid_system()
    L = C.ic0(A)
    lowA = sp.tril(A).tocsr()
    # same pattern as the lower triangle of A
    assert np.array_equal((abs(L) > 0).astype(int).toarray(), (abs(lowA) > 0).astype(int).toarray())
    LLt = (L @ L.T).toarray()
    Ad = A.toarray()
    mask = lowA.toarray() != 0
    err = np.abs(LLt - Ad)[mask].max() / np.abs(Ad).max()
    dropped = np.abs(LLt - Ad)[~mask & np.tril(np.ones_like(mask), -1).astype(bool)].max()
    print(f"(L L^T - A) on the pattern {err:.2e}; dropped fill reaches {dropped:.2e}")
    assert err <= 1e-13
    assert dropped > 1e-6          # fill was dropped: this is not the exact factor


def test_fsai_full_pattern_is_the_exact_inverse_factor():
    rng = np.random.default_rng(4)
    X = rng.normal(size=(9, 9))
    A = sp.csr_matrix(X @ X.T + 9 * np.eye(9))
    G = C.fsai(A).toarray()
    L = np.linalg.cholesky(A.toarray())
    err = np.abs(G - np.linalg.inv(L)).max()
    print(f"FSAI (full pattern) vs L^-1 {err:.2e}")
    assert err <= 1e-13
    assert np.abs(G.T @ G - np.linalg.inv(A.toarray())).max() <= 1e-13


def test_fsai_defining_equations_on_grid_system():
    A = grid_system(stencil=-2)
    G = C.fsai(A)
    lowA = sp.tril(A).tocsr()
    assert np.array_equal((abs(G) > 0).astype(int).toarray(), (abs(lowA) > 0).astype(int).toarray())
    GA = (G @ A).toarray()
    mask = (lowA.toarray() != 0) & ~np.eye(A.shape[0], dtype=bool)
    off = np.abs(GA[mask]).max()
    dg = np.abs(np.diag((G @ A @ G.T).toarray()) - 1).max()
    print(f"(G A) off the diagonal on the pattern {off:.2e}; diag(G A G^T) - 1 {dg:.2e}")
    assert off <= 1e-12 and dg <= 1e-12
    # fsai_row gives the same row as the whole-matrix routine
    S, g = C.fsai_row(A, 57)
    assert np.allclose(G[57, S].toarray().ravel(), g, rtol=0, atol=1e-15)


def test_ic0_and_fsai_pcg_reach_the_direct_solution():
    A = grid_system(H=20, W=23, lam=300.0)
    rhs = np.random.default_rng(6).normal(size=(A.shape[0], 3))
    exact = O.DirectSolver(A)(rhs)
    kappa = O.jacobi_condition_number(A)
    tol = 1e-10
    counts = {}
    for name, ap in (("jacobi", lambda r: r / A.diagonal()[:, None]), ("ic0", C.ic0_apply(C.ic0(A))),
                     ("fsai", C.fsai_apply(C.fsai(A)))):
        x, it = pcg_preconditioned(A, rhs, np.zeros_like(rhs), ap, tol, 5000)
        e = np.linalg.norm(x - exact) / np.linalg.norm(exact)
        counts[name] = int(it.max())
        assert e <= kappa * tol * 4, (name, e)
    print("PCG iterations", counts)
    assert counts["ic0"] < counts["jacobi"] and counts["fsai"] < counts["jacobi"]
