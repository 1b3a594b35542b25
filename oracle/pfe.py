"""FP64 oracle for piecewise flat embeddings (PFE) — test infrastructure only.

What it computes, with the passage each piece follows:

* Graph and weights — Sec. II (background): heat-kernel weights
  w_ij = exp(-||x_i - x_j||^2 / (2 sigma^2)) on the graph's edges; degree matrix
  D = diag(W 1) (Eq. 1 and Algorithm 1, degree step).
* M — Sec. II, definition of the edge-difference matrix: one row per edge
  (i, j), i < j, holding +w_ij in column i and -w_ij in column j.  Only edges of
  the neighbourhood graph are kept (rows of zero weight are inert).
* System matrix — Eq. (13): A = lambda/2 M^T M + r/2 D, the same for all d
  columns and for every inner solve.
* Split Bregman (Algorithm 2 with Eqs. (9), (10), (13)): per inner step
  rhs = lambda/2 M^T (d - b) + r/2 D^{1/2} (P - B), Y = A^{-1} rhs,
  t = M Y + b, d = Shrink(t, 1/lambda), b = t - d.
  Reading of the right-hand side: Eq. (6)/(13) print Q2 = B - P; the
  stationarity condition of the least-squares objective in Algorithm 2 gives
  P - B, which is used here (pinned by tests: argmin check and lambda = 0 case).
* Stage II (Sec. IV, experiments): after the SOC iterations, Split-Bregman
  iterations alone with the orthogonality constraint relaxed; read as
  Algorithm 2 run with P and B frozen at their final values.
* SOC outer loop (Algorithm 1): b and d start at zero for every outer step;
  Z = D^{1/2} Y + B; P = argmin ||P - Z|| s.t. P^T P = I, i.e. the polar factor
  of Z (default), or the Cholesky-QR factor Z R^{-1} (option); B = Z - P.
  Reading: Algorithm 1's Y-update prints "- P + P"; it is read as "- P + B",
  as in Eq. (5) and Algorithm 2.
* PCG — Sec. III (last paragraph): the d systems of Eq. (13) solved together,
  here as d independent preconditioned CG recurrences (Barrett et al.'s
  template), each column frozen once ||r_c|| <= tol ||rhs_c||.
* Laplacian-eigenmap initialisation — Sec. I: (D - W) y = mu D y, vectors
  2..d+1, D-normalised, sign fixed so the largest-magnitude entry is positive.

Layouts: Y, P, B are n x d float64; the split variables b and d ("dd" here, to
keep it apart from the dimension d) are |E| x d with rows in the edge order
(i, j), i < j, sorted lexicographically.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

__all__ = [
    "grid_edges", "heat_kernel", "Graph", "build_grid_graph", "build_edge_graph",
    "system_matrix", "shrink", "sb_rhs", "DirectSolver", "CGSolver", "pcg",
    "sb_inner_step", "split_bregman", "p_update", "soc_outer_step", "orthonormalize_init",
    "PFEState", "pfe_run", "objective", "constraint_residual", "split_residual",
    "le_init", "shrink_active_scale", "kron_L", "kron_Dt", "vec", "unvec",
    "kronecker_memory", "kmeans_agreement", "jacobi_condition_number",
]


# ----------------------------------------------------------------------------
# Graph construction (Sec. II)
# ----------------------------------------------------------------------------

def grid_offsets(stencil: int):
    """Forward neighbour offsets (dy, dx) of a pixel grid: those whose linear
    offset dy*W + dx is positive.  stencil 4 / 8 are the 4- and 8-neighbourhoods;
    stencil -R is the (2R+1)^2 window minus its centre (Chebyshev radius R)."""
    if stencil == 4:
        offs = [(0, 1), (1, 0)]
    elif stencil == 8:
        offs = [(0, 1), (1, -1), (1, 0), (1, 1)]
    elif stencil < 0:
        R = -stencil
        offs = [(dy, dx) for dy in range(0, R + 1) for dx in range(-R, R + 1)
                if (dy > 0 or dx > 0)]
    else:
        raise ValueError(f"unsupported stencil {stencil}")
    return offs


def grid_edges(H: int, W: int, stencil: int):
    """Undirected edges (i, j), i < j, of the pixel grid, sorted lexicographically.
    Vertex index is y*W + x."""
    ii, jj = [], []
    ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    for dy, dx in grid_offsets(stencil):
        y2, x2 = ys + dy, xs + dx
        ok = (y2 >= 0) & (y2 < H) & (x2 >= 0) & (x2 < W)
        ii.append((ys * W + xs)[ok])
        jj.append((y2 * W + x2)[ok])
    i = np.concatenate(ii).astype(np.int64)
    j = np.concatenate(jj).astype(np.int64)
    order = np.lexsort((j, i))
    return i[order], j[order]


def heat_kernel(dist2, sigma: float):
    """w = exp(-||x_i - x_j||^2 / (2 sigma^2))  (Sec. II, heat kernel)."""
    return np.exp(-np.asarray(dist2, dtype=np.float64) / (2.0 * sigma * sigma))


@dataclass
class Graph:
    n: int
    ei: np.ndarray            # |E| lower endpoints
    ej: np.ndarray            # |E| upper endpoints (ei < ej)
    w: np.ndarray             # |E| weights, float64
    D: np.ndarray = field(init=False)       # degrees d_i = sum_j w_ij
    M: sp.csr_matrix = field(init=False)    # |E| x n edge-difference matrix

    def __post_init__(self):
        if np.any(self.ei >= self.ej):
            raise ValueError("edges must satisfy i < j")
        E = len(self.w)
        # D = diag(W 1): each undirected edge adds w to both endpoints (Eq. 1).
        self.D = (np.bincount(self.ei, weights=self.w, minlength=self.n)
                  + np.bincount(self.ej, weights=self.w, minlength=self.n))
        if np.any(self.D <= 0.0):
            raise ValueError("isolated vertex: a zero degree makes A singular")
        rows = np.concatenate([np.arange(E), np.arange(E)])
        cols = np.concatenate([self.ei, self.ej])
        vals = np.concatenate([self.w, -self.w])
        self.M = sp.csr_matrix((vals, (rows, cols)), shape=(E, self.n))

    @property
    def n_edges(self) -> int:
        return len(self.w)

    def adjacency(self) -> sp.csr_matrix:
        Wm = sp.csr_matrix((self.w, (self.ei, self.ej)), shape=(self.n, self.n))
        return (Wm + Wm.T).tocsr()


def build_grid_graph(feat, H: int, W: int, stencil: int, sigma: float) -> Graph:
    """Pixel graph: one vertex per pixel, edges inside the stencil, heat-kernel
    weights on the feature rows (Sec. II; Sec. IV uses RGB on a 4-neighbourhood)."""
    x = np.asarray(feat, dtype=np.float64).reshape(H * W, -1)
    i, j = grid_edges(H, W, stencil)
    diff = x[i] - x[j]
    w = heat_kernel(np.einsum("ij,ij->i", diff, diff), sigma)
    return Graph(H * W, i, j, w)


def build_edge_graph(n: int, src, dst, dist2, sigma: float) -> Graph:
    """Graph from an undirected edge list with squared distances."""
    a = np.asarray(src, dtype=np.int64)
    b = np.asarray(dst, dtype=np.int64)
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    order = np.lexsort((hi, lo))
    return Graph(n, lo[order], hi[order], heat_kernel(np.asarray(dist2)[order], sigma))


# ----------------------------------------------------------------------------
# Operators (Eqs. 7-13) and the shrink of Algorithm 2
# ----------------------------------------------------------------------------

def system_matrix(g: Graph, lam: float, r: float) -> sp.csc_matrix:
    """A = lambda/2 M^T M + r/2 D   (Eq. 13)."""
    return (0.5 * lam * (g.M.T @ g.M) + 0.5 * r * sp.diags(g.D)).tocsc()


def shrink(y, gamma):
    """Shrink(y, gamma) = sign(y) * max(|y| - gamma, 0), elementwise (Algorithm 2)."""
    y = np.asarray(y, dtype=np.float64)
    return np.sign(y) * np.maximum(np.abs(y) - gamma, 0.0)


def sb_rhs(g: Graph, P, B, b, dd, lam: float, r: float):
    """Right-hand side of Eq. (13): lambda/2 M^T Q1 + r/2 D^{1/2} Q2 with
    Q1 = d - b (Eq. 13) and Q2 = P - B (sign reading, see module docstring)."""
    return 0.5 * lam * (g.M.T @ (dd - b)) + 0.5 * r * np.sqrt(g.D)[:, None] * (P - B)


class DirectSolver:
    """Sparse direct solve of A Y = rhs; A is factored once (it does not change
    between inner solves, Eq. 13)."""

    def __init__(self, A):
        self.A = A.tocsc()
        self.lu = spla.splu(self.A)
        self.last_iters = None

    def __call__(self, rhs, x0=None):
        return self.lu.solve(np.asarray(rhs, dtype=np.float64))


def pcg(A, rhs, x0, minv_diag=None, tol=1e-12, maxit=10000):
    """Preconditioned CG on the d columns of rhs, each its own recurrence
    (Barrett et al., PCG template).  Preconditioner: z = minv_diag * r (Jacobi
    when minv_diag = 1/diag(A)); None means no preconditioning.

    A column stops when ||r_c|| <= tol ||rhs_c||; a zero right-hand side gives
    x_c = 0.  Returns (x, iterations per column, final relative residuals).
    """
    rhs = np.asarray(rhs, dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    d = rhs.shape[1]
    bnorm = np.linalg.norm(rhs, axis=0)
    zero = bnorm == 0.0
    x[:, zero] = 0.0
    r = rhs - A @ x
    iters = np.zeros(d, dtype=np.int64)
    active = ~zero & (np.linalg.norm(r, axis=0) > tol * bnorm)
    p = np.zeros_like(x)
    rho_old = np.ones(d)
    for _ in range(maxit):
        if not active.any():
            break
        z = r * minv_diag[:, None] if minv_diag is not None else r.copy()
        rho = np.einsum("ij,ij->j", r, z)
        first = iters == 0
        beta = np.where(first, 0.0, rho / np.where(first, 1.0, rho_old))
        p = np.where(active[None, :], z + beta[None, :] * p, p)
        q = A @ p
        pq = np.einsum("ij,ij->j", p, q)
        alpha = np.where(active, rho / np.where(active, pq, 1.0), 0.0)
        x += alpha[None, :] * p
        r -= alpha[None, :] * q
        rho_old = np.where(active, rho, rho_old)
        iters += active
        active &= np.linalg.norm(r, axis=0) > tol * bnorm
    rel = np.where(zero, 0.0, np.linalg.norm(r, axis=0) / np.where(zero, 1.0, bnorm))
    return x, iters, rel


class CGSolver:
    """The oracle's own FP64 Jacobi-PCG, for graphs too large to factor."""

    def __init__(self, A, tol=1e-12, maxit=20000):
        self.A = A.tocsr()
        self.minv = 1.0 / self.A.diagonal()
        self.tol, self.maxit = tol, maxit
        self.last_iters = None

    def __call__(self, rhs, x0=None):
        if x0 is None:
            x0 = np.zeros_like(rhs)
        x, it, _ = pcg(self.A, rhs, x0, self.minv, self.tol, self.maxit)
        self.last_iters = it
        return x


# ----------------------------------------------------------------------------
# Algorithms 1 and 2
# ----------------------------------------------------------------------------

def sb_inner_step(g: Graph, solve, Y, P, B, b, dd, lam: float, r: float):
    """One Split-Bregman iteration in the compact form (Algorithm 2 with
    Eq. 13 for the least-squares step and Eqs. 9-10 for the shrink and Bregman
    steps).  Returns (Y, b, dd) of the next iteration."""
    rhs = sb_rhs(g, P, B, b, dd, lam, r)
    Y = solve(rhs, Y)
    t = g.M @ Y + b                                      # vec(M Y) + b
    gamma = np.inf if lam == 0 else 1.0 / lam
    dd_new = shrink(t, gamma)                            # Eq. 9
    b_new = t - dd_new                                   # Eq. 10
    return Y, b_new, dd_new


def p_update(Z, mode: str = "polar"):
    """argmin_P ||P - Z||_F s.t. P^T P = I (Algorithm 1, P-update).

    'polar': the orthogonal polar factor U V^T from the thin SVD Z = U S V^T,
    which is the exact minimiser.  'chol': Cholesky QR, Z R^{-1} with
    R^T R = Z^T Z (feasible, not the minimiser)."""
    Z = np.asarray(Z, dtype=np.float64)
    if mode == "polar":
        U, _, Vt = np.linalg.svd(Z, full_matrices=False)
        return U @ Vt
    if mode == "chol":
        R = np.linalg.cholesky(Z.T @ Z).T      # upper triangular
        return sla.solve_triangular(R, Z.T, trans="T", lower=False).T
    raise ValueError(mode)


def split_bregman(g: Graph, solve, Y, P, B, lam: float, r: float, n_iter: int):
    """SplitBregman(M, D, P, B) of Algorithm 2 for a fixed number of
    iterations: b = d = 0 at the start, then n_iter inner steps with P and B
    held fixed.  Returns (Y, b, dd) after the last step.

    This is both the Y-update inside a SOC iteration and, run on its own with
    the final P and B, Stage II of the two-stage procedure of the experiments
    (Sec. IV: orthogonality no longer enforced, only Split-Bregman iterations;
    reading: P and B frozen at the values Stage I ends with)."""
    d = Y.shape[1]
    b = np.zeros((g.n_edges, d))
    dd = np.zeros((g.n_edges, d))
    for _ in range(n_iter):
        Y, b, dd = sb_inner_step(g, solve, Y, P, B, b, dd, lam, r)
    return Y, b, dd


def soc_outer_step(g: Graph, solve, Y, P, B, lam, r, n_inner, mode="polar",
                   return_split=False):
    """One SOC iteration (Algorithm 1): the Y-update by n_inner Split-Bregman
    iterations started from b = d = 0 (Algorithm 2 initialisation), then the
    P-update and the B-update."""
    Y, b, dd = split_bregman(g, solve, Y, P, B, lam, r, n_inner)
    Z = np.sqrt(g.D)[:, None] * Y + B
    P = p_update(Z, mode)
    B = Z - P
    if return_split:
        return Y, P, B, b, dd
    return Y, P, B


def orthonormalize_init(g: Graph, Y0):
    """Y0 <- Y0 R^{-1}, R^T R = Y0^T D Y0 (Cholesky), so that Y^T D Y = I."""
    Y0 = np.asarray(Y0, dtype=np.float64)
    G = Y0.T @ (g.D[:, None] * Y0)
    R = np.linalg.cholesky(G).T
    return sla.solve_triangular(R, Y0.T, trans="T", lower=False).T


@dataclass
class PFEState:
    Y: np.ndarray
    P: np.ndarray
    B: np.ndarray
    history: list = field(default_factory=list)

    def yhat(self, g: Graph):
        """Feasible embedding D^{-1/2} P, which satisfies Yhat^T D Yhat = I."""
        return self.P / np.sqrt(g.D)[:, None]


def pfe_run(g: Graph, Y0, lam, r, n_outer, n_inner, mode="polar",
            orthonormalize=True, solver=None, monitor=False) -> PFEState:
    """SOC (Algorithm 1) with its Y-update by Split Bregman (Algorithm 2), for
    fixed iteration counts.  Initialisation: P = D^{1/2} Y0, B = 0."""
    Y = orthonormalize_init(g, Y0) if orthonormalize else np.asarray(Y0, np.float64)
    P = np.sqrt(g.D)[:, None] * Y
    B = np.zeros_like(Y)
    solve = solver if solver is not None else DirectSolver(system_matrix(g, lam, r))
    st = PFEState(Y, P, B)
    for _ in range(n_outer):
        Y, P, B = soc_outer_step(g, solve, Y, P, B, lam, r, n_inner, mode)
        st = PFEState(Y, P, B, st.history)
        if monitor:
            yh = st.yhat(g)
            st.history.append(dict(objective=objective(g, yh),
                                   constraint=constraint_residual(g, yh),
                                   split=split_residual(g, Y, P)))
    return st


# ----------------------------------------------------------------------------
# Monitors
# ----------------------------------------------------------------------------

def objective(g: Graph, Y):
    """||M Y||_1 = sum over undirected edges of w_ij ||y_i - y_j||_1 (Eq. 5's
    l1 term; Eq. 1 counts each edge twice)."""
    return float(np.abs(g.M @ Y).sum())


def constraint_residual(g: Graph, Y):
    """max |Y^T D Y - I| (Eq. 1 constraint)."""
    d = Y.shape[1]
    return float(np.abs(Y.T @ (g.D[:, None] * Y) - np.eye(d)).max())


def split_residual(g: Graph, Y, P):
    """||D^{1/2} Y - P||_F / ||P||_F (Eq. 2 split constraint)."""
    return float(np.linalg.norm(np.sqrt(g.D)[:, None] * Y - P) / np.linalg.norm(P))


def shrink_active_scale(g: Graph, Y, q: float = 0.99):
    """c = 1 / (q-quantile of |M Y|) (order statistic floor(q (N-1)) of the
    sorted values).  Using lambda = r = c keeps the conditioning of A and puts
    the shrink threshold 1/lambda at that quantile."""
    v = np.sort(np.abs(g.M @ Y).reshape(-1))
    return 1.0 / v[int(np.floor(q * (v.size - 1)))]


# ----------------------------------------------------------------------------
# Laplacian eigenmaps initialisation (Sec. I)
# ----------------------------------------------------------------------------

def le_init(g: Graph, d: int, dense_max: int = 2500):
    """Eigenvectors 2..d+1 of (D - W) y = mu D y, scaled so y^T D y = 1, with the
    largest-magnitude entry of each made positive.  Returns (Y, mu)."""
    Wm = g.adjacency()
    Lap = (sp.diags(g.D) - Wm).tocsc()
    Dm = sp.diags(g.D).tocsc()
    if g.n <= dense_max:
        mu, V = sla.eigh(Lap.toarray(), np.diag(g.D))
        mu, V = mu[1:d + 1], V[:, 1:d + 1]
    else:
        mu, V = spla.eigsh(Lap, k=d + 1, M=Dm, sigma=-1e-8, which="LM")
        order = np.argsort(mu)
        mu, V = mu[order][1:d + 1], V[:, order][:, 1:d + 1]
    V = V / np.sqrt(np.einsum("ij,i,ij->j", V, g.D, V))[None, :]
    idx = np.argmax(np.abs(V), axis=0)
    V = V * np.sign(V[idx, np.arange(d)])[None, :]
    return V, mu


# ----------------------------------------------------------------------------
# Kronecker (vectorised) forms, Eqs. (3)-(6) — small graphs only
# ----------------------------------------------------------------------------

def vec(Z):
    """Stack the columns of Z (Sec. III definition of vec)."""
    return np.asarray(Z).reshape(-1, order="F")


def unvec(v, rows):
    return np.asarray(v).reshape(rows, -1, order="F")


def kron_L(g: Graph, d: int):
    """L = I_d (x) M  (Eq. 3)."""
    return sp.kron(sp.identity(d), g.M).tocsr()


def kron_Dt(g: Graph, d: int):
    """D~ = I_d (x) D  (Eq. 4)."""
    return sp.kron(sp.identity(d), sp.diags(g.D)).tocsr()


def kronecker_memory(n: int, d: int, edges_per_vertex: int, bytes_per_value: int = 8):
    """Sizes of the Kronecker-form operators in the memory example that opens
    Sec. III.

    W stores edges_per_vertex nonzeros per vertex.  M has one row per vertex
    pair, n(n-1)/2 rows, and the example counts two nonzeros of M for each
    nonzero of W (every neighbour relation listed from both ends).  L = I_d (x) M
    (Eq. 3) repeats M's nonzeros d times; D~ = I_d (x) D (Eq. 4) is diagonal."""
    rows_M = n * (n - 1) // 2
    nnz_W = edges_per_vertex * n
    nnz_M = 2 * nnz_W
    return dict(
        W_bytes=nnz_W * bytes_per_value,
        Y_bytes=n * d * bytes_per_value,
        M_shape=(rows_M, n), M_nnz=nnz_M, M_bytes=nnz_M * bytes_per_value,
        L_shape=(d * rows_M, d * n), L_nnz=d * nnz_M, L_bytes=d * nnz_M * bytes_per_value,
        Dt_shape=(d * n, d * n), Dt_nnz=d * n, Dt_bytes=d * n * bytes_per_value,
        inverse_bytes=(d * n) ** 2 * bytes_per_value,
    )


# ----------------------------------------------------------------------------
# Evaluation helpers
# ----------------------------------------------------------------------------

def kmeans_agreement(Y_ref, Y_other, k: int, seed: int = 0):
    """k-means labels of two embeddings from the same initial centroids
    (k-means++ seeded on Y_ref), matched by the Hungarian method on the confusion
    matrix.  Returns (fraction of vertices whose labels agree, labels_ref)."""
    from scipy.optimize import linear_sum_assignment
    from sklearn.cluster import KMeans, kmeans_plusplus

    Y_ref = np.asarray(Y_ref, dtype=np.float64)
    Y_other = np.asarray(Y_other, dtype=np.float64)
    init, _ = kmeans_plusplus(Y_ref, n_clusters=k, random_state=seed)
    la = KMeans(n_clusters=k, init=init, n_init=1, random_state=seed).fit_predict(Y_ref)
    lb = KMeans(n_clusters=k, init=init, n_init=1, random_state=seed).fit_predict(Y_other)
    C = np.zeros((k, k), dtype=np.int64)
    np.add.at(C, (la, lb), 1)
    ri, ci = linear_sum_assignment(-C)
    return C[ri, ci].sum() / len(la), la


def jacobi_condition_number(A):
    """kappa(D_A^{-1/2} A D_A^{-1/2}) by dense eigenvalues (small A only)."""
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A)
    s = 1.0 / np.sqrt(np.diag(Ad))
    ev = np.linalg.eigvalsh(s[:, None] * Ad * s[None, :])
    return ev[-1] / ev[0]
