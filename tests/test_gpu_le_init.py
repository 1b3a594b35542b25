"""GPU Laplacian-eigenmap initialisation (pfe_le_init) against the oracle's
generalised eigensolver (oracle.le_init: dense eigh on small graphs, shift-invert
Lanczos on larger ones), Sec. I: the d smallest nontrivial solutions of
(D - W) y = mu D y.

Compared: the eigenvalues; the subspace (largest principal-angle sine, in the
D inner product, between the GPU's and the oracle's span of the constant
vector and y_1 .. y_d, which is well determined when mu_d < mu_{d+1} even
where single eigenvectors are not); D-orthonormality; and, on a graph whose
eigenvalues are well separated, the sign-fixed columns one by one."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_helpers import banner, gpu_graph, oracle_graph

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def d_orthonormal(B, D):
    """B R^{-1} with R^T R = B^T D B (columns D-orthonormal, same span)."""
    R = np.linalg.cholesky(B.T @ (D[:, None] * B)).T
    return np.linalg.solve(R.T, B.T).T


def sin_angle(Ya, Yb, D):
    """Largest principal-angle sine, in the D inner product, between
    span{1, Ya} and span{1, Yb}.  The trivial solution is included: the
    smallest nontrivial eigenvalues of a nearly disconnected graph lie within
    ~1e-12 of zero, so the solvers fix span{y_2 .. y_{d+1}} only up to a
    rounding-level mixture with the constant vector, while the span with it is
    separated from the rest of the spectrum by mu_{d+2}.  Computed as the norm
    of the D-projection residual (no 1 - cos^2 cancellation)."""
    one = np.ones((len(D), 1))
    A = d_orthonormal(np.hstack([one, Ya]), D)
    B = d_orthonormal(np.hstack([one, Yb]), D)
    Z = A - B @ (B.T @ (D[:, None] * A))
    return float(np.linalg.norm(np.sqrt(D)[:, None] * Z, 2))


def start_block(n, k, seed):
    return np.random.default_rng(seed).normal(size=(n, k))


def run(wl, d, k, tol, seed=1, max_iter=300):
    from paper_1612_06496_amd import le_init
    G = gpu_graph(wl)
    Y, mu, info = le_init(G, d, start_block(wl.n, k, seed), tol=tol, max_iter=max_iter)
    G.close()
    return Y.cpu().numpy(), mu, info


@pytest.mark.parametrize("name,d,k", [("gmm_one", 6, 12), ("voronoi64_4nbr", 4, 10), ("voronoi48x40_r2", 5, 12)])
def test_le_init_matches_oracle_small(name, d, k):
    banner(f"LE init vs oracle: {name} d={d} k={k}")
    if name == "gmm_one":
        wl = synth.edges_workload("gmm_one", 1500, 3, 1, 8, 4, d=d)     # one Gaussian cloud: distinct eigenvalues
    else:
        wl = synth.make_workload(name, 0)
    g = oracle_graph(wl)
    Yo, muo = O.le_init(g, d)
    Yg, mug, info = run(wl, d, k, tol=1e-13)
    ortho = np.abs(Yg.T @ (g.D[:, None] * Yg) - np.eye(d)).max()
    sa = sin_angle(Yg, Yo, g.D)
    emu = np.abs(mug - muo).max()
    print(f"{info}; mu gpu {mug} oracle {muo}; |dmu| {emu:.2e}; sin angle {sa:.2e}; D-orthonormality {ortho:.2e}")
    assert info["converged"] == 1
    assert ortho <= 1e-10
    assert emu <= 1e-10 * max(1.0, muo.max()) + 1e-13
    assert sa <= 1e-8
    if name == "gmm_one":
        # well separated eigenvalues: every sign-fixed column equals the oracle's
        gaps = np.diff(np.concatenate([[0.0], muo, [np.inf]]))
        assert gaps.min() > 1e-3 * muo.max()
        col = np.abs(Yg - Yo).max(axis=0) / np.abs(Yo).max(axis=0)
        print("column errors", col)
        assert col.max() <= 1e-6


def test_le_init_headline_image_subspace():
    """481x321 image, d = 10: the eigenvalues mu_2 .. mu_11 lie between 2e-15
    and 2e-8 with mu_12 ~ 9e-8, so single eigenvectors are fixed only up to
    rotations inside near-degenerate clusters; the span of the ten is fixed."""
    banner("LE init vs oracle: 481x321, d = 10")
    wl = synth.make_workload("voronoi481x321_8nbr", 0)
    g = oracle_graph(wl)
    Yo, muo = O.le_init(g, wl.d)
    Yg, mug, info = run(wl, wl.d, 32, tol=1e-13, max_iter=400)
    ortho = np.abs(Yg.T @ (g.D[:, None] * Yg) - np.eye(wl.d)).max()
    sa = sin_angle(Yg, Yo, g.D)
    emu = np.abs(mug - muo).max()
    print(f"{info}; |dmu| {emu:.2e} (mu up to {muo.max():.2e}); sin angle {sa:.2e}; D-orthonormality {ortho:.2e}")
    assert info["converged"] == 1
    assert ortho <= 1e-10
    assert emu <= 1e-12
    assert sa <= 1e-6


def test_le_init_argument_checks():
    from paper_1612_06496_amd import Graph, le_init
    from paper_1612_06496_amd import _lib as L
    banner("LE init argument checks")
    wl = synth.make_workload("voronoi64_4nbr", 0)
    G = gpu_graph(wl)
    with pytest.raises(L.PFEError):
        le_init(G, 5, start_block(wl.n, 4, 0))          # k < d
    with pytest.raises(L.PFEError):
        le_init(G, 4, start_block(wl.n, 33, 0))         # k > 32
    U = Graph.union([G, gpu_graph(wl)])
    with pytest.raises(L.PFEError):
        le_init(U, 4, start_block(U.n, 8, 0))           # unions are not one graph
