"""GPU k-means (pfe_kmeans, through the C ABI) against the oracle's Lloyd
iterations from the same initial centroids.  Both decide the nearest centroid
in FP64 by the same sequence of roundings, so labels and iteration counts must
agree exactly; centroids (means summed in different orders) to 1e-12."""
import numpy as np
import pytest

import oracle as O
import synth
from oracle import kmeans as KM
from gpu_helpers import banner, gpu_graph, oracle_graph, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def clustered(n, d, K, seed):
    """Seeded rows around K centres of mixed spread (some clusters overlap)."""
    rng = np.random.default_rng(seed)
    centres = rng.normal(0.0, 1.0, size=(K, d))
    lab = rng.integers(0, K, size=n)
    return centres[lab] + rng.uniform(0.1, 0.6, size=(K, 1))[lab] * rng.normal(size=(n, d))


CASES = [(20000, 3, 5, "f32"), (20000, 10, 40, "f32"), (12000, 20, 17, "f64"), (9000, 32, 64, "f32"),
         (154401, 10, 40, "f32")]


@pytest.mark.parametrize("n,d,K,dt", CASES, ids=[f"n{c[0]}_d{c[1]}_K{c[2]}_{c[3]}" for c in CASES])
def test_kmeans_matches_oracle(n, d, K, dt):
    from paper_1612_06496_amd import kmeans
    banner(f"k-means n={n} d={d} K={K} {dt}")
    X = clustered(n, d, K, seed=n + d)
    X = X.astype(np.float32) if dt == "f32" else X
    C0 = X[np.random.default_rng(5).choice(n, K, replace=False)].astype(np.float64)
    Y = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    lab, cen, it = kmeans(Y, C0, 200)
    lab_o, cen_o, it_o = KM.lloyd(X.astype(np.float64), C0, 200)
    e = np.abs(cen.cpu().numpy() - cen_o).max() / np.abs(cen_o).max()
    diff = int(np.count_nonzero(lab.cpu().numpy() != lab_o))
    print(f"iterations {it} (oracle {it_o}); labels differing {diff}; centroid rel err {e:.2e}")
    assert it == it_o
    assert diff == 0
    assert e <= 1e-12


def test_kmeans_centroid_without_rows_stays():
    from paper_1612_06496_amd import kmeans
    banner("k-means: a centroid without rows keeps its place")
    X = clustered(5000, 4, 3, seed=9)
    C0 = np.vstack([X[:3], np.full((1, 4), 1e3)])
    lab, cen, it = kmeans(X, C0, 100)
    lab_o, cen_o, it_o = KM.lloyd(X, C0, 100)
    assert it == it_o and np.array_equal(lab.cpu().numpy(), lab_o)
    assert np.array_equal(cen.cpu().numpy()[3], C0[3])
    assert not np.any(lab.cpu().numpy() == 3)


def test_kmeans_rejects_bad_arguments():
    from paper_1612_06496_amd import kmeans
    from paper_1612_06496_amd._lib import PFEError
    banner("k-means argument checks")
    X = np.zeros((10, 4))
    with pytest.raises(PFEError):
        kmeans(X, np.zeros((300, 4)), 10)       # K above 256
    with pytest.raises(PFEError):
        kmeans(X, np.zeros((3, 4)), 0)          # no iteration
    with pytest.raises(PFEError):
        kmeans(np.zeros((10, 40)), np.zeros((3, 40)), 10)   # d above 32


def test_segmentation_pipeline_matches_oracle_pipeline():
    """Embedding then k-means, each side on its own: GPU PFE (FP32) and GPU
    k-means against the oracle's PFE and k-means, from the same initial rows;
    labels agree on >= 99 % of the pixels after Hungarian matching."""
    from paper_1612_06496_amd import Solver, kmeans
    wl = synth.make_workload("voronoi96x80_8nbr", 0)
    banner("segmentation: GPU PFE + GPU k-means vs oracle PFE + oracle k-means")
    g = oracle_graph(wl)
    Y0 = O.orthonormalize_init(g, wl.y0)
    c = O.shrink_active_scale(g, Y0)
    ref = O.pfe_run(g, Y0, c, c, wl.n_outer, wl.n_inner)
    S = Solver(gpu_graph(wl), Y0, lam=c, r=c, n_inner=wl.n_inner, tol=1e-6, maxit=2000, init_ortho=False)
    S.solve(wl.n_outer)
    yh = S.get("Yhat")
    K = wl.n_clusters
    rows = np.random.default_rng(3).choice(g.n, K, replace=False)
    lab, _, it = kmeans(yh, yh[torch.as_tensor(rows, device="cuda")].double(), 300)
    yh_o = ref.yhat(g)
    lab_o, _, it_o = KM.lloyd(yh_o, yh_o[rows], 300)
    agree = KM.label_agreement(lab_o, lab.cpu().numpy(), K)
    print(f"label agreement {agree:.4f}; k-means iterations {it} (oracle {it_o}); "
          f"Yhat rel {rel(yh.cpu().numpy(), yh_o):.2e}")
    assert agree >= 0.99
