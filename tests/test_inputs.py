"""Seeded input generators (CPU): the k-NN search used for large point clouds
(torch, float32 candidates re-ranked in float64) returns exactly the edge list
of the float64 brute force used for small ones, and brute-force checks of the
neighbour property on a tiny cloud."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("n,m,k", [(1500, 32, 16), (700, 3, 5)])
def test_torch_knn_matches_float64_brute_force(n, m, k):
    pts, _ = synth.gaussian_mixture(n, m, 6, 11)
    a = synth.knn_edge_list(pts, k)
    b = synth.knn_edge_list_torch(pts, k, device="cpu", block=256)
    assert np.array_equal(a[0], b[0].numpy()) and np.array_equal(a[1], b[1].numpy())
    assert np.allclose(a[2], b[2].numpy(), rtol=1e-12, atol=1e-12)
    assert np.allclose(np.sort(a[3]), np.sort(b[3].numpy()), rtol=1e-12, atol=1e-12)


def test_knn_neighbour_property_tiny():
    """Every point's k nearest (by an explicit O(n^2) loop) are among its edges,
    edges are unique pairs src < dst, and each vertex has at least k of them."""
    pts, _ = synth.gaussian_mixture(60, 4, 3, 2)
    k = 4
    src, dst, d2, _ = synth.knn_edge_list_torch(pts, k, device="cpu", block=16)
    src, dst = src.numpy(), dst.numpy()
    assert np.all(src < dst)
    pairs = set(zip(src.tolist(), dst.tolist()))
    assert len(pairs) == len(src)
    x = pts.astype(np.float64)
    for i in range(len(x)):
        dist = [((x[i] - x[j]) ** 2).sum() if j != i else np.inf for j in range(len(x))]
        for j in np.argsort(dist, kind="stable")[:k]:
            assert (min(i, j), max(i, j)) in pairs
    deg = np.bincount(np.concatenate([src, dst]), minlength=len(x))
    assert deg.min() >= k


def test_rcm_relabel_is_a_graph_isomorphism():
    """Relabelling keeps the edge set (up to the permutation) and its weights,
    and yields sorted unique pairs src < dst."""
    from synth.workloads import rcm_relabel
    pts, labels = synth.gaussian_mixture(400, 5, 4, 3)
    src, dst, d2, _ = synth.knn_edge_list(pts, 6)
    s2, t2, w2, perm, lab2 = rcm_relabel(len(pts), src, dst, d2, labels)
    assert np.all(s2 < t2)
    key = s2.astype(np.int64) * len(pts) + t2
    assert np.all(np.diff(key) > 0)
    assert np.array_equal(lab2, labels[perm])
    back = {(min(perm[a], perm[b]), max(perm[a], perm[b])): w for a, b, w in zip(s2, t2, w2)}
    orig = {(a, b): w for a, b, w in zip(src.tolist(), dst.tolist(), d2)}
    assert back.keys() == orig.keys()
    assert all(back[k] == orig[k] for k in orig)
