"""Pins for the oracle's k-means (Lloyd iterations from given centroids)
against scikit-learn's Lloyd k-means, the fixed-point property, and exact
recovery of well-separated clusters."""
import numpy as np

from oracle import kmeans as KM


def blobs(n_per, K, d, spread, seed):
    rng = np.random.default_rng(seed)
    centers = rng.normal(0.0, 10.0, size=(K, d))
    truth = np.repeat(np.arange(K), n_per)
    Y = centers[truth] + spread * rng.normal(size=(n_per * K, d))
    perm = rng.permutation(len(Y))
    return Y[perm], truth[perm]


def test_lloyd_matches_scikit_learn_from_the_same_centroids():
    from sklearn.cluster import KMeans
    rng = np.random.default_rng(1)
    Y = rng.normal(size=(3000, 6)) + np.repeat(rng.normal(0, 2.0, size=(12, 6)), 250, axis=0)
    C0 = Y[rng.choice(len(Y), 12, replace=False)]
    lab, C, it = KM.lloyd(Y, C0, 300)
    km = KMeans(n_clusters=12, init=C0, n_init=1, max_iter=300, tol=0.0, algorithm="lloyd").fit(Y)
    print(f"iterations {it} (scikit-learn {km.n_iter_}); centroid diff {np.abs(C - km.cluster_centers_).max():.2e}")
    assert np.array_equal(lab, km.labels_)
    assert np.abs(C - km.cluster_centers_).max() <= 1e-12


def test_lloyd_converged_state_is_a_fixed_point():
    rng = np.random.default_rng(2)
    Y = rng.normal(size=(2000, 4))
    C0 = Y[:9]
    lab, C, it = KM.lloyd(Y, C0, 1000)
    assert it < 1000
    # every row is at its nearest centroid, every centroid is its rows' mean
    D = ((Y[:, None, :] - C[None, :, :]) ** 2).sum(axis=2)
    assert np.array_equal(lab, np.argmin(D, axis=1))
    for k in range(9):
        assert np.allclose(C[k], Y[lab == k].mean(axis=0), rtol=0, atol=1e-14)


def test_lloyd_recovers_well_separated_clusters():
    Y, truth = blobs(50, 7, 5, 0.1, 3)
    C0 = np.stack([Y[np.flatnonzero(truth == k)[0]] for k in range(7)])
    lab, _, it = KM.lloyd(Y, C0, 50)
    assert np.array_equal(lab, truth) and it == 2
    assert KM.label_agreement(lab, (truth + 3) % 7, 7) == 1.0
