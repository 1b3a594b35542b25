"""FP64 oracle for the k-means step of the segmentation experiment — test
infrastructure only (see the package docstring for who may call it).

Sec. IV segments an image by k-means clustering of its embedding.  Reading:
Lloyd's algorithm from given initial centroids (choosing them is the caller's
random draw).  One iteration assigns every row of Y to its nearest centroid —
squared Euclidean distance summed over the coordinates in order, each term
(y_c - m_c)^2 rounded on its own (no fused multiply-add), ties to the lowest
centroid index — and then moves every centroid that has rows to their mean (a
centroid without rows stays).  It stops after max_iter iterations or after an
iteration in which no label changed.

Parity status: pinned in tests/test_oracle_kmeans.py (scikit-learn's Lloyd
k-means from the same initial centroids; the fixed-point property at
convergence; well-separated clusters recovered exactly).
"""
from __future__ import annotations

import numpy as np

__all__ = ["lloyd", "label_agreement"]


def lloyd(Y, C0, max_iter: int):
    """Returns (labels int32 n, centroids K x d, iterations run)."""
    Y = np.asarray(Y, dtype=np.float64)
    C = np.array(C0, dtype=np.float64, copy=True)
    n, d = Y.shape
    K = C.shape[0]
    labels = np.full(n, -1, dtype=np.int64)
    it = 0
    for it in range(1, max_iter + 1):
        dist = np.zeros((n, K))
        for c in range(d):
            diff = Y[:, c, None] - C[None, :, c]
            dist += diff * diff
        new = np.argmin(dist, axis=1)          # first minimum: lowest index on ties
        changed = int(np.count_nonzero(new != labels))
        labels = new
        for k in range(K):
            rows = labels == k
            if rows.any():
                C[k] = Y[rows].mean(axis=0)
        if changed == 0:
            break
    return labels.astype(np.int32), C, it


def label_agreement(la, lb, K: int) -> float:
    """Fraction of rows whose labels agree after matching the two labelings by
    the Hungarian method on their confusion matrix."""
    from scipy.optimize import linear_sum_assignment
    M = np.zeros((K, K), dtype=np.int64)
    np.add.at(M, (np.asarray(la), np.asarray(lb)), 1)
    ri, ci = linear_sum_assignment(-M)
    return M[ri, ci].sum() / len(la)
