"""Gaussian-mixture point clouds and their symmetrised k-nearest-neighbour lists.

Points: n samples in R^m from a C-component mixture with means ~ N(0, 4 I),
identity covariance and mixture weights ~ Dirichlet(1); component counts are
multinomial.  The neighbour list is exact Euclidean k-NN (self excluded, ties to
the lower index) made symmetric by union; it is an input artefact, like the
pixel grid of an image.
"""
from __future__ import annotations

import numpy as np


def gaussian_mixture(n: int, m: int, components: int, seed: int):
    """Return (points[n, m] float32, labels[n] int32)."""
    rng = np.random.default_rng(seed)
    means = rng.normal(0.0, 2.0, size=(components, m))
    weights = rng.dirichlet(np.ones(components))
    counts = rng.multinomial(n, weights)
    labels = np.repeat(np.arange(components, dtype=np.int32), counts)
    rng.shuffle(labels)
    pts = means[labels] + rng.normal(0.0, 1.0, size=(n, m))
    return pts.astype(np.float32), labels


def knn_edge_list(points: np.ndarray, k: int, block: int = 4096):
    """Exact k-NN by blocked brute force in float64.

    Returns (src, dst, dist2, knn_dist): undirected pairs src < dst sorted
    lexicographically, their squared distances (float64), and the n*k k-NN
    distances (for bandwidth choices).  Intended for modest n (tests); the cost is
    O(n^2 m).
    """
    x = points.astype(np.float64)
    n = x.shape[0]
    sq = np.einsum("ij,ij->i", x, x)
    nbr = np.empty((n, k), dtype=np.int64)
    nd2 = np.empty((n, k), dtype=np.float64)
    for b0 in range(0, n, block):
        b1 = min(n, b0 + block)
        d2 = sq[b0:b1, None] + sq[None, :] - 2.0 * (x[b0:b1] @ x.T)
        np.maximum(d2, 0.0, out=d2)
        d2[np.arange(b1 - b0), np.arange(b0, b1)] = np.inf
        # stable sort on (distance, index): lower index wins ties
        idx = np.argsort(d2, axis=1, kind="stable")[:, :k]
        nbr[b0:b1] = idx
        nd2[b0:b1] = np.take_along_axis(d2, idx, axis=1)
    rows = np.repeat(np.arange(n, dtype=np.int64), k)
    cols = nbr.reshape(-1)
    lo = np.minimum(rows, cols)
    hi = np.maximum(rows, cols)
    key = np.unique(lo * n + hi)
    src = (key // n).astype(np.int32)
    dst = (key % n).astype(np.int32)
    diff = x[src] - x[dst]
    dist2 = np.einsum("ij,ij->i", diff, diff)
    return src, dst, dist2, np.sqrt(nd2.reshape(-1))


def knn_edge_list_torch(points, k: int, device="cuda", block: int = 4096, cand: int = 0):
    """Exact k-NN of a large point cloud with torch on `device`, as
    knn_edge_list returns it (src < dst unique pairs sorted lexicographically,
    float64 squared distances, the n*k k-NN distances), as torch tensors on the
    device.

    Candidates per point: the `cand` (default 2k) smallest float32 squared
    distances of a blocked GEMM; they are re-ranked by float64 distance and the
    k nearest kept (self excluded; equal float64 distances, which these
    continuous draws do not produce, would be ordered by candidate rank, not by
    index).  The float32 candidate set holds the k nearest whenever the float32
    rounding of a squared distance, about 1e-7 of the squared norms, is below
    the gap between the k-th and the cand-th nearest distance.
    """
    import torch
    cand = cand or 2 * k
    x32 = torch.as_tensor(points, dtype=torch.float32, device=device)
    x64 = x32.double()
    n = x32.shape[0]
    sq32 = (x32 * x32).sum(1)
    nbr = torch.empty((n, k), dtype=torch.int64, device=device)
    nd2 = torch.empty((n, k), dtype=torch.float64, device=device)
    ar = torch.arange(n, device=device)
    for b0 in range(0, n, block):
        b1 = min(n, b0 + block)
        d2 = sq32[b0:b1, None] + sq32[None, :] - 2.0 * (x32[b0:b1] @ x32.T)
        d2[ar[: b1 - b0], ar[b0:b1]] = float("inf")
        ci = torch.topk(d2, cand, dim=1, largest=False).indices
        del d2
        diff = x64[b0:b1, None, :] - x64[ci]
        e2 = (diff * diff).sum(2)
        e2[ci == ar[b0:b1, None]] = float("inf")
        o = torch.argsort(e2, dim=1, stable=True)[:, :k]
        nbr[b0:b1] = torch.gather(ci, 1, o)
        nd2[b0:b1] = torch.gather(e2, 1, o)
    rows = ar.repeat_interleave(k)
    cols = nbr.reshape(-1)
    lo = torch.minimum(rows, cols)
    hi = torch.maximum(rows, cols)
    key = torch.unique(lo * n + hi)
    src = (key // n).to(torch.int32)
    dst = (key % n).to(torch.int32)
    diff = x64[src.long()] - x64[dst.long()]
    dist2 = (diff * diff).sum(1)
    return src, dst, dist2, torch.sqrt(nd2.reshape(-1))
