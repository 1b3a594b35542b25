"""Named synthetic workloads (sizes, value distributions and iteration counts).

Every workload is fully determined by its name and seed.  ``lam``/``r`` set to
None means the shrink-active choice lambda = r = c, where c is derived from the
initial embedding by the method itself (1 / 0.99-quantile of |M Y0|).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from .voronoi import voronoi_image, image_features, batch_image_shapes
from .points import gaussian_mixture, knn_edge_list, knn_edge_list_torch
from .embed import smooth_y0, gaussian_y0


@dataclass
class Workload:
    name: str
    kind: str                      # "grid" or "edges"
    n: int
    d: int
    sigma: float
    n_outer: int
    n_inner: int
    tol: float
    lam: Optional[float]
    r: Optional[float]
    n_clusters: int
    y0: np.ndarray                 # float32 n x d, not orthonormalised
    labels: np.ndarray             # ground-truth cell / component of each vertex
    H: int = 0
    W: int = 0
    stencil: int = 0               # 4, 8, or -R for a Chebyshev window of radius R
    feat: Optional[np.ndarray] = None   # float32 n x m (grid)
    src: Optional[np.ndarray] = None    # int32 (edges)
    dst: Optional[np.ndarray] = None
    dist2: Optional[np.ndarray] = None  # float64 (edges)
    fp64: bool = False
    meta: dict = field(default_factory=dict)


def grid_workload(name, H, W, K, noise, seed, *, gradient=0.0, with_xy=False,
                  stencil=4, sigma=0.1, d=4, lam=None, r=None, n_outer=10,
                  n_inner=5, tol=1e-6, fp64=False, y0_seed=None):
    rgb, labels = voronoi_image(H, W, K, noise, seed, gradient=gradient)
    feat = image_features(rgb, with_xy)
    y0 = smooth_y0(H, W, d, seed + 7919 if y0_seed is None else y0_seed)
    return Workload(name=name, kind="grid", n=H * W, d=d, sigma=sigma,
                    n_outer=n_outer, n_inner=n_inner, tol=tol, lam=lam, r=r,
                    n_clusters=K, y0=y0, labels=labels.reshape(-1), H=H, W=W,
                    stencil=stencil, feat=feat, fp64=fp64,
                    meta=dict(seed=seed, noise=noise, gradient=gradient, K=K))


def edges_workload(name, n, m, components, k, seed, *, d=20, n_outer=20,
                   n_inner=10, tol=1e-6, lam=None, r=None):
    pts, labels = gaussian_mixture(n, m, components, seed)
    src, dst, dist2, knn_dist = knn_edge_list(pts, k)
    sigma = float(np.median(knn_dist))
    y0 = gaussian_y0(n, d, seed + 7919)
    return Workload(name=name, kind="edges", n=n, d=d, sigma=sigma,
                    n_outer=n_outer, n_inner=n_inner, tol=tol, lam=lam, r=r,
                    n_clusters=components, y0=y0, labels=labels, src=src,
                    dst=dst, dist2=dist2, meta=dict(seed=seed, k=k, m=m))


WORKLOADS = {
    # 64x64, 5 cells, noise 0.05, RGB, 4-neighbour, sigma 0.1, d=4, lambda=r=1,
    # 10 outer x 5 inner, solver tolerance 1e-8 in FP64.
    "voronoi64_4nbr": dict(H=64, W=64, K=5, noise=0.05, stencil=4, d=4,
                           lam=1.0, r=1.0, n_outer=10, n_inner=5, tol=1e-8,
                           fp64=True),
    # 481x321 (BSDS image shape), 40 cells with smooth colour gradients, noise
    # 0.03, RGB + scaled xy, 8-neighbour, sigma 0.1, d=10, 20 outer x 10 inner,
    # solver tolerance 1e-6 in FP32.
    "voronoi481x321_8nbr": dict(H=321, W=481, K=40, noise=0.03, gradient=0.3,
                                with_xy=True, stencil=8, d=10, n_outer=20,
                                n_inner=10, tol=1e-6),
    # 1024x1024, 200 cells, noise 0.05, RGB, 5x5 window (radius 2), d=16.
    "voronoi1024_r2": dict(H=1024, W=1024, K=200, noise=0.05, stencil=-2, d=16,
                           n_outer=20, n_inner=10, tol=1e-6),
    # Small stand-ins with the same structure, sized for tests.
    "voronoi96x80_8nbr": dict(H=80, W=96, K=8, noise=0.03, gradient=0.3,
                              with_xy=True, stencil=8, d=10, n_outer=4,
                              n_inner=4, tol=1e-6),
    "voronoi48x40_r2": dict(H=40, W=48, K=6, noise=0.05, stencil=-2, d=16,
                            n_outer=3, n_inner=3, tol=1e-6),
}


# Gaussian-mixture point clouds with symmetrised exact k-NN graphs (edge
# lists), generated on a torch device (2 M points: about 4e12 candidate
# distances): 20 components in R^32, means N(0, 4 I), unit covariance,
# Dirichlet(1) weights, k = 16, sigma = median k-NN distance, d = 20.
EDGE_WORKLOADS = {
    "gmm2m_knn16": dict(n=2_000_000, m=32, components=20, k=16, d=20, n_outer=20, n_inner=10, tol=1e-6),
    # same distribution at a tenth of the size (training graphs for the learned
    # preconditioner of the 2 M-point graph)
    "gmm200k_knn16": dict(n=200_000, m=32, components=20, k=16, d=20, n_outer=20, n_inner=10, tol=1e-6),
    # the same graphs with the vertices relabelled in reverse Cuthill-McKee
    # order (input preparation that gives neighbour gathers locality; the
    # sampled points are i.i.d., so their order is arbitrary)
    "gmm2m_knn16_rcm": dict(n=2_000_000, m=32, components=20, k=16, d=20, n_outer=20, n_inner=10, tol=1e-6,
                            order="rcm"),
    "gmm200k_knn16_rcm": dict(n=200_000, m=32, components=20, k=16, d=20, n_outer=20, n_inner=10, tol=1e-6,
                              order="rcm"),
}


def rcm_relabel(n: int, src, dst, dist2, *arrays):
    """Relabel the vertices of an edge list (src < dst unique pairs) in reverse
    Cuthill-McKee order.  Returns (src', dst', dist2', perm, relabelled arrays):
    new vertex k is old vertex perm[k]; pairs re-sorted lexicographically;
    per-vertex arrays reordered."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import reverse_cuthill_mckee
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    A = sp.coo_matrix((np.ones(src.size, np.int8), (src, dst)), shape=(n, n)).tocsr()
    perm = reverse_cuthill_mckee((A + A.T).tocsr(), symmetric_mode=True).astype(np.int64)
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n, dtype=np.int64)
    a, b = inv[src], inv[dst]
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    order = np.argsort(lo * n + hi, kind="stable")
    out = [lo[order].astype(np.int32), hi[order].astype(np.int32), np.asarray(dist2)[order], perm]
    return tuple(out) + tuple(np.asarray(x)[perm] for x in arrays)


def make_edges_workload(name: str, seed: int = 0, device="cuda") -> Workload:
    """A named point-cloud workload; src, dst, dist2 are torch tensors on
    `device` (the k-NN search runs there)."""
    import torch
    if name not in EDGE_WORKLOADS:
        raise KeyError(f"unknown edge workload {name!r}; known: {sorted(EDGE_WORKLOADS)}")
    cfg = dict(EDGE_WORKLOADS[name])
    n, m, comps, k = cfg.pop("n"), cfg.pop("m"), cfg.pop("components"), cfg.pop("k")
    order = cfg.pop("order", None)
    pts, labels = gaussian_mixture(n, m, comps, seed)
    src, dst, dist2, knn_dist = knn_edge_list_torch(pts, k, device=device)
    sigma = float(torch.median(knn_dist))
    if order == "rcm":
        s2, d2, w2, perm, labels = rcm_relabel(n, src.cpu().numpy(), dst.cpu().numpy(), dist2.cpu().numpy(), labels)
        src = torch.as_tensor(s2, device=device)
        dst = torch.as_tensor(d2, device=device)
        dist2 = torch.as_tensor(w2, device=device)
    y0 = gaussian_y0(n, cfg["d"], seed + 7919)
    return Workload(name=name, kind="edges", n=n, d=cfg["d"], sigma=sigma,
                    n_outer=cfg["n_outer"], n_inner=cfg["n_inner"], tol=cfg["tol"], lam=None, r=None,
                    n_clusters=comps, y0=y0, labels=labels, src=src, dst=dst, dist2=dist2,
                    meta=dict(seed=seed, k=k, m=m))


# Batches of uneven images (one problem per image, solved side by side):
# W ~ U{wmin..wmax}, H ~ U{hmin..hmax}, one child seed per image; every image
# otherwise as its single-image counterpart.
BATCHES = {
    # 64 images of 128..512 x 128..384 pixels, each as the 481x321 workload.
    "voronoi_batch64_8nbr": dict(count=64, K=40, noise=0.03, gradient=0.3,
                                 with_xy=True, stencil=8, d=10, n_outer=20,
                                 n_inner=10, tol=1e-6),
    # Small stand-in for tests: 5 images of 24..64 x 20..48 pixels.
    "voronoi_batch5_8nbr": dict(count=5, wmin=24, wmax=64, hmin=20, hmax=48,
                                K=6, noise=0.03, gradient=0.3, with_xy=True,
                                stencil=8, d=6, n_outer=3, n_inner=3, tol=1e-6),
}


def make_batch(name: str, seed: int = 0) -> list:
    """The images of a named batch as single-image workloads, in batch order."""
    if name not in BATCHES:
        raise KeyError(f"unknown batch {name!r}; known: {sorted(BATCHES)}")
    cfg = dict(BATCHES[name])
    count = cfg.pop("count")
    lim = {k: cfg.pop(k) for k in ("wmin", "wmax", "hmin", "hmax") if k in cfg}
    shapes = batch_image_shapes(count, seed, **lim)
    return [grid_workload(f"{name}[{k}]", H, W, seed=s, **cfg) for k, (H, W, s) in enumerate(shapes)]


def make_workload(name: str, seed: int = 0) -> Workload:
    if name not in WORKLOADS:
        raise KeyError(f"unknown workload {name!r}; known: {sorted(WORKLOADS)}")
    cfg = dict(WORKLOADS[name])
    return grid_workload(name, seed=seed, **cfg)
