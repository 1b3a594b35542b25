"""Synthetic Voronoi images standing in for natural-image segmentation inputs.

An image of H rows and W columns is split into K Voronoi cells around sites drawn
uniformly in [0, W) x [0, H).  Each pixel centre (x + 0.5, y + 0.5) takes the cell
of its nearest site (ties go to the lowest site index).  Each cell gets a colour
drawn uniformly in [0, 1]^3, optionally with a smooth linear colour gradient, and
i.i.d. Gaussian noise is added to every channel without clipping.
"""
from __future__ import annotations

import numpy as np


def voronoi_image(H: int, W: int, K: int, noise: float, seed: int,
                  gradient: float = 0.0):
    """Return (rgb[H, W, 3] float64, labels[H, W] int32).

    gradient > 0 adds, per cell k, colour = c_k + G_k (u - s_k) where u is the
    pixel position scaled to [0, 1]^2, s_k the scaled site and the entries of
    G_k (3x2) are uniform in (-gradient, gradient).
    """
    rng = np.random.default_rng(seed)
    sites = np.empty((K, 2))
    sites[:, 0] = rng.uniform(0.0, W, size=K)   # x
    sites[:, 1] = rng.uniform(0.0, H, size=K)   # y
    colours = rng.uniform(0.0, 1.0, size=(K, 3))
    grads = rng.uniform(-gradient, gradient, size=(K, 3, 2)) if gradient > 0 else None

    labels = np.empty((H, W), dtype=np.int32)
    xs = np.arange(W, dtype=np.float64) + 0.5
    rows_per_chunk = max(1, (1 << 21) // max(1, W * K))
    for y0 in range(0, H, rows_per_chunk):
        y1 = min(H, y0 + rows_per_chunk)
        ys = np.arange(y0, y1, dtype=np.float64) + 0.5
        px = np.broadcast_to(xs[None, :], (y1 - y0, W)).reshape(-1)
        py = np.broadcast_to(ys[:, None], (y1 - y0, W)).reshape(-1)
        d2 = (px[:, None] - sites[None, :, 0]) ** 2 + (py[:, None] - sites[None, :, 1]) ** 2
        labels[y0:y1] = np.argmin(d2, axis=1).reshape(y1 - y0, W)

    rgb = colours[labels]
    if grads is not None:
        ux = np.arange(W, dtype=np.float64) / max(1, W - 1)
        uy = np.arange(H, dtype=np.float64) / max(1, H - 1)
        su = np.stack([sites[:, 0] / max(1, W - 1), sites[:, 1] / max(1, H - 1)], axis=1)
        du_x = ux[None, :] - su[labels][..., 0]
        du_y = uy[:, None] - su[labels][..., 1]
        g = grads[labels]                      # H, W, 3, 2
        rgb = rgb + g[..., 0] * du_x[..., None] + g[..., 1] * du_y[..., None]
    rgb = rgb + rng.normal(0.0, noise, size=rgb.shape)
    return rgb, labels


def image_features(rgb: np.ndarray, with_xy: bool) -> np.ndarray:
    """Per-pixel feature rows, row-major over (y, x): RGB, optionally followed by
    x/(W-1), y/(H-1).  Returned as float32 so both implementations read identical
    values."""
    H, W, _ = rgb.shape
    cols = [rgb.reshape(-1, 3)]
    if with_xy:
        ux = np.arange(W, dtype=np.float64) / max(1, W - 1)
        uy = np.arange(H, dtype=np.float64) / max(1, H - 1)
        cols.append(np.broadcast_to(ux[None, :], (H, W)).reshape(-1, 1))
        cols.append(np.broadcast_to(uy[:, None], (H, W)).reshape(-1, 1))
    return np.ascontiguousarray(np.concatenate(cols, axis=1), dtype=np.float32)


def batch_image_shapes(count: int, seed: int, wmin=128, wmax=512, hmin=128, hmax=384):
    """Uneven image sizes for a batch: W ~ U{wmin..wmax}, H ~ U{hmin..hmax}, and one
    child seed per image."""
    rng = np.random.default_rng(seed)
    Ws = rng.integers(wmin, wmax + 1, size=count)
    Hs = rng.integers(hmin, hmax + 1, size=count)
    seeds = rng.integers(0, 2**31 - 1, size=count)
    return [(int(h), int(w), int(s)) for h, w, s in zip(Hs, Ws, seeds)]
