"""Initial embeddings Y0 (n x d) drawn at random.

Neither generator orthonormalises: making Y0 satisfy Y^T D Y = I is part of the
method's initialisation and is done by each implementation itself.
"""
from __future__ import annotations

import numpy as np


def smooth_y0(H: int, W: int, d: int, seed: int, n_waves: int = 6) -> np.ndarray:
    """Smooth random fields on an H x W pixel grid: each column is a sum of a few
    low-frequency cosines with random frequencies, phases and amplitudes, plus a
    constant.  Returns float32 n x d, rows ordered (y, x)."""
    rng = np.random.default_rng(seed)
    u = np.arange(W, dtype=np.float64) / max(1, W - 1)
    v = np.arange(H, dtype=np.float64) / max(1, H - 1)
    U = np.broadcast_to(u[None, :], (H, W)).reshape(-1)
    V = np.broadcast_to(v[:, None], (H, W)).reshape(-1)
    Y = np.empty((H * W, d))
    for c in range(d):
        col = np.full(H * W, rng.normal())
        for _ in range(n_waves):
            fx, fy = rng.uniform(-3.0, 3.0, size=2)
            ph = rng.uniform(0.0, 2 * np.pi)
            amp = rng.normal()
            col += amp * np.cos(2 * np.pi * (fx * U + fy * V) + ph)
        Y[:, c] = col
    return Y.astype(np.float32)


def gaussian_y0(n: int, d: int, seed: int) -> np.ndarray:
    """i.i.d. standard normal entries, float32 n x d."""
    rng = np.random.default_rng(seed)
    return rng.normal(size=(n, d)).astype(np.float32)
