"""FP64 oracle for the learned sparse-factor preconditioner — test infrastructure only.

The paper preconditions its PCG with incomplete Cholesky (Sec. III, last
paragraph).  This module is the reference for a learned alternative built
beside it: M^{-1} = G^T G with

    G = Gt D_A^{-1/2},  Gt lower triangular on the pattern of A, diag(Gt) > 0,

so that M^{-1} is symmetric positive definite for every value of the network's
weights, and Gt = I reproduces Jacobi (diag(A)^{-1}) exactly.  The entries of
Gt come from a two-layer message-passing network (hidden width 16) evaluated on
the scaled matrix At = D_A^{-1/2} A D_A^{-1/2}:

    x_i    = [1, sum_j |At_ij|, max_j |At_ij|, deg_i / deg_max]
    agg1_i = sum_{j in N(i)} (-At_ij) x_j
    h1_i   = relu(W1s x_i + W1m agg1_i + b1)
    agg2_i = sum_{j in N(i)} (-At_ij) h1_j
    h2_i   = relu(W2s h1_i + W2m agg2_i + b2)
    U_i = u.h2_i,  V_i = v.h2_i,  Z_i = q.h2_i + bd
    Gt_ij = At_ij (U_i + V_j + c)   (j < i, j in N(i)),   Gt_ii = softplus(Z_i)

Training minimises mean_k ||At Gt^T Gt rho_k - rho_k||^2 over unit-norm
residual samples rho_k in the scaled space (rho = D_A^{-1/2} r / ||.||).

Matrix products of the network use bfloat16 weights and bfloat16 inputs with
wider accumulation; ``bf16=True`` emulates that rounding (straight-through for
gradients).  Everything else is float64.  Gradients come from torch CPU
float64 autograd and are pinned against central finite differences.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import torch

from .pfe import Graph, system_matrix

HIDDEN = 16
NFEAT = 4
# parameter vector layout (float32 on the device, float64 here)
LAYOUT = [("W1s", (HIDDEN, NFEAT)), ("W1m", (HIDDEN, NFEAT)), ("b1", (HIDDEN,)),
          ("W2s", (HIDDEN, HIDDEN)), ("W2m", (HIDDEN, HIDDEN)), ("b2", (HIDDEN,)),
          ("u", (HIDDEN,)), ("v", (HIDDEN,)), ("q", (HIDDEN,)), ("c", (1,)), ("bd", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in LAYOUT)          # 722
SOFTPLUS_ONE = math.log(math.e - 1.0)                       # softplus(SOFTPLUS_ONE) = 1


def unpack(theta):
    out, k = {}, 0
    for name, shape in LAYOUT:
        m = int(np.prod(shape))
        out[name] = theta[k:k + m].reshape(shape)
        k += m
    return out


def identity_params(seed: int = 0, scale: float = 0.1) -> np.ndarray:
    """Random hidden layers, zero output weights: Gt = I (Jacobi) at the start."""
    rng = np.random.default_rng(seed)
    th = np.zeros(NPARAM)
    p = unpack(th)
    for name in ("W1s", "W1m", "W2s", "W2m"):
        p[name][...] = rng.normal(0.0, scale, size=p[name].shape)
    for name in ("b1", "b2"):
        p[name][...] = rng.normal(0.0, scale, size=p[name].shape)
    p["bd"][0] = SOFTPLUS_ONE
    return th


class ScaledSystem:
    """A = lambda/2 M^T M + r/2 D (Eq. 13), its diagonal, and the scaled
    off-diagonal entries At_ij on the directed slots of the graph."""

    def __init__(self, g: Graph, lam: float, r: float):
        self.g = g
        self.A = system_matrix(g, lam, r).tocsr()
        self.dA = self.A.diagonal().copy()
        n = g.n
        # directed slots (i -> j), both orientations, sorted by (i, j)
        si = np.concatenate([g.ei, g.ej])
        sj = np.concatenate([g.ej, g.ei])
        w = np.concatenate([g.w, g.w])
        order = np.lexsort((sj, si))
        self.si, self.sj, w = si[order], sj[order], w[order]
        self.at = -0.5 * lam * w * w / np.sqrt(self.dA[self.si] * self.dA[self.sj])
        self.n = n
        deg = np.bincount(self.si, minlength=n)
        absat = np.abs(self.at)
        s = np.bincount(self.si, weights=absat, minlength=n)
        m = np.zeros(n)
        np.maximum.at(m, self.si, absat)
        self.x = np.stack([np.ones(n), s, m, deg / max(1, deg.max())], axis=1)
        self.At = sp.csr_matrix((self.at, (self.si, self.sj)), shape=(n, n)) + sp.identity(n)


def _bf16(t: torch.Tensor) -> torch.Tensor:
    """Round to bfloat16 (round-to-nearest-even), straight-through gradient."""
    return t + (t.to(torch.bfloat16).to(torch.float64) - t).detach()


def factor(theta, S: ScaledSystem, bf16: bool = True):
    """Network forward: returns (gvals per slot (value of Gt on the slot's
    edge, i.e. Gt_{max(i,j), min(i,j)}), diag of Gt), torch float64."""
    th = theta if isinstance(theta, torch.Tensor) else torch.tensor(theta, dtype=torch.float64)
    p = unpack(th)
    rnd = _bf16 if bf16 else (lambda t: t)
    si = torch.from_numpy(S.si)
    sj = torch.from_numpy(S.sj)
    at = torch.from_numpy(S.at)
    x = torch.from_numpy(S.x)

    def agg(h):
        out = torch.zeros_like(h)
        return out.index_add(0, si, (-at)[:, None] * h[sj])

    a1 = agg(x)
    h1 = torch.relu(rnd(x) @ rnd(p["W1s"]).T + rnd(a1) @ rnd(p["W1m"]).T + p["b1"])
    a2 = agg(h1)
    h2 = torch.relu(rnd(h1) @ rnd(p["W2s"]).T + rnd(a2) @ rnd(p["W2m"]).T + p["b2"])
    h2r = rnd(h2)
    U = h2r @ rnd(p["u"])
    V = h2r @ rnd(p["v"])
    Z = h2r @ rnd(p["q"]) + p["bd"][0]
    lo = torch.maximum(si, sj)
    hi = torch.minimum(si, sj)
    gvals = at * (U[lo] + V[hi] + p["c"][0])
    diag = torch.nn.functional.softplus(Z)
    return gvals, diag


def factor_matrix(gvals, diag, S: ScaledSystem) -> sp.csr_matrix:
    """Gt as a sparse lower-triangular matrix."""
    gv = gvals.detach().numpy() if isinstance(gvals, torch.Tensor) else gvals
    dg = diag.detach().numpy() if isinstance(diag, torch.Tensor) else diag
    low = S.sj < S.si
    L = sp.csr_matrix((gv[low], (S.si[low], S.sj[low])), shape=(S.n, S.n))
    return (L + sp.diags(dg)).tocsr()


def loss(theta, S: ScaledSystem, rho, bf16: bool = True):
    """mean_k ||At Gt^T Gt rho_k - rho_k||^2 for the columns rho_k of rho."""
    gvals, diag = factor(theta, S, bf16)
    si = torch.from_numpy(S.si)
    sj = torch.from_numpy(S.sj)
    at = torch.from_numpy(S.at)
    R = torch.as_tensor(rho, dtype=torch.float64)
    low = sj < si
    up = sj > si

    def gmul(y):       # Gt y
        out = diag[:, None] * y
        return out.index_add(0, si[low], gvals[low][:, None] * y[sj[low]])

    def gtmul(y):      # Gt^T y
        out = diag[:, None] * y
        return out.index_add(0, si[up], gvals[up][:, None] * y[sj[up]])

    def amul(y):       # At y (unit diagonal)
        return y.index_add(0, si, at[:, None] * y[sj])

    y3 = amul(gtmul(gmul(R)))
    return ((y3 - R) ** 2).sum() / R.shape[1]


def loss_and_grad(theta, S: ScaledSystem, rho, bf16: bool = True):
    th = torch.tensor(np.asarray(theta, dtype=np.float64), requires_grad=True)
    L = loss(th, S, rho, bf16)
    L.backward()
    return float(L.detach()), th.grad.numpy().copy()


def apply_preconditioner(gvals, diag, S: ScaledSystem, r):
    """z = D_A^{-1/2} Gt^T Gt D_A^{-1/2} r (columns of r)."""
    Gt = factor_matrix(gvals, diag, S)
    s = 1.0 / np.sqrt(S.dA)
    return s[:, None] * (Gt.T @ (Gt @ (s[:, None] * r)))


def pcg_preconditioned(A, rhs, x0, apply_minv, tol, maxit):
    """PCG (Barrett et al.) with per-column scalars and a general
    preconditioner apply_minv(r) -> z; same stopping rule as the oracle's
    Jacobi PCG.  Returns (x, iterations per column)."""
    rhs = np.asarray(rhs, dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    d = rhs.shape[1]
    bnorm = np.linalg.norm(rhs, axis=0)
    r = rhs - A @ x
    iters = np.zeros(d, dtype=np.int64)
    active = (bnorm > 0) & (np.linalg.norm(r, axis=0) > tol * bnorm)
    p = np.zeros_like(x)
    rho_old = np.ones(d)
    for _ in range(maxit):
        if not active.any():
            break
        z = apply_minv(r)
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
    return x, iters


def adam_step(theta, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba), bias-corrected; returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
