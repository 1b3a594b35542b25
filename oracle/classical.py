"""FP64 oracle for classical sparse preconditioners of the PCG — test
infrastructure only (see the package docstring for who may call it).

* IC(0) — the preconditioner the paper uses (Sec. III, closing paragraph: PCG
  preconditioned by an incomplete Cholesky factorisation).  Reading: the
  zero-fill variant of Meijerink and van der Vorst.  The factor L is lower
  triangular, keeps exactly the pattern of the lower triangle of A, and
  satisfies (L L^T)_ij = A_ij for every (i, j) in that pattern; it is computed
  by the Cholesky recurrences with every update outside the pattern dropped.
  M^{-1} r = L^{-T} L^{-1} r.
* FSAI — not in the paper: the factorized sparse approximate inverse of
  Kolotilina and Yeremin on the same lower pattern.  Row i of G is supported on
  S_i = {i} and the lower neighbours of i; it solves A[S_i, S_i] g = e_i and is
  scaled so that (G A G^T)_ii = 1.  M^{-1} = G^T G.  It has the form of the
  learned factor (G = Gt D_A^{-1/2} with Gt lower triangular on the pattern of
  A), so it is that factor's non-learned counterpart.

Both act on the system matrix A of Eq. (13) given as a scipy sparse matrix.
Parity status: pinned in tests/test_oracle_classical.py (IC(0) equals the
exact Cholesky factor where no fill is dropped and meets its defining
equations on a grid system; FSAI recovers an inverse factor that has the
pattern exactly and meets its defining equations; both PCGs reach the direct
solution within the condition-number bound).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

__all__ = ["lower_pattern", "ic0", "fsai_row", "fsai", "ic0_apply", "fsai_apply"]


def lower_pattern(A, i):
    """Sorted column indices j < i with a stored entry in row i of A (CSR)."""
    cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
    return np.sort(cols[cols < i])


def ic0(A) -> sp.csr_matrix:
    """Zero-fill incomplete Cholesky factor L (lower triangular, CSR).

    Row by row: for each j in the lower pattern of row i, in increasing order,
    L_ij = (A_ij - sum_k L_ik L_jk) / L_jj over the k < j present in both rows;
    then L_ii = sqrt(A_ii - sum_{j<i} L_ij^2).  A non-positive pivot raises."""
    A = sp.csr_matrix(A, dtype=np.float64)
    A.sort_indices()
    n = A.shape[0]
    rows = []
    for i in range(n):
        lo, hi = A.indptr[i], A.indptr[i + 1]
        cols, vals = A.indices[lo:hi], A.data[lo:hi]
        Li = {}
        aii = 0.0
        for j, aij in zip(cols, vals):
            j = int(j)
            if j > i:
                break
            if j == i:
                aii = float(aij)
                continue
            Lj = rows[j]
            s = float(aij)
            for k, lik in Li.items():          # every k here is < j
                ljk = Lj.get(k)
                if ljk is not None:
                    s -= lik * ljk
            Li[j] = s / Lj[j]
        piv = aii - sum(v * v for v in Li.values())
        if not piv > 0.0:
            raise ValueError(f"IC(0) breakdown at row {i} (pivot {piv})")
        Li[i] = math.sqrt(piv)
        rows.append(Li)
    ri = np.repeat(np.arange(n), [len(r) for r in rows])
    ci = np.fromiter((k for r in rows for k in r.keys()), dtype=np.int64, count=len(ri))
    vi = np.fromiter((v for r in rows for v in r.values()), dtype=np.float64, count=len(ri))
    return sp.csr_matrix((vi, (ri, ci)), shape=(n, n))


def _row_dicts(A):
    A = sp.csr_matrix(A, dtype=np.float64)
    A.sort_indices()
    return [dict(zip(A.indices[A.indptr[i]:A.indptr[i + 1]].tolist(), A.data[A.indptr[i]:A.indptr[i + 1]].tolist()))
            for i in range(A.shape[0])]


def _fsai_row(R, i):
    S = sorted(j for j in R[i] if j < i) + [i]
    As = np.array([[R[a].get(b, 0.0) for b in S] for a in S])
    e = np.zeros(len(S))
    e[-1] = 1.0
    gh = np.linalg.solve(As, e)
    return np.array(S), gh / math.sqrt(gh[-1])


def fsai_row(A, i):
    """(S_i, g): the pattern of row i of the FSAI factor (sorted, i last) and
    its values."""
    A = sp.csr_matrix(A, dtype=np.float64)
    rows = set(A.indices[A.indptr[i]:A.indptr[i + 1]].tolist()) | {i}
    R = {k: dict(zip(A.indices[A.indptr[k]:A.indptr[k + 1]].tolist(), A.data[A.indptr[k]:A.indptr[k + 1]].tolist()))
         for k in rows}
    return _fsai_row(R, i)


def fsai(A) -> sp.csr_matrix:
    """FSAI factor G (lower triangular, CSR) on the lower pattern of A."""
    R = _row_dicts(A)
    n = len(R)
    ri, ci, vi = [], [], []
    for i in range(n):
        S, g = _fsai_row(R, i)
        ri.append(np.full(len(S), i))
        ci.append(S)
        vi.append(g)
    return sp.csr_matrix((np.concatenate(vi), (np.concatenate(ri), np.concatenate(ci))), shape=(n, n))


def ic0_apply(L):
    """r -> L^{-T} L^{-1} r (columns of r)."""
    L = sp.csr_matrix(L)
    Lt = sp.csr_matrix(L.T)

    def apply(r):
        y = spla.spsolve_triangular(L, r, lower=True)
        return spla.spsolve_triangular(Lt, y, lower=False)
    return apply


def fsai_apply(G):
    """r -> G^T G r (columns of r)."""
    G = sp.csr_matrix(G)
    Gt = sp.csr_matrix(G.T)
    return lambda r: Gt @ (G @ r)
