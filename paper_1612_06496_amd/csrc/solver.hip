// The PFE hot path on gfx950: Split-Bregman inner iterations (Algorithm 2 in
// the compact form of Eqs. 9, 10, 13), their PCG least-squares solve
// (Sec. III), and the SOC P/B-update (Algorithm 1).
//
// Layout: every n x d block is row-major (d values per vertex); the
// Split-Bregman variables are stored per directed CSR slot (i -> j) with the
// orientation "i minus j", so each vertex owns the slots of its own row and
// every phase is atomic-free.  The two copies of an undirected edge are exact
// negatives of each other (the shrink and the clamp are odd functions and
// w (y_i - y_j) = -(w (y_j - y_i)) exactly), which keeps them consistent.
//
// Work decomposition: a phase is executed by nblk workgroups; workgroup lb
// owns the contiguous row range [lb n / nblk, (lb+1) n / nblk) and walks it
// R = blockDim / d rows at a time with thread t on (row t / d, column t % d),
// so consecutive lanes touch consecutive elements and gathers of neighbour
// rows stay coalesced on image grids.  Per-column reductions are FP64: each
// workgroup writes one partial per column, and one workgroup sums the partials
// in a fixed order (deterministic results).  Workgroup indices are remapped so
// that each XCD owns one contiguous eighth of the rows.
#include <cfloat>
#include <cmath>
#include <cstring>
#include <algorithm>

#include "common.hpp"

namespace pfe {

enum Phase : int {
    PH_E0 = 0,      // first inner solve: rhs = r/2 D^{1/2}(P - B), r0 = rhs - A x
    PH_EU = 1,      // shrink + Bregman on the edges, next rhs, optionally r0
    PH_R0 = 2,      // r0 = rhs - A x from a stored rhs
    PH_A = 3,       // p = z + beta p, q = A p, p^T q
    PH_B = 4,       // x += alpha p, r -= alpha q, r^T z, r^T r
    PH_GRAM = 5,    // Z = D^{1/2} Y + B, Z^T Z
    PH_APPLY = 6,   // P = Z T, B = Z - P
    PH_RHS = 7,     // rhs from stored b, d (no r0)
    PH_ZERO = 8     // zero the solution columns whose rhs is zero
};

template <typename T>
struct KA {
    int n, d, R, nblk;
    const int* rowptr;
    const int* col;
    const T* w;
    const T* diagA;
    const T* invdiag;
    const T* sqrtD;
    const T* isqrtD;
    const double* degree;
    T* x;              // PCG iterate
    T* Y;
    T* P;
    T* B;
    T* bs;             // Split-Bregman b per slot
    T* ds;             // Split-Bregman d per slot (keep_split)
    T* rhs;
    T* r;
    T* pA;
    T* pB;
    T* q;
    double* part;
    Scal* S;
    unsigned* bar;
    T c_off;           // lambda / 2: A_ij = -c_off w_ij^2, rhs edge factor
    T gamma;           // shrink threshold 1 / lambda
    T half_r;          // r / 2
    double tol2;
    int maxit;
    int keep_split;
    int store_rhs;
    int b_zero;        // first edge update of a SOC iteration: b starts from 0
    int ortho;         // PFE_POLAR / PFE_CHOL
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int logical_block(int nblk) {
    int b = blockIdx.x;
    if ((nblk % kNumXcd) == 0) return (b % kNumXcd) * (nblk / kNumXcd) + b / kNumXcd;
    return b;
}

__device__ __forceinline__ void row_range(int lb, int nblk, int n, int& rb, int& re) {
    rb = (int)(((long long)n * lb) / nblk);
    re = (int)(((long long)n * (lb + 1)) / nblk);
}

__device__ __forceinline__ int ld_flag(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_flag(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T> __device__ __forceinline__ T fma_t(T a, T b, T c);
template <> __device__ __forceinline__ float fma_t<float>(float a, float b, float c) { return __fmaf_rn(a, b, c); }
template <> __device__ __forceinline__ double fma_t<double>(double a, double b, double c) { return __fma_rn(a, b, c); }
template <typename T> __device__ __forceinline__ T mul_t(T a, T b);
template <> __device__ __forceinline__ float mul_t<float>(float a, float b) { return __fmul_rn(a, b); }
template <> __device__ __forceinline__ double mul_t<double>(double a, double b) { return __dmul_rn(a, b); }

// Shrink(y, g) = sign(y) max(|y| - g, 0) written as max(y - g, 0) + min(y + g, 0)
// (one rounding, the same as the definition in Algorithm 2).
template <typename T>
__device__ __forceinline__ T shrink(T y, T g) {
    return fmax(y - g, T(0)) + fmin(y + g, T(0));
}

// Jacobi-preconditioned residual z = r / diag(A)
template <typename T>
__device__ __forceinline__ T zval(const KA<T>& a, int i, size_t e) {
    return mul_t(a.invdiag[i], a.r[e]);
}

// Z = D^{1/2} Y + B of the P-update
template <typename T>
__device__ __forceinline__ T zrow(const KA<T>& a, int i, size_t e) {
    return fma_t(a.sqrtD[i], a.Y[e], a.B[e]);
}

// per-thread FP64 accumulators -> one partial per (quantity, column) per workgroup
template <int NQ>
__device__ void block_partials(const double (&acc)[NQ], double* sh, int d, int R, double* part,
                               int nblk, int lb) {
    const int t = threadIdx.x;
    const int B = blockDim.x;
#pragma unroll
    for (int q = 0; q < NQ; ++q) sh[q * B + t] = (t < R * d) ? acc[q] : 0.0;
    __syncthreads();
    if (t < NQ * d) {
        int q = t / d, c = t - q * d;
        double s = 0.0;
        for (int k = 0; k < R; ++k) s += sh[q * B + k * d + c];
        part[((size_t)q * nblk + lb) * d + c] = s;
    }
    __syncthreads();
}

// out[k] = sum over workgroups b (in order) of part[(k / d) * nblk + b) * d + k % d]
// for k < nq * d; runs on one workgroup; sh needs >= max(blockDim, nq*d) doubles.
__device__ void reduce_parts(const double* part, int nblk, int d, int nq, double* out, double* sh) {
    const int pairs = nq * d;
    int team = (int)blockDim.x / pairs;
    if (team > 32) team = 32;
    if (team < 1) team = 1;
    for (int idx = threadIdx.x; idx < pairs * team; idx += blockDim.x) {
        int pr = idx / team, s = idx - pr * team;
        int q = pr / d, c = pr - q * d;
        const double* base = part + (size_t)q * nblk * d + c;
        double acc = 0.0;
        for (int b = s; b < nblk; b += team) acc += base[(size_t)b * d];
        sh[idx] = acc;
    }
    __syncthreads();
    for (int pr = threadIdx.x; pr < pairs; pr += blockDim.x) {
        double acc = 0.0;
        for (int s = 0; s < team; ++s) acc += sh[pr * team + s];
        out[pr] = acc;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Phases (each called by every workgroup for its rows)
// ---------------------------------------------------------------------------

// PH_E0 / PH_EU / PH_R0 / PH_RHS.  For every owned element (i, c):
//   EU : t = w (y_i - y_j) + b_s ; d_s = Shrink(t, 1/lambda) ; b_s = t - d_s   (Eqs. 9, 10)
//        rhs = lambda/2 sum_s w (d_s - b_s) + r/2 D^{1/2} (P - B)               (Eq. 13)
//   E0 : rhs = r/2 D^{1/2} (P - B)                   (b = d = 0 at the first inner step)
//   R0 : rhs from the stored rhs
//   RHS: rhs from the stored b and d
//   then (unless RHS) r = rhs - A x, with the FP64 partials of r^T z, r^T r, rhs^T rhs.
template <typename T>
__device__ void ph_residual(const KA<T>& a, int lb, int mode, int do_r0, double* sh) {
    const int d = a.d, R = a.R, t = threadIdx.x;
    int rb, re;
    row_range(lb, a.nblk, a.n, rb, re);
    double acc[3] = {0.0, 0.0, 0.0};
    if (t < R * d) {
        const int rl = t / d, c = t - rl * d;
        for (int i = rb + rl; i < re; i += R) {
            const size_t e = (size_t)i * d + c;
            const int s0 = a.rowptr[i], s1 = a.rowptr[i + 1];
            const T xi = a.x[e];
            T accR = T(0), accA = T(0);
            if (mode == PH_EU) {
                const T yi = a.Y[e];
                for (int s = s0; s < s1; ++s) {
                    const int j = a.col[s];
                    const T ww = a.w[s];
                    const size_t ej = (size_t)j * d + c;
                    const T yj = a.Y[ej];
                    const size_t es = (size_t)s * d + c;
                    const T bold = a.b_zero ? T(0) : a.bs[es];
                    const T tv = fma_t(ww, yi - yj, bold);
                    const T dv = shrink(tv, a.gamma);
                    const T bn = tv - dv;
                    a.bs[es] = bn;
                    if (a.keep_split) a.ds[es] = dv;
                    accR = fma_t(ww, dv - bn, accR);
                    if (do_r0) accA = fma_t(mul_t(ww, ww), a.x[ej], accA);
                }
            } else if (mode == PH_RHS) {
                for (int s = s0; s < s1; ++s) {
                    const size_t es = (size_t)s * d + c;
                    accR = fma_t(a.w[s], a.ds[es] - a.bs[es], accR);
                }
            } else if (do_r0) {
                for (int s = s0; s < s1; ++s) {
                    const int j = a.col[s];
                    const T ww = a.w[s];
                    accA = fma_t(mul_t(ww, ww), a.x[(size_t)j * d + c], accA);
                }
            }
            T rhs;
            if (mode == PH_R0) {
                rhs = a.rhs[e];
            } else {
                const T split = mul_t(a.half_r, mul_t(a.sqrtD[i], a.P[e] - a.B[e]));
                rhs = (mode == PH_E0) ? split : fma_t(a.c_off, accR, split);
                if (a.store_rhs || mode == PH_RHS) a.rhs[e] = rhs;
            }
            if (do_r0) {
                const T ax = fma_t(a.diagA[i], xi, -mul_t(a.c_off, accA));
                const T rv = rhs - ax;
                a.r[e] = rv;
                const T zv = mul_t(a.invdiag[i], rv);
                acc[0] += (double)rv * (double)zv;
                acc[1] += (double)rv * (double)rv;
                acc[2] += (double)rhs * (double)rhs;
            }
        }
    }
    if (do_r0) block_partials<3>(acc, sh, d, R, a.part, a.nblk, lb);
}

// PH_A: p_new = z + beta p_old (z = r / diag A), q = A p_new, partial p^T q.
// Neighbour values of p_new are recomputed from r and p_old, bit-identical to
// what their owner stores, so no separate p-update pass is needed.
template <typename T>
__device__ void ph_a(const KA<T>& a, int lb, double* sh) {
    const int d = a.d, R = a.R, t = threadIdx.x;
    int rb, re;
    row_range(lb, a.nblk, a.n, rb, re);
    const int it = ld_flag(&a.S->it);
    const bool first = (it == 0);
    T* pnew = (it & 1) ? a.pB : a.pA;
    const T* pold = (it & 1) ? a.pA : a.pB;
    double acc[1] = {0.0};
    if (t < R * d) {
        const int rl = t / d, c = t - rl * d;
        const T beta = (T)a.S->beta[c];
        for (int i = rb + rl; i < re; i += R) {
            const size_t e = (size_t)i * d + c;
            const T zi = zval(a, i, e);
            const T pi = first ? zi : fma_t(beta, pold[e], zi);
            const int s0 = a.rowptr[i], s1 = a.rowptr[i + 1];
            T accA = T(0);
            for (int s = s0; s < s1; ++s) {
                const int j = a.col[s];
                const T ww = a.w[s];
                const size_t ej = (size_t)j * d + c;
                const T zj = zval(a, j, ej);
                const T pj = first ? zj : fma_t(beta, pold[ej], zj);
                accA = fma_t(mul_t(ww, ww), pj, accA);
            }
            const T qi = fma_t(a.diagA[i], pi, -mul_t(a.c_off, accA));
            pnew[e] = pi;
            a.q[e] = qi;
            acc[0] += (double)pi * (double)qi;
        }
    }
    block_partials<1>(acc, sh, d, R, a.part, a.nblk, lb);
}

// PH_B: x += alpha p, r -= alpha q, partials of r^T z and r^T r.
template <typename T>
__device__ void ph_b(const KA<T>& a, int lb, double* sh) {
    const int d = a.d, R = a.R, t = threadIdx.x;
    int rb, re;
    row_range(lb, a.nblk, a.n, rb, re);
    const int it = ld_flag(&a.S->it);
    const T* p = (it & 1) ? a.pB : a.pA;
    double acc[2] = {0.0, 0.0};
    if (t < R * d) {
        const int rl = t / d, c = t - rl * d;
        const T alpha = (T)a.S->alpha[c];
        for (int i = rb + rl; i < re; i += R) {
            const size_t e = (size_t)i * d + c;
            const T xv = fma_t(alpha, p[e], a.x[e]);
            const T rv = fma_t(-alpha, a.q[e], a.r[e]);
            a.x[e] = xv;
            a.r[e] = rv;
            const T zv = mul_t(a.invdiag[i], rv);
            acc[0] += (double)rv * (double)zv;
            acc[1] += (double)rv * (double)rv;
        }
    }
    block_partials<2>(acc, sh, d, R, a.part, a.nblk, lb);
}

// PH_ZERO: x_c = 0 for columns with a zero right-hand side
template <typename T>
__device__ void ph_zero(const KA<T>& a, int lb) {
    const int d = a.d, R = a.R, t = threadIdx.x;
    int rb, re;
    row_range(lb, a.nblk, a.n, rb, re);
    if (t < R * d) {
        const int rl = t / d, c = t - rl * d;
        if (!a.S->zero[c]) return;
        for (int i = rb + rl; i < re; i += R) a.x[(size_t)i * d + c] = T(0);
    }
}

// PH_GRAM: FP64 Gram matrix of Z (mode 0: Z = D^{1/2} Y + B; mode 1: Z = D^{1/2} Y),
// upper triangle packed, one partial per workgroup.
template <typename T>
__device__ void ph_gram(const KA<T>& a, int lb, int mode, double* sh) {
    const int d = a.d, R = a.R, t = threadIdx.x;
    const int npair = d * (d + 1) / 2;
    int rb, re;
    row_range(lb, a.nblk, a.n, rb, re);
    double* zt = sh;                  // R x d staged rows
    // pair decode (row-major upper triangle): k -> (pa, pb), pa <= pb
    int pa[2] = {0, 0}, pb[2] = {0, 0};
    for (int h = 0; h < 2; ++h) {
        int k = t + h * (int)blockDim.x;
        if (k < npair) {
            int r = 0, off = 0;
            while (off + (d - r) <= k) { off += d - r; ++r; }
            pa[h] = r;
            pb[h] = r + (k - off);
        }
    }
    double acc[2] = {0.0, 0.0};
    for (int base = rb; base < re; base += R) {
        int rows = min(R, re - base);
        if (t < rows * d) {
            int rl = t / d, c = t - rl * d;
            int i = base + rl;
            size_t e = (size_t)i * d + c;
            T z = (mode == 0) ? zrow(a, i, e) : mul_t(a.sqrtD[i], a.Y[e]);
            zt[t] = (double)z;
        }
        __syncthreads();
        for (int h = 0; h < 2; ++h) {
            int k = t + h * (int)blockDim.x;
            if (k < npair) {
                double s = acc[h];
                for (int rr = 0; rr < rows; ++rr) s += zt[rr * d + pa[h]] * zt[rr * d + pb[h]];
                acc[h] = s;
            }
        }
        __syncthreads();
    }
    for (int h = 0; h < 2; ++h) {
        int k = t + h * (int)blockDim.x;
        if (k < npair) a.part[(size_t)lb * npair + k] = acc[h];
    }
}

// PH_APPLY: mode 0 (P-update): P = Z T, B = Z - P with Z = D^{1/2} Y + B;
//           mode 1 (initial orthonormalisation): Y <- Y T, P = D^{1/2} Y, B = 0.
template <typename T>
__device__ void ph_apply(const KA<T>& a, int lb, int mode, double* sh) {
    const int d = a.d, R = a.R, t = threadIdx.x;
    int rb, re;
    row_range(lb, a.nblk, a.n, rb, re);
    double* Ts = sh;                  // d x d
    double* zt = sh + kMaxD * kMaxD;  // R x d
    for (int k = t; k < d * d; k += blockDim.x) Ts[k] = a.S->T[(k / d) * kMaxD + (k % d)];
    for (int base = rb; base < re; base += R) {
        int rows = min(R, re - base);
        __syncthreads();
        if (t < rows * d) {
            int rl = t / d, c = t - rl * d;
            int i = base + rl;
            size_t e = (size_t)i * d + c;
            T z = (mode == 0) ? zrow(a, i, e) : a.Y[e];
            zt[t] = (double)z;
        }
        __syncthreads();
        if (t < rows * d) {
            int rl = t / d, c = t - rl * d;
            int i = base + rl;
            size_t e = (size_t)i * d + c;
            double s = 0.0;
            for (int k = 0; k < d; ++k) s += zt[rl * d + k] * Ts[k * d + c];
            if (mode == 0) {
                a.P[e] = (T)s;
                a.B[e] = (T)(zt[t] - s);
            } else {
                T y = (T)s;
                a.Y[e] = y;
                a.P[e] = mul_t(a.sqrtD[i], y);
                a.B[e] = T(0);
            }
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Finalisers (one workgroup, after every workgroup has written its partials)
// ---------------------------------------------------------------------------

// after PH_E0 / PH_EU / PH_R0: start of a PCG solve
template <typename T>
__device__ void fin_init(const KA<T>& a, double* sh) {
    const int d = a.d;
    double* out = sh + 1024;
    reduce_parts(a.part, a.nblk, d, 3, out, sh);
    if (threadIdx.x == 0) {
        int any = 0;
        for (int c = 0; c < d; ++c) {
            double rz = out[c], rr = out[d + c], bb = out[2 * d + c];
            a.S->rho[c] = rz;
            a.S->rr[c] = rr;
            a.S->bnorm2[c] = bb;
            a.S->beta[c] = 0.0;
            a.S->alpha[c] = 0.0;
            a.S->iters[c] = 0;
            int z = (bb == 0.0);
            a.S->zero[c] = z;
            int act = !z && (rr > a.tol2 * bb);
            a.S->active[c] = act;
            any |= act;
        }
        a.S->it = 0;
        a.S->done = !any;
    }
}

// after PH_A: alpha = rho / p^T q per active column; breakdown check
template <typename T>
__device__ void fin_a(const KA<T>& a, double* sh) {
    const int d = a.d;
    double* out = sh + 1024;
    reduce_parts(a.part, a.nblk, d, 1, out, sh);
    if (threadIdx.x == 0) {
        int bad = 0;
        for (int c = 0; c < d; ++c) {
            double al = 0.0;
            if (a.S->active[c]) {
                double pq = out[c];
                al = a.S->rho[c] / pq;
                if (!(pq > 0.0) || !isfinite(al)) { bad = 1; al = 0.0; }
            }
            a.S->alpha[c] = al;
        }
        if (bad) {
            a.S->status = PFE_E_NOT_SPD;
            a.S->done = 1;
        }
    }
}

// after PH_B: beta, convergence, iteration count, statistics
template <typename T>
__device__ void fin_b(const KA<T>& a, double* sh) {
    const int d = a.d;
    double* out = sh + 1024;
    reduce_parts(a.part, a.nblk, d, 2, out, sh);
    if (threadIdx.x == 0) {
        int any = 0;
        for (int c = 0; c < d; ++c) {
            int act = a.S->active[c];
            double rz = out[c], rr = out[d + c];
            if (act) {
                a.S->beta[c] = rz / a.S->rho[c];
                a.S->rho[c] = rz;
                a.S->rr[c] = rr;
                a.S->iters[c] += 1;
                act = rr > a.tol2 * a.S->bnorm2[c];
                if (!isfinite(rr)) { a.S->status = PFE_E_NOT_SPD; act = 0; }
            } else {
                a.S->beta[c] = 0.0;
            }
            a.S->active[c] = act;
            any |= act;
        }
        int it = a.S->it + 1;
        a.S->it = it;
        if (any && it >= a.maxit) {
            if (a.S->status == 0) a.S->status = PFE_E_NOCONV;
            any = 0;
        }
        a.S->done = !any;
    }
}

// called by thread 0 when a solve ends: accumulate statistics
template <typename T>
__device__ void solve_stats(const KA<T>& a) {
    int d = a.d, mx = 0;
    double rel = 0.0;
    for (int c = 0; c < d; ++c) {
        mx = max(mx, a.S->iters[c]);
        double bb = a.S->bnorm2[c];
        if (bb > 0.0) rel = fmax(rel, sqrt(a.S->rr[c] / bb));
    }
    a.S->solves += 1;
    a.S->iters_total += mx;
    a.S->iters_max = max(a.S->iters_max, mx);
    a.S->iters_last = mx;
    a.S->relres_max = fmax(a.S->relres_max, rel);
}

// d x d factor of the P-update, FP64, one workgroup.
//   G = Z^T Z (sum of the packed partials), Cholesky G = L L^T (rank check),
//   CHOL / init: T = L^{-T}  (Z T = Z R^{-1}, R = L^T);
//   POLAR: T = G^{-1/2} by the coupled Newton-Schulz iteration on G / s,
//   s = ||G||_inf, so that Z T is the orthogonal polar factor of Z.
template <typename T>
__device__ void fin_gram(const KA<T>& a, int mode, double* sh) {
    const int d = a.d, t = threadIdx.x, nb = blockDim.x;
    const int npair = d * (d + 1) / 2;
    // layout in sh: [0,1024) reduce scratch, G at 1024, L at 2048, M0 at 2048+1024...
    double* G = sh + 1024;
    double* L = sh + 2048;
    double* Ym = sh + 3072;
    double* Zm = sh + 3072 + 512;   // only for d <= 22 (d*d <= 512); larger d uses Gm
    double* red = sh + 4096;
    // packed partials: part[lb * npair + k], summed in workgroup order
    reduce_parts(a.part, a.nblk, npair, 1, L, sh);
    for (int k = t; k < npair; k += nb) {
        int r = 0, off = 0;
        while (off + (d - r) <= k) { off += d - r; ++r; }
        int cc = r + (k - off);
        G[r * d + cc] = L[k];
        G[cc * d + r] = L[k];
    }
    __syncthreads();
    // Cholesky (lower), on a copy in L
    for (int k = t; k < d * d; k += nb) L[k] = G[k];
    __shared__ int s_bad;
    if (t == 0) s_bad = 0;
    __syncthreads();
    for (int k = 0; k < d; ++k) {
        if (t == 0) {
            // a pivot that lost all but ~13 digits of G_kk means rank deficiency
            double v = L[k * d + k];
            if (!(v > 1e-13 * G[k * d + k]) || !isfinite(v)) { s_bad = 1; v = 1.0; }
            L[k * d + k] = sqrt(v);
        }
        __syncthreads();
        for (int i = k + 1 + t; i < d; i += nb) L[i * d + k] /= L[k * d + k];
        __syncthreads();
        for (int idx = t; idx < d * d; idx += nb) {
            int i = idx / d, j = idx - i * d;
            if (j > k && i >= j) L[i * d + j] -= L[i * d + k] * L[j * d + k];
        }
        __syncthreads();
    }
    if (s_bad) {
        if (t == 0) {
            a.S->ortho_ok = 0;
            a.S->status = PFE_E_RANK;
        }
        __syncthreads();
        return;
    }
    if (mode == 1 || a.ortho == PFE_CHOL) {
        // T = L^{-T}: column c of L^{-1} by forward substitution, T[a][c] = Linv[c][a]
        for (int c = t; c < d; c += nb) {
            for (int i = 0; i < d; ++i) {
                double s = (i == c) ? 1.0 : 0.0;
                for (int k = c; k < i; ++k) s -= L[i * d + k] * Ym[k * kMaxD + c];
                Ym[i * kMaxD + c] = (i < c) ? 0.0 : s / L[i * d + i];
            }
        }
        __syncthreads();
        for (int idx = t; idx < d * d; idx += nb) {
            int r = idx / d, c = idx - r * d;
            a.S->T[r * kMaxD + c] = Ym[c * kMaxD + r];
        }
    } else {
        // coupled Newton-Schulz for (G/s)^{-1/2}
        __shared__ double s_scale;
        if (t == 0) {
            double s = 0.0;
            for (int i = 0; i < d; ++i) {
                double rs = 0.0;
                for (int j = 0; j < d; ++j) rs += fabs(G[i * d + j]);
                s = fmax(s, rs);
            }
            s_scale = s;
        }
        __syncthreads();
        const double s = s_scale;
        double* Yk = Ym;          // d x d, stride d
        double* Zk = L;           // reuse L storage (Cholesky no longer needed)
        double* Mk = G;           // reuse G storage
        double* Wk = Zm;          // scratch
        const int dd = d * d;
        double* big = sh;         // when d*d > 512, scratch lives in the reduce area
        if (dd > 512) Wk = big;
        for (int k = t; k < dd; k += nb) {
            Yk[k] = G[k] / s;
            Zk[k] = ((k / d) == (k % d)) ? 1.0 : 0.0;
        }
        __syncthreads();
        __shared__ double s_err;
        double prev = INFINITY;
        for (int iter = 0; iter < 100; ++iter) {
            // M = Z Y
            double emax = 0.0;
            for (int k = t; k < dd; k += nb) {
                int i = k / d, j = k - i * d;
                double acc = 0.0;
                for (int m = 0; m < d; ++m) acc += Zk[i * d + m] * Yk[m * d + j];
                Wk[k] = acc;
                emax = fmax(emax, fabs(acc - ((i == j) ? 1.0 : 0.0)));
            }
            red[t] = emax;
            __syncthreads();
            if (t == 0) {
                double e = 0.0;
                for (int k = 0; k < nb; ++k) e = fmax(e, red[k]);
                s_err = e;
            }
            __syncthreads();
            // stop at rounding level: tiny, or no longer shrinking quadratically
            if (s_err < 1e-14 || !isfinite(s_err) || (s_err < 1e-11 && s_err > 0.25 * prev)) break;
            prev = s_err;
            // T = (3 I - M) / 2, kept in Mk
            for (int k = t; k < dd; k += nb) {
                int i = k / d, j = k - i * d;
                Mk[k] = 0.5 * (((i == j) ? 3.0 : 0.0) - Wk[k]);
            }
            __syncthreads();
            // Y <- Y T (into Wk), Z <- T Z (into Yk after copy)
            for (int k = t; k < dd; k += nb) {
                int i = k / d, j = k - i * d;
                double acc = 0.0;
                for (int m = 0; m < d; ++m) acc += Yk[i * d + m] * Mk[m * d + j];
                Wk[k] = acc;
            }
            __syncthreads();
            for (int k = t; k < dd; k += nb) Yk[k] = Wk[k];
            __syncthreads();
            for (int k = t; k < dd; k += nb) {
                int i = k / d, j = k - i * d;
                double acc = 0.0;
                for (int m = 0; m < d; ++m) acc += Mk[i * d + m] * Zk[m * d + j];
                Wk[k] = acc;
            }
            __syncthreads();
            for (int k = t; k < dd; k += nb) Zk[k] = Wk[k];
            __syncthreads();
        }
        const double is = 1.0 / sqrt(s);
        for (int k = t; k < dd; k += nb) {
            int r = k / d, c = k - r * d;
            a.S->T[r * kMaxD + c] = Zk[k] * is;
        }
        if (t == 0 && !(s_err < 1e-10)) {
            a.S->ortho_ok = 0;
            a.S->status = PFE_E_RANK;
            return;
        }
    }
    if (t == 0) a.S->ortho_ok = 1;
}

// ---------------------------------------------------------------------------
// Grid-wide synchronisation
// ---------------------------------------------------------------------------

// Fences: one thread per workgroup publishes and acquires.  __syncthreads()
// completes the stores of every wave of the workgroup (the vector L1 is
// write-through), so thread 0's agent-scope release covers them, and its
// agent-scope acquire invalidates the caches the whole workgroup reads through.
__device__ __forceinline__ void fence_acquire_agent() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// Multi-launch path: the last workgroup to finish a phase runs its finaliser.
__device__ bool last_block(unsigned* counter, unsigned nblk) {
    __shared__ int s_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = (prev == nblk - 1);
        if (s_last) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    return s_last;
}

// Persistent path: barrier over all co-resident workgroups; the last to
// arrive runs fin() before releasing the others.  Waiters poll with relaxed
// loads (no cache invalidation per poll) and acquire once.  The wait is
// bounded: after kSpinLimit polls a workgroup raises abort_flag and the kernel
// unwinds (every later barrier returns at once).
constexpr long long kSpinLimit = 1ll << 25;

template <class F>
__device__ bool grid_sync(unsigned* bar, unsigned nblk, Scal* S, F&& fin) {
    __shared__ int s_last;
    __shared__ int s_abort;
    __syncthreads();
    if (threadIdx.x == 0) {
        s_abort = 0;
        unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned prev = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = (prev == nblk - 1);
        if (!s_last) {
            long long spins = 0;
            while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(1);
                if ((++spins & 1023) == 0) {
                    if (ld_flag(&S->abort_flag) || spins > kSpinLimit) {
                        st_flag(&S->abort_flag, 1);
                        s_abort = 1;
                        break;
                    }
                }
            }
            fence_acquire_agent();
        }
    }
    __syncthreads();
    if (s_abort) return false;
    if (s_last) {
        fin();
        __syncthreads();
        if (threadIdx.x == 0) {
            __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    }
    return true;
}

struct NoFin {
    __device__ void operator()() const {}
};

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// One phase per launch; the last workgroup finalises.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_phase(KA<T> a, int ph, int mode, int do_r0) {
    __shared__ double sh[kSmemDoubles];
    const int lb = logical_block(a.nblk);
    if ((ph == PH_A || ph == PH_B) && ld_flag(&a.S->done)) return;
    switch (ph) {
        case PH_E0: case PH_EU: case PH_R0: case PH_RHS:
            ph_residual(a, lb, ph, do_r0, sh);
            if (do_r0 && last_block(a.bar, a.nblk)) fin_init(a, sh);
            break;
        case PH_A:
            ph_a(a, lb, sh);
            if (last_block(a.bar, a.nblk)) fin_a(a, sh);
            break;
        case PH_B:
            ph_b(a, lb, sh);
            if (last_block(a.bar, a.nblk)) {
                fin_b(a, sh);
                if (threadIdx.x == 0 && a.S->done) solve_stats(a);
            }
            break;
        case PH_ZERO:
            ph_zero(a, lb);
            break;
        case PH_GRAM:
            ph_gram(a, lb, mode, sh);
            if (last_block(a.bar, a.nblk)) fin_gram(a, mode, sh);
            break;
        case PH_APPLY:
            if (!ld_flag(&a.S->ortho_ok)) return;
            ph_apply(a, lb, mode, sh);
            break;
    }
}

// statistics when a solve finished before its first iteration
template <typename T>
__global__ void k_stats_if_done(KA<T> a) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && a.S->done && a.S->it == 0) solve_stats(a);
}

struct Plan {
    int l_begin;      // first inner index of the first SOC iteration
    int n_inner;      // inner iterations per SOC iteration
    int n_outer;      // SOC iterations to run
    int skip_last_eu; // the edge update after the last solve is not needed
};

// Persistent path: whole SOC iterations in one cooperative launch.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_soc(KA<T> a_in, Plan plan) {
    KA<T> a = a_in;
    __shared__ double sh[kSmemDoubles];
    const int lb = logical_block(a.nblk);
    const unsigned nb = (unsigned)a.nblk;
    Scal* S = a.S;
    int l0 = plan.l_begin;
    for (int outer = 0; outer < plan.n_outer; ++outer) {
        for (int l = l0; l < plan.n_inner; ++l) {
            a.b_zero = (l == 1);
            ph_residual(a, lb, (l == 0) ? PH_E0 : PH_EU, 1, sh);
            if (!grid_sync(a.bar, nb, S, [&] { fin_init(a, sh); })) return;
            while (!ld_flag(&S->done)) {
                ph_a(a, lb, sh);
                if (!grid_sync(a.bar, nb, S, [&] { fin_a(a, sh); })) return;
                if (ld_flag(&S->done)) break;
                ph_b(a, lb, sh);
                if (!grid_sync(a.bar, nb, S, [&] { fin_b(a, sh); })) return;
            }
            if (lb == 0 && threadIdx.x == 0) solve_stats(a);
            int any_zero = 0;
            for (int c = 0; c < a.d; ++c) any_zero |= a.S->zero[c];
            if (any_zero) {
                // columns with a zero right-hand side: x_c = 0
                ph_zero(a, lb);
                if (!grid_sync(a.bar, nb, S, NoFin{})) return;
            }
        }
        l0 = 0;
        ph_gram(a, lb, 0, sh);
        if (!grid_sync(a.bar, nb, S, [&] { fin_gram(a, 0, sh); })) return;
        if (ld_flag(&S->ortho_ok)) ph_apply(a, lb, 0, sh);
        else return;
        // P, B of each row are written and read by the same workgroup; the
        // next barrier (after the first residual phase) orders the rest.
    }
}

template <typename T>
__global__ void k_spmm(KA<T> a, const T* __restrict__ X, T* __restrict__ Q) {
    const int d = a.d, R = a.R, t = threadIdx.x;
    const int lb = blockIdx.x;
    int rb, re;
    row_range(lb, gridDim.x, a.n, rb, re);
    if (t >= R * d) return;
    const int rl = t / d, c = t - rl * d;
    for (int i = rb + rl; i < re; i += R) {
        const size_t e = (size_t)i * d + c;
        T acc = T(0);
        for (int s = a.rowptr[i]; s < a.rowptr[i + 1]; ++s) {
            const T ww = a.w[s];
            acc = fma_t(mul_t(ww, ww), X[(size_t)a.col[s] * d + c], acc);
        }
        Q[e] = fma_t(a.diagA[i], X[e], -mul_t(a.c_off, acc));
    }
}

// diagonal of A = lambda/2 M^T M + r/2 D in FP64, and D^{+-1/2}
template <typename T>
__global__ void k_diag(int n, const double* __restrict__ degree, const double* __restrict__ wsq,
                       double half_lam, double half_r, T* diagA, T* invdiag, T* sqrtD, T* isqrtD) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double da = half_lam * wsq[i] + half_r * degree[i];
    diagA[i] = (T)da;
    invdiag[i] = (T)(1.0 / da);
    sqrtD[i] = (T)sqrt(degree[i]);
    isqrtD[i] = (T)(1.0 / sqrt(degree[i]));
}

// per-slot state <-> per-undirected-edge blocks (orientation: lower index minus upper)
template <typename T>
__global__ void k_slots_to_edges(int n, int d, const int* __restrict__ rowptr, const int* __restrict__ col,
                                 const int* __restrict__ eid, const T* __restrict__ s, T* __restrict__ e) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
        if (col[k] <= i) continue;
        size_t eo = (size_t)eid[k] * d, so = (size_t)k * d;
        for (int c = 0; c < d; ++c) e[eo + c] = s[so + c];
    }
}

template <typename T>
__global__ void k_edges_to_slots(int n, int d, const int* __restrict__ rowptr, const int* __restrict__ col,
                                 const int* __restrict__ eid, const T* __restrict__ e, T* __restrict__ s) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
        size_t eo = (size_t)eid[k] * d, so = (size_t)k * d;
        bool up = col[k] > i;
        for (int c = 0; c < d; ++c) s[so + c] = up ? e[eo + c] : -e[eo + c];
    }
}

template <typename T>
__global__ void k_yhat(size_t nd, int d, const T* __restrict__ isqrtD, const T* __restrict__ P, T* __restrict__ out) {
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nd) return;
    out[e] = mul_t(isqrtD[e / d], P[e]);
}

// Monitors: objective ||M Yhat||_1 (FP64 over upper slots), ||D^{1/2}Y - P||^2,
// ||P||^2, Gram P^T P and Yhat^T D Yhat (packed); one partial set per block.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_monitor(KA<T> a) {
    __shared__ double sh[kSmemDoubles];
    const int d = a.d, R = a.R, t = threadIdx.x;
    const int lb = blockIdx.x;
    const int npair = d * (d + 1) / 2;
    const int nq = 3 + 2 * npair;     // objective, split^2, P^2, PtP pairs, YDY pairs
    int rb, re;
    row_range(lb, a.nblk, a.n, rb, re);
    double* pz = sh;             // R x d P rows
    double* yz = sh + kBlock;    // R x d Yhat rows
    double obj = 0.0, spl = 0.0, pp = 0.0;
    double g1[2] = {0.0, 0.0}, g2[2] = {0.0, 0.0};
    int pa[2] = {0, 0}, pb[2] = {0, 0};
    for (int h = 0; h < 2; ++h) {
        int k = t + h * (int)blockDim.x;
        if (k < npair) {
            int r = 0, off = 0;
            while (off + (d - r) <= k) { off += d - r; ++r; }
            pa[h] = r;
            pb[h] = r + (k - off);
        }
    }
    for (int base = rb; base < re; base += R) {
        int rows = min(R, re - base);
        if (t < rows * d) {
            int rl = t / d, c = t - rl * d;
            int i = base + rl;
            size_t e = (size_t)i * d + c;
            T yh = mul_t(a.isqrtD[i], a.P[e]);
            for (int s = a.rowptr[i]; s < a.rowptr[i + 1]; ++s) {
                int j = a.col[s];
                if (j <= i) continue;
                T yj = mul_t(a.isqrtD[j], a.P[(size_t)j * d + c]);
                obj += fabs((double)a.w[s] * ((double)yh - (double)yj));
            }
            double dv = (double)mul_t(a.sqrtD[i], a.Y[e]) - (double)a.P[e];
            spl += dv * dv;
            pp += (double)a.P[e] * (double)a.P[e];
            pz[t] = (double)a.P[e];
            yz[t] = (double)yh * sqrt(a.degree[i]);
        }
        __syncthreads();
        for (int h = 0; h < 2; ++h) {
            int k = t + h * (int)blockDim.x;
            if (k < npair)
                for (int rr = 0; rr < rows; ++rr) {
                    g1[h] += pz[rr * d + pa[h]] * pz[rr * d + pb[h]];
                    g2[h] += yz[rr * d + pa[h]] * yz[rr * d + pb[h]];
                }
        }
        __syncthreads();
    }
    // block sums of obj, spl, pp
    double* red = sh + 2 * kBlock;
    red[t] = obj;
    red[kBlock + t] = spl;
    red[2 * kBlock + t] = pp;
    __syncthreads();
    double* out = a.part + (size_t)lb * nq;
    if (t < 3) {
        double s = 0.0;
        for (int k = 0; k < (int)blockDim.x; ++k) s += red[t * kBlock + k];
        out[t] = s;
    }
    for (int h = 0; h < 2; ++h) {
        int k = t + h * (int)blockDim.x;
        if (k < npair) {
            out[3 + k] = g1[h];
            out[3 + npair + k] = g2[h];
        }
    }
    if (last_block(a.bar, a.nblk)) {
        for (int k = t; k < nq; k += blockDim.x) {
            double s = 0.0;
            for (int b = 0; b < a.nblk; ++b) s += a.part[(size_t)b * nq + k];
            sh[k] = s;
        }
        __syncthreads();
        if (t == 0) {
            double cmax = 0.0, omax = 0.0;
            for (int k = 0; k < npair; ++k) {
                int r = 0, off = 0;
                while (off + (d - r) <= k) { off += d - r; ++r; }
                int cc = r + (k - off);
                double id = (r == cc) ? 1.0 : 0.0;
                omax = fmax(omax, fabs(sh[3 + k] - id));
                cmax = fmax(cmax, fabs(sh[3 + npair + k] - id));
            }
            a.S->mon[0] = sh[0];
            a.S->mon[1] = cmax;
            a.S->mon[2] = sqrt(sh[1]) / sqrt(sh[2]);
            a.S->mon[3] = omax;
        }
    }
}

// |M Y| histogram passes for the exact order statistic (radix select on the
// bit pattern of the non-negative value, 3 passes of 12 + 12 + 8 bits).
template <typename T> struct Bits;
template <> struct Bits<float> { typedef unsigned U; static constexpr int W = 32; };
template <> struct Bits<double> { typedef unsigned long long U; static constexpr int W = 64; };

template <typename T>
__global__ void k_hist(KA<T> a, int shift, int nbits, unsigned long long prefix, int pshift,
                       unsigned* __restrict__ hist) {
    typedef typename Bits<T>::U U;
    const int d = a.d;
    __shared__ unsigned sh[4096];
    const int nbins = 1 << nbits;
    for (int k = threadIdx.x; k < nbins; k += blockDim.x) sh[k] = 0;
    __syncthreads();
    size_t total = (size_t)a.n * d;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        int i = (int)(e / d), c = (int)(e - (size_t)i * d);
        T yi = a.Y[e];
        for (int s = a.rowptr[i]; s < a.rowptr[i + 1]; ++s) {
            int j = a.col[s];
            if (j <= i) continue;
            T v = fabs(mul_t(a.w[s], yi - a.Y[(size_t)j * d + c]));
            U u;
            memcpy(&u, &v, sizeof(T));
            if (pshift < Bits<T>::W && (unsigned long long)(u >> pshift) != prefix) continue;
            atomicAdd(&sh[(unsigned)((u >> shift) & (U)(nbins - 1))], 1u);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nbins; k += blockDim.x)
        if (sh[k]) atomicAdd(&hist[k], sh[k]);
}

}  // namespace pfe

// ===========================================================================
// Host side
// ===========================================================================
using namespace pfe;

struct pfe_ctx {
    pfe_graph* g = nullptr;
    pfe_params prm{};
    hipStream_t stream = nullptr;
    int device = 0;
    int esz = 4;
    int64_t n = 0, d = 0, slots = 0;
    int inner = 0;           // inner iterations done in the current SOC iteration
    int nblk = 0;            // workgroups of the multi-launch path
    int nblk_coop = 0;       // workgroups of the persistent path
    void* Y = nullptr; void* P = nullptr; void* B = nullptr;
    void* bs = nullptr; void* ds = nullptr;
    void* rhs = nullptr; void* r = nullptr; void* pA = nullptr; void* pB = nullptr; void* q = nullptr;
    void* diagA = nullptr; void* invdiag = nullptr; void* sqrtD = nullptr; void* isqrtD = nullptr;
    double* part = nullptr;
    size_t part_doubles = 0;
    Scal* S = nullptr;
    unsigned* bar = nullptr;
    unsigned* hist = nullptr;
};

namespace {

template <typename T>
KA<T> make_args(pfe_ctx* c, int nblk) {
    KA<T> a{};
    a.n = (int)c->n;
    a.d = (int)c->d;
    a.R = kBlock / (int)c->d;
    a.nblk = nblk;
    a.rowptr = c->g->rowptr;
    a.col = c->g->col;
    if (sizeof(T) == 4) a.w = (const T*)c->g->w32; else a.w = (const T*)c->g->w64;
    a.diagA = (const T*)c->diagA;
    a.invdiag = (const T*)c->invdiag;
    a.sqrtD = (const T*)c->sqrtD;
    a.isqrtD = (const T*)c->isqrtD;
    a.degree = c->g->degree;
    a.x = (T*)c->Y;
    a.Y = (T*)c->Y;
    a.P = (T*)c->P;
    a.B = (T*)c->B;
    a.bs = (T*)c->bs;
    a.ds = (T*)c->ds;
    a.rhs = (T*)c->rhs;
    a.r = (T*)c->r;
    a.pA = (T*)c->pA;
    a.pB = (T*)c->pB;
    a.q = (T*)c->q;
    a.part = c->part;
    a.S = c->S;
    a.bar = c->bar;
    a.c_off = (T)(0.5 * c->prm.lambda);
    a.gamma = (c->prm.lambda > 0.0) ? (T)(1.0 / c->prm.lambda) : (T)INFINITY;
    a.half_r = (T)(0.5 * c->prm.r);
    a.tol2 = c->prm.tol * c->prm.tol;
    a.maxit = c->prm.maxit;
    a.keep_split = c->prm.keep_split;
    a.store_rhs = 0;
    a.ortho = c->prm.ortho;
    return a;
}

template <typename T>
pfe_status launch_phase(pfe_ctx* c, const KA<T>& a, int ph, int mode, int do_r0) {
    hipLaunchKernelGGL(k_phase<T>, dim3(a.nblk), dim3(kBlock), 0, c->stream, a, ph, mode, do_r0);
    PFE_CHECK_HIP(hipGetLastError());
    return PFE_OK;
}

#define PFE_TRY(x) do { pfe_status s__ = (x); if (s__ != PFE_OK) return s__; } while (0)

// Multi-launch PCG loop after a residual phase; the host polls the done flag
// every few iterations.
template <typename T>
pfe_status pcg_loop_mk(pfe_ctx* c, const KA<T>& a) {
    hipLaunchKernelGGL(k_stats_if_done<T>, dim3(1), dim3(64), 0, c->stream, a);
    int it = 0;
    const int chunk = 4;
    int done = 0;
    while (true) {
        for (int k = 0; k < chunk; ++k) {
            PFE_TRY(launch_phase(c, a, PH_A, 0, 0));
            PFE_TRY(launch_phase(c, a, PH_B, 0, 0));
        }
        it += chunk;
        PFE_CHECK_HIP(hipMemcpyAsync(&done, &c->S->done, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        PFE_CHECK_HIP(hipStreamSynchronize(c->stream));
        if (done || it > c->prm.maxit + chunk) break;
    }
    PFE_TRY(launch_phase(c, a, PH_ZERO, 0, 0));
    return PFE_OK;
}

template <typename T>
pfe_status inner_mk(pfe_ctx* c, bool store_next) {
    KA<T> a = make_args<T>(c, c->nblk);
    // residual / rhs for this solve
    if (c->inner == 0) {
        PFE_TRY(launch_phase(c, a, PH_E0, 0, 1));
    } else {
        PFE_TRY(launch_phase(c, a, PH_R0, 0, 1));
    }
    PFE_TRY(pcg_loop_mk(c, a));
    // edge update of this inner step and rhs of the next one
    KA<T> b = a;
    b.store_rhs = 1;
    b.b_zero = (c->inner == 0);
    PFE_TRY(launch_phase(c, b, PH_EU, 0, 0));
    (void)store_next;
    c->inner += 1;
    return PFE_OK;
}

template <typename T>
pfe_status ortho_mk(pfe_ctx* c, int mode) {
    KA<T> a = make_args<T>(c, c->nblk);
    PFE_TRY(launch_phase(c, a, PH_GRAM, mode, 0));
    PFE_TRY(launch_phase(c, a, PH_APPLY, mode, 0));
    return PFE_OK;
}

template <typename T>
pfe_status outer_mk(pfe_ctx* c) {
    while (c->inner < c->prm.n_inner) PFE_TRY(inner_mk<T>(c, true));
    PFE_TRY(ortho_mk<T>(c, 0));
    c->inner = 0;
    return PFE_OK;
}

template <typename T>
pfe_status outer_coop(pfe_ctx* c, int n_outer) {
    KA<T> a = make_args<T>(c, c->nblk_coop);
    Plan plan{c->inner, c->prm.n_inner, n_outer, 1};
    if (c->inner > 0) {
        // resuming mid-iteration: the next solve starts from the stored rhs
        KA<T> m = make_args<T>(c, c->nblk);
        PFE_TRY(launch_phase(c, m, PH_R0, 0, 1));
        PFE_TRY(pcg_loop_mk(c, m));
        KA<T> b = m;
        b.store_rhs = 1;
        c->inner += 1;
        if (c->inner < c->prm.n_inner) PFE_TRY(launch_phase(c, b, PH_EU, 0, 0));
        // the remaining inner steps of this SOC iteration use the multi-launch path
        while (c->inner < c->prm.n_inner) PFE_TRY(inner_mk<T>(c, true));
        PFE_TRY(ortho_mk<T>(c, 0));
        c->inner = 0;
        n_outer -= 1;
        plan.l_begin = 0;
        if (n_outer == 0) return PFE_OK;
    }
    plan.n_outer = n_outer;
    PFE_CHECK_HIP(hipMemsetAsync(c->bar, 0, 2 * sizeof(unsigned), c->stream));
    void* args[] = {(void*)&a, (void*)&plan};
    PFE_CHECK_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_soc<T>), dim3(a.nblk),
                                             dim3(kBlock), args, 0, c->stream));
    c->inner = 0;
    return PFE_OK;
}

pfe_status read_info(pfe_ctx* c, pfe_step_info* info) {
    Scal h;
    PFE_CHECK_HIP(hipMemcpyAsync(&h, c->S, sizeof(Scal), hipMemcpyDeviceToHost, c->stream));
    PFE_CHECK_HIP(hipStreamSynchronize(c->stream));
    if (h.abort_flag) { set_error("grid barrier timed out"); return PFE_E_HIP; }
    if (info) {
        info->solves = h.solves;
        info->cg_iters_total = h.iters_total;
        info->cg_iters_max = h.iters_max;
        info->cg_iters_last = h.iters_last;
        info->rel_res_max = h.relres_max;
        info->status = h.status;
        info->fallbacks = h.fallbacks;
    }
    if (h.status != 0) {
        set_error("%s", pfe_status_string((pfe_status)h.status));
        return (pfe_status)h.status;
    }
    return PFE_OK;
}

pfe_status reset_stats(pfe_ctx* c) {
    // statistics and status are the tail of Scal starting at 'status'
    size_t off = offsetof(Scal, status);
    PFE_CHECK_HIP(hipMemsetAsync((char*)c->S + off, 0, sizeof(int), c->stream));
    off = offsetof(Scal, solves);
    PFE_CHECK_HIP(hipMemsetAsync((char*)c->S + off, 0, sizeof(Scal) - off, c->stream));
    return PFE_OK;
}

template <typename T>
pfe_status set_diag(pfe_ctx* c) {
    int n = (int)c->n;
    hipLaunchKernelGGL(k_diag<T>, dim3((n + 255) / 256), dim3(256), 0, c->stream, n, c->g->degree, c->g->wsq,
                       0.5 * c->prm.lambda, 0.5 * c->prm.r, (T*)c->diagA, (T*)c->invdiag, (T*)c->sqrtD,
                       (T*)c->isqrtD);
    PFE_CHECK_HIP(hipGetLastError());
    return PFE_OK;
}

void free_ctx(pfe_ctx* c) {
    void* bufs[] = {c->Y, c->P, c->B, c->bs, c->ds, c->rhs, c->r, c->pA, c->pB, c->q,
                    c->diagA, c->invdiag, c->sqrtD, c->isqrtD, c->part, c->S, c->bar, c->hist};
    for (void* p : bufs)
        if (p) (void)hipFree(p);
}

bool params_ok(const pfe_params* p, int64_t n) {
    if (p->d < 1 || p->d > kMaxD || p->d >= n) { set_error("d must be in [1, %d] and below n", kMaxD); return false; }
    if (!(p->lambda >= 0.0) || !std::isfinite(p->lambda)) { set_error("lambda must be >= 0"); return false; }
    if (!(p->r > 0.0) || !std::isfinite(p->r)) { set_error("r must be > 0"); return false; }
    if (p->n_inner < 1) { set_error("n_inner must be >= 1"); return false; }
    if (!(p->tol > 0.0) || p->maxit < 1) { set_error("tol must be > 0 and maxit >= 1"); return false; }
    if (p->precond != PFE_JACOBI) { set_error("preconditioner not available"); return false; }
    if (p->ortho != PFE_POLAR && p->ortho != PFE_CHOL) { set_error("unknown ortho mode"); return false; }
    if (p->dtype != PFE_FP32 && p->dtype != PFE_FP64) { set_error("unknown dtype"); return false; }
    return true;
}

template <typename T>
pfe_status monitor_impl(pfe_ctx* c, pfe_monitors* out) {
    KA<T> a = make_args<T>(c, c->nblk);
    hipLaunchKernelGGL(k_monitor<T>, dim3(a.nblk), dim3(kBlock), 0, c->stream, a);
    PFE_CHECK_HIP(hipGetLastError());
    double mon[4];
    PFE_CHECK_HIP(hipMemcpyAsync(mon, c->S->mon, sizeof(mon), hipMemcpyDeviceToHost, c->stream));
    PFE_CHECK_HIP(hipStreamSynchronize(c->stream));
    out->objective = mon[0];
    out->constraint = mon[1];
    out->split = mon[2];
    out->orthogonality = mon[3];
    return PFE_OK;
}

template <typename T>
pfe_status quantile_impl(pfe_ctx* c, double q, double* out) {
    typedef typename Bits<T>::U U;
    KA<T> a = make_args<T>(c, c->nblk);
    const int W = Bits<T>::W;
    // passes over the top bits; float: 12+12+8, double: 16+16+16+16
    int widths[4];
    int np;
    if (W == 32) { widths[0] = 12; widths[1] = 12; widths[2] = 8; np = 3; }
    else { widths[0] = 12; widths[1] = 12; widths[2] = 12; widths[3] = 12; np = 4; }
    unsigned long long total = (unsigned long long)c->g->n_edges * c->d;
    if (total == 0) { set_error("no edges"); return PFE_E_STATE; }
    unsigned long long k = (unsigned long long)floor(q * (double)(total - 1));
    unsigned long long prefix = 0;
    int consumed = 0;
    std::vector<unsigned> h(4096);
    for (int pz = 0; pz < np; ++pz) {
        int nb = widths[pz];
        int shift = W - consumed - nb;
        PFE_CHECK_HIP(hipMemsetAsync(c->hist, 0, sizeof(unsigned) * 4096, c->stream));
        int pshift = W - consumed;   // consumed == 0 -> no prefix filter (pshift == W)
        hipLaunchKernelGGL(k_hist<T>, dim3(1024), dim3(256), 0, c->stream, a, shift, nb, prefix, pshift, c->hist);
        PFE_CHECK_HIP(hipGetLastError());
        PFE_CHECK_HIP(hipMemcpyAsync(h.data(), c->hist, sizeof(unsigned) * 4096, hipMemcpyDeviceToHost, c->stream));
        PFE_CHECK_HIP(hipStreamSynchronize(c->stream));
        unsigned long long cum = 0;
        int bin = 0;
        for (; bin < (1 << nb); ++bin) {
            if (cum + h[bin] > k) break;
            cum += h[bin];
        }
        if (bin == (1 << nb)) { set_error("quantile selection failed"); return PFE_E_STATE; }
        k -= cum;
        prefix = (prefix << nb) | (unsigned long long)bin;
        consumed += nb;
        if (W == 64 && pz == np - 1 && consumed < W) {
            // remaining low bits are not resolved; the value is the bin's lower edge
        }
    }
    U u = (U)(prefix << (W - consumed));
    T v;
    memcpy(&v, &u, sizeof(T));
    *out = (double)v;
    return PFE_OK;
}

}  // namespace

extern "C" {

pfe_status pfe_init(pfe_graph* g, const pfe_params* p, const void* Y0, hipStream_t stream, pfe_ctx** out) {
    if (!g || !p || !Y0 || !out) { set_error("pfe_init: null argument"); return PFE_E_ARG; }
    *out = nullptr;
    if (!params_ok(p, g->n)) return PFE_E_ARG;
    pfe_ctx* c = new pfe_ctx();
    c->g = g;
    c->prm = *p;
    c->stream = stream;
    PFE_CHECK_HIP(hipGetDevice(&c->device));
    c->esz = (p->dtype == PFE_FP64) ? 8 : 4;
    c->n = g->n;
    c->d = p->d;
    c->slots = g->slots;
    const size_t nd = (size_t)c->n * c->d * c->esz;
    const size_t sd = (size_t)(c->slots + 1) * c->d * c->esz;
    const size_t nv = (size_t)c->n * c->esz;
    // workgroup counts
    int ncu = 0;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) { delete c; set_error("hipGetDeviceProperties failed"); return PFE_E_HIP; }
    ncu = prop.multiProcessorCount;
    const int R = kBlock / (int)c->d;
    int64_t want = (c->n + R - 1) / R;
    c->nblk = (int)std::max<int64_t>(1, std::min<int64_t>(want, 2048));
    if (c->nblk >= kNumXcd) c->nblk -= c->nblk % kNumXcd;
    int occ = 0;
    hipError_t oe = (p->dtype == PFE_FP64)
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)k_soc<double>, kBlock, 0)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)k_soc<float>, kBlock, 0);
    if (oe != hipSuccess) occ = 0;
    int per_cu = std::max(0, std::min(occ, 2));
    c->nblk_coop = per_cu * ncu;
    if (c->nblk_coop > want) c->nblk_coop = (int)std::max<int64_t>(kNumXcd, want - want % kNumXcd);
    if (c->nblk_coop >= kNumXcd) c->nblk_coop -= c->nblk_coop % kNumXcd;
    int npair = (int)(c->d * (c->d + 1) / 2);
    int nblk_max = std::max(c->nblk, c->nblk_coop);
    c->part_doubles = (size_t)nblk_max * std::max<int64_t>(3 * c->d, 3 + 2 * npair) + 64;
    hipError_t e = hipSuccess;
#define ALLOC(ptr, bytes) do { if (e == hipSuccess) e = hipMalloc((void**)&(ptr), (bytes)); } while (0)
    ALLOC(c->Y, nd); ALLOC(c->P, nd); ALLOC(c->B, nd);
    ALLOC(c->bs, sd);
    if (p->keep_split) ALLOC(c->ds, sd);
    ALLOC(c->rhs, nd); ALLOC(c->r, nd); ALLOC(c->pA, nd); ALLOC(c->pB, nd); ALLOC(c->q, nd);
    ALLOC(c->diagA, nv); ALLOC(c->invdiag, nv); ALLOC(c->sqrtD, nv); ALLOC(c->isqrtD, nv);
    ALLOC(c->part, sizeof(double) * c->part_doubles);
    ALLOC(c->S, sizeof(Scal));
    ALLOC(c->bar, 64 * sizeof(unsigned));
    ALLOC(c->hist, 4096 * sizeof(unsigned));
#undef ALLOC
    if (e != hipSuccess) {
        free_ctx(c);
        delete c;
        return hip_fail(e, "hipMalloc (context)", __FILE__, __LINE__);
    }
    pfe_status s = PFE_OK;
    do {
        if (hipMemsetAsync(c->S, 0, sizeof(Scal), stream) != hipSuccess ||
            hipMemsetAsync(c->bar, 0, 64 * sizeof(unsigned), stream) != hipSuccess ||
            hipMemsetAsync(c->bs, 0, sd, stream) != hipSuccess ||
            hipMemsetAsync(c->pA, 0, nd, stream) != hipSuccess ||
            hipMemsetAsync(c->pB, 0, nd, stream) != hipSuccess ||
            (c->ds && hipMemsetAsync(c->ds, 0, sd, stream) != hipSuccess) ||
            hipMemcpyAsync(c->Y, Y0, nd, hipMemcpyDeviceToDevice, stream) != hipSuccess) {
            s = hip_fail(hipGetLastError(), "context initialisation", __FILE__, __LINE__);
            break;
        }
        s = (p->dtype == PFE_FP64) ? set_diag<double>(c) : set_diag<float>(c);
        if (s != PFE_OK) break;
        if (p->init_ortho) {
            s = (p->dtype == PFE_FP64) ? ortho_mk<double>(c, 1) : ortho_mk<float>(c, 1);
        } else {
            // P = D^{1/2} Y, B = 0 through the same apply pass with T = I
            Scal hS;
            memset(&hS, 0, sizeof(hS));
            for (int k = 0; k < c->d; ++k) hS.T[k * kMaxD + k] = 1.0;
            hS.ortho_ok = 1;
            if (hipMemcpyAsync(c->S, &hS, sizeof(Scal), hipMemcpyHostToDevice, stream) != hipSuccess) {
                s = PFE_E_HIP; break;
            }
            KA<float> af; KA<double> ad;
            if (p->dtype == PFE_FP64) { ad = make_args<double>(c, c->nblk); s = launch_phase(c, ad, PH_APPLY, 1, 0); }
            else { af = make_args<float>(c, c->nblk); s = launch_phase(c, af, PH_APPLY, 1, 0); }
            if (hipStreamSynchronize(stream) != hipSuccess) s = PFE_E_HIP;
        }
        if (s != PFE_OK) break;
        Scal h;
        if (hipMemcpyAsync(&h, c->S, sizeof(Scal), hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess) { s = PFE_E_HIP; break; }
        if (!h.ortho_ok || h.status == PFE_E_RANK) {
            set_error("pfe_init: Y0 is rank deficient (Y0^T D Y0 not positive definite)");
            s = PFE_E_RANK;
            break;
        }
        s = reset_stats(c);
    } while (0);
    if (s != PFE_OK) {
        (void)hipStreamSynchronize(stream);
        free_ctx(c);
        delete c;
        return s;
    }
    *out = c;
    return PFE_OK;
}

pfe_status pfe_set_penalties(pfe_ctx* c, double lambda, double r) {
    if (!c) { set_error("null context"); return PFE_E_ARG; }
    pfe_params p = c->prm;
    p.lambda = lambda;
    p.r = r;
    if (!params_ok(&p, c->n)) return PFE_E_ARG;
    c->prm = p;
    return (p.dtype == PFE_FP64) ? set_diag<double>(c) : set_diag<float>(c);
}

pfe_status pfe_step(pfe_ctx* c, int granularity, pfe_step_info* info) {
    if (!c) { set_error("null context"); return PFE_E_ARG; }
    if (info) PFE_TRY(reset_stats(c));
    pfe_status s;
    const bool f64 = c->prm.dtype == PFE_FP64;
    if (granularity == PFE_INNER) {
        if (c->inner >= c->prm.n_inner) { set_error("all inner iterations done; call pfe_step(PFE_OUTER)"); return PFE_E_STATE; }
        s = f64 ? inner_mk<double>(c, true) : inner_mk<float>(c, true);
    } else if (granularity == PFE_OUTER) {
        if (c->prm.persistent && c->nblk_coop >= kNumXcd && c->inner < c->prm.n_inner)
            s = f64 ? outer_coop<double>(c, 1) : outer_coop<float>(c, 1);
        else
            s = f64 ? outer_mk<double>(c) : outer_mk<float>(c);
    } else {
        set_error("unknown granularity");
        return PFE_E_ARG;
    }
    if (s != PFE_OK) return s;
    if (info) return read_info(c, info);
    return PFE_OK;
}

pfe_status pfe_solve(pfe_ctx* c, int n_outer, pfe_step_info* info) {
    if (!c || n_outer < 0) { set_error("pfe_solve: bad argument"); return PFE_E_ARG; }
    if (info) PFE_TRY(reset_stats(c));
    const bool f64 = c->prm.dtype == PFE_FP64;
    if (c->prm.persistent && c->nblk_coop >= kNumXcd && n_outer > 0 && c->inner < c->prm.n_inner) {
        PFE_TRY(f64 ? outer_coop<double>(c, n_outer) : outer_coop<float>(c, n_outer));
    } else {
        for (int k = 0; k < n_outer; ++k) PFE_TRY(f64 ? outer_mk<double>(c) : outer_mk<float>(c));
    }
    if (info) return read_info(c, info);
    return PFE_OK;
}

pfe_status pfe_stats(pfe_ctx* c, pfe_step_info* out, int reset) {
    if (!c || !out) { set_error("pfe_stats: null argument"); return PFE_E_ARG; }
    pfe_status s = read_info(c, out);
    if (reset) PFE_TRY(reset_stats(c));
    return s;
}

pfe_status pfe_get(pfe_ctx* c, int which, void* dst) {
    if (!c || !dst) { set_error("pfe_get: null argument"); return PFE_E_ARG; }
    const size_t nd = (size_t)c->n * c->d * c->esz;
    hipStream_t st = c->stream;
    const int n = (int)c->n, d = (int)c->d;
    switch (which) {
        case PFE_Y: PFE_CHECK_HIP(hipMemcpyAsync(dst, c->Y, nd, hipMemcpyDeviceToDevice, st)); break;
        case PFE_P: PFE_CHECK_HIP(hipMemcpyAsync(dst, c->P, nd, hipMemcpyDeviceToDevice, st)); break;
        case PFE_B: PFE_CHECK_HIP(hipMemcpyAsync(dst, c->B, nd, hipMemcpyDeviceToDevice, st)); break;
        case PFE_RHS: PFE_CHECK_HIP(hipMemcpyAsync(dst, c->rhs, nd, hipMemcpyDeviceToDevice, st)); break;
        case PFE_YHAT: {
            size_t ne = (size_t)c->n * c->d;
            if (c->esz == 8)
                hipLaunchKernelGGL(k_yhat<double>, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st, ne, d,
                                   (const double*)c->isqrtD, (const double*)c->P, (double*)dst);
            else
                hipLaunchKernelGGL(k_yhat<float>, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st, ne, d,
                                   (const float*)c->isqrtD, (const float*)c->P, (float*)dst);
            PFE_CHECK_HIP(hipGetLastError());
            break;
        }
        case PFE_BSPLIT:
        case PFE_DSPLIT: {
            void* src = (which == PFE_BSPLIT) ? c->bs : c->ds;
            if (!src) { set_error("pfe_get: split variable d not kept (keep_split = 0)"); return PFE_E_STATE; }
            if (c->inner == 0) {
                // b and d restart from zero at every SOC iteration
                PFE_CHECK_HIP(hipMemsetAsync(dst, 0, (size_t)c->g->n_edges * d * c->esz, st));
                break;
            }
            if (c->esz == 8)
                hipLaunchKernelGGL(k_slots_to_edges<double>, dim3((n + 255) / 256), dim3(256), 0, st, n, d,
                                   c->g->rowptr, c->g->col, c->g->eid, (const double*)src, (double*)dst);
            else
                hipLaunchKernelGGL(k_slots_to_edges<float>, dim3((n + 255) / 256), dim3(256), 0, st, n, d,
                                   c->g->rowptr, c->g->col, c->g->eid, (const float*)src, (float*)dst);
            PFE_CHECK_HIP(hipGetLastError());
            break;
        }
        default: set_error("pfe_get: unknown block %d", which); return PFE_E_ARG;
    }
    PFE_CHECK_HIP(hipStreamSynchronize(st));
    return PFE_OK;
}

pfe_status pfe_set(pfe_ctx* c, int which, const void* src) {
    if (!c || !src) { set_error("pfe_set: null argument"); return PFE_E_ARG; }
    const size_t nd = (size_t)c->n * c->d * c->esz;
    hipStream_t st = c->stream;
    const int n = (int)c->n, d = (int)c->d;
    switch (which) {
        case PFE_Y: PFE_CHECK_HIP(hipMemcpyAsync(c->Y, src, nd, hipMemcpyDeviceToDevice, st)); break;
        case PFE_P: PFE_CHECK_HIP(hipMemcpyAsync(c->P, src, nd, hipMemcpyDeviceToDevice, st)); break;
        case PFE_B: PFE_CHECK_HIP(hipMemcpyAsync(c->B, src, nd, hipMemcpyDeviceToDevice, st)); break;
        case PFE_BSPLIT:
        case PFE_DSPLIT: {
            void* dstp = (which == PFE_BSPLIT) ? c->bs : c->ds;
            if (!dstp) { set_error("pfe_set: split variable d not kept (keep_split = 0)"); return PFE_E_STATE; }
            if (c->esz == 8)
                hipLaunchKernelGGL(k_edges_to_slots<double>, dim3((n + 255) / 256), dim3(256), 0, st, n, d,
                                   c->g->rowptr, c->g->col, c->g->eid, (const double*)src, (double*)dstp);
            else
                hipLaunchKernelGGL(k_edges_to_slots<float>, dim3((n + 255) / 256), dim3(256), 0, st, n, d,
                                   c->g->rowptr, c->g->col, c->g->eid, (const float*)src, (float*)dstp);
            PFE_CHECK_HIP(hipGetLastError());
            break;
        }
        default: set_error("pfe_set: block %d cannot be set", which); return PFE_E_ARG;
    }
    // the stored rhs follows the state when mid-way through a SOC iteration
    if (c->inner > 0 && c->ds) {
        if (c->esz == 8) { KA<double> a = make_args<double>(c, c->nblk); PFE_TRY(launch_phase(c, a, PH_RHS, 0, 0)); }
        else { KA<float> a = make_args<float>(c, c->nblk); PFE_TRY(launch_phase(c, a, PH_RHS, 0, 0)); }
    }
    PFE_CHECK_HIP(hipStreamSynchronize(st));
    return PFE_OK;
}

pfe_status pfe_get_inner_index(pfe_ctx* c, int* inner_index) {
    if (!c || !inner_index) { set_error("null argument"); return PFE_E_ARG; }
    *inner_index = c->inner;
    return PFE_OK;
}

pfe_status pfe_set_inner_index(pfe_ctx* c, int inner_index) {
    if (!c) { set_error("null context"); return PFE_E_ARG; }
    if (inner_index < 0 || inner_index > c->prm.n_inner) { set_error("inner index out of range"); return PFE_E_ARG; }
    if (inner_index > 0 && !c->ds) { set_error("resuming inside a SOC iteration needs keep_split = 1"); return PFE_E_STATE; }
    c->inner = inner_index;
    if (inner_index == 0) {
        PFE_CHECK_HIP(hipMemsetAsync(c->bs, 0, (size_t)(c->slots + 1) * c->d * c->esz, c->stream));
        if (c->ds) PFE_CHECK_HIP(hipMemsetAsync(c->ds, 0, (size_t)(c->slots + 1) * c->d * c->esz, c->stream));
    } else {
        if (c->esz == 8) { KA<double> a = make_args<double>(c, c->nblk); PFE_TRY(launch_phase(c, a, PH_RHS, 0, 0)); }
        else { KA<float> a = make_args<float>(c, c->nblk); PFE_TRY(launch_phase(c, a, PH_RHS, 0, 0)); }
    }
    PFE_CHECK_HIP(hipStreamSynchronize(c->stream));
    return PFE_OK;
}

pfe_status pfe_monitor(pfe_ctx* c, pfe_monitors* out) {
    if (!c || !out) { set_error("pfe_monitor: null argument"); return PFE_E_ARG; }
    return (c->esz == 8) ? monitor_impl<double>(c, out) : monitor_impl<float>(c, out);
}

pfe_status pfe_apply_A(pfe_ctx* c, const void* X, void* Q) {
    if (!c || !X || !Q) { set_error("pfe_apply_A: null argument"); return PFE_E_ARG; }
    if (c->esz == 8) {
        KA<double> a = make_args<double>(c, c->nblk);
        hipLaunchKernelGGL(k_spmm<double>, dim3(a.nblk), dim3(kBlock), 0, c->stream, a, (const double*)X, (double*)Q);
    } else {
        KA<float> a = make_args<float>(c, c->nblk);
        hipLaunchKernelGGL(k_spmm<float>, dim3(a.nblk), dim3(kBlock), 0, c->stream, a, (const float*)X, (float*)Q);
    }
    PFE_CHECK_HIP(hipGetLastError());
    PFE_CHECK_HIP(hipStreamSynchronize(c->stream));
    return PFE_OK;
}

pfe_status pfe_pcg(pfe_ctx* c, const void* RHS, void* X, int32_t* iters, pfe_step_info* info) {
    if (!c || !RHS || !X) { set_error("pfe_pcg: null argument"); return PFE_E_ARG; }
    PFE_TRY(reset_stats(c));
    if (c->esz == 8) {
        KA<double> a = make_args<double>(c, c->nblk);
        a.x = (double*)X;
        a.rhs = (double*)RHS;
        PFE_TRY(launch_phase(c, a, PH_R0, 0, 1));
        PFE_TRY(pcg_loop_mk(c, a));
    } else {
        KA<float> a = make_args<float>(c, c->nblk);
        a.x = (float*)X;
        a.rhs = (float*)RHS;
        PFE_TRY(launch_phase(c, a, PH_R0, 0, 1));
        PFE_TRY(pcg_loop_mk(c, a));
    }
    if (iters) {
        PFE_CHECK_HIP(hipMemcpyAsync(iters, c->S->iters, sizeof(int) * c->d, hipMemcpyDeviceToHost, c->stream));
    }
    return read_info(c, info);
}

pfe_status pfe_edge_quantile(pfe_ctx* c, double q, double* out) {
    if (!c || !out || !(q >= 0.0 && q <= 1.0)) { set_error("pfe_edge_quantile: bad argument"); return PFE_E_ARG; }
    return (c->esz == 8) ? quantile_impl<double>(c, q, out) : quantile_impl<float>(c, q, out);
}

void pfe_destroy_ctx(pfe_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free_ctx(c);
    delete c;
}

}  // extern "C"
