// Laplacian-eigenmap initialisation of the embedding (Sec. I: the smallest
// nontrivial solutions of the generalised eigenproblem (D - W) y = mu D y,
// the spectral embedding the piecewise flat embedding starts from and refines).
//
// With z = D^{1/2} y the problem is the symmetric one N z = (1 - mu) z for the
// normalised adjacency N = D^{-1/2} W D^{-1/2}, whose spectrum lies in [-1, 1];
// the smallest mu are the largest eigenvalues of N.  The trivial solution
// (mu = 0, z0 = D^{1/2} 1 / sqrt(vol)) is known exactly and projected out of
// every iterate, so the block converges to eigenvectors 2, 3, ... of the pencil.
//
// Method: Chebyshev-filtered subspace iteration (in the manner of Zhou and
// Saad) on a block of k >= d vectors.  Each outer iteration applies the
// degree-m Chebyshev polynomial of the first kind that maps the unwanted
// interval [-1, a] onto [-1, 1] (a: the smallest Ritz value of the block),
// so the components of eigenvalues above a grow by T_m at that eigenvalue
// (scaled three-term recurrence, no overflow); then the block is deflated
// against z0, D-orthonormalised by Cholesky QR (twice), and rotated onto the
// Ritz vectors of N (Rayleigh-Ritz: the k x k matrix X^T N X diagonalised by
// cyclic Jacobi rotations).  The degree doubles while an iteration reduces the
// largest residual ||N x_i - theta_i x_i|| of the d wanted Ritz pairs by less
// than a factor 10 (up to degree 1024).  Everything is FP64; reductions are per-workgroup partial
// sums added in a fixed order.  Output: y_i = D^{-1/2} x_i for the d largest
// Ritz values (y^T D y = 1), mu_i = 1 - theta_i, each column's sign fixed so
// that its entry of largest magnitude (lowest row on ties) is positive.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"

namespace pfe {

constexpr int kLeMaxK = 32;      // block width
constexpr int kLeThreads = 256;
constexpr int kLeGramBlocks = 1024;
constexpr int kLeMaxDegree = 1024;

// ---- block kernels (n x k row-major FP64) ----------------------------------

// out = alpha (N X) + beta X + gamma Xp  (Xp may be null)
__global__ void __launch_bounds__(kLeThreads) k_le_cheb(int n, int k, const int* __restrict__ rowptr,
                                                       const int* __restrict__ col, const double* __restrict__ w,
                                                       const double* __restrict__ isd, const double* __restrict__ X,
                                                       const double* __restrict__ Xp, double alpha, double beta,
                                                       double gamma, double* __restrict__ out) {
    const int64_t ne = (int64_t)n * k;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / k), c = (int)(e - (int64_t)i * k);
        double acc = 0.0;
        const int s1 = rowptr[i + 1];
        for (int s = rowptr[i]; s < s1; ++s) {
            const int j = col[s];
            acc = fma(w[s] * isd[j], X[(int64_t)j * k + c], acc);
        }
        double v = alpha * (isd[i] * acc) + beta * X[e];
        if (Xp) v += gamma * Xp[e];
        out[e] = v;
    }
}

// partial sums of A^T B (ka x kb) over row ranges: part[blk][a * kb + b]
__global__ void __launch_bounds__(kLeThreads) k_le_gram(int n, int ka, int kb, const double* __restrict__ A,
                                                       const double* __restrict__ B, double* __restrict__ part) {
    const int pairs = ka * kb;
    const int per = (n + gridDim.x - 1) / gridDim.x;
    const int r0 = blockIdx.x * per, r1 = min(n, r0 + per);
    for (int p = threadIdx.x; p < pairs; p += blockDim.x) {
        const int a = p / kb, b = p - a * kb;
        double acc = 0.0;
        for (int i = r0; i < r1; ++i) acc = fma(A[(int64_t)i * ka + a], B[(int64_t)i * kb + b], acc);
        part[(size_t)blockIdx.x * pairs + p] = acc;
    }
}

// out[p] = sum over the nblk partials, in block order
__global__ void k_le_gram_sum(int nblk, int pairs, const double* __restrict__ part, double* __restrict__ out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= pairs) return;
    double acc = 0.0;
    for (int b = 0; b < nblk; ++b) acc += part[(size_t)b * pairs + p];
    out[p] = acc;
}

// X <- X - z0 (z0^T X), with zx = z0^T X (1 x k)
__global__ void k_le_deflate(int n, int k, const double* __restrict__ z0, const double* __restrict__ zx,
                             double* __restrict__ X) {
    const int64_t ne = (int64_t)n * k;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / k), c = (int)(e - (int64_t)i * k);
        X[e] = fma(-z0[i], zx[c], X[e]);
    }
}

// out = X T (T: k x kt, row stride kLeMaxK), out n x kt
__global__ void k_le_rot(int n, int k, int kt, const double* __restrict__ X, const double* __restrict__ T,
                         double* __restrict__ out) {
    __shared__ double sT[kLeMaxK * kLeMaxK];
    for (int p = threadIdx.x; p < kLeMaxK * kLeMaxK; p += blockDim.x) sT[p] = T[p];
    __syncthreads();
    const int64_t ne = (int64_t)n * kt;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / kt), c = (int)(e - (int64_t)i * kt);
        double acc = 0.0;
        for (int m = 0; m < k; ++m) acc = fma(X[(int64_t)i * k + m], sT[m * kLeMaxK + c], acc);
        out[e] = acc;
    }
}

// ---- small dense kernels (one workgroup) -----------------------------------

// T = R^{-1} for the Cholesky factor G = R^T R (upper R), so that X T has
// orthonormal columns; flag[0] = 1 when G is not positive definite
__global__ void __launch_bounds__(kLeThreads) k_le_cholinv(int k, const double* __restrict__ G, double* __restrict__ T,
                                                           int* __restrict__ flag) {
    __shared__ double L[kLeMaxK * kLeMaxK];
    __shared__ double Li[kLeMaxK * kLeMaxK];
    __shared__ int bad;
    const int t = threadIdx.x;
    for (int p = t; p < k * k; p += blockDim.x) L[p] = G[p];
    if (t == 0) bad = 0;
    __syncthreads();
    for (int j = 0; j < k; ++j) {
        if (t == 0) {
            double v = L[j * k + j];
            if (!(v > 1e-300) || !isfinite(v)) { bad = 1; v = 1.0; }
            L[j * k + j] = sqrt(v);
        }
        __syncthreads();
        for (int i = j + 1 + t; i < k; i += blockDim.x) L[i * k + j] /= L[j * k + j];
        __syncthreads();
        for (int p = t; p < k * k; p += blockDim.x) {
            const int i = p / k, c = p - i * k;
            if (c > j && i >= c) L[i * k + c] -= L[i * k + j] * L[c * k + j];
        }
        __syncthreads();
    }
    // Li = L^{-1} column by column (lower triangular), T = Li^T (upper)
    for (int c = t; c < k; c += blockDim.x)
        for (int i = 0; i < k; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int m = c; m < i; ++m) s -= L[i * k + m] * Li[m * kLeMaxK + c];
            Li[i * kLeMaxK + c] = (i < c) ? 0.0 : s / L[i * k + i];
        }
    __syncthreads();
    for (int p = t; p < kLeMaxK * kLeMaxK; p += blockDim.x) {
        const int r = p / kLeMaxK, c = p - r * kLeMaxK;
        T[p] = (r < k && c < k) ? Li[c * kLeMaxK + r] : 0.0;
    }
    if (t == 0 && bad) flag[0] = 1;
}

// Symmetric eigendecomposition of H (k x k, row-major) by cyclic Jacobi
// rotations in round-robin order (k/2 disjoint rotations per round, padded to
// even k): V (row stride kLeMaxK) holds the eigenvectors in its columns,
// ordered by decreasing eigenvalue, theta the eigenvalues.
__global__ void __launch_bounds__(kLeThreads) k_le_eig(int k, const double* __restrict__ Hin, double* __restrict__ V,
                                                       double* __restrict__ theta) {
    constexpr int M = kLeMaxK;
    __shared__ double H[M * M];
    __shared__ double Q[M * M];
    __shared__ double cs[M / 2], sn[M / 2];
    __shared__ int pp[M / 2], qq[M / 2];
    __shared__ double off;
    __shared__ int order[M];
    const int t = threadIdx.x;
    const int ke = k + (k & 1);            // even size with an inert extra index
    for (int p = t; p < M * M; p += blockDim.x) {
        const int r = p / M, c = p - r * M;
        H[p] = (r < k && c < k) ? Hin[r * k + c] : 0.0;
        Q[p] = (r == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    double scale = 0.0;
    for (int p = 0; p < k * k; ++p) scale = fmax(scale, fabs(H[(p / k) * M + p % k]));
    for (int sweep = 0; sweep < 60; ++sweep) {
        if (t == 0) {
            double s = 0.0;
            for (int r = 0; r < k; ++r)
                for (int c = r + 1; c < k; ++c) s = fmax(s, fabs(H[r * M + c]));
            off = s;
        }
        __syncthreads();
        if (!(off > 1e-16 * scale)) break;
        for (int round = 0; round < ke - 1; ++round) {
            // round-robin pairing: index ke-1 fixed, the others rotate
            if (t < ke / 2) {
                int a = (t == 0) ? ke - 1 : (round + t) % (ke - 1);
                int b = (round + ke - 1 - t) % (ke - 1);
                if (t == 0) b = round % (ke - 1);
                const int p = min(a, b), q = max(a, b);
                pp[t] = p;
                qq[t] = q;
                double c = 1.0, s = 0.0;
                if (q < k && p != q) {
                    const double hpq = H[p * M + q];
                    if (hpq != 0.0) {
                        const double tau = (H[q * M + q] - H[p * M + p]) / (2.0 * hpq);
                        const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + tt * tt);
                        s = tt * c;
                    }
                }
                cs[t] = c;
                sn[t] = s;
            }
            __syncthreads();
            // rows p, q of H: H <- J^T H
            for (int idx = t; idx < (ke / 2) * k; idx += blockDim.x) {
                const int pr = idx / k, col = idx - pr * k;
                const int p = pp[pr], q = qq[pr];
                if (q >= k || p == q) continue;
                const double c = cs[pr], s = sn[pr];
                const double hp = H[p * M + col], hq = H[q * M + col];
                H[p * M + col] = c * hp - s * hq;
                H[q * M + col] = s * hp + c * hq;
            }
            __syncthreads();
            // columns p, q of H and of Q: H <- H J, Q <- Q J
            for (int idx = t; idx < (ke / 2) * k; idx += blockDim.x) {
                const int pr = idx / k, row = idx - pr * k;
                const int p = pp[pr], q = qq[pr];
                if (q >= k || p == q) continue;
                const double c = cs[pr], s = sn[pr];
                const double hp = H[row * M + p], hq = H[row * M + q];
                H[row * M + p] = c * hp - s * hq;
                H[row * M + q] = s * hp + c * hq;
                const double vp = Q[row * M + p], vq = Q[row * M + q];
                Q[row * M + p] = c * vp - s * vq;
                Q[row * M + q] = s * vp + c * vq;
            }
            __syncthreads();
        }
    }
    if (t == 0) {
        // decreasing eigenvalues (stable: ties keep the index order)
        for (int i = 0; i < k; ++i) order[i] = i;
        for (int i = 1; i < k; ++i) {
            const int v = order[i];
            int j = i - 1;
            while (j >= 0 && H[order[j] * M + order[j]] < H[v * M + v]) { order[j + 1] = order[j]; --j; }
            order[j + 1] = v;
        }
    }
    __syncthreads();
    for (int p = t; p < M * M; p += blockDim.x) {
        const int r = p / M, c = p - r * M;
        V[p] = (r < k && c < k) ? Q[r * M + order[c]] : 0.0;
    }
    for (int c = t; c < k; c += blockDim.x) theta[c] = H[order[c] * M + order[c]];
}

// per-workgroup (max |y|, lowest row) of each column c < d of y = D^{-1/2} X
// (X an n x ld block)
__global__ void __launch_bounds__(kLeThreads) k_le_argmax(int n, int ld, int d, const double* __restrict__ X,
                                                         const double* __restrict__ isd, double* __restrict__ pv,
                                                         int* __restrict__ pi) {
    __shared__ double sv[kLeThreads];
    __shared__ int si[kLeThreads];
    const int per = (n + gridDim.x - 1) / gridDim.x;
    const int r0 = blockIdx.x * per, r1 = min(n, r0 + per);
    for (int c = 0; c < d; ++c) {
        double bv = -1.0;
        int bi = INT32_MAX;
        for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
            const double v = fabs(isd[i] * X[(int64_t)i * ld + c]);
            if (v > bv) { bv = v; bi = i; }      // rows visited in increasing order per thread
        }
        sv[threadIdx.x] = bv;
        si[threadIdx.x] = bi;
        __syncthreads();
        for (int h = blockDim.x / 2; h > 0; h >>= 1) {
            if (threadIdx.x < h) {
                const double ov = sv[threadIdx.x + h];
                const int oi = si[threadIdx.x + h];
                if (ov > sv[threadIdx.x] || (ov == sv[threadIdx.x] && oi < si[threadIdx.x])) {
                    sv[threadIdx.x] = ov;
                    si[threadIdx.x] = oi;
                }
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            pv[(size_t)blockIdx.x * d + c] = sv[0];
            pi[(size_t)blockIdx.x * d + c] = si[0];
        }
        __syncthreads();
    }
}

// Y (n x d) = sign_c D^{-1/2} X[:, c] with sign_c making the entry of largest
// magnitude positive (the partials of k_le_argmax reduced in block order)
__global__ void k_le_output(int n, int ld, int d, int nblk, const double* __restrict__ X,
                            const double* __restrict__ isd, const double* __restrict__ pv, const int* __restrict__ pi,
                            double* __restrict__ Y) {
    __shared__ double sgn[kLeMaxK];
    if (threadIdx.x < d) {
        const int c = threadIdx.x;
        double bv = -1.0;
        int bi = INT32_MAX;
        for (int b = 0; b < nblk; ++b) {
            const double v = pv[(size_t)b * d + c];
            const int i = pi[(size_t)b * d + c];
            if (v > bv || (v == bv && i < bi)) { bv = v; bi = i; }
        }
        sgn[c] = (bi < n && X[(int64_t)bi * ld + c] < 0.0) ? -1.0 : 1.0;
    }
    __syncthreads();
    const int64_t ne = (int64_t)n * d;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / d), c = (int)(e - (int64_t)i * d);
        Y[e] = sgn[c] * isd[i] * X[(int64_t)i * ld + c];
    }
}

// R = NX - X diag(theta): the Ritz residuals, formed explicitly (their norms
// are far below the rounding of ||N x||^2 - theta^2)
__global__ void k_le_resid(int n, int k, const double* __restrict__ NX, const double* __restrict__ X,
                           const double* __restrict__ theta, double* __restrict__ R) {
    const int64_t ne = (int64_t)n * k;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e % k);
        R[e] = fma(-theta[c], X[e], NX[e]);
    }
}

__global__ void k_le_isd(int n, const double* __restrict__ deg, double vol, double* __restrict__ isd,
                         double* __restrict__ z0) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    isd[i] = 1.0 / sqrt(deg[i]);
    z0[i] = sqrt(deg[i] / vol);
}

__global__ void k_le_sum(int n, const double* __restrict__ v, double* __restrict__ out) {
    // one workgroup: fixed-order strided partials, then a tree
    __shared__ double red[kLeThreads];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += v[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// ---- host driver ------------------------------------------------------------

struct LeWork {
    int n = 0, k = 0;
    hipStream_t st = nullptr;
    const int* rowptr = nullptr;
    const int* col = nullptr;
    const double* w = nullptr;
    double* isd = nullptr;
    double* z0 = nullptr;
    double* X = nullptr;     // current block
    double* Y1 = nullptr;    // recurrence buffers / N X
    double* Y2 = nullptr;
    double* part = nullptr;  // Gram partials
    double* small = nullptr; // k x k results, transforms, Ritz values
    int* flag = nullptr;
    unsigned grid = 1;
};

static unsigned le_grid(int64_t ne) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((ne + 255) / 256, 8192)); }

// G (ka x kb, stored at dst) = A^T B
static pfe_status le_gram(LeWork& L, int ka, int kb, const double* A, const double* B, double* dst) {
    const int nblk = std::min(kLeGramBlocks, std::max(1, L.n / 64));
    hipLaunchKernelGGL(k_le_gram, dim3(nblk), dim3(kLeThreads), 0, L.st, L.n, ka, kb, A, B, L.part);
    hipLaunchKernelGGL(k_le_gram_sum, dim3((ka * kb + 255) / 256), dim3(256), 0, L.st, nblk, ka * kb, L.part, dst);
    PFE_CHECK_HIP(hipGetLastError());
    return PFE_OK;
}

static pfe_status le_apply(LeWork& L, const double* X, const double* Xp, double alpha, double beta, double gamma,
                           double* out) {
    hipLaunchKernelGGL(k_le_cheb, dim3(L.grid), dim3(kLeThreads), 0, L.st, L.n, L.k, L.rowptr, L.col, L.w, L.isd,
                       X, Xp, alpha, beta, gamma, out);
    PFE_CHECK_HIP(hipGetLastError());
    return PFE_OK;
}

// X <- X - z0 z0^T X, then X <- X R^{-1} (Cholesky QR), twice
static pfe_status le_orthonormalise(LeWork& L, double* X, double* tmp) {
    double* G = L.small;                       // k x k
    double* T = L.small + kLeMaxK * kLeMaxK;   // transform
    double* zx = L.small + 2 * kLeMaxK * kLeMaxK;
    for (int pass = 0; pass < 2; ++pass) {
        PFE_TRY_STATUS(le_gram(L, 1, L.k, L.z0, X, zx));
        hipLaunchKernelGGL(k_le_deflate, dim3(L.grid), dim3(kLeThreads), 0, L.st, L.n, L.k, L.z0, zx, X);
        PFE_TRY_STATUS(le_gram(L, L.k, L.k, X, X, G));
        hipLaunchKernelGGL(k_le_cholinv, dim3(1), dim3(kLeThreads), 0, L.st, L.k, G, T, L.flag);
        hipLaunchKernelGGL(k_le_rot, dim3(L.grid), dim3(kLeThreads), 0, L.st, L.n, L.k, L.k, X, T, tmp);
        PFE_CHECK_HIP(hipGetLastError());
        PFE_CHECK_HIP(hipMemcpyAsync(X, tmp, sizeof(double) * (size_t)L.n * L.k, hipMemcpyDeviceToDevice, L.st));
    }
    return PFE_OK;
}

}  // namespace pfe

using namespace pfe;

extern "C" pfe_status pfe_le_init(const pfe_graph* g, int d, const double* X0, int k, double tol, int max_iter,
                                  double* Y, double* mu, pfe_le_info* info, hipStream_t stream) {
    if (info) *info = pfe_le_info{};
    if (!g || !X0 || !Y || d < 1 || k < d || k > kLeMaxK || !(tol > 0.0) || max_iter < 1 ||
        (int64_t)k + 1 >= g->n || g->n >= (int64_t)INT32_MAX) {
        set_error("pfe_le_init: bad argument (1 <= d <= k <= %d, k + 1 < n, tol > 0, max_iter >= 1)", kLeMaxK);
        return PFE_E_ARG;
    }
    if (g->seg_row0.size() != 2) {
        set_error("pfe_le_init: one graph (not a union of several)");
        return PFE_E_ARG;
    }
    LeWork L;
    L.n = (int)g->n;
    L.k = k;
    L.st = stream;
    L.rowptr = g->rowptr;
    L.col = g->col;
    L.w = g->w64;
    L.grid = le_grid((int64_t)L.n * k);
    const size_t nk = (size_t)L.n * k;
    const int nblk_g = std::min(kLeGramBlocks, std::max(1, L.n / 64));
    pfe_status s = PFE_OK;
    std::vector<void*> bufs;
    auto grab = [&](void** p, size_t bytes) {
        if (s != PFE_OK) return;
        if (dev_alloc(p, bytes) != hipSuccess) { s = hip_fail(hipErrorOutOfMemory, "pfe_le_init allocation", __FILE__, __LINE__); return; }
        bufs.push_back(*p);
    };
    grab((void**)&L.isd, sizeof(double) * L.n);
    grab((void**)&L.z0, sizeof(double) * L.n);
    grab((void**)&L.X, sizeof(double) * nk);
    grab((void**)&L.Y1, sizeof(double) * nk);
    grab((void**)&L.Y2, sizeof(double) * nk);
    grab((void**)&L.part, sizeof(double) * (size_t)nblk_g * kLeMaxK * kLeMaxK);
    grab((void**)&L.small, sizeof(double) * 8 * kLeMaxK * kLeMaxK);
    grab((void**)&L.flag, sizeof(int) * 4);
    double* pv = nullptr;
    int* pi = nullptr;
    grab((void**)&pv, sizeof(double) * 1024 * kLeMaxK);
    grab((void**)&pi, sizeof(int) * 1024 * kLeMaxK);
    int iters = 0, degree = 16, conv = 0;
    double res = INFINITY;
    do {
        if (s != PFE_OK) break;
        if (hipMemsetAsync(L.flag, 0, sizeof(int) * 4, stream) != hipSuccess) { s = PFE_E_HIP; break; }
        // D^{-1/2}, z0 = D^{1/2} 1 / sqrt(vol)
        double* vol_d = L.small + 7 * kLeMaxK * kLeMaxK;
        hipLaunchKernelGGL(k_le_sum, dim3(1), dim3(kLeThreads), 0, stream, L.n, g->degree, vol_d);
        double vol = 0.0;
        if (hipMemcpyAsync(&vol, vol_d, sizeof(double), hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess) { s = PFE_E_HIP; break; }
        hipLaunchKernelGGL(k_le_isd, dim3((L.n + 255) / 256), dim3(256), 0, stream, L.n, g->degree, vol, L.isd, L.z0);
        if (hipMemcpyAsync(L.X, X0, sizeof(double) * nk, hipMemcpyDeviceToDevice, stream) != hipSuccess) { s = PFE_E_HIP; break; }
        if ((s = le_orthonormalise(L, L.X, L.Y1)) != PFE_OK) break;
        double* H = L.small + 3 * kLeMaxK * kLeMaxK;
        double* V = L.small + 4 * kLeMaxK * kLeMaxK;
        double* theta = L.small + 5 * kLeMaxK * kLeMaxK;
        double* R = L.small + 6 * kLeMaxK * kLeMaxK;   // residual Gram diagonal source
        std::vector<double> th(k), rg((size_t)k * k);
        double prev_res = INFINITY;
        for (int it = 0; it <= max_iter; ++it) {
            // Rayleigh-Ritz: N X, H = X^T N X, X <- X V, (N X) <- (N X) V
            if ((s = le_apply(L, L.X, nullptr, 1.0, 0.0, 0.0, L.Y1)) != PFE_OK) break;
            if ((s = le_gram(L, k, k, L.X, L.Y1, H)) != PFE_OK) break;
            hipLaunchKernelGGL(k_le_eig, dim3(1), dim3(kLeThreads), 0, stream, k, H, V, theta);
            hipLaunchKernelGGL(k_le_rot, dim3(L.grid), dim3(kLeThreads), 0, stream, L.n, k, k, L.X, V, L.Y2);
            if (hipMemcpyAsync(L.X, L.Y2, sizeof(double) * nk, hipMemcpyDeviceToDevice, stream) != hipSuccess) { s = PFE_E_HIP; break; }
            hipLaunchKernelGGL(k_le_rot, dim3(L.grid), dim3(kLeThreads), 0, stream, L.n, k, k, L.Y1, V, L.Y2);
            // residuals R = N X - X diag(theta) and their Gram matrix (diagonal used)
            hipLaunchKernelGGL(k_le_resid, dim3(L.grid), dim3(kLeThreads), 0, stream, L.n, k, L.Y2, L.X, theta, L.Y1);
            if ((s = le_gram(L, k, k, L.Y1, L.Y1, R)) != PFE_OK) break;
            int bad = 0;
            if (hipMemcpyAsync(th.data(), theta, sizeof(double) * k, hipMemcpyDeviceToHost, stream) != hipSuccess ||
                hipMemcpyAsync(rg.data(), R, sizeof(double) * k * k, hipMemcpyDeviceToHost, stream) != hipSuccess ||
                hipMemcpyAsync(&bad, L.flag, sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess ||
                hipStreamSynchronize(stream) != hipSuccess) { s = PFE_E_HIP; break; }
            if (bad) { set_error("pfe_le_init: the block lost rank (start block X0 deficient?)"); s = PFE_E_RANK; break; }
            res = 0.0;
            for (int i = 0; i < d; ++i) res = std::max(res, std::sqrt(std::max(0.0, rg[(size_t)i * k + i])));
            iters = it;
            if (res <= tol) { conv = 1; break; }
            if (it == max_iter) break;
            // (capped so that the filtered block stays well conditioned for Cholesky QR)
            if (it > 0 && res > 0.1 * prev_res) degree = std::min(2 * degree, kLeMaxDegree);
            prev_res = res;
            // Chebyshev filter of degree `degree` on [-1, a], a = smallest Ritz value
            const double a = th[k - 1], lo = -1.0;
            const double e = 0.5 * (a - lo), c = 0.5 * (a + lo);
            const double top = th[0];
            double sigma = e / (top - c);
            const double sigma1 = sigma;
            // Y1 = (N X - c X) sigma1 / e
            if ((s = le_apply(L, L.X, nullptr, sigma1 / e, -c * sigma1 / e, 0.0, L.Y1)) != PFE_OK) break;
            double* prev = L.X;
            double* cur = L.Y1;
            double* nxt = L.Y2;
            for (int j = 2; j <= degree && s == PFE_OK; ++j) {
                const double sigma_new = 1.0 / (2.0 / sigma1 - sigma);
                s = le_apply(L, cur, prev, 2.0 * sigma_new / e, -2.0 * c * sigma_new / e, -sigma * sigma_new, nxt);
                double* tmp = prev;
                prev = cur;
                cur = nxt;
                nxt = tmp;
                sigma = sigma_new;
            }
            if (s != PFE_OK) break;
            if (cur != L.X &&
                hipMemcpyAsync(L.X, cur, sizeof(double) * nk, hipMemcpyDeviceToDevice, stream) != hipSuccess) { s = PFE_E_HIP; break; }
            if ((s = le_orthonormalise(L, L.X, L.Y1)) != PFE_OK) break;
        }
        if (s != PFE_OK) break;
        if (mu) for (int i = 0; i < d; ++i) mu[i] = 1.0 - th[i];
        // sign-fixed output
        const int nb = std::min(1024, std::max(1, L.n / 256));
        hipLaunchKernelGGL(k_le_argmax, dim3(nb), dim3(kLeThreads), 0, stream, L.n, k, d, L.X, L.isd, pv, pi);
        hipLaunchKernelGGL(k_le_output, dim3(L.grid), dim3(kLeThreads), 0, stream, L.n, k, d, nb, L.X, L.isd, pv, pi, Y);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(stream) != hipSuccess) { s = PFE_E_HIP; break; }
    } while (0);
    (void)hipStreamSynchronize(stream);
    for (void* p : bufs) (void)dev_free(p);
    if (info) {
        info->iterations = iters;
        info->degree = degree;
        info->residual = res;
        info->converged = conv;
    }
    if (s == PFE_OK && !conv) {
        set_error("pfe_le_init: residual %.3g above tol after %d iterations", res, iters);
        return PFE_E_NOCONV;
    }
    return s;
}
