// Learned sparse-factor preconditioner: inference and training kernels.
//
// M^{-1} = G^T G with G = Gt D_A^{-1/2}, Gt lower triangular on the pattern of
// A = lambda/2 M^T M + r/2 D (Eq. 13) with a positive (softplus) diagonal, so
// M^{-1} is SPD for any weights and Gt = I is exactly Jacobi.  The entries of
// Gt come from a two-layer message-passing network of width 16 evaluated on
// the scaled matrix At = D_A^{-1/2} A D_A^{-1/2}:
//   x_i    = [1, sum_j |At_ij|, max_j |At_ij|, deg_i / deg_max]
//   agg1_i = sum_j (-At_ij) x_j,          h1_i = relu(W1s x_i + W1m agg1_i + b1)
//   agg2_i = sum_j (-At_ij) h1_j,         h2_i = relu(W2s h1_i + W2m agg2_i + b2)
//   U_i = u.h2_i, V_i = v.h2_i, Z_i = q.h2_i + bd
//   Gt_ij = At_ij (U_i + V_j + c) (j < i),  Gt_ii = softplus(Z_i)
// The dense products run on MFMA (bf16 weights and inputs, fp32 accumulation,
// one wavefront per 16 vertices); aggregation, the factor, the loss chain and
// the backward pass are fp32 with fp64 reductions.  Training minimises
// mean_k ||At Gt^T Gt rho_k - rho_k||^2 over unit-norm scaled residuals
// rho = D_A^{-1/2} r / ||D_A^{-1/2} r|| with Adam.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace pfe {
namespace mp {

constexpr int kH = 16;
constexpr int kNP = 722;
// parameter vector layout
constexpr int oW1s = 0, oW1m = 64, ob1 = 128, oW2s = 144, oW2m = 400, ob2 = 656;
constexpr int ou = 672, ov = 688, oq = 704, oc = 720, obd = 721;
constexpr int kTB = 256;

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ unsigned short f2bf(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float rbf(float f) { return __uint_as_float(((unsigned)f2bf(f)) << 16); }

__device__ __forceinline__ float softplus(float z) { return fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))); }
__device__ __forceinline__ float sigmoid(float z) { return 1.f / (1.f + expf(-z)); }

struct View {
    int n, K, deg_max;
    const int* rowptr;
    const int* scol;
    const int* seid;
    const double* sw64;
    const double* degree;
    const double* wsq;
    double half_lam, half_r;
};

__device__ __forceinline__ void slots(const View& v, int i, int& s0, int& cnt, int& st) {
    if (v.K > 0) { s0 = i; cnt = v.K; st = v.n; }
    else { s0 = v.rowptr[i]; cnt = v.rowptr[i + 1] - s0; st = 1; }
}

// At per slot and node features
__global__ void k_prep(View v, float* __restrict__ at, float* __restrict__ x) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= v.n) return;
    const double di = v.half_lam * v.wsq[i] + v.half_r * v.degree[i];
    int s0, cnt, st;
    slots(v, i, s0, cnt, st);
    float sabs = 0.f, mabs = 0.f;
    int deg = 0;
    for (int k = 0; k < cnt; ++k) {
        int s = s0 + k * st;
        int j = v.scol[s];
        double w = v.sw64[s];
        double dj = v.half_lam * v.wsq[j] + v.half_r * v.degree[j];
        float a = (float)(-v.half_lam * w * w / sqrt(di * dj));
        at[s] = a;
        sabs += fabsf(a);
        mabs = fmaxf(mabs, fabsf(a));
        deg += (v.seid[s] >= 0);
    }
    x[i * 4 + 0] = 1.f;
    x[i * 4 + 1] = sabs;
    x[i * 4 + 2] = mabs;
    x[i * 4 + 3] = (float)deg / (float)max(1, v.deg_max);
}

// out_i = sum_s (-At_s) in_j  (F features per vertex): F / 4 threads per
// vertex, each summing four consecutive features (one slot load and one
// 16-byte gather per slot, issued for eight slots at a time), every feature in
// slot order
template <int F>
__global__ void k_agg(View v, const float* __restrict__ at, const float* __restrict__ in, float* __restrict__ out) {
    static_assert(F % 4 == 0, "four features per thread");
    constexpr int L = F / 4, G = 8;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= v.n * L) return;
    const int i = e / L, f0 = (e - i * L) * 4;
    int s0, cnt, st;
    slots(v, i, s0, cnt, st);
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    int k = 0;
    for (; k + G <= cnt; k += G) {
        float w[G];
        f4 x[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int s = s0 + (k + g) * st;
            w[g] = -at[s];
            x[g] = *reinterpret_cast<const f4*>(in + (size_t)v.scol[s] * F + f0);
        }
#pragma unroll
        for (int g = 0; g < G; ++g)
            for (int t = 0; t < 4; ++t) acc[t] = fmaf(w[g], x[g][t], acc[t]);
    }
    for (; k < cnt; ++k) {
        const int s = s0 + k * st;
        const float w = -at[s];
        const f4 x = *reinterpret_cast<const f4*>(in + (size_t)v.scol[s] * F + f0);
        for (int t = 0; t < 4; ++t) acc[t] = fmaf(w, x[t], acc[t]);
    }
    *reinterpret_cast<f4*>(out + (size_t)i * F + f0) = acc;
}

// MFMA tile: D[m][o] += sum_k A[m][k] B[k][o] for a 16x16x16 bf16 block.  Lane l
// supplies A[l % 16][4 (l / 16) + t] and B[4 (l / 16) + t][l % 16], t < 4, and
// receives D[4 (l / 16) + t][l % 16].
__device__ __forceinline__ f4 mfma16(const float (&a)[4], const float (&b)[4], f4 acc) {
    s4 av, bv;
    for (int t = 0; t < 4; ++t) {
        av[t] = (short)f2bf(a[t]);
        bv[t] = (short)f2bf(b[t]);
    }
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
}

// Dense layers, one wavefront per 16 vertices (blockDim = 256: 64 vertices).
// layer 1: in = [x (4), agg1 (4)]; layer 2: in = [h1 (16), agg2 (16)];
// output: in = h2, out columns (U, V, Z - bd).
template <int LAYER>
__global__ void __launch_bounds__(kTB) k_dense(int n, const float* __restrict__ theta, const float* __restrict__ in_a,
                                               const float* __restrict__ in_b, float* __restrict__ pre,
                                               float* __restrict__ act) {
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * kTB + threadIdx.x) >> 6;
    const int base = wave * 16;
    if (base >= n) return;
    const int m = lane & 15, kg = lane >> 4;
    const int node = base + m;
    const bool ok = node < n;
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    float a[4], b[4];
    const int o = m;   // B column owned by this lane
    if (LAYER == 1) {
        for (int t = 0; t < 4; ++t) {
            a[t] = (ok && kg == 0) ? in_a[node * 4 + t] : (ok && kg == 1) ? in_b[node * 4 + t] : 0.f;
            b[t] = (kg == 0) ? theta[oW1s + o * 4 + t] : (kg == 1) ? theta[oW1m + o * 4 + t] : 0.f;
        }
        acc = mfma16(a, b, acc);
    } else if (LAYER == 2) {
        for (int t = 0; t < 4; ++t) {
            a[t] = ok ? in_a[node * kH + 4 * kg + t] : 0.f;
            b[t] = theta[oW2s + o * kH + 4 * kg + t];
        }
        acc = mfma16(a, b, acc);
        for (int t = 0; t < 4; ++t) {
            a[t] = ok ? in_b[node * kH + 4 * kg + t] : 0.f;
            b[t] = theta[oW2m + o * kH + 4 * kg + t];
        }
        acc = mfma16(a, b, acc);
    } else {
        for (int t = 0; t < 4; ++t) {
            a[t] = ok ? in_a[node * kH + 4 * kg + t] : 0.f;
            const int k = 4 * kg + t;
            b[t] = (o == 0) ? theta[ou + k] : (o == 1) ? theta[ov + k] : (o == 2) ? theta[oq + k] : 0.f;
        }
        acc = mfma16(a, b, acc);
    }
    for (int t = 0; t < 4; ++t) {
        const int row = base + 4 * kg + t;
        if (row >= n) continue;
        if (LAYER == 3) {
            if (o < 3) pre[row * 3 + o] = acc[t];
        } else {
            const float bias = theta[(LAYER == 1 ? ob1 : ob2) + o];
            const float p = acc[t] + bias;
            pre[row * kH + o] = p;
            act[row * kH + o] = fmaxf(p, 0.f);
        }
    }
}

// Gt on every slot (value of the edge's lower-triangular entry) and its diagonal
template <typename T>
__global__ void k_factor(View v, const float* __restrict__ theta, const float* __restrict__ at,
                         const float* __restrict__ uvz, T* __restrict__ gval, T* __restrict__ gdiag) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= v.n) return;
    const float c = theta[oc];
    int s0, cnt, st;
    slots(v, i, s0, cnt, st);
    for (int k = 0; k < cnt; ++k) {
        int s = s0 + k * st;
        int j = v.scol[s];
        int lo = max(i, j), hi = min(i, j);
        gval[s] = (T)(at[s] * (uvz[lo * 3 + 0] + uvz[hi * 3 + 1] + c));
    }
    gdiag[i] = (T)softplus(uvz[i * 3 + 2] + theta[obd]);
}

// ---- loss chain on k sample columns (n x k, row-major, fp32) -----------------

// y = Gt x (lower) or Gt^T x (upper)
template <bool LOWER>
__global__ void k_gmul(View v, int kc, const float* __restrict__ gval, const float* __restrict__ gdiag,
                       const float* __restrict__ x, float* __restrict__ y) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= v.n * kc) return;
    int i = e / kc, c = e - i * kc;
    int s0, cnt, st;
    slots(v, i, s0, cnt, st);
    float acc = gdiag[i] * x[e];
    for (int k = 0; k < cnt; ++k) {
        int s = s0 + k * st;
        int j = v.scol[s];
        if (LOWER ? (j < i) : (j > i)) acc = fmaf(gval[s], x[j * kc + c], acc);
    }
    y[e] = acc;
}

// y = At x (unit diagonal)
__global__ void k_amul(View v, int kc, const float* __restrict__ at, const float* __restrict__ x,
                       float* __restrict__ y) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= v.n * kc) return;
    int i = e / kc, c = e - i * kc;
    int s0, cnt, st;
    slots(v, i, s0, cnt, st);
    float acc = x[e];
    for (int k = 0; k < cnt; ++k) {
        int s = s0 + k * st;
        acc = fmaf(at[s], x[v.scol[s] * kc + c], acc);
    }
    y[e] = acc;
}

// per-block fp64 partial sums of one value per (element): out[blk * kc + c]
template <class F>
__device__ void col_partials(int n, int kc, F&& val, double* out) {
    __shared__ double sh[kTB];
    // threads walk elements of their block range; accumulate per column in LDS
    const int nb = gridDim.x;
    const int rows_per = (n + nb - 1) / nb;
    const int r0 = blockIdx.x * rows_per, r1 = min(n, r0 + rows_per);
    for (int c0 = 0; c0 < kc; c0 += 1) {
        double acc = 0.0;
        for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) acc += val(i, c0);
        sh[threadIdx.x] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int t = 0; t < (int)blockDim.x; ++t) s += sh[t];
            out[blockIdx.x * kc + c0] = s;
        }
        __syncthreads();
    }
}

// column norms of D_A^{-1/2} r: partials
template <typename T>
__global__ void k_sample_norm(View v, int kc, const T* __restrict__ r, double* __restrict__ part) {
    col_partials(v.n, kc, [&](int i, int c) {
        double di = v.half_lam * v.wsq[i] + v.half_r * v.degree[i];
        double z = (double)r[(size_t)i * kc + c] / sqrt(di);
        return z * z;
    }, part);
}

__global__ void k_sum_partials(int nb, int kc, const double* __restrict__ part, double* __restrict__ out) {
    int c = threadIdx.x;
    if (c >= kc) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[b * kc + c];
    out[c] = s;
}

template <typename T>
__global__ void k_sample_scale(View v, int kc, const T* __restrict__ r, const double* __restrict__ nrm2,
                               float* __restrict__ rho) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= v.n * kc) return;
    int i = e / kc, c = e - i * kc;
    double di = v.half_lam * v.wsq[i] + v.half_r * v.degree[i];
    double nn = nrm2[c];
    rho[e] = (nn > 0.0) ? (float)((double)r[e] / sqrt(di) / sqrt(nn)) : 0.f;
}

// e = y3 - rho: partial sums of e^2 per column; stores 2 e / k
__global__ void k_resid(View v, int kc, const float* __restrict__ y3, const float* __restrict__ rho,
                        float* __restrict__ escaled, double* __restrict__ part) {
    const int nb = gridDim.x;
    const int rows_per = (v.n + nb - 1) / nb;
    const int r0 = blockIdx.x * rows_per, r1 = min(v.n, r0 + rows_per);
    for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x)
        for (int c = 0; c < kc; ++c) {
            float ev = y3[i * kc + c] - rho[i * kc + c];
            escaled[i * kc + c] = 2.f * ev / (float)kc;
        }
    col_partials(v.n, kc, [&](int i, int c) {
        double ev = (double)y3[i * kc + c] - (double)rho[i * kc + c];
        return ev * ev;
    }, part);
}

// gradient of the loss with respect to every slot value and the diagonal:
// dGt_lo,hi = sum_c dy1_lo rho_hi + y1_lo dy2_hi  (stored on both directions)
__global__ void k_dfactor(View v, int kc, const float* __restrict__ rho, const float* __restrict__ y1,
                          const float* __restrict__ dy1, const float* __restrict__ dy2,
                          float* __restrict__ dgval, float* __restrict__ dgdiag) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= v.n) return;
    // sum over the kc sample columns (in column order) of dy1_lo rho_hi + y1_lo dy2_hi,
    // four columns per 16-byte load when kc allows
    auto pair = [&](int lo, int hi) {
        const float* a = dy1 + (size_t)lo * kc;
        const float* b = rho + (size_t)hi * kc;
        const float* c = y1 + (size_t)lo * kc;
        const float* d = dy2 + (size_t)hi * kc;
        float acc = 0.f;
        if ((kc & 3) == 0) {
            for (int q = 0; q < kc; q += 4) {
                const f4 av = *reinterpret_cast<const f4*>(a + q), bv = *reinterpret_cast<const f4*>(b + q);
                const f4 cv = *reinterpret_cast<const f4*>(c + q), dv = *reinterpret_cast<const f4*>(d + q);
                for (int t = 0; t < 4; ++t) acc += av[t] * bv[t] + cv[t] * dv[t];
            }
        } else {
            for (int q = 0; q < kc; ++q) acc += a[q] * b[q] + c[q] * d[q];
        }
        return acc;
    };
    int s0, cnt, st;
    slots(v, i, s0, cnt, st);
    for (int k = 0; k < cnt; ++k) {
        int s = s0 + k * st;
        int j = v.scol[s];
        dgval[s] = (j != i) ? pair(max(i, j), min(i, j)) : 0.f;
    }
    dgdiag[i] = pair(i, i);
}

// output layer backward: dU, dV, dZ per vertex and dpre2
__global__ void k_out_bwd(View v, const float* __restrict__ theta, const float* __restrict__ at,
                          const float* __restrict__ dgval, const float* __restrict__ dgdiag,
                          const float* __restrict__ uvz, const float* __restrict__ pre2,
                          float* __restrict__ duvz, float* __restrict__ dpre2) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= v.n) return;
    int s0, cnt, st;
    slots(v, i, s0, cnt, st);
    float dU = 0.f, dV = 0.f;
    for (int k = 0; k < cnt; ++k) {
        int s = s0 + k * st;
        int j = v.scol[s];
        float g = dgval[s] * at[s];
        if (j < i) dU += g;
        else if (j > i) dV += g;
    }
    float dZ = dgdiag[i] * sigmoid(uvz[i * 3 + 2] + theta[obd]);
    duvz[i * 3 + 0] = dU;
    duvz[i * 3 + 1] = dV;
    duvz[i * 3 + 2] = dZ;
    for (int k = 0; k < kH; ++k) {
        float dh = dU * rbf(theta[ou + k]) + dV * rbf(theta[ov + k]) + dZ * rbf(theta[oq + k]);
        dpre2[i * kH + k] = (pre2[i * kH + k] > 0.f) ? dh : 0.f;
    }
}

// layer 2 backward to the vertex: dh1 (through W2s) and dagg2 (through W2m)
__global__ void k_l2_bwd(int n, const float* __restrict__ theta, const float* __restrict__ dpre2,
                         float* __restrict__ dh1, float* __restrict__ dagg2) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * kH) return;
    int i = e / kH, k = e - i * kH;
    float a = 0.f, b = 0.f;
    for (int o = 0; o < kH; ++o) {
        float d = dpre2[i * kH + o];
        a = fmaf(rbf(theta[oW2s + o * kH + k]), d, a);
        b = fmaf(rbf(theta[oW2m + o * kH + k]), d, b);
    }
    dh1[e] = a;
    dagg2[e] = b;
}

// dpre1 = (dh1 + At-aggregated dagg2) masked by relu
__global__ void k_l1_mask(int n, const float* __restrict__ dh1, const float* __restrict__ t,
                          const float* __restrict__ pre1, float* __restrict__ dpre1) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * kH) return;
    dpre1[e] = (pre1[e] > 0.f) ? dh1[e] + t[e] : 0.f;
}

// Weight gradients: per-block fp64 partials of all kNP entries.  Inputs of the
// dense products enter rounded to bf16, as in the forward pass.
struct WG {
    int n;
    const float *x, *agg1, *h1, *agg2, *h2, *dpre1, *dpre2, *duvz;
};

__global__ void __launch_bounds__(kTB) k_wgrad(WG w, double* __restrict__ part) {
    constexpr int CH = 32;
    __shared__ float sx[CH][4], sa1[CH][4], sh1[CH][kH], sa2[CH][kH], sh2[CH][kH], sd1[CH][kH], sd2[CH][kH],
        sdu[CH][3];
    const int nb = gridDim.x;
    const int rows_per = (w.n + nb - 1) / nb;
    const int r0 = blockIdx.x * rows_per, r1 = min(w.n, r0 + rows_per);
    double acc[3] = {0.0, 0.0, 0.0};
    for (int b0 = r0; b0 < r1; b0 += CH) {
        const int rows = min(CH, r1 - b0);
        for (int k = threadIdx.x; k < rows * kH; k += blockDim.x) {
            int rr = k / kH, f = k - rr * kH, i = b0 + rr;
            sh1[rr][f] = rbf(w.h1[i * kH + f]);
            sa2[rr][f] = rbf(w.agg2[i * kH + f]);
            sh2[rr][f] = rbf(w.h2[i * kH + f]);
            sd1[rr][f] = w.dpre1[i * kH + f];
            sd2[rr][f] = w.dpre2[i * kH + f];
            if (f < 4) {
                sx[rr][f] = rbf(w.x[i * 4 + f]);
                sa1[rr][f] = rbf(w.agg1[i * 4 + f]);
            }
            if (f < 3) sdu[rr][f] = w.duvz[i * 3 + f];
        }
        __syncthreads();
        for (int h = 0; h < 3; ++h) {
            const int p = threadIdx.x + h * kTB;
            if (p >= kNP) break;
            double s = 0.0;
            for (int rr = 0; rr < rows; ++rr) {
                float g;
                if (p < oW1m) { int o = (p - oW1s) / 4, k = (p - oW1s) % 4; g = sd1[rr][o] * sx[rr][k]; }
                else if (p < ob1) { int o = (p - oW1m) / 4, k = (p - oW1m) % 4; g = sd1[rr][o] * sa1[rr][k]; }
                else if (p < oW2s) { g = sd1[rr][p - ob1]; }
                else if (p < oW2m) { int o = (p - oW2s) / kH, k = (p - oW2s) % kH; g = sd2[rr][o] * sh1[rr][k]; }
                else if (p < ob2) { int o = (p - oW2m) / kH, k = (p - oW2m) % kH; g = sd2[rr][o] * sa2[rr][k]; }
                else if (p < ou) { g = sd2[rr][p - ob2]; }
                else if (p < ov) { g = sdu[rr][0] * sh2[rr][p - ou]; }
                else if (p < oq) { g = sdu[rr][1] * sh2[rr][p - ov]; }
                else if (p < oc) { g = sdu[rr][2] * sh2[rr][p - oq]; }
                else if (p == oc) { g = sdu[rr][0]; }
                else { g = sdu[rr][2]; }
                s += (double)g;
            }
            acc[h] += s;
        }
        __syncthreads();
    }
    for (int h = 0; h < 3; ++h) {
        const int p = threadIdx.x + h * kTB;
        if (p < kNP) part[(size_t)blockIdx.x * kNP + p] = acc[h];
    }
}

__global__ void k_wgrad_sum(int nb, const double* __restrict__ part, float* __restrict__ grad) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNP) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[(size_t)b * kNP + p];
    grad[p] = (float)s;
}

// Adam (bias-corrected), fp32 master weights
__global__ void k_adam(float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, float lr, float b1, float b2, float eps, int t) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNP) return;
    float mm = b1 * m[p] + (1.f - b1) * g[p];
    float vv = b2 * v[p] + (1.f - b2) * g[p] * g[p];
    m[p] = mm;
    v[p] = vv;
    float mh = mm / (1.f - powf(b1, (float)t));
    float vh = vv / (1.f - powf(b2, (float)t));
    theta[p] -= lr * mh / (sqrtf(vh) + eps);
}

}  // namespace mp
}  // namespace pfe

using namespace pfe;
using namespace pfe::mp;

// Network weights, Adam state and per-graph scratch (grown on demand).
struct pfe_mpnn {
    float* theta = nullptr;   // kNP, device
    float* m = nullptr;
    float* v = nullptr;
    float* grad = nullptr;
    int t = 0;
    int64_t cap_n = 0, cap_s = 0;
    int cap_k = 0;
    float *at = nullptr, *x = nullptr, *agg1 = nullptr, *pre1 = nullptr, *h1 = nullptr, *agg2 = nullptr,
          *pre2 = nullptr, *h2 = nullptr, *uvz = nullptr, *gval = nullptr, *gdiag = nullptr;
    float *rho = nullptr, *y1 = nullptr, *y2 = nullptr, *y3 = nullptr, *es = nullptr, *dy2 = nullptr, *dy1 = nullptr;
    float *dgval = nullptr, *dgdiag = nullptr, *duvz = nullptr, *dpre2 = nullptr, *dh1 = nullptr, *dagg2 = nullptr,
          *tbuf = nullptr, *dpre1 = nullptr;
    double* part = nullptr;
    double* nrm = nullptr;
};

namespace {

constexpr int kRedBlocks = 256;

void free_scratch(pfe_mpnn* w) {
    float** bufs[] = {&w->at, &w->x, &w->agg1, &w->pre1, &w->h1, &w->agg2, &w->pre2, &w->h2, &w->uvz, &w->gval,
                      &w->gdiag, &w->rho, &w->y1, &w->y2, &w->y3, &w->es, &w->dy2, &w->dy1, &w->dgval, &w->dgdiag,
                      &w->duvz, &w->dpre2, &w->dh1, &w->dagg2, &w->tbuf, &w->dpre1};
    for (float** b : bufs)
        if (*b) { (void)dev_free(*b); *b = nullptr; }
    if (w->part) { (void)dev_free(w->part); w->part = nullptr; }
    if (w->nrm) { (void)dev_free(w->nrm); w->nrm = nullptr; }
    w->cap_n = w->cap_s = 0;
    w->cap_k = 0;
}

pfe_status ensure(pfe_mpnn* w, int64_t n, int64_t ns, int k) {
    if (n <= w->cap_n && ns <= w->cap_s && k <= w->cap_k) return PFE_OK;
    free_scratch(w);
    const int64_t nk = n * std::max(k, 1);
    hipError_t e = hipSuccess;
#define AL(p, cnt) do { if (e == hipSuccess) e = dev_alloc((void**)&(p), sizeof(float) * (size_t)(cnt)); } while (0)
    AL(w->at, ns); AL(w->x, n * 4); AL(w->agg1, n * 4); AL(w->pre1, n * kH); AL(w->h1, n * kH);
    AL(w->agg2, n * kH); AL(w->pre2, n * kH); AL(w->h2, n * kH); AL(w->uvz, n * 3); AL(w->gval, ns);
    AL(w->gdiag, n); AL(w->rho, nk); AL(w->y1, nk); AL(w->y2, nk); AL(w->y3, nk); AL(w->es, nk);
    AL(w->dy2, nk); AL(w->dy1, nk); AL(w->dgval, ns); AL(w->dgdiag, n); AL(w->duvz, n * 3);
    AL(w->dpre2, n * kH); AL(w->dh1, n * kH); AL(w->dagg2, n * kH); AL(w->tbuf, n * kH); AL(w->dpre1, n * kH);
#undef AL
    if (e == hipSuccess) e = dev_alloc((void**)&w->part, sizeof(double) * (size_t)kRedBlocks * kNP);
    if (e == hipSuccess) e = dev_alloc((void**)&w->nrm, sizeof(double) * 64);
    if (e != hipSuccess) {
        free_scratch(w);
        return hip_fail(e, "device allocation (network scratch)", __FILE__, __LINE__);
    }
    w->cap_n = n;
    w->cap_s = ns;
    w->cap_k = std::max(k, 1);
    return PFE_OK;
}

inline unsigned nblk(int64_t items) { return (unsigned)((items + kTB - 1) / kTB); }

View make_view(const NetGraph& g) {
    View v;
    v.n = (int)g.n;
    v.K = g.ell_K;
    v.deg_max = g.deg_max;
    v.rowptr = g.rowptr;
    v.scol = g.scol;
    v.seid = g.seid;
    v.sw64 = g.sw64;
    v.degree = g.degree;
    v.wsq = g.wsq;
    v.half_lam = 0.5 * g.lambda;
    v.half_r = 0.5 * g.r;
    return v;
}

// forward pass up to the factor values (fp32 gval / gdiag in the scratch)
pfe_status forward(pfe_mpnn* w, const View& v, int64_t ns, hipStream_t st) {
    const int n = v.n;
    hipLaunchKernelGGL(k_prep, dim3(nblk(n)), dim3(kTB), 0, st, v, w->at, w->x);
    hipLaunchKernelGGL(k_agg<4>, dim3(nblk((int64_t)n)), dim3(kTB), 0, st, v, w->at, w->x, w->agg1);
    const unsigned gd = (unsigned)(((n + 15) / 16 + 3) / 4);
    hipLaunchKernelGGL(k_dense<1>, dim3(gd), dim3(kTB), 0, st, n, w->theta, w->x, w->agg1, w->pre1, w->h1);
    hipLaunchKernelGGL(k_agg<kH>, dim3(nblk((int64_t)n * (kH / 4))), dim3(kTB), 0, st, v, w->at, w->h1, w->agg2);
    hipLaunchKernelGGL(k_dense<2>, dim3(gd), dim3(kTB), 0, st, n, w->theta, w->h1, w->agg2, w->pre2, w->h2);
    hipLaunchKernelGGL(k_dense<3>, dim3(gd), dim3(kTB), 0, st, n, w->theta, w->h2, (const float*)nullptr, w->uvz,
                       (float*)nullptr);
    hipLaunchKernelGGL(k_factor<float>, dim3(nblk(n)), dim3(kTB), 0, st, v, w->theta, w->at, w->uvz, w->gval,
                       w->gdiag);
    PFE_CHECK_HIP(hipGetLastError());
    (void)ns;
    return PFE_OK;
}

}  // namespace

namespace pfe {

pfe_status mpnn_factor(pfe_mpnn* w, const NetGraph& g, void* gval, void* gdiag, int esz, hipStream_t st) {
    PFE_TRY_STATUS(ensure(w, g.n, g.nslot, 1));
    View v = make_view(g);
    PFE_TRY_STATUS(forward(w, v, g.nslot, st));
    if (esz == 8) {
        hipLaunchKernelGGL(k_factor<double>, dim3(nblk(g.n)), dim3(kTB), 0, st, v, w->theta, w->at, w->uvz,
                           (double*)gval, (double*)gdiag);
    } else {
        PFE_CHECK_HIP(hipMemcpyAsync(gval, w->gval, sizeof(float) * g.nslot, hipMemcpyDeviceToDevice, st));
        PFE_CHECK_HIP(hipMemcpyAsync(gdiag, w->gdiag, sizeof(float) * g.n, hipMemcpyDeviceToDevice, st));
    }
    PFE_CHECK_HIP(hipGetLastError());
    return PFE_OK;
}

pfe_status mpnn_train_step(pfe_mpnn* w, const NetGraph& g, const void* samples, int esz, int kc, float lr,
                           double* loss, hipStream_t st) {
    PFE_TRY_STATUS(ensure(w, g.n, g.nslot, kc));
    View v = make_view(g);
    const int n = v.n;
    const int64_t nk = (int64_t)n * kc;
    PFE_TRY_STATUS(forward(w, v, g.nslot, st));
    // scaled, unit-norm samples
    if (esz == 8)
        hipLaunchKernelGGL(k_sample_norm<double>, dim3(kRedBlocks), dim3(kTB), 0, st, v, kc, (const double*)samples, w->part);
    else
        hipLaunchKernelGGL(k_sample_norm<float>, dim3(kRedBlocks), dim3(kTB), 0, st, v, kc, (const float*)samples, w->part);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, st, kRedBlocks, kc, w->part, w->nrm);
    if (esz == 8)
        hipLaunchKernelGGL(k_sample_scale<double>, dim3(nblk(nk)), dim3(kTB), 0, st, v, kc, (const double*)samples, w->nrm, w->rho);
    else
        hipLaunchKernelGGL(k_sample_scale<float>, dim3(nblk(nk)), dim3(kTB), 0, st, v, kc, (const float*)samples, w->nrm, w->rho);
    // y1 = Gt rho, y2 = Gt^T y1, y3 = At y2, loss and dL/dy3
    hipLaunchKernelGGL(k_gmul<true>, dim3(nblk(nk)), dim3(kTB), 0, st, v, kc, w->gval, w->gdiag, w->rho, w->y1);
    hipLaunchKernelGGL(k_gmul<false>, dim3(nblk(nk)), dim3(kTB), 0, st, v, kc, w->gval, w->gdiag, w->y1, w->y2);
    hipLaunchKernelGGL(k_amul, dim3(nblk(nk)), dim3(kTB), 0, st, v, kc, w->at, w->y2, w->y3);
    hipLaunchKernelGGL(k_resid, dim3(kRedBlocks), dim3(kTB), 0, st, v, kc, w->y3, w->rho, w->es, w->part);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, st, kRedBlocks, kc, w->part, w->nrm);
    // dy2 = At e, dy1 = Gt dy2
    hipLaunchKernelGGL(k_amul, dim3(nblk(nk)), dim3(kTB), 0, st, v, kc, w->at, w->es, w->dy2);
    hipLaunchKernelGGL(k_gmul<true>, dim3(nblk(nk)), dim3(kTB), 0, st, v, kc, w->gval, w->gdiag, w->dy2, w->dy1);
    hipLaunchKernelGGL(k_dfactor, dim3(nblk(n)), dim3(kTB), 0, st, v, kc, w->rho, w->y1, w->dy1, w->dy2, w->dgval,
                       w->dgdiag);
    // network backward
    hipLaunchKernelGGL(k_out_bwd, dim3(nblk(n)), dim3(kTB), 0, st, v, w->theta, w->at, w->dgval, w->dgdiag, w->uvz,
                       w->pre2, w->duvz, w->dpre2);
    hipLaunchKernelGGL(k_l2_bwd, dim3(nblk((int64_t)n * kH)), dim3(kTB), 0, st, n, w->theta, w->dpre2, w->dh1, w->dagg2);
    hipLaunchKernelGGL(k_agg<kH>, dim3(nblk((int64_t)n * (kH / 4))), dim3(kTB), 0, st, v, w->at, w->dagg2, w->tbuf);
    hipLaunchKernelGGL(k_l1_mask, dim3(nblk((int64_t)n * kH)), dim3(kTB), 0, st, n, w->dh1, w->tbuf, w->pre1, w->dpre1);
    WG wg{n, w->x, w->agg1, w->h1, w->agg2, w->h2, w->dpre1, w->dpre2, w->duvz};
    hipLaunchKernelGGL(k_wgrad, dim3(kRedBlocks), dim3(kTB), 0, st, wg, w->part);
    hipLaunchKernelGGL(k_wgrad_sum, dim3((kNP + 255) / 256), dim3(256), 0, st, kRedBlocks, w->part, w->grad);
    PFE_CHECK_HIP(hipGetLastError());
    if (loss) {
        std::vector<double> lc(kc);
        PFE_CHECK_HIP(hipMemcpyAsync(lc.data(), w->nrm, sizeof(double) * kc, hipMemcpyDeviceToHost, st));
        PFE_CHECK_HIP(hipStreamSynchronize(st));
        double s = 0.0;
        for (int c = 0; c < kc; ++c) s += lc[c];
        *loss = s / kc;
    }
    if (lr > 0.f) {
        w->t += 1;
        hipLaunchKernelGGL(k_adam, dim3((kNP + 255) / 256), dim3(256), 0, st, w->theta, w->m, w->v, w->grad, lr,
                           0.9f, 0.999f, 1e-8f, w->t);
        PFE_CHECK_HIP(hipGetLastError());
    }
    return PFE_OK;
}

}  // namespace pfe

extern "C" {

pfe_status pfe_mpnn_create(const float* params, pfe_mpnn** out) {
    if (!out) { set_error("pfe_mpnn_create: null argument"); return PFE_E_ARG; }
    *out = nullptr;
    pfe_mpnn* w = new pfe_mpnn();
    hipError_t e = dev_alloc((void**)&w->theta, sizeof(float) * kNP);
    if (e == hipSuccess) e = dev_alloc((void**)&w->m, sizeof(float) * kNP);
    if (e == hipSuccess) e = dev_alloc((void**)&w->v, sizeof(float) * kNP);
    if (e == hipSuccess) e = dev_alloc((void**)&w->grad, sizeof(float) * kNP);
    if (e != hipSuccess) {
        (void)dev_free(w->theta); (void)dev_free(w->m); (void)dev_free(w->v); (void)dev_free(w->grad);
        delete w;
        return hip_fail(e, "device allocation (network)", __FILE__, __LINE__);
    }
    std::vector<float> th(kNP, 0.f);
    if (params) {
        memcpy(th.data(), params, sizeof(float) * kNP);
    } else {
        th[obd] = (float)log(exp(1.0) - 1.0);   // Gt = I: the Jacobi preconditioner
    }
    if (hipMemcpy(w->theta, th.data(), sizeof(float) * kNP, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(w->m, 0, sizeof(float) * kNP) != hipSuccess || hipMemset(w->v, 0, sizeof(float) * kNP) != hipSuccess ||
        hipMemset(w->grad, 0, sizeof(float) * kNP) != hipSuccess) {
        pfe_mpnn_destroy(w);
        set_error("pfe_mpnn_create: initialisation copy failed");
        return PFE_E_HIP;
    }
    *out = w;
    return PFE_OK;
}

pfe_status pfe_mpnn_get_params(pfe_mpnn* w, float* params, float* grad) {
    if (!w) { set_error("pfe_mpnn_get_params: null network"); return PFE_E_ARG; }
    if (params) PFE_CHECK_HIP(hipMemcpy(params, w->theta, sizeof(float) * kNP, hipMemcpyDeviceToHost));
    if (grad) PFE_CHECK_HIP(hipMemcpy(grad, w->grad, sizeof(float) * kNP, hipMemcpyDeviceToHost));
    return PFE_OK;
}

pfe_status pfe_mpnn_set_params(pfe_mpnn* w, const float* params) {
    if (!w || !params) { set_error("pfe_mpnn_set_params: null argument"); return PFE_E_ARG; }
    PFE_CHECK_HIP(hipMemcpy(w->theta, params, sizeof(float) * kNP, hipMemcpyHostToDevice));
    PFE_CHECK_HIP(hipMemset(w->m, 0, sizeof(float) * kNP));
    PFE_CHECK_HIP(hipMemset(w->v, 0, sizeof(float) * kNP));
    w->t = 0;
    return PFE_OK;
}

// network file: 8-byte magic, uint32 parameter count, the parameters as
// little-endian float32 (the layout of PFE_MPNN_NPARAMS)
static const char kMpnnMagic[8] = {'P', 'F', 'E', 'M', 'P', 'N', 'N', '1'};

pfe_status pfe_mpnn_save(pfe_mpnn* w, const char* path) {
    if (!w || !path) { set_error("pfe_mpnn_save: null argument"); return PFE_E_ARG; }
    std::vector<float> th(kNP);
    const pfe_status st = pfe_mpnn_get_params(w, th.data(), nullptr);
    if (st != PFE_OK) return st;
    FILE* f = fopen(path, "wb");
    if (!f) { set_error("pfe_mpnn_save: cannot open %s", path); return PFE_E_ARG; }
    const uint32_t count = (uint32_t)kNP;
    const bool ok = fwrite(kMpnnMagic, 1, 8, f) == 8 && fwrite(&count, 4, 1, f) == 1 &&
                    fwrite(th.data(), sizeof(float), kNP, f) == (size_t)kNP;
    if (fclose(f) != 0 || !ok) { set_error("pfe_mpnn_save: write to %s failed", path); return PFE_E_ARG; }
    return PFE_OK;
}

pfe_status pfe_mpnn_load(const char* path, pfe_mpnn** out) {
    if (!path || !out) { set_error("pfe_mpnn_load: null argument"); return PFE_E_ARG; }
    *out = nullptr;
    FILE* f = fopen(path, "rb");
    if (!f) { set_error("pfe_mpnn_load: cannot open %s", path); return PFE_E_ARG; }
    char magic[8];
    uint32_t count = 0;
    std::vector<float> th(kNP);
    bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kMpnnMagic, 8) == 0 && fread(&count, 4, 1, f) == 1 &&
              count == (uint32_t)kNP && fread(th.data(), sizeof(float), kNP, f) == (size_t)kNP;
    char extra;
    ok = ok && fread(&extra, 1, 1, f) == 0;   // nothing after the parameters
    fclose(f);
    if (!ok) { set_error("pfe_mpnn_load: %s is not a network file of %d parameters", path, kNP); return PFE_E_ARG; }
    for (float v : th)
        if (!std::isfinite(v)) { set_error("pfe_mpnn_load: non-finite parameter in %s", path); return PFE_E_ARG; }
    return pfe_mpnn_create(th.data(), out);
}

void pfe_mpnn_destroy(pfe_mpnn* w) {
    if (!w) return;
    (void)hipDeviceSynchronize();
    free_scratch(w);
    (void)dev_free(w->theta); (void)dev_free(w->m); (void)dev_free(w->v); (void)dev_free(w->grad);
    delete w;
}

}  // extern "C"
