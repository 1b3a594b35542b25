// Graph construction on the device (Sec. II): CSR adjacency with both
// directions of every edge and heat-kernel weights w = exp(-||dx||^2 / 2 sigma^2)
// evaluated in FP64, degrees d_i = sum_j w_ij (Algorithm 1: D = diag(W 1)).
#include <cfloat>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <vector>
#include <algorithm>

#include "common.hpp"

namespace pfe {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

pfe_status hip_fail(hipError_t e, const char* what, const char* file, int line) {
    set_error("%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
    return (e == hipErrorOutOfMemory) ? PFE_E_NOMEM : PFE_E_HIP;
}

// ---------------------------------------------------------------------------
// Exclusive prefix sum of int32 counts (three passes: per-block scan, scan of
// block totals, offset add).  Used once per graph build.
// ---------------------------------------------------------------------------
constexpr int kScanBlock = 1024;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanBlock * kScanItems;

__device__ int block_exclusive_scan(int v, int* sh, int* total) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
        int add = (t >= off) ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    int incl = sh[t];
    if (total) *total = sh[kScanBlock - 1];
    __syncthreads();
    return incl - v;
}

__global__ void __launch_bounds__(kScanBlock)
k_scan_tiles(const int* __restrict__ in, int* __restrict__ out, int* __restrict__ tile_sum, int64_t n) {
    __shared__ int sh[kScanBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    int tot;
    int ex = block_exclusive_scan(s, sh, &tot);
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kScanBlock)
k_scan_sums(int* __restrict__ tile_sum, int ntiles, int* __restrict__ grand_total) {
    __shared__ int sh[kScanBlock];
    int carry = 0;
    for (int b0 = 0; b0 < ntiles; b0 += kScanBlock) {
        int i = b0 + threadIdx.x;
        int v = (i < ntiles) ? tile_sum[i] : 0;
        int tot;
        int ex = block_exclusive_scan(v, sh, &tot);
        if (i < ntiles) tile_sum[i] = ex + carry;
        carry += tot;
    }
    if (threadIdx.x == 0) *grand_total = carry;
}

__global__ void k_scan_add(int* __restrict__ out, const int* __restrict__ tile_sum, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += tile_sum[i / kScanTile];
}

// out[0..n) = exclusive scan of in[0..n); out[n] = total.  out must hold n + 1.
static pfe_status exclusive_scan(const int* in, int* out, int64_t n, hipStream_t st) {
    int64_t ntiles = (n + kScanTile - 1) / kScanTile;
    if (ntiles < 1) ntiles = 1;
    int* sums = nullptr;
    PFE_CHECK_HIP(dev_alloc_async((void**)&sums, sizeof(int) * ntiles, st));
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(kScanBlock), 0, st, in, out, sums, n);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, st, sums, (int)ntiles, out + n);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, out, sums, n);
    PFE_CHECK_HIP(hipGetLastError());
    PFE_CHECK_HIP(dev_free_async(sums, st));
    return PFE_OK;
}

// ---------------------------------------------------------------------------
// Pixel grids
// ---------------------------------------------------------------------------
constexpr int kMaxOffsets = 80;   // window radius up to 4
struct Stencil {
    int k;
    int dy[kMaxOffsets];
    int dx[kMaxOffsets];
};

// error bits written by the build kernels
enum : int {
    ERR_RANGE = 1, ERR_SELF = 2, ERR_DUP = 4, ERR_ISOLATED = 8, ERR_NONFINITE = 16, ERR_ASYM = 32
};

__global__ void k_grid_degree(int H, int W, Stencil st, int* __restrict__ deg) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)H * W) return;
    int y = (int)(i / W), x = (int)(i - (int64_t)y * W);
    int c = 0;
    for (int k = 0; k < st.k; ++k) {
        int yy = y + st.dy[k], xx = x + st.dx[k];
        c += (yy >= 0 && yy < H && xx >= 0 && xx < W);
    }
    deg[i] = c;
}

__global__ void k_grid_fill(int H, int W, int m, const float* __restrict__ feat, Stencil st,
                            double inv2s2, const int* __restrict__ rowptr, int* __restrict__ col,
                            double* __restrict__ w64) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)H * W) return;
    int y = (int)(i / W), x = (int)(i - (int64_t)y * W);
    int s = rowptr[i];
    const float* fi = feat + i * m;
    for (int k = 0; k < st.k; ++k) {
        int yy = y + st.dy[k], xx = x + st.dx[k];
        if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
        int64_t j = (int64_t)yy * W + xx;
        const float* fj = feat + j * m;
        double d2 = 0.0;
        for (int f = 0; f < m; ++f) {
            double df = (double)fi[f] - (double)fj[f];
            d2 += df * df;
        }
        col[s] = (int)j;
        w64[s] = exp(-d2 * inv2s2);
        ++s;
    }
}

// ---------------------------------------------------------------------------
// Edge lists
// ---------------------------------------------------------------------------
__global__ void k_edge_count(int64_t n, int64_t ne, const int32_t* __restrict__ src,
                             const int32_t* __restrict__ dst, int* __restrict__ deg, int* __restrict__ err) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    int a = src[e], b = dst[e];
    if (a < 0 || b < 0 || a >= n || b >= n) { atomicOr(err, ERR_RANGE); return; }
    if (a == b) { atomicOr(err, ERR_SELF); return; }
    atomicAdd(&deg[a], 1);
    atomicAdd(&deg[b], 1);
}

__global__ void k_edge_scatter(int64_t n, int64_t ne, const int32_t* __restrict__ src,
                               const int32_t* __restrict__ dst, const double* __restrict__ dist2,
                               double inv2s2, const int* __restrict__ rowptr, int* __restrict__ fill,
                               int* __restrict__ col, double* __restrict__ w64) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    int a = src[e], b = dst[e];
    if (a < 0 || b < 0 || a >= n || b >= n || a == b) return;
    double w = exp(-dist2[e] * inv2s2);
    int sa = rowptr[a] + atomicAdd(&fill[a], 1);
    int sb = rowptr[b] + atomicAdd(&fill[b], 1);
    col[sa] = b; w64[sa] = w;
    col[sb] = a; w64[sb] = w;
}

// Sort every row by column (insertion sort: rows are short) and flag duplicates.
__global__ void k_row_sort(int64_t n, const int* __restrict__ rowptr, int* __restrict__ col,
                           double* __restrict__ w64, int* __restrict__ err) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int s0 = rowptr[i], s1 = rowptr[i + 1];
    for (int s = s0 + 1; s < s1; ++s) {
        int c = col[s];
        double w = w64[s];
        int t = s - 1;
        while (t >= s0 && col[t] > c) {
            col[t + 1] = col[t];
            w64[t + 1] = w64[t];
            --t;
        }
        col[t + 1] = c;
        w64[t + 1] = w;
    }
    for (int s = s0 + 1; s < s1; ++s)
        if (col[s] == col[s - 1]) atomicOr(err, ERR_DUP);
}

// ---------------------------------------------------------------------------
// Common finish: FP32 weights, degrees, sum of squared weights, upper counts.
// ---------------------------------------------------------------------------
__global__ void k_row_finish(int64_t n, const int* __restrict__ rowptr, const int* __restrict__ col,
                             const double* __restrict__ w64, float* __restrict__ w32,
                             double* __restrict__ degree, double* __restrict__ wsq,
                             int* __restrict__ upper, int* __restrict__ err) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int s0 = rowptr[i], s1 = rowptr[i + 1];
    double dsum = 0.0, qsum = 0.0;
    int up = 0;
    for (int s = s0; s < s1; ++s) {
        double w = w64[s];
        if (!isfinite(w)) atomicOr(err, ERR_NONFINITE);
        w32[s] = (float)w;
        dsum += w;
        qsum += w * w;
        up += (col[s] > i);
    }
    degree[i] = dsum;
    wsq[i] = qsum;
    upper[i] = up;
    if (!(dsum >= (double)FLT_MIN)) atomicOr(err, ERR_ISOLATED);
}

// Reverse slot and undirected edge id of every slot.
__global__ void k_rev_eid(int64_t n, const int* __restrict__ rowptr, const int* __restrict__ col,
                          const int* __restrict__ upper, const int* __restrict__ uptr,
                          int* __restrict__ rev, int* __restrict__ eid, int* __restrict__ err) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int s0 = rowptr[i], s1 = rowptr[i + 1];
    for (int s = s0; s < s1; ++s) {
        int j = col[s];
        int lo = rowptr[j], hi = rowptr[j + 1] - 1, found = -1;
        while (lo <= hi) {
            int mid = (lo + hi) >> 1;
            int c = col[mid];
            if (c == (int)i) { found = mid; break; }
            if (c < (int)i) lo = mid + 1; else hi = mid - 1;
        }
        if (found < 0) { atomicOr(err, ERR_ASYM); rev[s] = s; eid[s] = 0; continue; }
        rev[s] = found;
        if (j > (int)i) {
            eid[s] = uptr[i] + (s - (s1 - upper[i]));
        } else {
            int j1 = rowptr[j + 1];
            eid[s] = uptr[j] + (found - (j1 - upper[j]));
        }
    }
}

// ELL copy of the CSR slots: slot k of row i at k * n + i.
__global__ void k_build_ell(int64_t n, int K, const int* __restrict__ rowptr, const int* __restrict__ col,
                            const float* __restrict__ w32, const double* __restrict__ w64,
                            const int* __restrict__ eid, int* __restrict__ s_col, float* __restrict__ s_w32,
                            double* __restrict__ s_w64, int* __restrict__ s_eid) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int s0 = rowptr[i], deg = rowptr[i + 1] - s0;
    for (int k = 0; k < K; ++k) {
        int64_t s = (int64_t)k * n + i;
        if (k < deg) {
            s_col[s] = col[s0 + k];
            s_w32[s] = w32[s0 + k];
            s_w64[s] = w64[s0 + k];
            s_eid[s] = eid[s0 + k];
        } else {
            s_col[s] = (int)i;
            s_w32[s] = 0.0f;
            s_w64[s] = 0.0;
            s_eid[s] = -1;
        }
    }
}

// Stencil-ordered ELL for pixel grids: slot k of row i is stencil offset k.
__global__ void k_build_stencil_ell(int H, int W, Stencil st, const int* __restrict__ rowptr,
                                    const int* __restrict__ col, const float* __restrict__ w32,
                                    const double* __restrict__ w64, const int* __restrict__ eid,
                                    int* __restrict__ s_col, float* __restrict__ s_w32,
                                    double* __restrict__ s_w64, int* __restrict__ s_eid, int* __restrict__ err) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)H * W;
    if (i >= n) return;
    int y = (int)(i / W), x = (int)(i - (int64_t)y * W);
    int s0 = rowptr[i], s1 = rowptr[i + 1];
    for (int k = 0; k < st.k; ++k) {
        int64_t s = (int64_t)k * n + i;
        int yy = y + st.dy[k], xx = x + st.dx[k];
        int slot = -1;
        if (yy >= 0 && yy < H && xx >= 0 && xx < W) {
            int j = yy * W + xx;
            int lo = s0, hi = s1 - 1;
            while (lo <= hi) {
                int mid = (lo + hi) >> 1;
                if (col[mid] == j) { slot = mid; break; }
                if (col[mid] < j) lo = mid + 1; else hi = mid - 1;
            }
            if (slot < 0) atomicOr(err, ERR_ASYM);
        }
        if (slot >= 0) {
            s_col[s] = col[slot];
            s_w32[s] = w32[slot];
            s_w64[s] = w64[slot];
            s_eid[s] = eid[slot];
        } else {
            s_col[s] = (int)i;
            s_w32[s] = 0.0f;
            s_w64[s] = 0.0;
            s_eid[s] = -1;
        }
    }
}

// dst[i] = src[i] + add (negative entries kept as they are when keep_neg)
__global__ void k_add_int(int64_t n, const int* __restrict__ src, int add, int keep_neg, int* __restrict__ dst) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int v = src[i];
    dst[i] = (keep_neg && v < 0) ? v : v + add;
}

__global__ void k_max_deg(int64_t n, const int* __restrict__ rowptr, int* __restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    atomicMax(out, rowptr[i + 1] - rowptr[i]);
}

// grid-stride 16-byte copy
// Plain copy for the bandwidth probe: each thread keeps kCopyUnroll 16-byte
// loads in flight (issued together, then their stores), grid-stride over the
// buffer, streaming (non-temporal) accesses.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kCopyUnroll = 4;
constexpr int kCopyThreads = 256;

__global__ void __launch_bounds__(kCopyThreads) k_stream_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                               size_t n16) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (kCopyUnroll - 1) * stride < n16; i += kCopyUnroll * stride) {
        u32x4 v[kCopyUnroll];
#pragma unroll
        for (int k = 0; k < kCopyUnroll; ++k) v[k] = __builtin_nontemporal_load(src + i + k * stride);
#pragma unroll
        for (int k = 0; k < kCopyUnroll; ++k) __builtin_nontemporal_store(v[k], dst + i + k * stride);
    }
    for (; i < n16; i += stride) dst[i] = src[i];
}

static void free_graph_buffers(pfe_graph* g) {
    if (!g) return;
    (void)dev_free(g->rowptr); (void)dev_free(g->col); (void)dev_free(g->rev); (void)dev_free(g->eid);
    (void)dev_free(g->w32); (void)dev_free(g->w64); (void)dev_free(g->degree); (void)dev_free(g->wsq);
    if (g->ell_K > 0) {
        (void)dev_free(g->s_col); (void)dev_free(g->s_w32); (void)dev_free(g->s_w64); (void)dev_free(g->s_eid);
    }
}

static const char* graph_err_text(int e) {
    if (e & ERR_RANGE) return "edge endpoint out of range";
    if (e & ERR_SELF) return "self loop in edge list";
    if (e & ERR_DUP) return "duplicate edge";
    if (e & ERR_NONFINITE) return "non-finite edge weight";
    if (e & ERR_ISOLATED) return "isolated vertex (degree below FLT_MIN)";
    if (e & ERR_ASYM) return "adjacency not symmetric";
    return "invalid graph";
}

static pfe_status build_impl(const pfe_graph_desc* d, hipStream_t st, pfe_graph* g) {
    const double inv2s2 = 1.0 / (2.0 * d->sigma * d->sigma);
    const int TB = 256;
    int* deg = nullptr;
    int* err = nullptr;
    int* fill = nullptr;
    int* upper = nullptr;
    void* tmp_in = nullptr;      // device copies of host inputs
    void* tmp_in2 = nullptr;
    void* tmp_in3 = nullptr;
    int64_t n = g->n;
    unsigned gridN = (unsigned)((n + TB - 1) / TB);
    PFE_CHECK_HIP(dev_alloc_async((void**)&deg, sizeof(int) * (n + 1), st));
    PFE_CHECK_HIP(dev_alloc_async((void**)&err, sizeof(int), st));
    PFE_CHECK_HIP(hipMemsetAsync(deg, 0, sizeof(int) * (n + 1), st));
    PFE_CHECK_HIP(hipMemsetAsync(err, 0, sizeof(int), st));
    PFE_CHECK_HIP(dev_alloc((void**)&g->rowptr, sizeof(int) * (n + 1)));

    if (d->kind == PFE_GRID) {
        Stencil sten{};
        std::vector<std::pair<int, int>> offs;
        if (d->stencil == 4) offs = {{-1, 0}, {0, -1}, {0, 1}, {1, 0}};
        else if (d->stencil == 8) offs = {{-1, -1}, {-1, 0}, {-1, 1}, {0, -1}, {0, 1}, {1, -1}, {1, 0}, {1, 1}};
        else {
            int R = -d->stencil;
            for (int dy = -R; dy <= R; ++dy)
                for (int dx = -R; dx <= R; ++dx)
                    if (dy || dx) offs.push_back({dy, dx});
        }
        sten.k = (int)offs.size();
        for (int k = 0; k < sten.k; ++k) { sten.dy[k] = offs[k].first; sten.dx[k] = offs[k].second; }
        const float* feat = d->feat;
        size_t fbytes = sizeof(float) * (size_t)n * d->m;
        if (!d->on_device) {
            PFE_CHECK_HIP(dev_alloc_async(&tmp_in, fbytes, st));
            PFE_CHECK_HIP(hipMemcpyAsync(tmp_in, d->feat, fbytes, hipMemcpyHostToDevice, st));
            feat = (const float*)tmp_in;
        }
        hipLaunchKernelGGL(k_grid_degree, dim3(gridN), dim3(TB), 0, st, d->H, d->W, sten, deg);
        pfe_status s = exclusive_scan(deg, g->rowptr, n, st);
        if (s != PFE_OK) return s;
        int total = 0;
        PFE_CHECK_HIP(hipMemcpyAsync(&total, g->rowptr + n, sizeof(int), hipMemcpyDeviceToHost, st));
        PFE_CHECK_HIP(hipStreamSynchronize(st));
        g->slots = total;
        PFE_CHECK_HIP(dev_alloc((void**)&g->col, sizeof(int) * (g->slots + 1)));
        PFE_CHECK_HIP(dev_alloc((void**)&g->w64, sizeof(double) * (g->slots + 1)));
        hipLaunchKernelGGL(k_grid_fill, dim3(gridN), dim3(TB), 0, st, d->H, d->W, d->m, feat, sten,
                           inv2s2, g->rowptr, g->col, g->w64);
        hipLaunchKernelGGL(k_row_sort, dim3(gridN), dim3(TB), 0, st, n, g->rowptr, g->col, g->w64, err);
    } else {
        int64_t ne = d->n_edges;
        const int32_t* src = d->src;
        const int32_t* dst = d->dst;
        const double* dist2 = d->dist2;
        if (!d->on_device) {
            PFE_CHECK_HIP(dev_alloc_async(&tmp_in, sizeof(int32_t) * (ne + 1), st));
            PFE_CHECK_HIP(dev_alloc_async(&tmp_in2, sizeof(int32_t) * (ne + 1), st));
            PFE_CHECK_HIP(dev_alloc_async(&tmp_in3, sizeof(double) * (ne + 1), st));
            PFE_CHECK_HIP(hipMemcpyAsync(tmp_in, src, sizeof(int32_t) * ne, hipMemcpyHostToDevice, st));
            PFE_CHECK_HIP(hipMemcpyAsync(tmp_in2, dst, sizeof(int32_t) * ne, hipMemcpyHostToDevice, st));
            PFE_CHECK_HIP(hipMemcpyAsync(tmp_in3, dist2, sizeof(double) * ne, hipMemcpyHostToDevice, st));
            src = (const int32_t*)tmp_in;
            dst = (const int32_t*)tmp_in2;
            dist2 = (const double*)tmp_in3;
        }
        unsigned gridE = (unsigned)((ne + TB - 1) / TB);
        if (ne > 0)
            hipLaunchKernelGGL(k_edge_count, dim3(gridE), dim3(TB), 0, st, n, ne, src, dst, deg, err);
        pfe_status s = exclusive_scan(deg, g->rowptr, n, st);
        if (s != PFE_OK) return s;
        int total = 0, herr = 0;
        PFE_CHECK_HIP(hipMemcpyAsync(&total, g->rowptr + n, sizeof(int), hipMemcpyDeviceToHost, st));
        PFE_CHECK_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
        PFE_CHECK_HIP(hipStreamSynchronize(st));
        if (herr) { set_error("pfe_build_graph: %s", graph_err_text(herr)); return PFE_E_GRAPH; }
        g->slots = total;
        PFE_CHECK_HIP(dev_alloc((void**)&g->col, sizeof(int) * (g->slots + 1)));
        PFE_CHECK_HIP(dev_alloc((void**)&g->w64, sizeof(double) * (g->slots + 1)));
        PFE_CHECK_HIP(dev_alloc_async((void**)&fill, sizeof(int) * (n + 1), st));
        PFE_CHECK_HIP(hipMemsetAsync(fill, 0, sizeof(int) * (n + 1), st));
        if (ne > 0)
            hipLaunchKernelGGL(k_edge_scatter, dim3(gridE), dim3(TB), 0, st, n, ne, src, dst, dist2,
                               inv2s2, g->rowptr, fill, g->col, g->w64);
        hipLaunchKernelGGL(k_row_sort, dim3(gridN), dim3(TB), 0, st, n, g->rowptr, g->col, g->w64, err);
    }
    g->n_edges = g->slots / 2;
    PFE_CHECK_HIP(dev_alloc((void**)&g->w32, sizeof(float) * (g->slots + 1)));
    PFE_CHECK_HIP(dev_alloc((void**)&g->rev, sizeof(int) * (g->slots + 1)));
    PFE_CHECK_HIP(dev_alloc((void**)&g->eid, sizeof(int) * (g->slots + 1)));
    PFE_CHECK_HIP(dev_alloc((void**)&g->degree, sizeof(double) * n));
    PFE_CHECK_HIP(dev_alloc((void**)&g->wsq, sizeof(double) * n));
    PFE_CHECK_HIP(dev_alloc_async((void**)&upper, sizeof(int) * (n + 1), st));
    hipLaunchKernelGGL(k_row_finish, dim3(gridN), dim3(TB), 0, st, n, g->rowptr, g->col, g->w64, g->w32,
                       g->degree, g->wsq, upper, err);
    int* uptr = deg;   // reuse: exclusive scan of upper counts
    pfe_status s = exclusive_scan(upper, uptr, n, st);
    if (s != PFE_OK) return s;
    hipLaunchKernelGGL(k_rev_eid, dim3(gridN), dim3(TB), 0, st, n, g->rowptr, g->col, upper, uptr,
                       g->rev, g->eid, err);
    PFE_CHECK_HIP(hipGetLastError());
    int herr = 0;
    PFE_CHECK_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
    PFE_CHECK_HIP(dev_free_async(deg, st));
    PFE_CHECK_HIP(dev_free_async(err, st));
    PFE_CHECK_HIP(dev_free_async(upper, st));
    if (fill) PFE_CHECK_HIP(dev_free_async(fill, st));
    if (tmp_in) PFE_CHECK_HIP(dev_free_async(tmp_in, st));
    if (tmp_in2) PFE_CHECK_HIP(dev_free_async(tmp_in2, st));
    if (tmp_in3) PFE_CHECK_HIP(dev_free_async(tmp_in3, st));
    PFE_CHECK_HIP(hipStreamSynchronize(st));
    if (herr) { set_error("pfe_build_graph: %s", graph_err_text(herr)); return PFE_E_GRAPH; }

    // slot layout for the solver: ELL when padding to the largest degree costs
    // at most a quarter more slots (pixel stencils), CSR otherwise.
    int* dmax = nullptr;
    PFE_CHECK_HIP(dev_alloc((void**)&dmax, sizeof(int)));
    PFE_CHECK_HIP(hipMemsetAsync(dmax, 0, sizeof(int), st));
    hipLaunchKernelGGL(k_max_deg, dim3(gridN), dim3(TB), 0, st, n, g->rowptr, dmax);
    PFE_CHECK_HIP(hipMemcpyAsync(&g->max_deg, dmax, sizeof(int), hipMemcpyDeviceToHost, st));
    PFE_CHECK_HIP(hipStreamSynchronize(st));
    PFE_CHECK_HIP(dev_free(dmax));
    const int64_t ell_slots = (int64_t)g->max_deg * n;
    if (d->kind == PFE_GRID) {
        // stencil-ordered ELL (every pixel grid qualifies)
        Stencil sten{};
        std::vector<std::pair<int, int>> offs;
        if (d->stencil == 4) offs = {{-1, 0}, {0, -1}, {0, 1}, {1, 0}};
        else if (d->stencil == 8) offs = {{-1, -1}, {-1, 0}, {-1, 1}, {0, -1}, {0, 1}, {1, -1}, {1, 0}, {1, 1}};
        else {
            int R = -d->stencil;
            for (int dy = -R; dy <= R; ++dy)
                for (int dx = -R; dx <= R; ++dx)
                    if (dy || dx) offs.push_back({dy, dx});
        }
        sten.k = (int)offs.size();
        for (int k = 0; k < sten.k; ++k) {
            sten.dy[k] = offs[k].first;
            sten.dx[k] = offs[k].second;
        }
        const int64_t ns = (int64_t)sten.k * n;
        if (ns >= (int64_t)INT32_MAX) { set_error("pfe_build_graph: graph too large"); return PFE_E_ARG; }
        g->ell_K = sten.k;
        g->stencil = 1;
        g->nslot = ns;
        PFE_CHECK_HIP(dev_alloc((void**)&g->s_col, sizeof(int) * ns));
        PFE_CHECK_HIP(dev_alloc((void**)&g->s_w32, sizeof(float) * ns));
        PFE_CHECK_HIP(dev_alloc((void**)&g->s_w64, sizeof(double) * ns));
        PFE_CHECK_HIP(dev_alloc((void**)&g->s_eid, sizeof(int) * ns));
        int* err2 = nullptr;
        PFE_CHECK_HIP(dev_alloc((void**)&err2, sizeof(int)));
        PFE_CHECK_HIP(hipMemsetAsync(err2, 0, sizeof(int), st));
        hipLaunchKernelGGL(k_build_stencil_ell, dim3(gridN), dim3(TB), 0, st, d->H, d->W, sten, g->rowptr, g->col,
                           g->w32, g->w64, g->eid, g->s_col, g->s_w32, g->s_w64, g->s_eid, err2);
        PFE_CHECK_HIP(hipGetLastError());
        int herr2 = 0;
        PFE_CHECK_HIP(hipMemcpyAsync(&herr2, err2, sizeof(int), hipMemcpyDeviceToHost, st));
        PFE_CHECK_HIP(hipStreamSynchronize(st));
        PFE_CHECK_HIP(dev_free(err2));
        if (herr2) { set_error("pfe_build_graph: %s", graph_err_text(herr2)); return PFE_E_GRAPH; }
    } else if (g->max_deg > 0 && 4 * ell_slots <= 5 * g->slots && ell_slots < (int64_t)INT32_MAX) {
        g->ell_K = g->max_deg;
        g->nslot = ell_slots;
        PFE_CHECK_HIP(dev_alloc((void**)&g->s_col, sizeof(int) * ell_slots));
        PFE_CHECK_HIP(dev_alloc((void**)&g->s_w32, sizeof(float) * ell_slots));
        PFE_CHECK_HIP(dev_alloc((void**)&g->s_w64, sizeof(double) * ell_slots));
        PFE_CHECK_HIP(dev_alloc((void**)&g->s_eid, sizeof(int) * ell_slots));
        hipLaunchKernelGGL(k_build_ell, dim3(gridN), dim3(TB), 0, st, n, g->ell_K, g->rowptr, g->col, g->w32,
                           g->w64, g->eid, g->s_col, g->s_w32, g->s_w64, g->s_eid);
        PFE_CHECK_HIP(hipGetLastError());
        PFE_CHECK_HIP(hipStreamSynchronize(st));
    } else {
        g->ell_K = 0;
        g->nslot = g->slots;
        g->s_col = g->col;
        g->s_w32 = g->w32;
        g->s_w64 = g->w64;
        g->s_eid = g->eid;
    }
    return PFE_OK;
}

}  // namespace pfe

using namespace pfe;

extern "C" {

const char* pfe_last_error(void) { return g_err; }

const char* pfe_status_string(pfe_status s) {
    switch (s) {
        case PFE_OK: return "ok";
        case PFE_E_ARG: return "invalid argument";
        case PFE_E_GRAPH: return "invalid graph";
        case PFE_E_HIP: return "HIP runtime error";
        case PFE_E_NOMEM: return "out of device memory";
        case PFE_E_NOT_SPD: return "conjugate gradient breakdown (matrix not SPD)";
        case PFE_E_RANK: return "rank-deficient embedding (Gram matrix not positive definite)";
        case PFE_E_NOCONV: return "conjugate gradient did not converge within maxit";
        case PFE_E_STATE: return "request not valid in the current state";
    }
    return "unknown status";
}

pfe_status pfe_build_graph(const pfe_graph_desc* d, hipStream_t stream, pfe_graph** out) {
    g_err[0] = 0;
    if (!d || !out) { set_error("pfe_build_graph: null argument"); return PFE_E_ARG; }
    *out = nullptr;
    if (!(d->sigma > 0.0) || !std::isfinite(d->sigma)) { set_error("pfe_build_graph: sigma must be > 0"); return PFE_E_ARG; }
    int64_t n = 0;
    if (d->kind == PFE_GRID) {
        if (d->H < 1 || d->W < 1 || d->m < 1 || d->m > 4096 || !d->feat) {
            set_error("pfe_build_graph: bad grid description (H, W, m, feat)");
            return PFE_E_ARG;
        }
        if (!(d->stencil == 4 || d->stencil == 8 || (d->stencil < 0 && d->stencil >= -4))) {
            set_error("pfe_build_graph: stencil must be 4, 8 or -R with 1 <= R <= 4");
            return PFE_E_ARG;
        }
        n = (int64_t)d->H * d->W;
    } else if (d->kind == PFE_EDGES) {
        if (d->n < 2 || d->n_edges < 0 || (d->n_edges > 0 && (!d->src || !d->dst || !d->dist2))) {
            set_error("pfe_build_graph: bad edge-list description");
            return PFE_E_ARG;
        }
        if (2 * d->n_edges >= (int64_t)INT32_MAX) { set_error("pfe_build_graph: too many edges"); return PFE_E_ARG; }
        n = d->n;
    } else {
        set_error("pfe_build_graph: unknown kind %d", d->kind);
        return PFE_E_ARG;
    }
    if (n >= (int64_t)INT32_MAX / 2) { set_error("pfe_build_graph: too many vertices"); return PFE_E_ARG; }
    pfe_graph* g = new pfe_graph();
    PFE_CHECK_HIP(hipGetDevice(&g->device));
    g->stream = stream;
    g->n = n;
    pfe_status s = build_impl(d, stream, g);
    if (s != PFE_OK) {
        (void)hipStreamSynchronize(stream);
        free_graph_buffers(g);
        delete g;
        return s;
    }
    g->seg_row0 = {0, g->n};
    g->seg_edge0 = {0, g->n_edges};
    g->seg_H = {d->kind == PFE_GRID ? d->H : 0};
    g->seg_W = {d->kind == PFE_GRID ? d->W : 0};
    *out = g;
    return PFE_OK;
}

pfe_status pfe_graph_union(const pfe_graph* const* parts, int count, hipStream_t stream, pfe_graph** out) {
    g_err[0] = 0;
    if (!parts || !out || count < 1) { set_error("pfe_graph_union: null argument or count < 1"); return PFE_E_ARG; }
    *out = nullptr;
    int dev = 0;
    PFE_CHECK_HIP(hipGetDevice(&dev));
    int64_t N = 0, SL = 0, E = 0, NS = 0;
    int K = -1, max_deg = 0;
    bool ell = true, sten = true;
    for (int p = 0; p < count; ++p) {
        const pfe_graph* q = parts[p];
        if (!q) { set_error("pfe_graph_union: part %d is null", p); return PFE_E_ARG; }
        if (q->device != dev) { set_error("pfe_graph_union: part %d lives on another device", p); return PFE_E_ARG; }
        N += q->n;
        SL += q->slots;
        E += q->n_edges;
        max_deg = std::max(max_deg, q->max_deg);
        if (K < 0) K = q->ell_K;
        ell = ell && q->ell_K > 0 && q->ell_K == K;
        sten = sten && q->stencil;
    }
    if (N >= (int64_t)INT32_MAX / 2 || SL >= (int64_t)INT32_MAX) { set_error("pfe_graph_union: union too large"); return PFE_E_ARG; }
    if (ell) {
        NS = (int64_t)K * N;
        if (NS >= (int64_t)INT32_MAX) ell = false;
    }
    pfe_graph* g = new pfe_graph();
    g->device = dev;
    g->stream = stream;
    g->n = N;
    g->slots = SL;
    g->n_edges = E;
    g->max_deg = max_deg;
    auto fail = [&](pfe_status s) {
        (void)hipStreamSynchronize(stream);
        free_graph_buffers(g);
        delete g;
        return s;
    };
    hipError_t e = hipSuccess;
#define UALLOC(ptr, bytes) do { if (e == hipSuccess) e = dev_alloc((void**)&(ptr), (bytes)); } while (0)
    UALLOC(g->rowptr, sizeof(int) * (N + 1));
    UALLOC(g->col, sizeof(int) * (SL + 1));
    UALLOC(g->rev, sizeof(int) * (SL + 1));
    UALLOC(g->eid, sizeof(int) * (SL + 1));
    UALLOC(g->w32, sizeof(float) * (SL + 1));
    UALLOC(g->w64, sizeof(double) * (SL + 1));
    UALLOC(g->degree, sizeof(double) * N);
    UALLOC(g->wsq, sizeof(double) * N);
    if (ell) {
        UALLOC(g->s_col, sizeof(int) * NS);
        UALLOC(g->s_w32, sizeof(float) * NS);
        UALLOC(g->s_w64, sizeof(double) * NS);
        UALLOC(g->s_eid, sizeof(int) * NS);
    }
#undef UALLOC
    if (e != hipSuccess) {
        if (!ell) g->ell_K = 0;   // nothing ELL-specific allocated
        else g->ell_K = K;
        return fail(hip_fail(e, "device allocation (graph union)", __FILE__, __LINE__));
    }
    g->ell_K = ell ? K : 0;
    const int TB = 256;
    int64_t V = 0, S = 0, Eo = 0;
    g->seg_row0.assign(1, 0);
    g->seg_edge0.assign(1, 0);
    g->seg_H.clear();
    g->seg_W.clear();
    for (int p = 0; p < count; ++p) {
        const pfe_graph* q = parts[p];
        const int64_t n = q->n, sl = q->slots;
        const unsigned gn = (unsigned)((n + TB - 1) / TB), gs = (unsigned)((sl + TB - 1) / TB);
        hipLaunchKernelGGL(k_add_int, dim3(gn), dim3(TB), 0, stream, n, q->rowptr, (int)S, 0, g->rowptr + V);
        if (sl > 0) {
            hipLaunchKernelGGL(k_add_int, dim3(gs), dim3(TB), 0, stream, sl, q->col, (int)V, 0, g->col + S);
            hipLaunchKernelGGL(k_add_int, dim3(gs), dim3(TB), 0, stream, sl, q->rev, (int)S, 0, g->rev + S);
            hipLaunchKernelGGL(k_add_int, dim3(gs), dim3(TB), 0, stream, sl, q->eid, (int)Eo, 0, g->eid + S);
            if (hipMemcpyAsync(g->w32 + S, q->w32, sizeof(float) * sl, hipMemcpyDeviceToDevice, stream) != hipSuccess ||
                hipMemcpyAsync(g->w64 + S, q->w64, sizeof(double) * sl, hipMemcpyDeviceToDevice, stream) != hipSuccess)
                return fail(hip_fail(hipGetLastError(), "hipMemcpyAsync (graph union)", __FILE__, __LINE__));
        }
        if (hipMemcpyAsync(g->degree + V, q->degree, sizeof(double) * n, hipMemcpyDeviceToDevice, stream) != hipSuccess ||
            hipMemcpyAsync(g->wsq + V, q->wsq, sizeof(double) * n, hipMemcpyDeviceToDevice, stream) != hipSuccess)
            return fail(hip_fail(hipGetLastError(), "hipMemcpyAsync (graph union)", __FILE__, __LINE__));
        if (ell) {
            for (int k = 0; k < K; ++k) {
                const int64_t so = (int64_t)k * n, dO = (int64_t)k * N + V;
                hipLaunchKernelGGL(k_add_int, dim3(gn), dim3(TB), 0, stream, n, q->s_col + so, (int)V, 0, g->s_col + dO);
                hipLaunchKernelGGL(k_add_int, dim3(gn), dim3(TB), 0, stream, n, q->s_eid + so, (int)Eo, 1, g->s_eid + dO);
                if (hipMemcpyAsync(g->s_w32 + dO, q->s_w32 + so, sizeof(float) * n, hipMemcpyDeviceToDevice, stream) != hipSuccess ||
                    hipMemcpyAsync(g->s_w64 + dO, q->s_w64 + so, sizeof(double) * n, hipMemcpyDeviceToDevice, stream) != hipSuccess)
                    return fail(hip_fail(hipGetLastError(), "hipMemcpyAsync (graph union)", __FILE__, __LINE__));
            }
        }
        hipError_t le = hipGetLastError();
        if (le != hipSuccess) return fail(hip_fail(le, "graph union kernels", __FILE__, __LINE__));
        V += n;
        S += sl;
        Eo += q->n_edges;
        for (size_t k = 1; k < q->seg_row0.size(); ++k) {
            g->seg_row0.push_back(g->seg_row0.back() + (q->seg_row0[k] - q->seg_row0[k - 1]));
            g->seg_edge0.push_back(g->seg_edge0.back() + (q->seg_edge0[k] - q->seg_edge0[k - 1]));
            g->seg_H.push_back(q->seg_H[k - 1]);
            g->seg_W.push_back(q->seg_W[k - 1]);
        }
    }
    const int last = (int)SL;
    if (hipMemcpyAsync(g->rowptr + N, &last, sizeof(int), hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return fail(hip_fail(hipGetLastError(), "graph union", __FILE__, __LINE__));
    if (ell) {
        g->nslot = NS;
        g->stencil = sten ? 1 : 0;
    } else {
        g->nslot = SL;
        g->s_col = g->col;
        g->s_w32 = g->w32;
        g->s_w64 = g->w64;
        g->s_eid = g->eid;
    }
    *out = g;
    return PFE_OK;
}

pfe_status pfe_graph_segments(const pfe_graph* g, int* count, int64_t* row0, int64_t* edge0) {
    if (!g || !count) { set_error("pfe_graph_segments: null argument"); return PFE_E_ARG; }
    *count = (int)g->seg_row0.size() - 1;
    for (size_t k = 0; k < g->seg_row0.size(); ++k) {
        if (row0) row0[k] = g->seg_row0[k];
        if (edge0) edge0[k] = g->seg_edge0[k];
    }
    return PFE_OK;
}

pfe_status pfe_graph_info(const pfe_graph* g, int64_t* n, int64_t* n_edges, int64_t* nnz_A) {
    if (!g) { set_error("pfe_graph_info: null graph"); return PFE_E_ARG; }
    if (n) *n = g->n;
    if (n_edges) *n_edges = g->n_edges;
    if (nnz_A) *nnz_A = g->n + g->slots;
    return PFE_OK;
}

pfe_status pfe_graph_csr(const pfe_graph* g, int32_t* rowptr, int32_t* col, float* w, double* degree) {
    if (!g) { set_error("pfe_graph_csr: null graph"); return PFE_E_ARG; }
    hipStream_t st = g->stream;
    if (rowptr) PFE_CHECK_HIP(hipMemcpyAsync(rowptr, g->rowptr, sizeof(int) * (g->n + 1), hipMemcpyDeviceToDevice, st));
    if (col) PFE_CHECK_HIP(hipMemcpyAsync(col, g->col, sizeof(int) * g->slots, hipMemcpyDeviceToDevice, st));
    if (w) PFE_CHECK_HIP(hipMemcpyAsync(w, g->w32, sizeof(float) * g->slots, hipMemcpyDeviceToDevice, st));
    if (degree) PFE_CHECK_HIP(hipMemcpyAsync(degree, g->degree, sizeof(double) * g->n, hipMemcpyDeviceToDevice, st));
    PFE_CHECK_HIP(hipStreamSynchronize(st));
    return PFE_OK;
}

pfe_status pfe_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t stream) {
    if (!src || !dst || (bytes % 16) != 0 || ((uintptr_t)src % 16) != 0 || ((uintptr_t)dst % 16) != 0) {
        set_error("pfe_stream_copy: pointers and size must be 16-byte aligned");
        return PFE_E_ARG;
    }
    const size_t n16 = bytes / 16;
    if (n16 == 0) return PFE_OK;
    // at most 16 workgroups per CU, fewer when the buffer is small
    const size_t per_block = (size_t)kCopyThreads * kCopyUnroll;
    const unsigned blocks = (unsigned)std::min<size_t>((n16 + per_block - 1) / per_block, 256 * 16);
    hipLaunchKernelGGL(k_stream_copy, dim3(blocks), dim3(kCopyThreads), 0, stream, (const u32x4*)src, (u32x4*)dst,
                       n16);
    PFE_CHECK_HIP(hipGetLastError());
    return PFE_OK;
}

void pfe_destroy_graph(pfe_graph* g) {
    if (!g) return;
    (void)hipStreamSynchronize(g->stream);
    free_graph_buffers(g);
    delete g;
}

}  // extern "C"
