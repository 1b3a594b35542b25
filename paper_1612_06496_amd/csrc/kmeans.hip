// k-means (Lloyd iterations) on the rows of an embedding: the clustering the
// segmentation experiment applies to the embedding (Sec. IV).
//
// Assignment: one thread per row; the K x d centroids sit in LDS (FP64), the
// row's d coordinates in registers (widened exactly from the storage type).
// The squared distance is summed over the coordinates in order with every
// product and sum rounded on its own (contraction off), so the nearest
// centroid (ties to the lowest index) is decided in FP64 by a fixed sequence
// of operations.  Update: one workgroup per (centroid, row slice) sums that
// centroid's rows in the slice (strided over the threads, then a fixed tree
// over the workgroup), and one thread per centroid coordinate adds the slices
// in order (deterministic); a centroid without rows keeps its position.
// Iterations run in groups launched back to back; a device flag makes the
// kernels of the iterations after convergence return at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "common.hpp"

namespace pfe {

constexpr int kKmMaxK = 256;
constexpr int kKmMaxKD = 8000;   // K * d doubles in LDS (62.5 KiB)
constexpr int kKmThreads = 256;

template <typename T, int DMAX>
__global__ void __launch_bounds__(kKmThreads) k_km_assign(const T* __restrict__ Y, int64_t n, int d,
                                                          const double* __restrict__ C, int K,
                                                          int32_t* __restrict__ labels, unsigned* __restrict__ st) {
#pragma clang fp contract(off)
    if (st[1]) return;   // converged in an earlier iteration of the chunk
    unsigned* changed = st;
    extern __shared__ double sc[];
    __shared__ unsigned s_changed;
    if (threadIdx.x == 0) s_changed = 0;
    for (int e = threadIdx.x; e < K * d; e += blockDim.x) sc[e] = C[e];
    __syncthreads();
    unsigned mine = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double y[DMAX];
#pragma unroll
        for (int c = 0; c < DMAX; ++c) y[c] = (c < d) ? (double)Y[i * d + c] : 0.0;
        double best = 0.0;
        int bk = -1;
        for (int k = 0; k < K; ++k) {
            const double* m = sc + k * d;
            double dist = 0.0;
#pragma unroll
            for (int c = 0; c < DMAX; ++c) {
                if (c < d) {
                    const double diff = y[c] - m[c];
                    const double sq = diff * diff;
                    dist = dist + sq;
                }
            }
            if (bk < 0 || dist < best) { best = dist; bk = k; }
        }
        if (labels[i] != bk) { labels[i] = bk; ++mine; }
    }
    if (mine) atomicAdd(&s_changed, mine);
    __syncthreads();
    if (threadIdx.x == 0 && s_changed) atomicAdd(changed, s_changed);
}

// sums of the rows of centroid k (blockIdx.x) in row slice s (blockIdx.y):
// part[(k S + s) (d + 1) + c] for the d coordinates, then the row count
template <typename T, int DMAX>
__global__ void __launch_bounds__(kKmThreads) k_km_partial(const T* __restrict__ Y, int64_t n, int d,
                                                           const int32_t* __restrict__ labels,
                                                           double* __restrict__ part, const unsigned* __restrict__ st) {
    if (st[1]) return;
    __shared__ double red[kKmThreads];
    const int k = blockIdx.x, sl = blockIdx.y, S = gridDim.y, t = threadIdx.x;
    const int64_t per = (n + S - 1) / S;
    const int64_t r0 = (int64_t)sl * per, r1 = (r0 + per < n) ? r0 + per : n;
    double acc[DMAX];
#pragma unroll
    for (int c = 0; c < DMAX; ++c) acc[c] = 0.0;
    double cnt = 0.0;
    for (int64_t i = r0 + t; i < r1; i += kKmThreads) {
        if (labels[i] != k) continue;
        cnt += 1.0;
#pragma unroll
        for (int c = 0; c < DMAX; ++c)
            if (c < d) acc[c] += (double)Y[i * d + c];
    }
    double* out = part + ((size_t)k * S + sl) * (d + 1);
    // fixed-order tree over the workgroup, one coordinate at a time (the count last)
#pragma unroll
    for (int c = 0; c <= DMAX; ++c) {
        if (c < d || c == DMAX) {
            red[t] = (c == DMAX) ? cnt : acc[c];
            __syncthreads();
            for (int h = kKmThreads / 2; h > 0; h >>= 1) {
                if (t < h) red[t] += red[t + h];
                __syncthreads();
            }
            if (t == 0) out[c == DMAX ? d : c] = red[0];
            __syncthreads();
        }
    }
}

// centroid k moves to the mean of its rows (slices summed in order); a
// centroid without rows stays
__global__ void k_km_move(const double* __restrict__ part, int K, int d, int S, double* __restrict__ C,
                          const unsigned* __restrict__ st) {
    if (st[1]) return;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= K * d) return;
    const int k = idx / d, c = idx - k * d;
    double sum = 0.0, cnt = 0.0;
    for (int sl = 0; sl < S; ++sl) {
        const double* p = part + ((size_t)k * S + sl) * (d + 1);
        sum += p[c];
        cnt += p[d];
    }
    if (cnt > 0.0) C[idx] = sum / cnt;
}

// start of a call: change count, converged flag and iteration count to zero
__global__ void k_km_clear(unsigned* st) {
    if (threadIdx.x < 3) st[threadIdx.x] = 0;
}

// before an iteration: clear the change count (unless converged)
__global__ void k_km_begin(unsigned* st) {
    if (threadIdx.x == 0 && !st[1]) st[0] = 0;
}

// after an iteration: count it, and stop when no label changed
__global__ void k_km_end(unsigned* st) {
    if (threadIdx.x == 0 && !st[1]) {
        st[2] += 1;
        if (st[0] == 0) st[1] = 1;
    }
}

__global__ void k_km_fill(int64_t n, int32_t v, int32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = v;
}

// iterations in chunks of kKmChunk launched back to back; the device state
// stops the kernels of an iteration after convergence, and the host reads it
// once per chunk
constexpr int kKmChunk = 8;

template <typename T, int DMAX>
pfe_status km_run(const T* Y, int64_t n, int d, int K, int max_iter, int32_t* labels, double* C, unsigned* st,
                  double* part, int S, int* iters, hipStream_t stream) {
    const int64_t want = (n + kKmThreads - 1) / kKmThreads;
    const unsigned grid = (unsigned)std::min<int64_t>(want, 4096);
    const size_t lds = sizeof(double) * (size_t)K * d;
    unsigned h[3] = {0, 0, 0};
    for (int done_it = 0; done_it < max_iter;) {
        const int chunk = std::min(kKmChunk, max_iter - done_it);
        for (int k = 0; k < chunk; ++k) {
            hipLaunchKernelGGL(k_km_begin, dim3(1), dim3(64), 0, stream, st);
            hipLaunchKernelGGL((k_km_assign<T, DMAX>), dim3(grid), dim3(kKmThreads), lds, stream, Y, n, d, C, K,
                               labels, st);
            hipLaunchKernelGGL((k_km_partial<T, DMAX>), dim3(K, S), dim3(kKmThreads), 0, stream, Y, n, d, labels,
                               part, st);
            hipLaunchKernelGGL(k_km_move, dim3((K * d + 255) / 256), dim3(256), 0, stream, part, K, d, S, C, st);
            hipLaunchKernelGGL(k_km_end, dim3(1), dim3(64), 0, stream, st);
        }
        PFE_CHECK_HIP(hipGetLastError());
        done_it += chunk;
        PFE_CHECK_HIP(hipMemcpyAsync(h, st, sizeof(h), hipMemcpyDeviceToHost, stream));
        PFE_CHECK_HIP(hipStreamSynchronize(stream));
        if (h[1]) break;
    }
    if (iters) *iters = (int)h[2];
    return PFE_OK;
}

template <typename T>
pfe_status km_dispatch(const T* Y, int64_t n, int d, int K, int max_iter, int32_t* labels, double* C,
                       unsigned* changed, double* part, int S, int* iters, hipStream_t st) {
    if (d <= 8) return km_run<T, 8>(Y, n, d, K, max_iter, labels, C, changed, part, S, iters, st);
    if (d <= 16) return km_run<T, 16>(Y, n, d, K, max_iter, labels, C, changed, part, S, iters, st);
    return km_run<T, 32>(Y, n, d, K, max_iter, labels, C, changed, part, S, iters, st);
}

bool km_args_ok(const void* Y, int64_t n, int d, int dtype, const double* C0, int K, int max_iter,
                const int32_t* labels, const double* centroids, const char* who) {
    if (!Y || !C0 || !labels || !centroids || n < 1 || n >= (int64_t)INT32_MAX || d < 1 || d > kMaxD || K < 1 ||
        K > kKmMaxK || K * d > kKmMaxKD || max_iter < 1 || (dtype != PFE_FP32 && dtype != PFE_FP64)) {
        set_error("%s: bad argument (1 <= d <= %d, 1 <= K <= %d, K d <= %d, max_iter >= 1)", who, kMaxD, kKmMaxK,
                  kKmMaxKD);
        return false;
    }
    return true;
}

// row slices of the centroid sums: about 4096 rows each, at most kKmMaxSlices
constexpr int kKmMaxSlices = 64;
inline int km_slices(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(kKmMaxSlices, n / 4096)); }

// Lloyd iterations with the caller's scratch: st (3 unsigned: change count,
// converged flag, iterations run) and part (K x S x (d + 1) doubles)
pfe_status km_call(const void* Y, int64_t n, int d, int dtype, const double* C0, int K, int max_iter, int32_t* labels,
                   double* centroids, int32_t* iters, unsigned* st, double* part, int S, hipStream_t stream) {
    if (centroids != C0)
        PFE_CHECK_HIP(hipMemcpyAsync(centroids, C0, sizeof(double) * (size_t)K * d, hipMemcpyDeviceToDevice, stream));
    hipLaunchKernelGGL(k_km_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, n, -1, labels);
    hipLaunchKernelGGL(k_km_clear, dim3(1), dim3(64), 0, stream, st);
    PFE_CHECK_HIP(hipGetLastError());
    int it = 0;
    pfe_status s = (dtype == PFE_FP64)
                       ? km_dispatch<double>((const double*)Y, n, d, K, max_iter, labels, centroids, st, part, S, &it,
                                             stream)
                       : km_dispatch<float>((const float*)Y, n, d, K, max_iter, labels, centroids, st, part, S, &it,
                                            stream);
    if (s == PFE_OK && iters) *iters = it;
    return s;
}

// Scratch of the allocation-free entry point: the three counters (padded to
// 256 bytes), then the slice sums of the largest call the argument checks
// allow (K d <= kKmMaxKD and K <= kKmMaxK, so K (d + 1) <= kKmMaxKD + kKmMaxK).
constexpr size_t kKmCounterBytes = 256;
constexpr size_t kKmScratchBytes =
    kKmCounterBytes + sizeof(double) * (size_t)(kKmMaxKD + kKmMaxK) * kKmMaxSlices;   // 4,227,328 bytes
static __device__ __align__(256) unsigned char scratch[kKmScratchBytes];

// device address of this GPU's copy of scratch, looked up once per device
// (with that device current) and kept; the array's host-side name is never
// passed to a kernel or a copy
constexpr int kKmMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kKmMaxDevices] = {};

pfe_status scratch_address(void** out) {
    int dev = 0;
    PFE_CHECK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kKmMaxDevices) {
        set_error("pfe_kmeans_noalloc: device index %d above %d", dev, kKmMaxDevices - 1);
        return PFE_E_ARG;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        PFE_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) { set_error("pfe_kmeans_noalloc: no device address for the scratch array"); return PFE_E_HIP; }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PFE_OK;
}

}  // namespace pfe

using namespace pfe;

extern "C" pfe_status pfe_kmeans(const void* Y, int64_t n, int d, int dtype, const double* C0, int K, int max_iter,
                                 int32_t* labels, double* centroids, int32_t* iters, hipStream_t stream) {
    if (!km_args_ok(Y, n, d, dtype, C0, K, max_iter, labels, centroids, "pfe_kmeans")) return PFE_E_ARG;
    const int S = km_slices(n);
    unsigned* changed = nullptr;   // device state: change count, converged flag, iterations run
    double* part = nullptr;        // K x S x (d + 1) slice sums
    PFE_CHECK_HIP(dev_alloc((void**)&changed, 3 * sizeof(unsigned)));
    hipError_t e = dev_alloc((void**)&part, sizeof(double) * (size_t)K * S * (d + 1));
    if (e != hipSuccess) {
        (void)dev_free(changed);
        return hip_fail(e, "device allocation (k-means)", __FILE__, __LINE__);
    }
    pfe_status s = km_call(Y, n, d, dtype, C0, K, max_iter, labels, centroids, iters, changed, part, S, stream);
    (void)hipStreamSynchronize(stream);
    (void)dev_free(part);
    (void)dev_free(changed);
    return s;
}

extern "C" pfe_status pfe_kmeans_noalloc(const void* Y, int64_t n, int d, int dtype, const double* C0, int K,
                                         int max_iter, int32_t* labels, double* centroids, int32_t* iters,
                                         hipStream_t stream) {
    if (!km_args_ok(Y, n, d, dtype, C0, K, max_iter, labels, centroids, "pfe_kmeans_noalloc")) return PFE_E_ARG;
    const int S = km_slices(n);
    const size_t need = kKmCounterBytes + sizeof(double) * (size_t)K * S * (d + 1);
    if (need > kKmScratchBytes) {
        set_error("pfe_kmeans_noalloc: needs %zu bytes of scratch, the static array holds %zu", need,
                  kKmScratchBytes);
        return PFE_E_ARG;
    }
    void* base = nullptr;
    PFE_TRY_STATUS(scratch_address(&base));
    unsigned* st = static_cast<unsigned*>(base);
    double* part = reinterpret_cast<double*>(static_cast<unsigned char*>(base) + kKmCounterBytes);
    pfe_status s = km_call(Y, n, d, dtype, C0, K, max_iter, labels, centroids, iters, st, part, S, stream);
    (void)hipStreamSynchronize(stream);
    return s;
}
