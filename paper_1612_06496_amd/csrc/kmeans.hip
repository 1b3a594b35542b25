// k-means (Lloyd iterations) on the rows of an embedding: the clustering the
// segmentation experiment applies to the embedding (Sec. IV).
//
// Assignment: one thread per row; the K x d centroids sit in LDS (FP64), the
// row's d coordinates in registers (widened exactly from the storage type).
// The squared distance is summed over the coordinates in order with every
// product and sum rounded on its own (contraction off), so the nearest
// centroid (ties to the lowest index) is decided in FP64 by a fixed sequence
// of operations.  Update: one workgroup per centroid; each thread sums the
// rows of that centroid among its strided share of the rows, then a fixed
// tree over the workgroup combines them (deterministic); a centroid without
// rows keeps its position.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "common.hpp"

namespace pfe {

constexpr int kKmMaxK = 256;
constexpr int kKmMaxKD = 8000;   // K * d doubles in LDS (62.5 KiB)
constexpr int kKmThreads = 256;

template <typename T, int DMAX>
__global__ void __launch_bounds__(kKmThreads) k_km_assign(const T* __restrict__ Y, int64_t n, int d,
                                                          const double* __restrict__ C, int K,
                                                          int32_t* __restrict__ labels, unsigned* __restrict__ changed) {
#pragma clang fp contract(off)
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

template <typename T, int DMAX>
__global__ void __launch_bounds__(kKmThreads) k_km_update(const T* __restrict__ Y, int64_t n, int d,
                                                          const int32_t* __restrict__ labels, double* __restrict__ C) {
    __shared__ double red[kKmThreads];
    __shared__ double sums[DMAX + 1];
    const int k = blockIdx.x, t = threadIdx.x;
    double acc[DMAX];
#pragma unroll
    for (int c = 0; c < DMAX; ++c) acc[c] = 0.0;
    double cnt = 0.0;
    for (int64_t i = t; i < n; i += kKmThreads) {
        if (labels[i] != k) continue;
        cnt += 1.0;
#pragma unroll
        for (int c = 0; c < DMAX; ++c)
            if (c < d) acc[c] += (double)Y[i * d + c];
    }
    // fixed-order tree over the workgroup, one coordinate at a time (the count last)
#pragma unroll
    for (int c = 0; c <= DMAX; ++c) {
        if (c < d || c == DMAX) {
            red[t] = (c == DMAX) ? cnt : acc[c];
            __syncthreads();
            for (int s = kKmThreads / 2; s > 0; s >>= 1) {
                if (t < s) red[t] += red[t + s];
                __syncthreads();
            }
            if (t == 0) sums[c] = red[0];
            __syncthreads();
        }
    }
    const double total = sums[DMAX];
    if (total > 0.0 && t < d) C[(size_t)k * d + t] = sums[t] / total;
}

__global__ void k_km_fill(int64_t n, int32_t v, int32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = v;
}

template <typename T, int DMAX>
pfe_status km_run(const T* Y, int64_t n, int d, int K, int max_iter, int32_t* labels, double* C, unsigned* changed,
                  int* iters, hipStream_t st) {
    const int64_t want = (n + kKmThreads - 1) / kKmThreads;
    const unsigned grid = (unsigned)std::min<int64_t>(want, 4096);
    const size_t lds = sizeof(double) * (size_t)K * d;
    int it = 0;
    for (it = 1; it <= max_iter; ++it) {
        PFE_CHECK_HIP(hipMemsetAsync(changed, 0, sizeof(unsigned), st));
        hipLaunchKernelGGL((k_km_assign<T, DMAX>), dim3(grid), dim3(kKmThreads), lds, st, Y, n, d, C, K, labels,
                           changed);
        hipLaunchKernelGGL((k_km_update<T, DMAX>), dim3(K), dim3(kKmThreads), 0, st, Y, n, d, labels, C);
        PFE_CHECK_HIP(hipGetLastError());
        unsigned h = 0;
        PFE_CHECK_HIP(hipMemcpyAsync(&h, changed, sizeof(unsigned), hipMemcpyDeviceToHost, st));
        PFE_CHECK_HIP(hipStreamSynchronize(st));
        if (h == 0) break;
    }
    if (iters) *iters = std::min(it, max_iter);
    return PFE_OK;
}

template <typename T>
pfe_status km_dispatch(const T* Y, int64_t n, int d, int K, int max_iter, int32_t* labels, double* C,
                       unsigned* changed, int* iters, hipStream_t st) {
    if (d <= 8) return km_run<T, 8>(Y, n, d, K, max_iter, labels, C, changed, iters, st);
    if (d <= 16) return km_run<T, 16>(Y, n, d, K, max_iter, labels, C, changed, iters, st);
    return km_run<T, 32>(Y, n, d, K, max_iter, labels, C, changed, iters, st);
}

}  // namespace pfe

using namespace pfe;

extern "C" pfe_status pfe_kmeans(const void* Y, int64_t n, int d, int dtype, const double* C0, int K, int max_iter,
                                 int32_t* labels, double* centroids, int32_t* iters, hipStream_t stream) {
    if (!Y || !C0 || !labels || !centroids || n < 1 || n >= (int64_t)INT32_MAX || d < 1 || d > kMaxD || K < 1 ||
        K > kKmMaxK || K * d > kKmMaxKD || max_iter < 1 || (dtype != PFE_FP32 && dtype != PFE_FP64)) {
        set_error("pfe_kmeans: bad argument (1 <= d <= %d, 1 <= K <= %d, K d <= %d, max_iter >= 1)", kMaxD, kKmMaxK,
                  kKmMaxKD);
        return PFE_E_ARG;
    }
    if (centroids != C0)
        PFE_CHECK_HIP(hipMemcpyAsync(centroids, C0, sizeof(double) * (size_t)K * d, hipMemcpyDeviceToDevice, stream));
    hipLaunchKernelGGL(k_km_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, n, -1, labels);
    PFE_CHECK_HIP(hipGetLastError());
    unsigned* changed = nullptr;
    PFE_CHECK_HIP(dev_alloc((void**)&changed, sizeof(unsigned)));
    int it = 0;
    pfe_status s = (dtype == PFE_FP64)
                       ? km_dispatch<double>((const double*)Y, n, d, K, max_iter, labels, centroids, changed, &it, stream)
                       : km_dispatch<float>((const float*)Y, n, d, K, max_iter, labels, centroids, changed, &it, stream);
    (void)hipStreamSynchronize(stream);
    (void)dev_free(changed);
    if (s == PFE_OK && iters) *iters = it;
    return s;
}
