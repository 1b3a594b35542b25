// Internal declarations shared by the libpfe translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "pfe.h"

namespace pfe {

void set_error(const char* fmt, ...);
pfe_status hip_fail(hipError_t e, const char* what, const char* file, int line);

// device memory of the library (the caller's allocator when one is installed)
hipError_t dev_alloc(void** p, size_t bytes);
hipError_t dev_free(void* p);
hipError_t dev_alloc_async(void** p, size_t bytes, hipStream_t st);
hipError_t dev_free_async(void* p, hipStream_t st);
template <typename T>
inline hipError_t dev_alloc(T** p, size_t bytes) { return dev_alloc(reinterpret_cast<void**>(p), bytes); }
template <typename T>
inline hipError_t dev_alloc_async(T** p, size_t bytes, hipStream_t st) {
    return dev_alloc_async(reinterpret_cast<void**>(p), bytes, st);
}

constexpr int kMaxD = 32;          // largest embedding dimension
constexpr int kNumXcd = 8;         // accelerator complex dies on MI355X
constexpr int kBlock = 512;        // threads per workgroup of the row-parallel phases
constexpr int kSmemDoubles = 4608; // LDS scratch per workgroup (36 KiB)

// Small solver state kept in device memory: per-column CG scalars, the d x d
// transform of the P-update, flags and statistics.
struct alignas(64) Scal {
    double rho[kMaxD];      // r^T z of the current iteration
    double alpha[kMaxD];
    double beta[kMaxD];
    double bnorm2[kMaxD];   // ||rhs_c||^2
    double rr[kMaxD];       // ||r_c||^2
    double T[kMaxD * kMaxD];  // d x d transform, row-major
    double mon[16];         // monitor results
    int iters[kMaxD];       // iterations of each column in the current solve
    int active[kMaxD];      // column still iterating
    int zero[kMaxD];        // column with a zero right-hand side
    int it;                 // iteration index of the current solve
    int done;               // current solve finished
    int status;             // worst status since the last reset (0 or PFE_E_*)
    int abort_flag;         // a grid barrier timed out
    int ortho_ok;           // the last Gram factorisation succeeded
    int saved_status;       // status set aside while a factor-preconditioned solve runs
    // statistics since the last reset
    long long solves;
    long long iters_total;
    int iters_max;
    int iters_last;
    double relres_max;
    int fallbacks;          // factor-preconditioned solves redone with Jacobi
    int pad2_;
};

}  // namespace pfe

struct pfe_mpnn;

namespace pfe {
// graph and system seen by the learned-preconditioner network
struct NetGraph {
    int64_t n = 0, nslot = 0;
    int ell_K = 0, deg_max = 0;
    const int* rowptr = nullptr;
    const int* scol = nullptr;
    const int* seid = nullptr;
    const double* sw64 = nullptr;
    const double* degree = nullptr;
    const double* wsq = nullptr;
    double lambda = 0.0, r = 0.0;
};
// Gt on every slot and its diagonal, in the context's element type
pfe_status mpnn_factor(pfe_mpnn* w, const NetGraph& g, void* gval, void* gdiag, int esz, hipStream_t st);
// one training step (lr == 0: gradient only) on k residual samples
pfe_status mpnn_train_step(pfe_mpnn* w, const NetGraph& g, const void* samples, int esz, int kc, float lr,
                           double* loss, hipStream_t st);
}  // namespace pfe

#define PFE_TRY_STATUS(x) do { pfe_status s__ = (x); if (s__ != PFE_OK) return s__; } while (0)

#define PFE_CHECK_HIP(expr)                                                   \
    do {                                                                      \
        hipError_t e__ = (expr);                                              \
        if (e__ != hipSuccess) return pfe::hip_fail(e__, #expr, __FILE__, __LINE__); \
    } while (0)

struct pfe_graph {
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t n = 0;
    int64_t n_edges = 0;
    int64_t slots = 0;        // 2 |E| directed adjacency entries
    // CSR adjacency (columns ascending within a row)
    int* rowptr = nullptr;    // n + 1
    int* col = nullptr;       // slots
    int* rev = nullptr;       // slot of the reverse direction
    int* eid = nullptr;       // undirected edge index (lexicographic (i, j), i < j)
    float* w32 = nullptr;     // heat-kernel weight per slot, FP32
    double* w64 = nullptr;    // same in FP64
    double* degree = nullptr; // d_i = sum_j w_ij (FP64)
    double* wsq = nullptr;    // sum_j w_ij^2 (FP64): diagonal of M^T M
    int max_deg = 0;
    // Slot layout used by the solver.  ELL (stencil-like graphs): K slots per
    // row, slot k of row i at index k * n + i, unused slots point at the row
    // itself with weight 0; otherwise the CSR order above (K = 0).
    int ell_K = 0;
    int64_t nslot = 0;        // slots in the solver layout (K n for ELL, 2|E| for CSR)
    int* s_col = nullptr;
    float* s_w32 = nullptr;
    double* s_w64 = nullptr;
    int* s_eid = nullptr;     // undirected edge of the slot, -1 for padding
    // Pixel grids: ELL slot k of every row is stencil offset k; slots that
    // leave the image have weight 0 and point at the row itself.
    int stencil = 0;
    // Block-diagonal batches: segment s owns the vertices [seg_row0[s],
    // seg_row0[s+1]) and the undirected edges [seg_edge0[s], seg_edge0[s+1]);
    // a graph built from one description is a single segment.
    std::vector<int64_t> seg_row0;
    std::vector<int64_t> seg_edge0;
    // image height and width of each segment (0 for edge-list graphs); a
    // segment's pixel (y, x) is vertex seg_row0 + y W + x
    std::vector<int> seg_H;
    std::vector<int> seg_W;
};
