// The PFE hot path on gfx950: Split-Bregman inner iterations (Algorithm 2 in
// the compact form of Eqs. 9, 10, 13), their PCG least-squares solve
// (Sec. III), and the SOC P/B-update (Algorithm 1).
//
// Layout.  Every n x d block is row-major (d values per vertex).  The
// Split-Bregman variables live per directed slot (i -> j) with the orientation
// "i minus j", so each vertex owns the slots of its own row and every phase is
// atomic-free; the two copies of an undirected edge stay exact negatives of each
// other because the shrink and the clamp are odd and w (y_i - y_j) is exactly
// -(w (y_j - y_i)).  Slots follow the graph's solver layout (ELL: slot k of row
// i at k n + i, so lanes on consecutive rows read consecutive slots; or CSR).
//
// Work decomposition.  A phase runs on nblk workgroups, each walking its rows
// R = blockDim / d at a time, thread t on (row t / d, column t % d):
// consecutive lanes touch consecutive elements and gathers of neighbour rows of
// an image stay coalesced.  Workgroup indices are remapped so that each XCD owns
// a contiguous band of rows.  Inside a band, a team of up to 64 workgroups of
// the same segment deals the band's R-row chunks out cyclically, so the team
// sweeps the band together and the rows a chunk gathers from (an image row
// above and below) are still in that XCD's L2 when they are read again; with
// teams of one workgroup each owns a contiguous range.  Per-column reductions
// are FP64: one partial per workgroup and column, summed in a fixed order
// (results are bitwise reproducible).
//
// PCG.  The d systems of Eq. 13 are solved together with per-column scalars by
// the Chronopoulos-Gear form of Jacobi-preconditioned CG, which needs a single
// global reduction per iteration.  Each iteration is one phase: a row updates
// its own p, s, x, r and forms w = A u with u = diag(A)^{-1} r, recomputing the
// neighbours' new u from their previous r, w, s (bit-identical to what their
// owners store), so an iteration costs one grid-wide synchronisation.
#include <cfloat>
#include <cmath>
#include <cstring>
#include <cstdlib>
#include <algorithm>
#include <type_traits>
#include <vector>

#include "common.hpp"

namespace pfe {

enum Phase : int {
    PH_E0 = 0,      // first inner solve: rhs = r/2 D^{1/2}(P - B), r0 = rhs - A x
    PH_EU = 1,      // shrink + Bregman on the edges, next rhs, optionally r0
    PH_R0 = 2,      // r0 = rhs - A x from a stored rhs
    PH_W0 = 3,      // w0 = A u0, gamma0 = r0.u0, delta0 = w0.u0
    PH_IT = 4,      // one CG iteration (p, s, x, r, w) and its dot products
    PH_GRAM = 5,    // Z = D^{1/2} Y + B, Z^T Z
    PH_APPLY = 6,   // P = Z T, B = Z - P
    PH_RHS = 7,     // rhs from stored b, d (no r0)
    PH_ZERO = 8,    // zero the solution columns whose rhs is zero
    // PCG with the learned factor M^{-1} = D_A^{-1/2} Gt^T Gt D_A^{-1/2}
    PH_LA = 9,      // p = z + beta p, q = A p, p.q
    PH_LC = 11,     // x += alpha p, r -= alpha q, y1 = Gt D_A^{-1/2} r
    PH_LD = 12,     // z = D_A^{-1/2} Gt^T y1, r.z, r.r
    PH_LCD = 13,    // LC and LD fused (strips with a two-radius halo)
    // factor-preconditioned CG in Chronopoulos-Gear form, one pass per iteration
    // (strips with a three-radius halo)
    PH_FW0 = 14,    // u0 = M^{-1} r0, w0 = A u0, gamma0 = r0.u0, delta0 = w0.u0
    PH_FIT = 15,    // one iteration: p, s, x, r, u = M^{-1} r, w = A u and their dots
    PH_GA = 16      // pixel launches: the CG iteration's own-row pass (kernel selection only)
};

// per (segment, column) CG state, struct of arrays of length nseg * d
struct ColState {
    double* gamma;    // r.u of the current iteration
    double* alpha;
    double* beta;
    double* bnorm2;   // ||rhs||^2
    double* rr;       // ||r||^2
    int* iters;
    int* active;
    int* zero;
};

template <typename T>
struct KA {
    int n, d, R, nblk, nseg, ell_K;
    const int* row0;       // nblk + 1 row boundaries of the logical workgroups
    const int* bit;        // per logical workgroup: first row, end row, stride (rows
                           // first + k stride + [0, R) below end are its own)
    const int* blk_seg;    // segment of each logical workgroup
    const int* seg_blk0;   // nseg + 1 first logical workgroup of each segment
    const int* geo;        // strip partitions: per logical workgroup {row0, W, H, x0, len, y0, y1, 0}
                           // (image pixels (y, x), y in [y0, y1), x in [x0, x0 + len)); else null
    const int* rowptr;     // CSR row pointers (used when ell_K == 0)
    const int* scol;       // solver slot layout
    const T* sw;
    const T* diagA;
    const T* invdiag;
    const T* sqrtD;
    const T* isqrtD;
    const double* degree;
    T* x;              // PCG iterate (Y, or a caller buffer)
    T* Y;
    T* P;
    T* B;
    T* bsb[2];         // Split-Bregman b: edge update m reads bsb[m & 1] and writes bsb[(m + 1) & 1]
                       // (one buffer, updated in place, with per-slot storage)
    T* ds;             // Split-Bregman d (keep_split), stored like b
    T* rhs;
    T* rb[2];          // r, double-buffered across iterations
    T* wb[2];          // w = A u
    T* sb[2];          // s = A p
    T* p;
    const T* gval;     // learned factor: Gt entry of each slot's edge
    const T* gdiag;    // its diagonal
    const T* isq;      // D_A^{-1/2}
    T* zl;             // preconditioned residual (learned path)
    T* y1;             // Gt D_A^{-1/2} r
    double* part;      // workgroup partials
    double* gpart;     // per-XCD-group partials
    double* Tm;        // d x d transforms (stride kMaxD), one per segment
    ColState cs;
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
    int bpar;          // parity m & 1 of this launch's edge update (which b buffer it reads)
    int bhalf;         // b, d once per undirected edge (pixel stencils) instead of per slot
    int ortho;         // PFE_POLAR / PFE_CHOL
    int sten;          // ELL slots in pixel-stencil order (lower neighbours first)
    const int* dact;   // per segment: active columns (the leading ones; the others stay zero), or null (all d)
    int pxl;           // per-row ("pixel") launch of the Jacobi PCG phases (geo: per workgroup
                       // {row0, W, H} of its image on pixel-stencil layouts, else null)
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int logical_block(int nblk) {
    int b = blockIdx.x;
    if ((nblk % kNumXcd) == 0) return (b % kNumXcd) * (nblk / kNumXcd) + b / kNumXcd;
    return b;
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

// slots of row i: s = s0 + k * stride, k < cnt.  KC > 0 is the ELL width known
// at compile time (the slot loops of the hot phases then unroll completely).
template <int KC = 0, typename T>
__device__ __forceinline__ void row_slots(const KA<T>& a, int i, int& s0, int& cnt, int& stride) {
    if constexpr (KC > 0) { s0 = i; cnt = KC; stride = a.n; }
    else if (a.ell_K > 0) { s0 = i; cnt = a.ell_K; stride = a.n; }
    else { s0 = a.rowptr[i]; cnt = a.rowptr[i + 1] - s0; stride = 1; }
}

// Storage of the split variables b and d.  Per directed slot, "row minus
// column", for every layout; on pixel-stencil layouts (bhalf) once per
// undirected edge instead: on the lower-neighbour slot k < K/2 of the edge's
// later pixel i (orientation y_i - y_j).  The earlier pixel j reaches it
// through its mirrored upper slot K-1-k with the opposite sign: the shrink and
// the clamp are odd and w (y_j - y_i) is exactly -(w (y_i - y_j)), so both
// endpoints form exactly opposite values from the same stored b, and only the
// owner writes (into the other buffer of the pair, as the other endpoint reads
// the old value in the same pass).  Returns the storage slot of slot k of row
// i (neighbour j), and whether this row owns it.
template <int KC, typename T>
__device__ __forceinline__ size_t split_slot(const KA<T>& a, int i, int k, int j, size_t sl, bool& owner) {
    if constexpr (KC > 0) {
        if (a.bhalf) {
            owner = k < KC / 2;
            return owner ? sl : (size_t)(KC - 1 - k) * a.n + j;
        }
    }
    owner = true;
    return sl;
}

// Z = D^{1/2} Y + B of the P-update
template <typename T>
__device__ __forceinline__ T zrow(const KA<T>& a, int i, size_t e) {
    return fma_t(a.sqrtD[i], a.Y[e], a.B[e]);
}

// The CG recurrences, written once so that a row and its neighbours evaluate
// them identically:  s_i = w_i + beta s_{i-1},  r_{i+1} = r_i - alpha s_i,
// u_{i+1} = r_{i+1} / diag(A).
template <typename T>
__device__ __forceinline__ T cg_s(bool first, T beta, T sprev, T w) { return first ? w : fma_t(beta, sprev, w); }
template <typename T>
__device__ __forceinline__ T cg_r(T alpha, T s, T r) { return fma_t(-alpha, s, r); }

// per-thread FP64 accumulators -> one partial per (quantity, column) per
// workgroup: staged in LDS, then one thread per (quantity, column) adds the
// rows in order.  (A version with one wavefront per pair and a butterfly of
// lane shuffles was slower in the persistent kernel: 397 against 424 SOC
// iterations/s on the 481 x 321 image.)
template <int NQ>
__device__ __forceinline__ void block_partials(const double (&acc)[NQ], double* sh, int d, int R, double* part,
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

// out[q * d + c] = sum over workgroups b in [b0, b1) of src[(q * stride + b) * d + c],
// in a fixed order; one workgroup; sh needs blockDim doubles (out must not
// overlap them).  Thread idx = s * pairs + pr (pr = q * d + c, so a wave reads
// consecutive columns of one workgroup) sums the workgroups b0 + s + k team, up
// to eight loads in flight; then the team's sums of each pair are added in s
// order.  The partials are usually written on other XCDs, so each round of
// loads is a trip beyond L2: the team is as large as makes one round of eight
// loads per thread, within the workgroup.
__device__ __forceinline__ void reduce_range(const double* src, int stride, int b0, int b1, int d, int nq, double* out,
                             double* sh) {
    constexpr int U = 8;
    const int pairs = nq * d;
    const int nb = b1 - b0;
    int team = (int)blockDim.x / pairs;
    team = min(team, (nb + U - 1) / U);
    if (team < 1) team = 1;
    for (int idx = threadIdx.x; idx < pairs * team; idx += blockDim.x) {
        const int s = idx / pairs, pr = idx - s * pairs;
        const int q = pr / d, c = pr - q * d;
        const double* base = src + (size_t)q * stride * d + c;
        double acc = 0.0;
        int b = b0 + s;
        for (; b + (U - 1) * team < b1; b += U * team) {
            double v[U];
#pragma unroll
            for (int k = 0; k < U; ++k) v[k] = base[(size_t)(b + k * team) * d];
#pragma unroll
            for (int k = 0; k < U; ++k) acc += v[k];
        }
        for (; b < b1; b += team) acc += base[(size_t)b * d];
        sh[idx] = acc;
    }
    __syncthreads();
    for (int pr = threadIdx.x; pr < pairs; pr += blockDim.x) {
        double acc = 0.0;
        for (int s = 0; s < team; ++s) acc += sh[s * pairs + pr];
        out[pr] = acc;
    }
    __syncthreads();
}

// Reduce the partials of segment sg into out[q * d + c] (nq quantities of d
// values).  With a single segment the per-XCD-group partials are summed.
template <typename T>
__device__ __forceinline__ void seg_sums(const KA<T>& a, int sg, int nq, int d, double* out, double* sh, bool grouped) {
    if (grouped) reduce_range(a.gpart, kNumXcd, 0, kNumXcd, d, nq, out, sh);
    else reduce_range(a.part, a.nblk, a.seg_blk0[sg], a.seg_blk0[sg + 1], d, nq, out, sh);
}

// Sums for the segments [sg0, sg0 + ns) at once: out[(k * nq + q) * d + c] for
// segment sg0 + k.  One segment: the team reduction above (or the per-XCD-group
// partials when grouped); several: one thread per (segment, quantity, column),
// summing the segment's workgroups in order.
template <typename T>
__device__ __forceinline__ void seg_sums_all(const KA<T>& a, int sg0, int ns, int nq, double* out, double* sh,
                                             bool grouped) {
    const int d = a.d;
    if (a.nseg == 1) { seg_sums(a, 0, nq, d, out, sh, grouped); return; }
    const int per = nq * d;
    for (int idx = threadIdx.x; idx < ns * per; idx += blockDim.x) {
        const int k = idx / per, rem = idx - k * per, q = rem / d, c = rem - q * d;
        const int sg = sg0 + k;
        const double* base = a.part + (size_t)q * a.nblk * d + c;
        const int b0 = a.seg_blk0[sg], b1 = a.seg_blk0[sg + 1];
        double acc = 0.0;
#pragma unroll 8
        for (int b = b0; b < b1; ++b) acc += base[(size_t)b * d];
        out[idx] = acc;
    }
    __syncthreads();
}

// segments per pass of a finaliser (their sums share sh[1024, 4608))
__device__ __forceinline__ int seg_chunk(int nq, int d) {
    const int c = (kSmemDoubles - 1024) / (nq * d);
    return c < 1 ? 1 : c;
}

// ---------------------------------------------------------------------------
// Phases (each called by every workgroup for its rows)
// ---------------------------------------------------------------------------
// With the ELL width KC known at compile time the slot loops run in groups of
// up to 8 slots: the group's slot indices and weights are loaded together, then
// all of its neighbour gathers, then the arithmetic in slot order (the same
// operations in the same order as the generic loop), so one wave keeps many
// independent loads in flight instead of waiting on each slot.
// (GM: largest group, 8 in the one-phase kernels, 4 in the persistent kernel
// whose registers are shared by every phase)
// unroll factor of the plain slot loops (compiled width or generic CSR rows)
template <int KC>
constexpr int kSlotUnroll = KC > 0 ? 4 : 2;

// slots per group of the loops over rows of any length (general CSR layout)
constexpr int kGenGroup = 4;
// the per-row kernels' slot groups on general layouts (one thread per row and
// up to four columns: fewer threads per row, so more slots in flight each; on
// the 200k k-NN graph 8 ran a SOC iteration in 20.0 ms, 4 in 21.3)
constexpr int kRowGroup = 8;

template <int KC, int GM>
constexpr int slot_group() { return KC <= 0 ? 1 : (KC <= GM ? KC : GM); }

// LDS copy of the constant per-row data a workgroup of the persistent kernel
// reads in every phase (ELL slot columns and weights, diag(A), its inverse,
// D^{1/2}), filled once per launch when the workgroup's rows fit: the slot
// lookups of the gathers then cost an LDS access instead of a global one.
// Layout: chunk p of the workgroup (its p-th R-row chunk), row rl of the chunk:
// col/w at (p KC + k) R + rl, per-row values at p R + rl.
template <typename T>
struct RowCache {
    const int* col = nullptr;
    const T* w = nullptr;
    const T* inv = nullptr;
    const T* dA = nullptr;
    const T* sq = nullptr;
};

template <typename T>
__host__ __device__ constexpr size_t row_cache_bytes(int np, int R, int K) {
    return (size_t)np * R * ((size_t)K * (sizeof(int) + sizeof(T)) + 3 * sizeof(T));
}

template <typename T, int KC>
__device__ __forceinline__ RowCache<T> fill_row_cache(const KA<T>& a, int lb, unsigned char* lds, int np) {
    const int R = a.R;
    const int rb = a.bit[3 * lb], re = a.bit[3 * lb + 1], rs = a.bit[3 * lb + 2];
    int* col = reinterpret_cast<int*>(lds);
    T* w = reinterpret_cast<T*>(col + (size_t)np * KC * R);
    T* inv = w + (size_t)np * KC * R;
    T* dA = inv + (size_t)np * R;
    T* sq = dA + (size_t)np * R;
    for (int idx = threadIdx.x; idx < np * R; idx += blockDim.x) {
        const int p = idx / R, rl = idx - p * R;
        const int i = rb + p * rs + rl;
        if (i < re) {
            inv[idx] = a.invdiag[i];
            dA[idx] = a.diagA[i];
            sq[idx] = a.sqrtD[i];
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                const int sl = i + k * a.n;
                col[(p * KC + k) * R + rl] = a.scol[sl];
                w[(p * KC + k) * R + rl] = a.sw[sl];
            }
        }
    }
    __syncthreads();
    RowCache<T> rc;
    rc.col = col;
    rc.w = w;
    rc.inv = inv;
    rc.dA = dA;
    rc.sq = sq;
    return rc;
}

// Residual phases.  For every owned element (i, c):
//   EU : t = w (y_i - y_j) + b_s ; d_s = Shrink(t, 1/lambda) ; b_s = t - d_s   (Eqs. 9, 10)
//        rhs = lambda/2 sum_s w (d_s - b_s) + r/2 D^{1/2} (P - B)               (Eq. 13)
//   E0 : rhs = r/2 D^{1/2} (P - B)                   (b = d = 0 at the first inner step)
//   R0 : rhs from the stored rhs
//   RHS: rhs from the stored b and d
// then (unless RHS) r0 = rhs - A x, with FP64 partials of rhs^T rhs and r0^T r0.
template <int KC = 0, int GM = 8, bool LC = false, typename T>
__device__ __forceinline__ void ph_residual(const KA<T>& a, int lb, int mode, int do_r0, int b_zero, int par, double* sh,
                                            const RowCache<T>& rc = RowCache<T>()) {
    const int d = a.d, R = a.R, t = threadIdx.x;
    const T* bread = a.bsb[par & 1];
    T* bwrite = a.bsb[(par & 1) ^ 1];
    const int rb = a.bit[3 * lb], re = a.bit[3 * lb + 1], rs = a.bit[3 * lb + 2];
    double acc[2] = {0.0, 0.0};
    T* r0 = a.rb[0];
    if (t < R * d) {
        const int rl = t / d, c = t - rl * d;
        int p = 0;
        for (int i = rb + rl; i < re; i += rs, ++p) {
            const size_t e = (size_t)i * d + c;
            int s0, cnt, st;
            row_slots<KC>(a, i, s0, cnt, st);
            const T xi = a.x[e];
            T accR = T(0), accA = T(0);
            if (mode == PH_EU && KC > 0) {
                const T yi = a.Y[e];
                constexpr int G = slot_group<KC, GM>();
                for (int k0 = 0; k0 < cnt; k0 += G) {
                    int jj[G];
                    T ww[G], yj[G], bo[G], xj[G];
                    size_t ss[G];
                    bool own[G];
#pragma unroll
                    for (int k = 0; k < G; ++k) {
                        const int sl = s0 + (k0 + k) * st;
                        const int cix = (p * KC + k0 + k) * R + rl;
                        jj[k] = LC ? rc.col[cix] : a.scol[sl];
                        ww[k] = LC ? rc.w[cix] : a.sw[sl];
                        ss[k] = split_slot<KC>(a, i, k0 + k, jj[k], (size_t)sl, own[k]);
                        bo[k] = T(0);
                        if (!b_zero) {
                            const T b = bread[ss[k] * d + c];
                            bo[k] = own[k] ? b : -b;
                        }
                    }
#pragma unroll
                    for (int k = 0; k < G; ++k) {
                        const size_t ej = (size_t)jj[k] * d + c;
                        yj[k] = a.Y[ej];
                        xj[k] = do_r0 ? a.x[ej] : T(0);
                    }
#pragma unroll
                    for (int k = 0; k < G; ++k) {
                        const size_t es = ss[k] * d + c;
                        const T tv = fma_t(ww[k], yi - yj[k], bo[k]);
                        const T dv = shrink(tv, a.gamma);
                        const T bn = tv - dv;
                        if (own[k]) {
                            bwrite[es] = bn;
                            if (a.keep_split) a.ds[es] = dv;
                        }
                        accR = fma_t(ww[k], dv - bn, accR);
                        if (do_r0) accA = fma_t(mul_t(ww[k], ww[k]), xj[k], accA);
                    }
                }
            } else if (mode == PH_EU) {
                const T yi = a.Y[e];
#pragma unroll kSlotUnroll<KC>
                for (int k = 0; k < cnt; ++k) {
                    const int s = s0 + k * st;
                    const int j = a.scol[s];
                    const T ww = a.sw[s];
                    const size_t ej = (size_t)j * d + c;
                    const T yj = a.Y[ej];
                    const size_t es = (size_t)s * d + c;
                    const T bold = b_zero ? T(0) : bread[es];
                    const T tv = fma_t(ww, yi - yj, bold);
                    const T dv = shrink(tv, a.gamma);
                    const T bn = tv - dv;
                    bwrite[es] = bn;
                    if (a.keep_split) a.ds[es] = dv;
                    accR = fma_t(ww, dv - bn, accR);
                    if (do_r0) accA = fma_t(mul_t(ww, ww), a.x[ej], accA);
                }
            } else if (mode == PH_RHS) {
#pragma unroll kSlotUnroll<KC>
                for (int k = 0; k < cnt; ++k) {
                    const int s = s0 + k * st;
                    bool own;
                    const size_t es = split_slot<KC>(a, i, k, a.scol[s], (size_t)s, own) * d + c;
                    const T dmb = a.ds[es] - bread[es];
                    accR = fma_t(a.sw[s], own ? dmb : -dmb, accR);
                }
            } else if (do_r0 && KC > 0) {
                constexpr int G = slot_group<KC, GM>();
                for (int k0 = 0; k0 < cnt; k0 += G) {
                    int jj[G];
                    T ww[G], xj[G];
#pragma unroll
                    for (int k = 0; k < G; ++k) {
                        const int sl = s0 + (k0 + k) * st;
                        const int cix = (p * KC + k0 + k) * R + rl;
                        jj[k] = LC ? rc.col[cix] : a.scol[sl];
                        ww[k] = LC ? rc.w[cix] : a.sw[sl];
                    }
#pragma unroll
                    for (int k = 0; k < G; ++k) xj[k] = a.x[(size_t)jj[k] * d + c];
#pragma unroll
                    for (int k = 0; k < G; ++k) accA = fma_t(mul_t(ww[k], ww[k]), xj[k], accA);
                }
            } else if (do_r0) {
#pragma unroll kSlotUnroll<KC>
                for (int k = 0; k < cnt; ++k) {
                    const int s = s0 + k * st;
                    const T ww = a.sw[s];
                    accA = fma_t(mul_t(ww, ww), a.x[(size_t)a.scol[s] * d + c], accA);
                }
            }
            T rhs;
            if (mode == PH_R0) {
                rhs = a.rhs[e];
            } else {
                const T split = mul_t(a.half_r, mul_t(LC ? rc.sq[p * R + rl] : a.sqrtD[i], a.P[e] - a.B[e]));
                rhs = (mode == PH_E0) ? split : fma_t(a.c_off, accR, split);
                if (a.store_rhs || mode == PH_RHS) a.rhs[e] = rhs;
            }
            if (do_r0) {
                const T ax = fma_t(LC ? rc.dA[p * R + rl] : a.diagA[i], xi, -mul_t(a.c_off, accA));
                const T rv = rhs - ax;
                r0[e] = rv;
                acc[0] += (double)rhs * (double)rhs;
                acc[1] += (double)rv * (double)rv;
            }
        }
    }
    if (do_r0) block_partials<2>(acc, sh, d, R, a.part, a.nblk, lb);
}

// PH_W0: w0 = A u0 with u0 = r0 / diag(A); partials of r0.u0 and w0.u0.
template <int KC = 0, int GM = 8, bool LC = false, typename T>
__device__ __forceinline__ void ph_w0(const KA<T>& a, int lb, double* sh, const RowCache<T>& rc = RowCache<T>()) {
    const int d = a.d, R = a.R, t = threadIdx.x;
    const int rb = a.bit[3 * lb], re = a.bit[3 * lb + 1], rs = a.bit[3 * lb + 2];
    const T* r = a.rb[0];
    T* w = a.wb[0];
    double acc[2] = {0.0, 0.0};
    if (t < R * d) {
        const int rl = t / d, c = t - rl * d;
        int p = 0;
        for (int i = rb + rl; i < re; i += rs, ++p) {
            const size_t e = (size_t)i * d + c;
            int s0, cnt, st;
            row_slots<KC>(a, i, s0, cnt, st);
            const T ri = r[e];
            const T ui = mul_t(LC ? rc.inv[p * R + rl] : a.invdiag[i], ri);
            T accA = T(0);
            if constexpr (KC > 0) {
                constexpr int G = slot_group<KC, GM>();
                for (int k0 = 0; k0 < cnt; k0 += G) {
                    int jj[G];
                    T ww[G], rj[G], ij[G];
#pragma unroll
                    for (int k = 0; k < G; ++k) {
                        const int sl = s0 + (k0 + k) * st;
                        const int cix = (p * KC + k0 + k) * R + rl;
                        jj[k] = LC ? rc.col[cix] : a.scol[sl];
                        ww[k] = LC ? rc.w[cix] : a.sw[sl];
                    }
#pragma unroll
                    for (int k = 0; k < G; ++k) {
                        rj[k] = r[(size_t)jj[k] * d + c];
                        ij[k] = a.invdiag[jj[k]];
                    }
#pragma unroll
                    for (int k = 0; k < G; ++k) accA = fma_t(mul_t(ww[k], ww[k]), mul_t(ij[k], rj[k]), accA);
                }
            } else {
                // rows of any length: groups of kGenGroup slots (their column
                // and weight loads, then their gathers), then the tail
                int k = 0;
                for (; k + kGenGroup <= cnt; k += kGenGroup) {
                    int jj[kGenGroup];
                    T ww[kGenGroup], rj[kGenGroup], ij[kGenGroup];
#pragma unroll
                    for (int q = 0; q < kGenGroup; ++q) {
                        const int sl = s0 + (k + q) * st;
                        jj[q] = a.scol[sl];
                        ww[q] = a.sw[sl];
                    }
#pragma unroll
                    for (int q = 0; q < kGenGroup; ++q) {
                        rj[q] = r[(size_t)jj[q] * d + c];
                        ij[q] = a.invdiag[jj[q]];
                    }
#pragma unroll
                    for (int q = 0; q < kGenGroup; ++q) accA = fma_t(mul_t(ww[q], ww[q]), mul_t(ij[q], rj[q]), accA);
                }
                for (; k < cnt; ++k) {
                    const int s = s0 + k * st;
                    const int j = a.scol[s];
                    const T ww = a.sw[s];
                    const T uj = mul_t(a.invdiag[j], r[(size_t)j * d + c]);
                    accA = fma_t(mul_t(ww, ww), uj, accA);
                }
            }
            const T wi = fma_t(LC ? rc.dA[p * R + rl] : a.diagA[i], ui, -mul_t(a.c_off, accA));
            w[e] = wi;
            acc[0] += (double)ri * (double)ui;
            acc[1] += (double)wi * (double)ui;
        }
    }
    block_partials<2>(acc, sh, d, R, a.part, a.nblk, lb);
}

// PH_IT: CG iteration i = S->it with alpha_i, beta_i per (segment, column):
//   p_i = u_i + beta p_{i-1}, s_i = w_i + beta s_{i-1}, x += alpha p_i,
//   r_{i+1} = r_i - alpha s_i, u_{i+1} = r_{i+1} / diag(A), w_{i+1} = A u_{i+1};
// partials of r.u, w.u and r.r of iteration i+1.
//   it: iteration index; alphas, betas: the scalars per (segment, column).
template <int KC = 0, int GM = 8, bool LC = false, typename T>
__device__ __forceinline__ void ph_it(const KA<T>& a, int lb, double* sh, int it, const double* alphas,
                                      const double* betas, const RowCache<T>& rc = RowCache<T>()) {
    const int d = a.d, R = a.R, t = threadIdx.x;
    const int rb = a.bit[3 * lb], re = a.bit[3 * lb + 1], rs = a.bit[3 * lb + 2];
    const bool first = (it == 0);
    const int cur = it & 1, nxt = cur ^ 1;
    const T* r = a.rb[cur];
    const T* w = a.wb[cur];
    const T* sp = a.sb[cur];     // s_{i-1}
    T* rn = a.rb[nxt];
    T* wn = a.wb[nxt];
    T* sn = a.sb[nxt];           // s_i
    const int sg = a.blk_seg[lb];
    double acc[3] = {0.0, 0.0, 0.0};
    if (t < R * d) {
        const int rl = t / d, c = t - rl * d;
        const int ci = sg * d + c;
        const T alpha = (T)alphas[ci];
        const T beta = (T)betas[ci];
        int p = 0;
        for (int i = rb + rl; i < re; i += rs, ++p) {
            const size_t e = (size_t)i * d + c;
            int s0, cnt, st;
            row_slots<KC>(a, i, s0, cnt, st);
            // own-row loads are unconditional (selected below) so they issue together
            const T inv = LC ? rc.inv[p * R + rl] : a.invdiag[i];
            const T ri = r[e];
            const T pold = a.p[e];
            const T spi = sp[e];
            const T wi = w[e];
            const T ui = mul_t(inv, ri);
            const T pi = first ? ui : fma_t(beta, pold, ui);
            const T si = cg_s(first, beta, spi, wi);
            const T rn_i = cg_r(alpha, si, ri);
            const T un_i = mul_t(inv, rn_i);
            T accA = T(0);
            if constexpr (KC > 0) {
                constexpr int G = slot_group<KC, GM>();
                for (int k0 = 0; k0 < cnt; k0 += G) {
                    int jj[G];
                    T ww[G], spj[G], wj[G], rj[G], ij[G];
#pragma unroll
                    for (int k = 0; k < G; ++k) {
                        const int sl = s0 + (k0 + k) * st;
                        const int cix = (p * KC + k0 + k) * R + rl;
                        jj[k] = LC ? rc.col[cix] : a.scol[sl];
                        ww[k] = LC ? rc.w[cix] : a.sw[sl];
                    }
#pragma unroll
                    for (int k = 0; k < G; ++k) {
                        const size_t ej = (size_t)jj[k] * d + c;
                        spj[k] = sp[ej];
                        wj[k] = w[ej];
                        rj[k] = r[ej];
                        ij[k] = a.invdiag[jj[k]];
                    }
#pragma unroll
                    for (int k = 0; k < G; ++k) {
                        const T sj = cg_s(first, beta, spj[k], wj[k]);
                        const T uj = mul_t(ij[k], cg_r(alpha, sj, rj[k]));
                        accA = fma_t(mul_t(ww[k], ww[k]), uj, accA);
                    }
                }
            } else {
                int k = 0;
                for (; k + kGenGroup <= cnt; k += kGenGroup) {
                    int jj[kGenGroup];
                    T ww[kGenGroup], spj[kGenGroup], wj[kGenGroup], rj[kGenGroup], ij[kGenGroup];
#pragma unroll
                    for (int q = 0; q < kGenGroup; ++q) {
                        const int sl = s0 + (k + q) * st;
                        jj[q] = a.scol[sl];
                        ww[q] = a.sw[sl];
                    }
#pragma unroll
                    for (int q = 0; q < kGenGroup; ++q) {
                        const size_t ej = (size_t)jj[q] * d + c;
                        spj[q] = sp[ej];
                        wj[q] = w[ej];
                        rj[q] = r[ej];
                        ij[q] = a.invdiag[jj[q]];
                    }
#pragma unroll
                    for (int q = 0; q < kGenGroup; ++q) {
                        const T sj = cg_s(first, beta, spj[q], wj[q]);
                        const T uj = mul_t(ij[q], cg_r(alpha, sj, rj[q]));
                        accA = fma_t(mul_t(ww[q], ww[q]), uj, accA);
                    }
                }
                for (; k < cnt; ++k) {
                    const int s = s0 + k * st;
                    const int j = a.scol[s];
                    const T ww = a.sw[s];
                    const size_t ej = (size_t)j * d + c;
                    const T sj = cg_s(first, beta, sp[ej], w[ej]);
                    const T uj = mul_t(a.invdiag[j], cg_r(alpha, sj, r[ej]));
                    accA = fma_t(mul_t(ww, ww), uj, accA);
                }
            }
            const T wn_i = fma_t(LC ? rc.dA[p * R + rl] : a.diagA[i], un_i, -mul_t(a.c_off, accA));
            a.p[e] = pi;
            sn[e] = si;
            a.x[e] = fma_t(alpha, pi, a.x[e]);
            rn[e] = rn_i;
            wn[e] = wn_i;
            acc[0] += (double)rn_i * (double)un_i;
            acc[1] += (double)wn_i * (double)un_i;
            acc[2] += (double)rn_i * (double)rn_i;
        }
    }
    block_partials<3>(acc, sh, d, R, a.part, a.nblk, lb);
}

// General layouts (rows of any length, KC = 0): one CG iteration in two
// passes, so that the neighbour values gathered are u' alone (stored by its
// owner) rather than the three vectors r, w, s from which the one-pass form
// recomputes them; on graphs of high and uneven degree (k-NN graphs) the
// gathers dominate, and the extra grid synchronisation is the cheaper price.
// Vectors in place (no neighbour reads them): r = rb[0], w = wb[0], s = sb[0],
// u' in zl.
//   GA (own rows): u = r / diag(A), p = u + beta p, s = w + beta s,
//       x += alpha p, r' = r - alpha s, u' = r' / diag(A); partials of r'.u'
//       (quantity 0) and r'.r' (quantity 2)
//   GB: w' = A u'; partials of w'.u' (quantity 1)
// The iteration's finaliser (the one-pass one) reads the three quantities.
template <int NQ>
__device__ __forceinline__ void block_partials_at(const double (&acc)[NQ], const int (&qout)[NQ], double* sh, int d,
                                                  int R, double* part, int nblk, int lb) {
    const int t = threadIdx.x;
    const int B = blockDim.x;
#pragma unroll
    for (int q = 0; q < NQ; ++q) sh[q * B + t] = (t < R * d) ? acc[q] : 0.0;
    __syncthreads();
    if (t < NQ * d) {
        const int q = t / d, c = t - q * d;
        double s = 0.0;
        for (int k = 0; k < R; ++k) s += sh[q * B + k * d + c];
        part[((size_t)qout[q] * nblk + lb) * d + c] = s;
    }
    __syncthreads();
}

template <typename T>
__device__ __forceinline__ void ph_ga(const KA<T>& a, int lb, double* sh, int it, const double* alphas,
                                      const double* betas) {
    const int d = a.d, R = a.R, t = threadIdx.x;
    const int rb = a.bit[3 * lb], re = a.bit[3 * lb + 1], rs = a.bit[3 * lb + 2];
    const bool first = (it == 0);
    T* r = a.rb[0];
    T* w = a.wb[0];
    T* sv = a.sb[0];
    double acc[2] = {0.0, 0.0};
    if (t < R * d) {
        const int rl = t / d, c = t - rl * d;
        const int ci = a.blk_seg[lb] * d + c;
        const T alpha = (T)alphas[ci];
        const T beta = (T)betas[ci];
        for (int i = rb + rl; i < re; i += rs) {
            const size_t e = (size_t)i * d + c;
            const T inv = a.invdiag[i];
            const T ri = r[e];
            const T pold = a.p[e];
            const T spi = sv[e];
            const T wi = w[e];
            const T ui = mul_t(inv, ri);
            const T pi = first ? ui : fma_t(beta, pold, ui);
            const T si = cg_s(first, beta, spi, wi);
            const T rn_i = cg_r(alpha, si, ri);
            const T un_i = mul_t(inv, rn_i);
            a.p[e] = pi;
            sv[e] = si;
            a.x[e] = fma_t(alpha, pi, a.x[e]);
            r[e] = rn_i;
            a.zl[e] = un_i;
            acc[0] += (double)rn_i * (double)un_i;
            acc[1] += (double)rn_i * (double)rn_i;
        }
    }
    const int qo[2] = {0, 2};
    block_partials_at<2>(acc, qo, sh, d, R, a.part, a.nblk, lb);
}

template <typename T>
__device__ __forceinline__ void ph_gb(const KA<T>& a, int lb, double* sh) {
    const int d = a.d, R = a.R, t = threadIdx.x;
    const int rb = a.bit[3 * lb], re = a.bit[3 * lb + 1], rs = a.bit[3 * lb + 2];
    const T* u = a.zl;
    T* w = a.wb[0];
    double acc[1] = {0.0};
    if (t < R * d) {
        const int rl = t / d, c = t - rl * d;
        for (int i = rb + rl; i < re; i += rs) {
            const size_t e = (size_t)i * d + c;
            int s0, cnt, st;
            row_slots<0>(a, i, s0, cnt, st);
            const T ui = u[e];
            T accA = T(0);
            int k = 0;
            for (; k + kGenGroup <= cnt; k += kGenGroup) {
                int jj[kGenGroup];
                T ww[kGenGroup], uj[kGenGroup];
#pragma unroll
                for (int q = 0; q < kGenGroup; ++q) {
                    const int sl = s0 + (k + q) * st;
                    jj[q] = a.scol[sl];
                    ww[q] = a.sw[sl];
                }
#pragma unroll
                for (int q = 0; q < kGenGroup; ++q) uj[q] = u[(size_t)jj[q] * d + c];
#pragma unroll
                for (int q = 0; q < kGenGroup; ++q) accA = fma_t(mul_t(ww[q], ww[q]), uj[q], accA);
            }
            for (; k < cnt; ++k) {
                const int sl = s0 + k * st;
                const T ww = a.sw[sl];
                accA = fma_t(mul_t(ww, ww), u[(size_t)a.scol[sl] * d + c], accA);
            }
            const T wi = fma_t(a.diagA[i], ui, -mul_t(a.c_off, accA));
            w[e] = wi;
            acc[0] += (double)wi * (double)ui;
        }
    }
    const int qo[1] = {1};
    block_partials_at<1>(acc, qo, sh, d, R, a.part, a.nblk, lb);
}

// Learned-preconditioner PCG phases (standard PCG with M^{-1} = G^T G, one
// kernel per phase, three per iteration).  Buffers: q = wb[0]; p double
// buffered in sb[it & 1] (new) / sb[(it & 1) ^ 1] (previous); r double
// buffered in rb[it & 1] (before the update of iteration it) / rb[(it & 1) ^ 1]
// (after it), the initial residual in rb[0].
//   LA : p = z + beta p, q = A p, partials of p.q
//   LC : x += alpha p, r' = r - alpha q (own rows), y1 = Gt D_A^{-1/2} r' with
//        the neighbours' r' recomputed from their r and q (upd = 0: y1 from
//        the initial residual, no update)
//   LD : z = D_A^{-1/2} Gt^T y1, partials of r'.z and r'.r'
// On pixel-grid stencils the ELL slots [0, K/2) of a row are exactly its
// lower neighbours (raster order), [K/2, K) the upper ones; otherwise the
// column decides.
template <int H>
constexpr int half_group() { return H <= 0 ? 1 : (H % 8 == 0 ? 8 : (H % 6 == 0 ? 6 : (H % 4 == 0 ? 4 : H))); }

template <int KC = 0, typename T>
__device__ __forceinline__ void ph_lc(const KA<T>& a, int lb, int upd) {
    const int d = a.d, R = a.R, t = threadIdx.x;
    const int rb = a.bit[3 * lb], re = a.bit[3 * lb + 1], rs = a.bit[3 * lb + 2];
    const int it = upd ? ld_flag(&a.S->it) : 0;
    const T* r = a.rb[it & 1];
    T* rn = a.rb[(it & 1) ^ 1];
    const T* p = a.sb[it & 1];
    const T* q = a.wb[0];
    if (t >= R * d) return;
    const int rl = t / d, c = t - rl * d;
    const T alpha = upd ? (T)a.cs.alpha[a.blk_seg[lb] * d + c] : T(0);
    for (int i = rb + rl; i < re; i += rs) {
        const size_t e = (size_t)i * d + c;
        int s0, cnt, st;
        row_slots<KC>(a, i, s0, cnt, st);
        T ri = r[e];
        if (upd) {
            a.x[e] = fma_t(alpha, p[e], a.x[e]);
            ri = fma_t(-alpha, q[e], ri);
            rn[e] = ri;
        }
        T acc = mul_t(a.gdiag[i], mul_t(a.isq[i], ri));
        if (KC > 0 && a.sten) {
            constexpr int H = KC / 2, G = half_group<H>();
#pragma unroll
            for (int k0 = 0; k0 < H; k0 += G) {
                int jj[G];
                T gv[G], rj[G], qj[G], ij[G];
#pragma unroll
                for (int k = 0; k < G; ++k) {
                    const int sl = s0 + (k0 + k) * st;
                    jj[k] = a.scol[sl];
                    gv[k] = a.gval[sl];
                }
#pragma unroll
                for (int k = 0; k < G; ++k) {
                    const size_t ej = (size_t)jj[k] * d + c;
                    rj[k] = r[ej];
                    qj[k] = upd ? q[ej] : T(0);
                    ij[k] = a.isq[jj[k]];
                }
#pragma unroll
                for (int k = 0; k < G; ++k) {
                    const T rv = upd ? fma_t(-alpha, qj[k], rj[k]) : rj[k];
                    acc = fma_t(gv[k], mul_t(ij[k], rv), acc);
                }
            }
        } else {
#pragma unroll 2
            for (int k = 0; k < cnt; ++k) {
                const int s = s0 + k * st;
                const int j = a.scol[s];
                if (j < i) {
                    const size_t ej = (size_t)j * d + c;
                    const T rv = upd ? fma_t(-alpha, q[ej], r[ej]) : r[ej];
                    acc = fma_t(a.gval[s], mul_t(a.isq[j], rv), acc);
                }
            }
        }
        a.y1[e] = acc;
    }
}

template <int KC = 0, typename T>
__device__ __forceinline__ void ph_ld(const KA<T>& a, int lb, double* sh, int initial) {
    const int d = a.d, R = a.R, t = threadIdx.x;
    const int rb = a.bit[3 * lb], re = a.bit[3 * lb + 1], rs = a.bit[3 * lb + 2];
    const T* r = initial ? a.rb[0] : a.rb[(ld_flag(&a.S->it) & 1) ^ 1];
    double acc2[2] = {0.0, 0.0};
    if (t < R * d) {
        const int rl = t / d, c = t - rl * d;
        for (int i = rb + rl; i < re; i += rs) {
            const size_t e = (size_t)i * d + c;
            int s0, cnt, st;
            row_slots<KC>(a, i, s0, cnt, st);
            T acc = mul_t(a.gdiag[i], a.y1[e]);
            if (KC > 0 && a.sten) {
                constexpr int H = KC / 2, G = half_group<H>();
#pragma unroll
                for (int k0 = H; k0 < KC; k0 += G) {
                    int jj[G];
                    T gv[G], yj[G];
#pragma unroll
                    for (int k = 0; k < G; ++k) {
                        const int sl = s0 + (k0 + k) * st;
                        jj[k] = a.scol[sl];
                        gv[k] = a.gval[sl];
                    }
#pragma unroll
                    for (int k = 0; k < G; ++k) yj[k] = a.y1[(size_t)jj[k] * d + c];
#pragma unroll
                    for (int k = 0; k < G; ++k) acc = fma_t(gv[k], yj[k], acc);
                }
            } else {
#pragma unroll 2
                for (int k = 0; k < cnt; ++k) {
                    const int s = s0 + k * st;
                    const int j = a.scol[s];
                    if (j > i) acc = fma_t(a.gval[s], a.y1[(size_t)j * d + c], acc);
                }
            }
            const T z = mul_t(a.isq[i], acc);
            a.zl[e] = z;
            const T rv = r[e];
            acc2[0] += (double)rv * (double)z;
            acc2[1] += (double)rv * (double)rv;
        }
    }
    block_partials<2>(acc2, sh, d, R, a.part, a.nblk, lb);
}

template <int KC = 0, typename T>
__device__ __forceinline__ void ph_la(const KA<T>& a, int lb, double* sh) {
    const int d = a.d, R = a.R, t = threadIdx.x;
    const int rb = a.bit[3 * lb], re = a.bit[3 * lb + 1], rs = a.bit[3 * lb + 2];
    const int it = ld_flag(&a.S->it);
    const bool first = (it == 0);
    T* pnew = a.sb[it & 1];
    const T* pold = a.sb[(it & 1) ^ 1];
    T* q = a.wb[0];
    const int sg = a.blk_seg[lb];
    double acc1[1] = {0.0};
    if (t < R * d) {
        const int rl = t / d, c = t - rl * d;
        const T beta = (T)a.cs.beta[sg * d + c];
        for (int i = rb + rl; i < re; i += rs) {
            const size_t e = (size_t)i * d + c;
            int s0, cnt, st;
            row_slots<KC>(a, i, s0, cnt, st);
            const T zi = a.zl[e];
            const T po = pold[e];
            const T pi = first ? zi : fma_t(beta, po, zi);
            T acc = T(0);
            if constexpr (KC > 0) {
                constexpr int G = slot_group<KC, 8>();
#pragma unroll
                for (int k0 = 0; k0 < KC; k0 += G) {
                    int jj[G];
                    T ww[G], zj[G], pj[G];
#pragma unroll
                    for (int k = 0; k < G; ++k) {
                        const int sl = s0 + (k0 + k) * st;
                        jj[k] = a.scol[sl];
                        ww[k] = a.sw[sl];
                    }
#pragma unroll
                    for (int k = 0; k < G; ++k) {
                        const size_t ej = (size_t)jj[k] * d + c;
                        zj[k] = a.zl[ej];
                        pj[k] = pold[ej];
                    }
#pragma unroll
                    for (int k = 0; k < G; ++k) {
                        const T pv = first ? zj[k] : fma_t(beta, pj[k], zj[k]);
                        acc = fma_t(mul_t(ww[k], ww[k]), pv, acc);
                    }
                }
            } else {
#pragma unroll 2
                for (int k = 0; k < cnt; ++k) {
                    const int s = s0 + k * st;
                    const size_t ej = (size_t)a.scol[s] * d + c;
                    const T ww = a.sw[s];
                    const T pj = first ? a.zl[ej] : fma_t(beta, pold[ej], a.zl[ej]);
                    acc = fma_t(mul_t(ww, ww), pj, acc);
                }
            }
            const T qi = fma_t(a.diagA[i], pi, -mul_t(a.c_off, acc));
            pnew[e] = pi;
            q[e] = qi;
            acc1[0] += (double)pi * (double)qi;
        }
    }
    block_partials<1>(acc1, sh, d, R, a.part, a.nblk, lb);
}

// PH_ZERO: x_c = 0 for columns with a zero right-hand side
template <typename T>
__device__ __forceinline__ void ph_zero(const KA<T>& a, int lb, const int* zero) {
    const int d = a.d, R = a.R, t = threadIdx.x;
    const int rb = a.bit[3 * lb], re = a.bit[3 * lb + 1], rs = a.bit[3 * lb + 2];
    if (t < R * d) {
        const int rl = t / d, c = t - rl * d;
        if (!zero[a.blk_seg[lb] * d + c]) return;
        for (int i = rb + rl; i < re; i += rs) a.x[(size_t)i * d + c] = T(0);
    }
}

__device__ __forceinline__ void pair_of(int k, int d, int& pa, int& pb) {
    int r = 0, off = 0;
    while (off + (d - r) <= k) { off += d - r; ++r; }
    pa = r;
    pb = r + (k - off);
}

// PH_GRAM: FP64 Gram matrix of Z (mode 0: Z = D^{1/2} Y + B; mode 1: Z = D^{1/2} Y),
// upper triangle packed, one partial per workgroup.
template <typename T>
__device__ __forceinline__ void ph_gram(const KA<T>& a, int lb, int mode, double* sh) {
    const int d = a.d, R = a.R, t = threadIdx.x;
    const int npair = d * (d + 1) / 2;
    const int rb = a.bit[3 * lb], re = a.bit[3 * lb + 1], rs = a.bit[3 * lb + 2];
    double* zt = sh;                  // R x d staged rows
    // (pair, row slice) per thread: nsl slices of the staged rows per pair
    // (one when the pairs outnumber the threads: two pairs per thread), the
    // slices added in order at the end
    const int nsl = max(1, (int)blockDim.x / npair);
    const int sl = t / npair;
    int pa[2] = {0, 0}, pb[2] = {0, 0};
    for (int h = 0; h < 2; ++h) {
        int k = (nsl > 1) ? t - sl * npair : t + h * (int)blockDim.x;
        if (k < npair) pair_of(k, d, pa[h], pb[h]);
    }
    double acc[2] = {0.0, 0.0};
    // the factorisations that follow only ever clear this flag
    if (lb == 0 && t == 0) a.S->ortho_ok = 1;
    for (int base = rb; base < re; base += rs) {
        int rows = min(R, re - base);
        if (t < rows * d) {
            int rl = t / d, c = t - rl * d;
            int i = base + rl;
            size_t e = (size_t)i * d + c;
            T z = (mode == 0) ? zrow(a, i, e) : mul_t(a.sqrtD[i], a.Y[e]);
            zt[t] = (double)z;
        }
        __syncthreads();
        if (nsl > 1) {
            if (sl < nsl) {
                double s = acc[0];
                for (int rr = sl; rr < rows; rr += nsl) s += zt[rr * d + pa[0]] * zt[rr * d + pb[0]];
                acc[0] = s;
            }
        } else {
            for (int h = 0; h < 2; ++h) {
                int k = t + h * (int)blockDim.x;
                if (k < npair) {
                    double s = acc[h];
                    for (int rr = 0; rr < rows; ++rr) s += zt[rr * d + pa[h]] * zt[rr * d + pb[h]];
                    acc[h] = s;
                }
            }
        }
        __syncthreads();
    }
    if (nsl > 1) {
        double* red = sh + kBlock;    // beyond the staged rows
        if (sl < nsl) red[sl * npair + (t - sl * npair)] = acc[0];
        __syncthreads();
        if (t < npair) {
            double s = 0.0;
            for (int k = 0; k < nsl; ++k) s += red[k * npair + t];
            a.part[(size_t)lb * npair + t] = s;
        }
        __syncthreads();
        return;
    }
    for (int h = 0; h < 2; ++h) {
        int k = t + h * (int)blockDim.x;
        if (k < npair) a.part[(size_t)lb * npair + k] = acc[h];
    }
}

// PH_APPLY: mode 0 (P-update): P = Z T, B = Z - P with Z = D^{1/2} Y + B;
//           mode 1 (initial orthonormalisation): Y <- Y T, P = D^{1/2} Y, B = 0.
//           Tg: the segment's d x d transform (row stride kMaxD), global or LDS.
template <typename T>
__device__ __forceinline__ void ph_apply(const KA<T>& a, int lb, int mode, double* sh, const double* Tg) {
    const int d = a.d, R = a.R, t = threadIdx.x;
    const int rb = a.bit[3 * lb], re = a.bit[3 * lb + 1], rs = a.bit[3 * lb + 2];
    double* Ts = sh;                  // d x d
    double* zt = sh + kMaxD * kMaxD;  // R x d
    for (int k = t; k < d * d; k += blockDim.x) Ts[k] = Tg[(k / d) * kMaxD + (k % d)];
    for (int base = rb; base < re; base += rs) {
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
// Strip phases (pixel grids with a compiled stencil width, one launch per
// phase).  A workgroup owns the pixels x in [x0, x0 + len), y in [y0, y1) of
// one image and walks them one image row at a time.  Thread t holds element t
// of a ring row: pixel x0 - rho + t / d, column t % d, over the row segment
// [x0 - rho, x0 + len + rho).  The value each neighbour contributes (u_j of
// the CG iteration, x_j of A x) is formed once per pixel, by the thread that
// loaded it, into an LDS ring of 2 rho + 2 image rows, and the stencil sums
// read the ring; the loads of the next image row are issued before the
// arithmetic of the current one.  A thread's own pixel is the pixel it loads
// into the ring, so its own r, w, s come from the same loads.  The per-element
// arithmetic and the slot order are those of the row-chunk phases, so both
// give the same values element by element; only the per-workgroup partial
// sums group the rows differently.
// ---------------------------------------------------------------------------

// ELL slot k of a pixel grid is the stencil offset (dy, dx) of the (2 rho + 1)^2
// window in raster order without its centre (8 and 24 slots), or of the
// 4-neighbour cross in raster order.
template <int KC>
struct Sten {
    static constexpr int rho = (KC == 24) ? 2 : 1;
    static constexpr int side = 2 * rho + 1;
    static constexpr int ring = 2 * rho + 2;   // ring rows in LDS
    __device__ static constexpr int dy(int k) {
        return KC == 4 ? (k == 0 ? -1 : (k == 3 ? 1 : 0)) : ((k < KC / 2 ? k : k + 1) / side - rho);
    }
    __device__ static constexpr int dx(int k) {
        return KC == 4 ? (k == 1 ? -1 : (k == 2 ? 1 : 0)) : ((k < KC / 2 ? k : k + 1) % side - rho);
    }
    __device__ static constexpr int slot(int y) { return (y + 4 * ring) % ring; }   // y >= -2 rho
};

struct StripGeo {
    int row0, W, H, x0, len, y0, y1;
};

__device__ __forceinline__ StripGeo strip_geo(const int* geo, int lb) {
    const int* g = geo + 8 * lb;
    return StripGeo{g[0], g[1], g[2], g[3], g[4], g[5], g[6]};
}

// lane roles of a strip workgroup
struct StripLane {
    int c, px, span;
    bool loader, in_image, owner;
    __device__ StripLane(const StripGeo& g, int d, int rho) {
        const int t = threadIdx.x, q = t / d;
        c = t - q * d;
        span = g.len + 2 * rho;
        px = g.x0 - rho + q;
        loader = q < span;
        in_image = loader && px >= 0 && px < g.W;
        owner = q >= rho && q < rho + g.len;
    }
};

// Walk the strip of workgroup lb one image row at a time.
//   ld(j, e)    this lane's raw values of pixel j (element e = j d + c), loaded
//               LA image rows ahead of their publication; value-initialised
//               (zero) outside the image and outside the rows the strip reads
//   val(raw)    the value the lane publishes into the ring for its pixel
//   ldo(i, e)   an owner's further values of its pixel i, loaded LA rows ahead
//   body(i, e, raw, own, nb)  the arithmetic of owned pixel i, with nb(k) the
//               ring value of ELL slot k (zero outside the image)
// Ends with a workgroup barrier (the ring shares sh with the partial sums).
template <int KC, int LA = 1, typename T, class LD, class VAL, class LDO, class BODY>
__device__ __forceinline__ void strip_walk(const KA<T>& a, const StripGeo& g, const StripLane& ln, T* ring, LD&& ld,
                                           VAL&& val, LDO&& ldo, BODY&& body) {
    using S = Sten<KC>;
    constexpr int rho = S::rho;
    const int d = a.d, t = threadIdx.x;
    using Raw = decltype(ld(0, size_t(0)));
    using Own = decltype(ldo(0, size_t(0)));
    const int ylo = max(0, g.y0 - rho), yhi = min(g.H, g.y1 + rho);
    auto ldr = [&](int y) {
        Raw v{};
        if (ln.in_image && y >= ylo && y < yhi) {
            const int j = g.row0 + y * g.W + ln.px;
            v = ld(j, (size_t)j * d + ln.c);
        }
        return v;
    };
    auto ldw = [&](int y) {
        Own o{};
        if (ln.owner && y < g.y1) {
            const int i = g.row0 + y * g.W + ln.px;
            o = ldo(i, (size_t)i * d + ln.c);
        }
        return o;
    };
    if (g.len > 0 && g.y1 > g.y0) {
        constexpr int NR = rho + LA;   // raw rows held: y .. y + rho + LA - 1
        Raw raw[NR];
        Own own[LA];                   // own rows y .. y + LA - 1
#pragma unroll
        for (int k = 1; k <= rho; ++k)
            if (ln.loader) ring[S::slot(g.y0 - k) * kBlock + t] = val(ldr(g.y0 - k));
#pragma unroll
        for (int k = 0; k < NR; ++k) raw[k] = ldr(g.y0 + k);
#pragma unroll
        for (int k = 0; k < rho; ++k)
            if (ln.loader) ring[S::slot(g.y0 + k) * kBlock + t] = val(raw[k]);
#pragma unroll
        for (int k = 0; k < LA; ++k) own[k] = ldw(g.y0 + k);
        for (int y = g.y0; y < g.y1; ++y) {
            if (ln.loader) ring[S::slot(y + rho) * kBlock + t] = val(raw[rho]);
            const Raw rnext = ldr(y + NR);
            const Own onext = ldw(y + LA);
            __syncthreads();
            if (ln.owner) {
                const int i = g.row0 + y * g.W + ln.px;
                auto nb = [&](int k) { return ring[S::slot(y + S::dy(k)) * kBlock + t + S::dx(k) * d]; };
                body(i, (size_t)i * d + ln.c, raw[0], own[0], nb);
            }
#pragma unroll
            for (int k = 0; k + 1 < NR; ++k) raw[k] = raw[k + 1];
            raw[NR - 1] = rnext;
#pragma unroll
            for (int k = 0; k + 1 < LA; ++k) own[k] = own[k + 1];
            own[LA - 1] = onext;
        }
    }
    __syncthreads();
}

// CG iteration (the PH_IT arithmetic) over a strip
template <int KC, typename T>
__device__ __forceinline__ void st_it(const KA<T>& a, int lb, double* sh, int it, const double* alphas,
                                      const double* betas) {
    constexpr bool PW = KC <= 8;   // slot weights loaded one image row ahead with the rest
    const StripGeo g = strip_geo(a.geo, lb);
    const int d = a.d;
    const StripLane ln(g, d, Sten<KC>::rho);
    const bool first = (it == 0);
    const int cur = it & 1, nxt = cur ^ 1;
    const T* r = a.rb[cur];
    const T* w = a.wb[cur];
    const T* sp = a.sb[cur];
    T* rn = a.rb[nxt];
    T* wn = a.wb[nxt];
    T* sn = a.sb[nxt];
    const int ci = a.blk_seg[lb] * d + ln.c;
    const T alpha = (T)alphas[ci];
    const T beta = (T)betas[ci];
    struct Raw { T r, w, sp, inv; };
    struct Own { T p, x, dA, ww[PW ? KC : 1]; };
    double acc[3] = {0.0, 0.0, 0.0};
    strip_walk<KC, 2>(a, g, ln, reinterpret_cast<T*>(sh),
        [&](int j, size_t e) { return Raw{r[e], w[e], sp[e], a.invdiag[j]}; },
        // u_j = diag(A)^{-1} r_{j, i+1}: the neighbours' new u, as their owners form it
        [&](const Raw& v) { return mul_t(v.inv, cg_r(alpha, cg_s(first, beta, v.sp, v.w), v.r)); },
        [&](int i, size_t e) {
            Own o{};
            o.p = a.p[e];
            o.x = a.x[e];
            o.dA = a.diagA[i];
            if constexpr (PW) {
#pragma unroll
                for (int k = 0; k < KC; ++k) o.ww[k] = a.sw[(size_t)k * a.n + i];
            }
            return o;
        },
        [&](int i, size_t e, const Raw& v, const Own& own, auto&& nb) {
            const T ui = mul_t(v.inv, v.r);
            const T pi = first ? ui : fma_t(beta, own.p, ui);
            const T si = cg_s(first, beta, v.sp, v.w);
            const T rn_i = cg_r(alpha, si, v.r);
            const T un_i = mul_t(v.inv, rn_i);
            T accA = T(0);
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                const T wk = PW ? own.ww[PW ? k : 0] : a.sw[(size_t)k * a.n + i];
                accA = fma_t(mul_t(wk, wk), nb(k), accA);
            }
            const T wn_i = fma_t(own.dA, un_i, -mul_t(a.c_off, accA));
            a.p[e] = pi;
            sn[e] = si;
            a.x[e] = fma_t(alpha, pi, own.x);
            rn[e] = rn_i;
            wn[e] = wn_i;
            acc[0] += (double)rn_i * (double)un_i;
            acc[1] += (double)wn_i * (double)un_i;
            acc[2] += (double)rn_i * (double)rn_i;
        });
    block_partials<3>(acc, sh, d, kBlock / d, a.part, a.nblk, lb);
}

// w0 = A u0 with u0 = r0 / diag(A) (the PH_W0 arithmetic) over a strip
template <int KC, typename T>
__device__ __forceinline__ void st_w0(const KA<T>& a, int lb, double* sh) {
    const StripGeo g = strip_geo(a.geo, lb);
    const int d = a.d;
    const StripLane ln(g, d, Sten<KC>::rho);
    const T* r = a.rb[0];
    T* w = a.wb[0];
    struct Raw { T r, inv; };
    struct Own { T dA; };
    double acc[2] = {0.0, 0.0};
    strip_walk<KC>(a, g, ln, reinterpret_cast<T*>(sh),
        [&](int j, size_t e) { return Raw{r[e], a.invdiag[j]}; },
        [&](const Raw& v) { return mul_t(v.inv, v.r); },
        [&](int i, size_t) { return Own{a.diagA[i]}; },
        [&](int i, size_t e, const Raw& v, const Own& own, auto&& nb) {
            const T ui = mul_t(v.inv, v.r);
            T accA = T(0);
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                const T wk = a.sw[(size_t)k * a.n + i];
                accA = fma_t(mul_t(wk, wk), nb(k), accA);
            }
            const T wi = fma_t(own.dA, ui, -mul_t(a.c_off, accA));
            w[e] = wi;
            acc[0] += (double)v.r * (double)ui;
            acc[1] += (double)wi * (double)ui;
        });
    block_partials<2>(acc, sh, d, kBlock / d, a.part, a.nblk, lb);
}

// r0 = rhs - A x (PH_E0: rhs = r/2 D^{1/2}(P - B); PH_R0: the stored rhs) over
// a strip, with the partials of rhs.rhs and r0.r0 (the ph_residual arithmetic)
template <int KC, typename T>
__device__ __forceinline__ void st_res(const KA<T>& a, int lb, int mode, double* sh) {
    const StripGeo g = strip_geo(a.geo, lb);
    const int d = a.d;
    const StripLane ln(g, d, Sten<KC>::rho);
    T* r0 = a.rb[0];
    struct Raw { T x; };
    struct Own { T rhs, dA; };
    double acc[2] = {0.0, 0.0};
    strip_walk<KC>(a, g, ln, reinterpret_cast<T*>(sh),
        [&](int, size_t e) { return Raw{a.x[e]}; },
        [&](const Raw& v) { return v.x; },
        [&](int i, size_t e) {
            Own o{};
            o.rhs = (mode == PH_R0) ? a.rhs[e] : mul_t(a.half_r, mul_t(a.sqrtD[i], a.P[e] - a.B[e]));
            o.dA = a.diagA[i];
            return o;
        },
        [&](int i, size_t e, const Raw& v, const Own& own, auto&& nb) {
            T accA = T(0);
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                const T wk = a.sw[(size_t)k * a.n + i];
                accA = fma_t(mul_t(wk, wk), nb(k), accA);
            }
            if (mode != PH_R0 && a.store_rhs) a.rhs[e] = own.rhs;
            const T ax = fma_t(own.dA, v.x, -mul_t(a.c_off, accA));
            const T rv = own.rhs - ax;
            r0[e] = rv;
            acc[0] += (double)own.rhs * (double)own.rhs;
            acc[1] += (double)rv * (double)rv;
        });
    block_partials<2>(acc, sh, d, kBlock / d, a.part, a.nblk, lb);
}

// Edge update (the PH_EU arithmetic without r0) over a strip: per slot
// t = w (y_i - y_j) + b, d = Shrink(t, 1/lambda), b = t - d (Eqs. 9, 10), and
// rhs = lambda/2 sum w (d - b) + r/2 D^{1/2} (P - B) (Eq. 13), stored.
template <int KC, typename T>
__device__ __forceinline__ void st_eu(const KA<T>& a, int lb, double* sh) {
    constexpr bool PW = KC <= 8;   // slot weights and b loaded one image row ahead
    const StripGeo g = strip_geo(a.geo, lb);
    const int d = a.d;
    const StripLane ln(g, d, Sten<KC>::rho);
    const int b_zero = a.b_zero;
    const T* bread = a.bsb[a.bpar & 1];
    T* bwrite = a.bsb[(a.bpar & 1) ^ 1];
    // b of slot k of row i (the stored value, signed for this row)
    auto b_of = [&](int i, int k) {
        if (b_zero) return T(0);
        const size_t sl = (size_t)k * a.n + i;
        bool own;
        const size_t ss = split_slot<KC>(a, i, k, (a.bhalf && k >= KC / 2) ? a.scol[sl] : i, sl, own);
        const T b = bread[ss * d + ln.c];
        return own ? b : -b;
    };
    struct Raw { T y; };
    struct Own { T split, ww[PW ? KC : 1], bo[PW ? KC : 1]; };
    strip_walk<KC>(a, g, ln, reinterpret_cast<T*>(sh),
        [&](int, size_t e) { return Raw{a.Y[e]}; },
        [&](const Raw& v) { return v.y; },
        [&](int i, size_t e) {
            Own o{};
            o.split = mul_t(a.half_r, mul_t(a.sqrtD[i], a.P[e] - a.B[e]));
            if constexpr (PW) {
#pragma unroll
                for (int k = 0; k < KC; ++k) {
                    o.ww[k] = a.sw[(size_t)k * a.n + i];
                    o.bo[k] = b_of(i, k);
                }
            }
            return o;
        },
        [&](int i, size_t e, const Raw& v, const Own& own, auto&& nb) {
            T accR = T(0);
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                const size_t sl = (size_t)k * a.n + i;
                const T wk = PW ? own.ww[PW ? k : 0] : a.sw[sl];
                const T bo = PW ? own.bo[PW ? k : 0] : b_of(i, k);
                const T tv = fma_t(wk, v.y - nb(k), bo);
                const T dv = shrink(tv, a.gamma);
                const T bn = tv - dv;
                if (!a.bhalf || k < KC / 2) {
                    bwrite[sl * d + ln.c] = bn;
                    if (a.keep_split) a.ds[sl * d + ln.c] = dv;
                }
                accR = fma_t(wk, dv - bn, accR);
            }
            a.rhs[e] = fma_t(a.c_off, accR, own.split);
        });
}

// Learned-preconditioner PCG phases over a strip (the ph_la, ph_lc, ph_ld
// arithmetic; the stencil's slots [0, K/2) are a pixel's lower neighbours).
// LA: p = z + beta p, q = A p, partials of p.q
template <int KC, typename T>
__device__ __forceinline__ void st_la(const KA<T>& a, int lb, double* sh) {
    constexpr bool PW = KC <= 8;
    const StripGeo g = strip_geo(a.geo, lb);
    const int d = a.d;
    const StripLane ln(g, d, Sten<KC>::rho);
    const int it = ld_flag(&a.S->it);
    const bool first = (it == 0);
    T* pnew = a.sb[it & 1];
    const T* pold = a.sb[(it & 1) ^ 1];
    T* q = a.wb[0];
    const T beta = (T)a.cs.beta[a.blk_seg[lb] * d + ln.c];
    struct Raw { T z, po; };
    struct Own { T dA, ww[PW ? KC : 1]; };
    auto p_of = [&](const Raw& v) { return first ? v.z : fma_t(beta, v.po, v.z); };
    double acc1[1] = {0.0};
    strip_walk<KC>(a, g, ln, reinterpret_cast<T*>(sh),
        [&](int, size_t e) { return Raw{a.zl[e], pold[e]}; },
        p_of,
        [&](int i, size_t) {
            Own o{};
            o.dA = a.diagA[i];
            if constexpr (PW) {
#pragma unroll
                for (int k = 0; k < KC; ++k) o.ww[k] = a.sw[(size_t)k * a.n + i];
            }
            return o;
        },
        [&](int i, size_t e, const Raw& v, const Own& own, auto&& nb) {
            const T pi = p_of(v);
            T acc = T(0);
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                const T wk = PW ? own.ww[PW ? k : 0] : a.sw[(size_t)k * a.n + i];
                acc = fma_t(mul_t(wk, wk), nb(k), acc);
            }
            const T qi = fma_t(own.dA, pi, -mul_t(a.c_off, acc));
            pnew[e] = pi;
            q[e] = qi;
            acc1[0] += (double)pi * (double)qi;
        });
    block_partials<1>(acc1, sh, d, kBlock / d, a.part, a.nblk, lb);
}

// LC: x += alpha p, r' = r - alpha q (own pixels), y1 = Gt D_A^{-1/2} r' over
// the lower neighbours (upd = 0: y1 from the initial residual, no update)
template <int KC, typename T>
__device__ __forceinline__ void st_lc(const KA<T>& a, int lb, double* sh, int upd) {
    constexpr int H = KC / 2;
    const StripGeo g = strip_geo(a.geo, lb);
    const int d = a.d;
    const StripLane ln(g, d, Sten<KC>::rho);
    const int it = upd ? ld_flag(&a.S->it) : 0;
    const T* r = a.rb[it & 1];
    T* rn = a.rb[(it & 1) ^ 1];
    const T* p = a.sb[it & 1];
    const T* q = a.wb[0];
    const T alpha = upd ? (T)a.cs.alpha[a.blk_seg[lb] * d + ln.c] : T(0);
    struct Raw { T r, q, isq; };
    struct Own { T x, p, gd, gv[H]; };
    auto rv_of = [&](const Raw& v) { return upd ? fma_t(-alpha, v.q, v.r) : v.r; };
    strip_walk<KC>(a, g, ln, reinterpret_cast<T*>(sh),
        [&](int j, size_t e) { return Raw{r[e], upd ? q[e] : T(0), a.isq[j]}; },
        [&](const Raw& v) { return mul_t(v.isq, rv_of(v)); },
        [&](int i, size_t e) {
            Own o{};
            if (upd) {
                o.x = a.x[e];
                o.p = p[e];
            }
            o.gd = a.gdiag[i];
#pragma unroll
            for (int k = 0; k < H; ++k) o.gv[k] = a.gval[(size_t)k * a.n + i];
            return o;
        },
        [&](int, size_t e, const Raw& v, const Own& own, auto&& nb) {
            const T ri = rv_of(v);
            if (upd) {
                a.x[e] = fma_t(alpha, own.p, own.x);
                rn[e] = ri;
            }
            T acc = mul_t(own.gd, mul_t(v.isq, ri));
#pragma unroll
            for (int k = 0; k < H; ++k) acc = fma_t(own.gv[k], nb(k), acc);
            a.y1[e] = acc;
        });
}

// LD: z = D_A^{-1/2} Gt^T y1 over the upper neighbours, partials of r'.z, r'.r'
template <int KC, typename T>
__device__ __forceinline__ void st_ld(const KA<T>& a, int lb, double* sh, int initial) {
    constexpr int H = KC / 2;
    const StripGeo g = strip_geo(a.geo, lb);
    const int d = a.d;
    const StripLane ln(g, d, Sten<KC>::rho);
    const T* r = initial ? a.rb[0] : a.rb[(ld_flag(&a.S->it) & 1) ^ 1];
    struct Raw { T y1; };
    struct Own { T r, isq, gd, gv[KC - H]; };
    double acc2[2] = {0.0, 0.0};
    strip_walk<KC>(a, g, ln, reinterpret_cast<T*>(sh),
        [&](int, size_t e) { return Raw{a.y1[e]}; },
        [&](const Raw& v) { return v.y1; },
        [&](int i, size_t e) {
            Own o{};
            o.r = r[e];
            o.isq = a.isq[i];
            o.gd = a.gdiag[i];
#pragma unroll
            for (int k = H; k < KC; ++k) o.gv[k - H] = a.gval[(size_t)k * a.n + i];
            return o;
        },
        [&](int, size_t e, const Raw& v, const Own& own, auto&& nb) {
            T acc = mul_t(own.gd, v.y1);
#pragma unroll
            for (int k = H; k < KC; ++k) acc = fma_t(own.gv[k - H], nb(k), acc);
            const T z = mul_t(own.isq, acc);
            a.zl[e] = z;
            acc2[0] += (double)own.r * (double)z;
            acc2[1] += (double)own.r * (double)own.r;
        });
    block_partials<2>(acc2, sh, d, kBlock / d, a.part, a.nblk, lb);
}

// Factor-preconditioned CG in Chronopoulos-Gear form, one pass per
// iteration over a strip whose ring rows span three stencil radii on each
// side.  With M^{-1} = D_A^{-1/2} Gt^T Gt D_A^{-1/2}, iteration i updates
//   p = u + beta p, s = w + beta s, x += alpha p, r' = r - alpha s,
// forms u' = M^{-1} r' and w' = A u', and the partials of r'.u', w'.u', r'.r'
// (the same scalars and finaliser as the Jacobi iteration).  Per image row Y
// of the walk: publish D_A^{-1/2} r' of row Y (ring A), barrier, y1 = Gt
// D_A^{-1/2} r' of row Y over the lower neighbours (ring B), barrier,
// u' = D_A^{-1/2} Gt^T y1 of row Y - rho over the upper neighbours (ring C),
// barrier, then the owned pixels of row Y - 2 rho: w' = A u' from ring C and
// the vector updates.  r', y1 and u' of the halo pixels are formed from the
// neighbours' stored r, w, s with the arithmetic their owners use, so every
// value is the one the owner stores.  mode 0 (before the first iteration):
// r' = r0, u0 = M^{-1} r0, w0 = A u0 and the partials of r0.u0, w0.u0 (the
// w0-phase finaliser); nothing else is written.
template <int KC, typename T, int CPL>
struct FcgRings {
    static constexpr int rho = Sten<KC>::rho;
    static constexpr int na = rho + 1, nb = rho + 1, nc = 2 * rho + 1;
    static constexpr int rows = na + nb + nc;
    static constexpr int row_len = kBlock * CPL;   // elements of one ring row
    // LDS doubles: the three rings, or the partial sums and the finaliser's
    // scratch after the walk (the size the other phases use)
    static constexpr int ring_doubles = rows * row_len * (int)sizeof(T) / 8;
    static constexpr int doubles = ring_doubles > kSmemDoubles ? ring_doubles : kSmemDoubles;
};

// CPL consecutive values of a lane (CPL columns of one pixel), loaded and
// stored as one vector access
template <typename T, int CPL>
struct Lane { T v[CPL]; };
template <typename T, int CPL>
__device__ __forceinline__ Lane<T, CPL> ld_lane(const T* p) {
    Lane<T, CPL> o;
    if constexpr (CPL == 2) {
        typedef T V2 __attribute__((ext_vector_type(2)));
        const V2 x = *reinterpret_cast<const V2*>(p);
        o.v[0] = x[0];
        o.v[1] = x[1];
    } else {
#pragma unroll
        for (int j = 0; j < CPL; ++j) o.v[j] = p[j];
    }
    return o;
}
template <typename T, int CPL>
__device__ __forceinline__ void st_lane(T* p, const Lane<T, CPL>& o) {
    if constexpr (CPL == 2) {
        typedef T V2 __attribute__((ext_vector_type(2)));
        V2 x;
        x[0] = o.v[0];
        x[1] = o.v[1];
        *reinterpret_cast<V2*>(p) = x;
    } else {
#pragma unroll
        for (int j = 0; j < CPL; ++j) p[j] = o.v[j];
    }
}

// per-thread FP64 accumulators of CPL columns -> one partial per (quantity,
// column) per workgroup; lane t holds columns (t mod (d / CPL)) CPL + j of
// pixel t / (d / CPL); the sums over the pixels run in pixel order
template <int NQ, int CPL>
__device__ __forceinline__ void block_partials_cpl(const double (&acc)[NQ][CPL], double* sh, int d, double* part,
                                                   int nblk, int lb) {
    const int t = threadIdx.x;
    const int B = blockDim.x;
    const int dl = d / CPL;
    const int npx = B / dl;                  // pixels per workgroup row
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int j = 0; j < CPL; ++j) sh[q * B * CPL + t * CPL + j] = (t < npx * dl) ? acc[q][j] : 0.0;
    __syncthreads();
    if (t < NQ * d) {
        const int q = t / d, c = t - q * d;
        double s = 0.0;
        for (int k = 0; k < npx; ++k) s += sh[q * B * CPL + k * d + c];
        part[((size_t)q * nblk + lb) * d + c] = s;
    }
    __syncthreads();
}

template <int KC, int CPL, typename T>
__device__ __forceinline__ void st_fcg(const KA<T>& a, int lb, double* sh, int mode) {
    using S = Sten<KC>;
    using FR = FcgRings<KC, T, CPL>;
    using L = Lane<T, CPL>;
    constexpr int rho = S::rho, H = KC / 2, RL = FR::row_len;
    const StripGeo g = strip_geo(a.geo, lb);
    const int d = a.d, t = threadIdx.x, dl = d / CPL;
    const int qx = t / dl, c0 = (t - qx * dl) * CPL;   // pixel column of the lane, its first column
    const int lt = qx * d + c0;                        // the lane's first element in a ring row
    const int px = g.x0 - 3 * rho + qx;
    const bool loader = qx < g.len + 6 * rho;
    const bool in_image = loader && px >= 0 && px < g.W;
    const bool blane = in_image && qx >= rho && qx < g.len + 5 * rho;        // forms y1
    const bool clane = in_image && qx >= 2 * rho && qx < g.len + 4 * rho;    // forms u'
    const bool owner = qx >= 3 * rho && qx < g.len + 3 * rho;
    const bool iter = mode != 0;
    const int it = iter ? ld_flag(&a.S->it) : 0;
    const bool first = (it == 0);
    const int cur = it & 1, nxt = cur ^ 1;
    const T* r = a.rb[cur];
    const T* w = a.wb[cur];
    const T* sp = a.sb[cur];
    T* rn = a.rb[nxt];
    T* wn = iter ? a.wb[nxt] : a.wb[0];
    T* sn = a.sb[nxt];
    const int ci = a.blk_seg[lb] * d + c0;
    T alpha[CPL], beta[CPL];
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
        alpha[j] = iter ? (T)a.cs.alpha[ci + j] : T(0);
        beta[j] = iter ? (T)a.cs.beta[ci + j] : T(0);
    }
    T* ringA = reinterpret_cast<T*>(sh);             // D_A^{-1/2} r'
    T* ringB = ringA + FR::na * RL;                  // y1
    T* ringC = ringB + FR::nb * RL;                  // u'
    auto sa = [](int y) { return (y + 8 * FR::na) % FR::na; };
    auto sb_ = [](int y) { return (y + 8 * FR::nb) % FR::nb; };
    auto sc = [](int y) { return (y + 8 * FR::nc) % FR::nc; };
    struct Raw { L r, w, sp; T isq; };
    struct MidB { T gd, gv[H]; };
    struct MidC { T gd, isq, gv[KC - H]; };
    struct Own { Raw v; L p, x, u; T dA, ww[KC]; };
    const int yA0 = max(0, g.y0 - 2 * rho), yA1 = min(g.H, g.y1 + 2 * rho);   // rows of r' read
    auto ldr = [&](int y) {
        Raw v{};
        if (in_image && y >= yA0 && y < yA1) {
            const int j = g.row0 + y * g.W + px;
            const size_t e = (size_t)j * d + c0;
            v.r = ld_lane<T, CPL>(r + e);
            if (iter) {
                v.w = ld_lane<T, CPL>(w + e);
                if (!first) v.sp = ld_lane<T, CPL>(sp + e);
            }
            v.isq = a.isq[j];
        }
        return v;
    };
    auto ldb = [&](int y) {
        MidB m{};
        if (blane && y >= max(0, g.y0 - rho) && y < yA1) {
            const int j = g.row0 + y * g.W + px;
            m.gd = a.gdiag[j];
#pragma unroll
            for (int k = 0; k < H; ++k) m.gv[k] = a.gval[(size_t)k * a.n + j];
        }
        return m;
    };
    auto ldc = [&](int y) {
        MidC m{};
        if (clane && y >= max(0, g.y0 - rho) && y < min(g.H, g.y1 + rho)) {
            const int j = g.row0 + y * g.W + px;
            m.gd = a.gdiag[j];
            m.isq = a.isq[j];
#pragma unroll
            for (int k = H; k < KC; ++k) m.gv[k - H] = a.gval[(size_t)k * a.n + j];
        }
        return m;
    };
    // an owner's values of its pixel, its r, w, s included (loaded again
    // rather than carried through the rows of the walk, to keep registers)
    auto ldo = [&](int y) {
        Own o{};
        if (owner && y >= g.y0 && y < g.y1) {
            const int i = g.row0 + y * g.W + px;
            const size_t e = (size_t)i * d + c0;
            o.v.r = ld_lane<T, CPL>(r + e);
            if (iter) {
                o.v.w = ld_lane<T, CPL>(w + e);
                if (!first) o.v.sp = ld_lane<T, CPL>(sp + e);
                o.x = ld_lane<T, CPL>(a.x + e);
                o.u = ld_lane<T, CPL>(a.zl + e);
                if (!first) o.p = ld_lane<T, CPL>(a.p + e);
            }
            o.dA = a.diagA[i];
#pragma unroll
            for (int k = 0; k < KC; ++k) o.ww[k] = a.sw[(size_t)k * a.n + i];
        }
        return o;
    };
    // s and r' of a lane's pixel from its raw values (the owners' arithmetic)
    auto s_of = [&](const Raw& v, int j) { return cg_s(first, beta[j], v.sp.v[j], v.w.v[j]); };
    auto rp_of = [&](const Raw& v, int j) { return iter ? cg_r(alpha[j], s_of(v, j), v.r.v[j]) : v.r.v[j]; };
    double acc[3][CPL];
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int j = 0; j < CPL; ++j) acc[q][j] = 0.0;
    if (g.len > 0 && g.y1 > g.y0) {
        const int Yb = g.y0 - 2 * rho, Ye = g.y1 + 2 * rho;
        // every value a step uses is loaded one step ahead (the raw values two)
        Raw raw = ldr(Yb), rnext1 = ldr(Yb + 1);   // rows Y and Y + 1
        MidB mb = ldb(Yb);
        MidC mc = ldc(Yb - rho);
        Own own = ldo(Yb - 2 * rho);
        for (int Y = Yb; Y < Ye; ++Y) {
            const Raw rnext = ldr(Y + 2);
            const MidB mbn = ldb(Y + 1);
            const MidC mcn = ldc(Y + 1 - rho);
            const Own ownn = ldo(Y + 1 - 2 * rho);
            // A: publish D_A^{-1/2} r' of row Y (zero outside the image)
            if (loader) {
                L pa;
#pragma unroll
                for (int j = 0; j < CPL; ++j) pa.v[j] = mul_t(raw.isq, rp_of(raw, j));
                st_lane<T, CPL>(ringA + sa(Y) * RL + lt, pa);
            }
            __syncthreads();
            // B: y1 of row Y
            if (loader) {
                L y1{};
                if (blane && Y >= 0 && Y < g.H && Y >= g.y0 - rho) {
                    const L a0 = ld_lane<T, CPL>(ringA + sa(Y) * RL + lt);
#pragma unroll
                    for (int j = 0; j < CPL; ++j) y1.v[j] = mul_t(mb.gd, a0.v[j]);
#pragma unroll
                    for (int k = 0; k < H; ++k) {
                        const L an = ld_lane<T, CPL>(ringA + sa(Y + S::dy(k)) * RL + lt + S::dx(k) * d);
#pragma unroll
                        for (int j = 0; j < CPL; ++j) y1.v[j] = fma_t(mb.gv[k], an.v[j], y1.v[j]);
                    }
                }
                st_lane<T, CPL>(ringB + sb_(Y) * RL + lt, y1);
            }
            __syncthreads();
            // C: u' of row Y - rho
            const int Yc = Y - rho;
            if (loader && Yc >= g.y0 - rho) {
                L u{};
                if (clane && Yc >= 0 && Yc < g.H) {
                    const L b0 = ld_lane<T, CPL>(ringB + sb_(Yc) * RL + lt);
                    T accg[CPL];
#pragma unroll
                    for (int j = 0; j < CPL; ++j) accg[j] = mul_t(mc.gd, b0.v[j]);
#pragma unroll
                    for (int k = H; k < KC; ++k) {
                        const L bn = ld_lane<T, CPL>(ringB + sb_(Yc + S::dy(k)) * RL + lt + S::dx(k) * d);
#pragma unroll
                        for (int j = 0; j < CPL; ++j) accg[j] = fma_t(mc.gv[k - H], bn.v[j], accg[j]);
                    }
#pragma unroll
                    for (int j = 0; j < CPL; ++j) u.v[j] = mul_t(mc.isq, accg[j]);
                }
                st_lane<T, CPL>(ringC + sc(Yc) * RL + lt, u);
            }
            __syncthreads();
            // D: the owned pixels of row Y - 2 rho
            const int Yd = Y - 2 * rho;
            if (owner && Yd >= g.y0 && Yd < g.y1) {
                const int i = g.row0 + Yd * g.W + px;
                const size_t e = (size_t)i * d + c0;
                const L un = ld_lane<T, CPL>(ringC + sc(Yd) * RL + lt);
                T accA[CPL];
#pragma unroll
                for (int j = 0; j < CPL; ++j) accA[j] = T(0);
#pragma unroll
                for (int k = 0; k < KC; ++k) {
                    const T w2 = mul_t(own.ww[k], own.ww[k]);
                    const L cn = ld_lane<T, CPL>(ringC + sc(Yd + S::dy(k)) * RL + lt + S::dx(k) * d);
#pragma unroll
                    for (int j = 0; j < CPL; ++j) accA[j] = fma_t(w2, cn.v[j], accA[j]);
                }
                const Raw& v = own.v;
                L wnew, pi, si, ri, xn;
#pragma unroll
                for (int j = 0; j < CPL; ++j) {
                    wnew.v[j] = fma_t(own.dA, un.v[j], -mul_t(a.c_off, accA[j]));
                    if (iter) {
                        si.v[j] = s_of(v, j);
                        ri.v[j] = cg_r(alpha[j], si.v[j], v.r.v[j]);
                        pi.v[j] = first ? own.u.v[j] : fma_t(beta[j], own.p.v[j], own.u.v[j]);
                        xn.v[j] = fma_t(alpha[j], pi.v[j], own.x.v[j]);
                        acc[0][j] += (double)ri.v[j] * (double)un.v[j];
                        acc[2][j] += (double)ri.v[j] * (double)ri.v[j];
                    } else {
                        acc[0][j] += (double)v.r.v[j] * (double)un.v[j];
                    }
                    acc[1][j] += (double)wnew.v[j] * (double)un.v[j];
                }
                if (iter) {
                    st_lane<T, CPL>(a.p + e, pi);
                    st_lane<T, CPL>(sn + e, si);
                    st_lane<T, CPL>(a.x + e, xn);
                    st_lane<T, CPL>(rn + e, ri);
                }
                st_lane<T, CPL>(a.zl + e, un);
                st_lane<T, CPL>(wn + e, wnew);
            }
            raw = rnext1;
            rnext1 = rnext;
            mb = mbn;
            mc = mcn;
            own = ownn;
        }
    }
    __syncthreads();
    if (iter) {
        block_partials_cpl<3, CPL>(acc, sh, d, a.part, a.nblk, lb);
    } else {
        double acc2[2][CPL];
#pragma unroll
        for (int j = 0; j < CPL; ++j) { acc2[0][j] = acc[0][j]; acc2[1][j] = acc[1][j]; }
        block_partials_cpl<2, CPL>(acc2, sh, d, a.part, a.nblk, lb);
    }
}

// LC and LD fused (the ph_lc + ph_ld arithmetic) over a strip whose ring rows
// span two stencil radii on each side: x += alpha p and r' = r - alpha q on the
// owned pixels; y1 = Gt D_A^{-1/2} r' over the lower neighbours for every pixel
// within one radius of the strip, formed into a second LDS ring (not stored);
// z = D_A^{-1/2} Gt^T y1 over the upper neighbours on the owned pixels, with
// the partials of r'.z and r'.r' (upd = 0: from the initial residual).  Per
// image row y: publish isq r' of row y + rho, barrier, y1 of row y + rho,
// barrier, z of row y.
template <int KC, typename T>
__device__ __forceinline__ void st_lcd(const KA<T>& a, int lb, double* sh, int upd) {
    using S = Sten<KC>;
    constexpr int rho = S::rho, H = KC / 2, NS = rho + 2;
    const StripGeo g = strip_geo(a.geo, lb);
    const int d = a.d, t = threadIdx.x;
    const int qx = t / d, c = t - qx * d;
    const int span = g.len + 4 * rho;
    const int px = g.x0 - 2 * rho + qx;
    const bool loader = qx < span;
    const bool in_image = loader && px >= 0 && px < g.W;
    const bool mid = in_image && qx >= rho && qx < g.len + 3 * rho;   // forms y1 of its pixel
    const bool owner = qx >= 2 * rho && qx < g.len + 2 * rho;
    const int it = upd ? ld_flag(&a.S->it) : 0;
    const T* r = a.rb[it & 1];
    T* rn = a.rb[(it & 1) ^ 1];
    const T* p = a.sb[it & 1];
    const T* q = a.wb[0];
    const T alpha = upd ? (T)a.cs.alpha[a.blk_seg[lb] * d + c] : T(0);
    T* ringA = reinterpret_cast<T*>(sh);   // isq r'
    T* ringB = ringA + NS * kBlock;        // y1
    auto slot = [](int y) { return (y + 4 * NS) % NS; };
    const int ylo = max(0, g.y0 - rho), yhi = min(g.H, g.y1 + rho);    // rows of r' the strip reads
    struct Raw { T r, q, isq; };
    struct Mid { T gd, gv[H]; };
    struct Own { T x, p, gd, gv[KC - H]; };
    auto ldr = [&](int y) {
        Raw v{};
        if (in_image && y >= ylo && y < yhi) {
            const int j = g.row0 + y * g.W + px;
            const size_t e = (size_t)j * d + c;
            v.r = r[e];
            v.q = upd ? q[e] : T(0);
            v.isq = a.isq[j];
        }
        return v;
    };
    auto ldm = [&](int y) {
        Mid m{};
        if (mid && y < min(g.H, g.y1 + rho)) {
            const int j = g.row0 + y * g.W + px;
            m.gd = a.gdiag[j];
#pragma unroll
            for (int k = 0; k < H; ++k) m.gv[k] = a.gval[(size_t)k * a.n + j];
        }
        return m;
    };
    auto ldo = [&](int y) {
        Own o{};
        if (owner && y < g.y1) {
            const int i = g.row0 + y * g.W + px;
            const size_t e = (size_t)i * d + c;
            if (upd) {
                o.x = a.x[e];
                o.p = p[e];
            }
            o.gd = a.gdiag[i];
#pragma unroll
            for (int k = H; k < KC; ++k) o.gv[k - H] = a.gval[(size_t)k * a.n + i];
        }
        return o;
    };
    auto rv_of = [&](const Raw& v) { return upd ? fma_t(-alpha, v.q, v.r) : v.r; };
    // y1 of this lane's pixel at image row y (ring A holds rows y - rho .. y)
    auto y1_of = [&](int y, const Mid& m) {
        T acc = mul_t(m.gd, ringA[slot(y) * kBlock + t]);
#pragma unroll
        for (int k = 0; k < H; ++k) acc = fma_t(m.gv[k], ringA[slot(y + S::dy(k)) * kBlock + t + S::dx(k) * d], acc);
        return acc;
    };
    double acc2[2] = {0.0, 0.0};
    if (g.len > 0 && g.y1 > g.y0) {
        Raw raw[rho + 1];   // rows y .. y + rho of this lane
        // prime ring A with rows y0 - rho .. y0 + rho - 1 and ring B with rows y0 .. y0 + rho - 1
#pragma unroll
        for (int k = 1; k <= rho; ++k)
            if (loader) { const Raw v = ldr(g.y0 - k); ringA[slot(g.y0 - k) * kBlock + t] = mul_t(v.isq, rv_of(v)); }
#pragma unroll
        for (int k = 0; k <= rho; ++k) raw[k] = ldr(g.y0 + k);
#pragma unroll
        for (int k = 0; k < rho; ++k)
            if (loader) ringA[slot(g.y0 + k) * kBlock + t] = mul_t(raw[k].isq, rv_of(raw[k]));
        __syncthreads();
#pragma unroll
        for (int k = 0; k < rho; ++k) {
            const Mid m = ldm(g.y0 + k);
            if (loader) ringB[slot(g.y0 + k) * kBlock + t] = (mid && g.y0 + k < g.H) ? y1_of(g.y0 + k, m) : T(0);
        }
        __syncthreads();   // the first row overwrites a ring-A row the priming read
        Mid mcur = ldm(g.y0 + rho);
        Own own = ldo(g.y0);
        for (int y = g.y0; y < g.y1; ++y) {
            if (loader) ringA[slot(y + rho) * kBlock + t] = mul_t(raw[rho].isq, rv_of(raw[rho]));
            const Raw rnext = ldr(y + rho + 1);
            const Mid mnext = ldm(y + rho + 1);
            const Own onext = ldo(y + 1);
            __syncthreads();
            if (loader) ringB[slot(y + rho) * kBlock + t] = (mid && y + rho < g.H) ? y1_of(y + rho, mcur) : T(0);
            __syncthreads();
            if (owner) {
                const int i = g.row0 + y * g.W + px;
                const size_t e = (size_t)i * d + c;
                const T ri = rv_of(raw[0]);
                if (upd) {
                    a.x[e] = fma_t(alpha, own.p, own.x);
                    rn[e] = ri;
                }
                T acc = mul_t(own.gd, ringB[slot(y) * kBlock + t]);
#pragma unroll
                for (int k = H; k < KC; ++k)
                    acc = fma_t(own.gv[k - H], ringB[slot(y + S::dy(k)) * kBlock + t + S::dx(k) * d], acc);
                const T z = mul_t(raw[0].isq, acc);
                a.zl[e] = z;
                acc2[0] += (double)ri * (double)z;
                acc2[1] += (double)ri * (double)ri;
            }
#pragma unroll
            for (int k = 0; k < rho; ++k) raw[k] = raw[k + 1];
            raw[rho] = rnext;
            mcur = mnext;
            own = onext;
        }
    }
    __syncthreads();
    block_partials<2>(acc2, sh, d, kBlock / d, a.part, a.nblk, lb);
}

// ---------------------------------------------------------------------------
// Finalisers (one workgroup, after every workgroup has written its partials).
// 'grouped' means the per-XCD-group partials are already summed (one segment).
// ---------------------------------------------------------------------------

// after a residual phase: ||rhs||^2, ||r0||^2, convergence at iteration 0
template <typename T>
__device__ __forceinline__ void fin_res(const KA<T>& a, double* sh, bool grouped) {
    const int d = a.d;
    double* out = sh + 1024;
    __shared__ int s_any;
    if (threadIdx.x == 0) s_any = 0;
    const int chunk = seg_chunk(2, d);
    for (int sg0 = 0; sg0 < a.nseg; sg0 += chunk) {
        const int ns = min(chunk, a.nseg - sg0);
        seg_sums_all(a, sg0, ns, 2, out, sh, grouped);
        for (int idx = threadIdx.x; idx < ns * d; idx += blockDim.x) {
            const int k = idx / d, c = idx - k * d, ci = (sg0 + k) * d + c;
            const double* o = out + k * 2 * d;
            double bb = o[c], rr = o[d + c];
            a.cs.bnorm2[ci] = bb;
            a.cs.rr[ci] = rr;
            a.cs.iters[ci] = 0;
            a.cs.alpha[ci] = 0.0;
            a.cs.beta[ci] = 0.0;
            int z = (bb == 0.0);
            a.cs.zero[ci] = z;
            int act = !z && (rr > a.tol2 * bb);
            a.cs.active[ci] = act;
            if (act) atomicOr(&s_any, 1);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.S->it = 0;
        a.S->done = !s_any;
    }
}

// after PH_W0: alpha0 = gamma0 / delta0
template <typename T>
__device__ __forceinline__ void fin_w0(const KA<T>& a, double* sh, bool grouped) {
    const int d = a.d;
    double* out = sh + 1024;
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    const int chunk = seg_chunk(2, d);
    for (int sg0 = 0; sg0 < a.nseg; sg0 += chunk) {
        const int ns = min(chunk, a.nseg - sg0);
        seg_sums_all(a, sg0, ns, 2, out, sh, grouped);
        for (int idx = threadIdx.x; idx < ns * d; idx += blockDim.x) {
            const int k = idx / d, c = idx - k * d, ci = (sg0 + k) * d + c;
            const double* o = out + k * 2 * d;
            double g = o[c], dl = o[d + c];
            a.cs.gamma[ci] = g;
            double al = 0.0;
            if (a.cs.active[ci]) {
                al = g / dl;
                if (!(dl > 0.0) || !(g > 0.0) || !isfinite(al)) { s_bad = 1; al = 0.0; }
            }
            a.cs.alpha[ci] = al;
            a.cs.beta[ci] = 0.0;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && s_bad) {
        a.S->status = PFE_E_NOT_SPD;
        a.S->done = 1;
    }
}

// after PH_IT: convergence, beta, alpha of the next iteration, statistics
template <typename T>
__device__ __forceinline__ void fin_it(const KA<T>& a, double* sh, bool grouped) {
    const int d = a.d;
    double* out = sh + 1024;
    __shared__ int s_any, s_bad;
    if (threadIdx.x == 0) { s_any = 0; s_bad = 0; }
    const int chunk = seg_chunk(3, d);
    for (int sg0 = 0; sg0 < a.nseg; sg0 += chunk) {
        const int ns = min(chunk, a.nseg - sg0);
        seg_sums_all(a, sg0, ns, 3, out, sh, grouped);
        for (int idx = threadIdx.x; idx < ns * d; idx += blockDim.x) {
            const int k = idx / d, c = idx - k * d, ci = (sg0 + k) * d + c;
            const double* o = out + k * 3 * d;
            int act = a.cs.active[ci];
            if (act) {
                double g = o[c], dl = o[d + c], rr = o[2 * d + c];
                a.cs.iters[ci] += 1;
                a.cs.rr[ci] = rr;
                act = rr > a.tol2 * a.cs.bnorm2[ci];
                if (!isfinite(rr)) { s_bad = 1; act = 0; }
                if (act) {
                    double be = g / a.cs.gamma[ci];
                    double den = dl - be * g / a.cs.alpha[ci];
                    double al = g / den;
                    if (!(den > 0.0) || !isfinite(al) || !isfinite(be)) { s_bad = 1; act = 0; al = 0.0; be = 0.0; }
                    a.cs.beta[ci] = be;
                    a.cs.alpha[ci] = al;
                    a.cs.gamma[ci] = g;
                }
            }
            if (!act) {
                a.cs.alpha[ci] = 0.0;
                a.cs.beta[ci] = 0.0;
            }
            a.cs.active[ci] = act;
            if (act) atomicOr(&s_any, 1);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int any = s_any;
        if (s_bad) a.S->status = PFE_E_NOT_SPD;
        int it = a.S->it + 1;
        a.S->it = it;
        if (any && it >= a.maxit) {
            if (a.S->status == 0) a.S->status = PFE_E_NOCONV;
            any = 0;
        }
        a.S->done = !any;
    }
}

// learned path, after PH_LD: initial (before the first iteration) or after an
// iteration: convergence on ||r||, beta = (r.z)_new / (r.z)_old
template <typename T>
__device__ __forceinline__ void fin_ld(const KA<T>& a, double* sh, bool initial, bool grouped = false) {
    const int d = a.d;
    double* out = sh + 1024;
    __shared__ int s_any, s_bad;
    if (threadIdx.x == 0) { s_any = 0; s_bad = 0; }
    const int chunk = seg_chunk(2, d);
    for (int sg0 = 0; sg0 < a.nseg; sg0 += chunk) {
        const int ns = min(chunk, a.nseg - sg0);
        seg_sums_all(a, sg0, ns, 2, out, sh, grouped);
        for (int idx = threadIdx.x; idx < ns * d; idx += blockDim.x) {
            const int k = idx / d, c = idx - k * d, ci = (sg0 + k) * d + c;
            const double* o = out + k * 2 * d;
            int act = a.cs.active[ci];
            double g = o[c], rr = o[d + c];
            if (initial) {
                a.cs.gamma[ci] = g;
                a.cs.beta[ci] = 0.0;
                if (act && !(g > 0.0)) { s_bad = 1; act = 0; }
            } else if (act) {
                a.cs.iters[ci] += 1;
                a.cs.rr[ci] = rr;
                act = rr > a.tol2 * a.cs.bnorm2[ci];
                if (!isfinite(rr)) { s_bad = 1; act = 0; }
                if (act) {
                    double be = g / a.cs.gamma[ci];
                    if (!isfinite(be)) { s_bad = 1; act = 0; be = 0.0; }
                    a.cs.beta[ci] = be;
                    a.cs.gamma[ci] = g;
                }
            }
            if (!act) { a.cs.alpha[ci] = 0.0; a.cs.beta[ci] = 0.0; }
            a.cs.active[ci] = act;
            if (act) atomicOr(&s_any, 1);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int any = s_any;
        if (s_bad) a.S->status = PFE_E_NOT_SPD;
        if (!initial) {
            int it = a.S->it + 1;
            a.S->it = it;
            if (any && it >= a.maxit) {
                if (a.S->status == 0) a.S->status = PFE_E_NOCONV;
                any = 0;
            }
        }
        a.S->done = !any;
    }
}

// learned path, after PH_LA: alpha = (r.z) / (p.q)
template <typename T>
__device__ __forceinline__ void fin_la(const KA<T>& a, double* sh, bool grouped = false) {
    const int d = a.d;
    double* out = sh + 1024;
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    const int chunk = seg_chunk(1, d);
    for (int sg0 = 0; sg0 < a.nseg; sg0 += chunk) {
        const int ns = min(chunk, a.nseg - sg0);
        seg_sums_all(a, sg0, ns, 1, out, sh, grouped);
        for (int idx = threadIdx.x; idx < ns * d; idx += blockDim.x) {
            const int k = idx / d, c = idx - k * d, ci = (sg0 + k) * d + c;
            double al = 0.0;
            if (a.cs.active[ci]) {
                double pq = out[k * d + c];
                al = a.cs.gamma[ci] / pq;
                if (!(pq > 0.0) || !isfinite(al)) { s_bad = 1; al = 0.0; }
            }
            a.cs.alpha[ci] = al;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && s_bad) {
        a.S->status = PFE_E_NOT_SPD;
        a.S->done = 1;
    }
}

// called by one thread when a solve ends: accumulate statistics
template <typename T>
__device__ __forceinline__ void solve_stats(const KA<T>& a) {
    int mx = 0;
    double rel = 0.0;
    for (int ci = 0; ci < a.nseg * a.d; ++ci) {
        mx = max(mx, a.cs.iters[ci]);
        double bb = a.cs.bnorm2[ci];
        if (bb > 0.0) rel = fmax(rel, sqrt(a.cs.rr[ci] / bb));
    }
    a.S->solves += 1;
    a.S->iters_total += mx;
    a.S->iters_max = max(a.S->iters_max, mx);
    a.S->iters_last = mx;
    a.S->relres_max = fmax(a.S->relres_max, rel);
}

// d x d factor of the P-update for segment sg, FP64, one workgroup.
//   G = Z^T Z (packed, in gsum), Cholesky G = L L^T (rank check),
//   CHOL / init: T = L^{-T}  (Z T = Z R^{-1}, R = L^T);
//   POLAR: T = G^{-1/2} by the coupled Newton-Schulz iteration on G / s,
//   s = ||G||_inf, so that Z T is the orthogonal polar factor of Z.
// The transform goes to Tout (row stride kMaxD); report: record a failure in
// the solver flags.  Returns false when G is not (numerically) positive
// definite.  LDS use: sh[1024, 4608).
template <typename T>
__device__ __forceinline__ bool factor_gram(const KA<T>& a, int mode, const double* gsum, double* sh, double* Tout,
                                            bool report, int da) {
    // da <= a.d: the segment's active columns (the leading block of G is
    // factored; T is zero outside it, so inactive columns of P and B stay zero)
    const int dfull = a.d, d = da, t = threadIdx.x, nb = blockDim.x;
    const int npair = dfull * (dfull + 1) / 2;
    double* G = sh + 1024;
    double* L = sh + 2048;
    double* Ym = sh + 3072;
    double* Zm = sh + 3072 + 512;
    double* red = sh + 4096;
    for (int k = t; k < npair; k += nb) {
        int r, cc;
        pair_of(k, dfull, r, cc);
        if (r < d && cc < d) {
            G[r * d + cc] = gsum[k];
            G[cc * d + r] = gsum[k];
        }
    }
    if (d < dfull)
        for (int k = t; k < dfull * dfull; k += nb) {
            const int r = k / dfull, cc = k - r * dfull;
            if (r >= d || cc >= d) Tout[r * kMaxD + cc] = 0.0;
        }
    __syncthreads();
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
        if (t == 0 && report) {
            a.S->ortho_ok = 0;
            a.S->status = PFE_E_RANK;
        }
        __syncthreads();
        return false;
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
            Tout[r * kMaxD + c] = Ym[c * kMaxD + r];
        }
        __syncthreads();
        return true;
    }
    // coupled Newton-Schulz for (G/s)^{-1/2}
    __shared__ double s_scale, s_err;
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
    const int dd = d * d;
    double* Yk = Ym;
    double* Zk = L;           // the Cholesky factor is no longer needed
    double* Mk = G;
    double* Wk = (dd > 512) ? sh : Zm;
    for (int k = t; k < dd; k += nb) {
        Yk[k] = G[k] / s;
        Zk[k] = ((k / d) == (k % d)) ? 1.0 : 0.0;
    }
    __syncthreads();
    double prev = INFINITY;
    for (int iter = 0; iter < 100; ++iter) {
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
        const double err = s_err;
        // stop at rounding level: tiny, or no longer shrinking quadratically
        if (err < 1e-14 || !isfinite(err) || (err < 1e-11 && err > 0.25 * prev)) break;
        prev = err;
        for (int k = t; k < dd; k += nb) {
            int i = k / d, j = k - i * d;
            Mk[k] = 0.5 * (((i == j) ? 3.0 : 0.0) - Wk[k]);
        }
        __syncthreads();
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
        Tout[r * kMaxD + c] = Zk[k] * is;
    }
    const bool ok = s_err < 1e-10;
    if (t == 0 && !ok && report) {
        a.S->ortho_ok = 0;
        a.S->status = PFE_E_RANK;
    }
    __syncthreads();
    return ok;
}

// Gram sum of segment sg (grouped: the per-XCD-group partials of the single
// segment) and its factor, written to Tout.
// (gp: the per-XCD-group partial buffer when grouped)
template <typename T>
__device__ __forceinline__ bool seg_factor(const KA<T>& a, int sg, int mode, double* sh, bool grouped, double* Tout,
                                           bool report, const double* gp = nullptr) {
    const int npair = a.d * (a.d + 1) / 2;
    __shared__ double gsum[kMaxD * (kMaxD + 1) / 2];
    if (grouped) reduce_range(gp, kNumXcd, 0, kNumXcd, npair, 1, gsum, sh);
    else reduce_range(a.part, a.nblk, a.seg_blk0[sg], a.seg_blk0[sg + 1], npair, 1, gsum, sh);
    return factor_gram(a, mode, gsum, sh, Tout, report, a.dact ? a.dact[sg] : a.d);
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

// Persistent path: two-level barrier over all co-resident workgroups.
// Workgroups arrive on the counter of their XCD group (blockIdx % 8, one
// 128-byte line each); the last of a group optionally pre-reduces the group's
// partials (gfin), then arrives on the top counter.  The counters only grow
// during a launch (the host clears them before it), so the k-th barrier of a
// launch is complete when a group counter reaches k times the group size and
// the top counter k times the group count.  Without a finaliser the top counter
// is the release: everybody polls it with relaxed loads (no cache
// invalidation per poll) and then acquires.  With a finaliser the last group
// leader runs fin() and then bumps the generation word the others poll.  The
// wait is bounded: after kSpinLimit polls a workgroup raises abort_flag and the
// kernel unwinds (every later barrier then times out quickly).
constexpr long long kSpinLimit = 1ll << 25;
constexpr int kBarGen = 0;          // bar[0]: generation
constexpr int kBarTop = 32;         // bar[32]: top counter
constexpr int kBarGroup = 64;       // bar[64 + 32 g]: group counters
constexpr int kBarLast = 448;       // bar[448]: last-workgroup counter of the multi-launch path

struct NoFin;

// nbar: barriers this workgroup has passed in the current launch (every
// workgroup passes the same sequence)
template <class GF, class F>
__device__ __forceinline__ bool grid_sync(unsigned* bar, unsigned nblk, Scal* S, unsigned& nbar, GF&& gfin, F&& fin) {
    constexpr bool kFin = !std::is_same<typename std::decay<F>::type, NoFin>::value;
    __shared__ int s_role;     // 0 waiter, 1 group leader, 2 finalising leader
    __shared__ int s_abort;
    const unsigned g = blockIdx.x % kNumXcd;
    const unsigned gsize = nblk / kNumXcd;
    const unsigned k1 = ++nbar;
    __syncthreads();
    unsigned gen = 0;
    if (threadIdx.x == 0) {
        s_abort = 0;
        if (kFin) gen = __hip_atomic_load(&bar[kBarGen], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned prev = __hip_atomic_fetch_add(&bar[kBarGroup + 32 * g], 1u, __ATOMIC_RELEASE,
                                               __HIP_MEMORY_SCOPE_AGENT);
        s_role = (prev == gsize * k1 - 1) ? 1 : 0;
        if (s_role) fence_acquire_agent();
    }
    __syncthreads();
    if (s_role == 1) {
        gfin(g);
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned prev = __hip_atomic_fetch_add(&bar[kBarTop], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            s_role = (kFin && prev == kNumXcd * k1 - 1) ? 2 : 0;
        }
        __syncthreads();
    }
    if (kFin && s_role == 2) {
        fin();
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(&bar[kBarGen], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        return true;
    }
    if (threadIdx.x == 0) {
        long long spins = 0;
        while (kFin ? (__hip_atomic_load(&bar[kBarGen], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen)
                    : (__hip_atomic_load(&bar[kBarTop], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < kNumXcd * k1)) {
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
    __syncthreads();
    return !s_abort;
}

struct NoFin {
    __device__ void operator()() const {}
    __device__ void operator()(unsigned) const {}
};

// group pre-reduction of nq quantities of m values each (single segment):
// gpart[(q * 8 + g) * m + c] = sum over the group's workgroups
template <typename T>
__device__ __forceinline__ void group_reduce(const KA<T>& a, unsigned g, int m, int nq, double* sh, double* gp) {
    const int gs = a.nblk / kNumXcd;
    double* out = sh + 1024;
    reduce_range(a.part, a.nblk, (int)g * gs, (int)(g + 1) * gs, m, nq, out, sh);
    for (int k = threadIdx.x; k < nq * m; k += blockDim.x) {
        int q = k / m, c = k - q * m;
        gp[((size_t)q * kNumXcd + g) * m + c] = out[k];
    }
    __syncthreads();
}

// One-launch-per-phase kernels, single segment, a grid of whole XCD groups: the
// workgroup partials are summed in two levels instead of by one workgroup alone.
// The last workgroup of each XCD group (logical workgroups [g gs, (g + 1) gs),
// the ones launched on XCD g) sums its group's partials in order into gpart;
// the last of the eight group leaders returns true and runs the finaliser on the
// eight group sums (grouped).  Each level reads only a group's worth of
// partials, with many loads in flight, where one workgroup summing every
// partial waits on a long chain of memory round trips.
constexpr int kBarLastGroup = 456;   // bar[456 + 4 g]: group counters of the multi-launch path

template <typename T>
__device__ __forceinline__ bool grouped_fin(const KA<T>& a) {
    return a.nseg == 1 && a.nblk >= 8 * kNumXcd && (a.nblk % kNumXcd) == 0;
}

template <typename T>
__device__ bool last_block_grouped(const KA<T>& a, int nq, double* sh) {
    __shared__ int s_last;
    const unsigned g = blockIdx.x % kNumXcd;
    const unsigned gs = (unsigned)a.nblk / kNumXcd;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned* ctr = a.bar + kBarLastGroup + 4 * g;
        unsigned prev = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = (prev == gs - 1);
        if (s_last) __hip_atomic_store(ctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (!s_last) return false;
    group_reduce(a, g, a.d, nq, sh, a.gpart);
    return last_block(a.bar + kBarLast, kNumXcd);
}

// the last workgroup of a one-launch-per-phase kernel (grouped: see above);
// the finaliser then reads gpart when grouped_fin(a), else part
template <typename T>
__device__ __forceinline__ bool last_of_launch(const KA<T>& a, int nq, double* sh) {
    return grouped_fin(a) ? last_block_grouped(a, nq, sh) : last_block(a.bar + kBarLast, a.nblk);
}

// ---------------------------------------------------------------------------
// Per-workgroup CG state (persistent kernel, single segment).  After each grid
// barrier every workgroup sums the eight per-XCD-group partials itself, in the
// same order, and advances its own LDS copy of the column scalars and
// convergence flags (the copies stay bitwise identical), so the barrier only
// counts arrivals and no finaliser runs between the last arrival and the
// release.  Workgroup 0 records the statistics.
// ---------------------------------------------------------------------------
struct LocState {
    double gamma[kMaxD], alpha[kMaxD], beta[kMaxD], bnorm2[kMaxD], rr[kMaxD];
    int iters[kMaxD], active[kMaxD], zero[kMaxD];
    int it, done, status, any_zero;
};

// per-XCD-group partial buffer of the k-th barrier of a launch (two buffers:
// a workgroup may still read one while the next barrier's leaders write the other)
constexpr int kGroupStride = kNumXcd * (kMaxD * (kMaxD + 1) / 2 > 3 * kMaxD ? kMaxD * (kMaxD + 1) / 2 : 3 * kMaxD);

// sum of the eight per-XCD-group partials of quantity q, column c, in group
// order (the loads are independent, so one memory round trip)
__device__ __forceinline__ double group_total(const double* gp, int d, int q, int c) {
    const double* p = gp + (size_t)q * kNumXcd * d + c;
    double v[kNumXcd];
#pragma unroll
    for (int g = 0; g < kNumXcd; ++g) v[g] = p[(size_t)g * d];
    double acc = 0.0;
#pragma unroll
    for (int g = 0; g < kNumXcd; ++g) acc += v[g];
    return acc;
}

// The local finalisations run on the first wave only (lane c owns column c,
// d <= 32 < 64): its lanes load the group partials, advance the column
// scalars and vote on the flags; one workgroup barrier publishes the result.
template <typename T>
__device__ __forceinline__ void lfin_res(const KA<T>& a, LocState& L, const double* gp, double*) {
    const int d = a.d, t = threadIdx.x;
    if (t < 64) {
        int act = 0, zr = 0;
        if (t < d) {
            const double bb = group_total(gp, d, 0, t), rr = group_total(gp, d, 1, t);
            L.bnorm2[t] = bb;
            L.rr[t] = rr;
            L.iters[t] = 0;
            L.alpha[t] = 0.0;
            L.beta[t] = 0.0;
            zr = (bb == 0.0);
            act = !zr && (rr > a.tol2 * bb);
            L.zero[t] = zr;
            L.active[t] = act;
        }
        const bool any = __any(act), anyz = __any(zr);
        if (t == 0) {
            L.it = 0;
            L.done = !any;
            L.any_zero = anyz;
        }
    }
    __syncthreads();
}

template <typename T>
__device__ __forceinline__ void lfin_w0(const KA<T>& a, LocState& L, const double* gp, double*) {
    const int d = a.d, t = threadIdx.x;
    if (t < 64) {
        int bad = 0;
        if (t < d) {
            const double g = group_total(gp, d, 0, t), dl = group_total(gp, d, 1, t);
            L.gamma[t] = g;
            double al = 0.0;
            if (L.active[t]) {
                al = g / dl;
                if (!(dl > 0.0) || !(g > 0.0) || !isfinite(al)) { bad = 1; al = 0.0; }
            }
            L.alpha[t] = al;
            L.beta[t] = 0.0;
        }
        const bool anybad = __any(bad);
        if (t == 0 && anybad) {
            L.status = PFE_E_NOT_SPD;
            L.done = 1;
        }
    }
    __syncthreads();
}

template <typename T>
__device__ __forceinline__ void lfin_it(const KA<T>& a, LocState& L, const double* gp, double*) {
    const int d = a.d, t = threadIdx.x;
    if (t < 64) {
        int act = 0, bad = 0;
        if (t < d) {
            act = L.active[t];
            if (act) {
                const double g = group_total(gp, d, 0, t), dl = group_total(gp, d, 1, t),
                             rr = group_total(gp, d, 2, t);
                L.iters[t] += 1;
                L.rr[t] = rr;
                act = rr > a.tol2 * L.bnorm2[t];
                if (!isfinite(rr)) { bad = 1; act = 0; }
                if (act) {
                    double be = g / L.gamma[t];
                    double den = dl - be * g / L.alpha[t];
                    double al = g / den;
                    if (!(den > 0.0) || !isfinite(al) || !isfinite(be)) { bad = 1; act = 0; al = 0.0; be = 0.0; }
                    L.beta[t] = be;
                    L.alpha[t] = al;
                    L.gamma[t] = g;
                }
            }
            if (!act) {
                L.alpha[t] = 0.0;
                L.beta[t] = 0.0;
            }
            L.active[t] = act;
        }
        const bool any = __any(act), anybad = __any(bad);
        if (t == 0) {
            bool more = any;
            if (anybad) L.status = PFE_E_NOT_SPD;
            const int it = L.it + 1;
            L.it = it;
            if (more && it >= a.maxit) {
                if (L.status == 0) L.status = PFE_E_NOCONV;
                more = false;
            }
            L.done = !more;
        }
    }
    __syncthreads();
}

// statistics of a finished solve from the local state (one thread)
template <typename T>
__device__ __forceinline__ void solve_stats_loc(const KA<T>& a, const LocState& L) {
    int mx = 0;
    double rel = 0.0;
    for (int c = 0; c < a.d; ++c) {
        mx = max(mx, L.iters[c]);
        if (L.bnorm2[c] > 0.0) rel = fmax(rel, sqrt(L.rr[c] / L.bnorm2[c]));
    }
    a.S->solves += 1;
    a.S->iters_total += mx;
    a.S->iters_max = max(a.S->iters_max, mx);
    a.S->iters_last = mx;
    a.S->relres_max = fmax(a.S->relres_max, rel);
    if (L.status != 0 && (a.S->status == 0 || L.status == PFE_E_NOT_SPD)) a.S->status = L.status;
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// One phase per launch (the one-launch-per-phase path): a kernel per phase, the
// row-gathering ones specialised on the ELL width KC; the last workgroup to
// finish runs the finaliser.

// residual family (PH_E0, PH_EU, PH_R0, PH_RHS in ph)
template <typename T, int KC>
__global__ void __launch_bounds__(kBlock) k_residual(KA<T> a, int ph, int do_r0) {
    __shared__ double sh[kSmemDoubles];
    const int lb = logical_block(a.nblk);
    ph_residual<KC>(a, lb, ph, do_r0, a.b_zero, a.bpar, sh);
    if (do_r0 && last_of_launch(a, 2, sh)) fin_res(a, sh, grouped_fin(a));
}

template <typename T, int KC>
__global__ void __launch_bounds__(kBlock) k_cg_w0(KA<T> a) {
    __shared__ double sh[kSmemDoubles];
    if (ld_flag(&a.S->done)) return;
    const int lb = logical_block(a.nblk);
    ph_w0<KC>(a, lb, sh);
    if (last_of_launch(a, 2, sh)) fin_w0(a, sh, grouped_fin(a));
}

template <typename T, int KC>
__global__ void __launch_bounds__(kBlock) k_cg_it(KA<T> a) {
    __shared__ double sh[kSmemDoubles];
    if (ld_flag(&a.S->done)) return;
    const int lb = logical_block(a.nblk);
    ph_it<KC>(a, lb, sh, ld_flag(&a.S->it), a.cs.alpha, a.cs.beta);
    if (last_of_launch(a, 3, sh)) {
        fin_it(a, sh, grouped_fin(a));
        if (threadIdx.x == 0 && a.S->done) solve_stats(a);
    }
}

// general layouts: the CG iteration in two passes
template <typename T>
__global__ void __launch_bounds__(kBlock) k_cg_ga(KA<T> a) {
    __shared__ double sh[kSmemDoubles];
    if (ld_flag(&a.S->done)) return;
    ph_ga(a, logical_block(a.nblk), sh, ld_flag(&a.S->it), a.cs.alpha, a.cs.beta);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_cg_gb(KA<T> a) {
    __shared__ double sh[kSmemDoubles];
    if (ld_flag(&a.S->done)) return;
    ph_gb(a, logical_block(a.nblk), sh);
    if (last_of_launch(a, 3, sh)) {
        fin_it(a, sh, grouped_fin(a));
        if (threadIdx.x == 0 && a.S->done) solve_stats(a);
    }
}

// strip kernels (pixel grids): the residual with r0, w0 and the CG iteration
template <typename T, int KC>
__global__ void __launch_bounds__(kBlock) k_st_res(KA<T> a, int ph) {
    __shared__ double sh[kSmemDoubles];
    const int lb = logical_block(a.nblk);
    st_res<KC>(a, lb, ph, sh);
    if (last_of_launch(a, 2, sh)) fin_res(a, sh, grouped_fin(a));
}

template <typename T, int KC>
__global__ void __launch_bounds__(kBlock) k_st_w0(KA<T> a) {
    __shared__ double sh[kSmemDoubles];
    if (ld_flag(&a.S->done)) return;
    const int lb = logical_block(a.nblk);
    st_w0<KC>(a, lb, sh);
    if (last_of_launch(a, 2, sh)) fin_w0(a, sh, grouped_fin(a));
}

template <typename T, int KC>
__global__ void __launch_bounds__(kBlock) k_st_it(KA<T> a) {
    __shared__ double sh[kSmemDoubles];
    if (ld_flag(&a.S->done)) return;
    const int lb = logical_block(a.nblk);
    st_it<KC>(a, lb, sh, ld_flag(&a.S->it), a.cs.alpha, a.cs.beta);
    if (last_of_launch(a, 3, sh)) {
        fin_it(a, sh, grouped_fin(a));
        if (threadIdx.x == 0 && a.S->done) solve_stats(a);
    }
}

template <typename T, int KC>
__global__ void __launch_bounds__(kBlock) k_st_eu(KA<T> a) {
    __shared__ double sh[kSmemDoubles];
    st_eu<KC>(a, logical_block(a.nblk), sh);
}

// V consecutive columns of one row as one 4-, 8- or 16-byte access: an aligned
// array of V elements (the loads and stores move the whole array; the lanes are
// plain array elements, so no element is written through a pointer of another type)
template <typename T, int V>
struct alignas(sizeof(T) * V) Lanes {
    T v[V];
};
template <typename T, int V>
__device__ __forceinline__ Lanes<T, V> ld_lanes(const T* p) { return *reinterpret_cast<const Lanes<T, V>*>(p); }
template <typename T, int V>
__device__ __forceinline__ void st_lanes(T* p, const Lanes<T, V>& x) { *reinterpret_cast<Lanes<T, V>*>(p) = x; }

// The stencil slots of the edge update for pixel i at (py, px) of a W x H
// image (GEO; otherwise the slot columns): b once per undirected edge (own
// slots kk < KC/2 stored by this pixel, the others read negated from the later
// neighbour), Eqs. 9-10 per slot, acc += w (d - b) in slot order.  With AX the
// same loop also sums w^2 y_j over the slots for A y, and both sums run in the
// visiting order (nothing is held: the registers go to the caller's residual).
template <typename T, int KC, int V, bool GEO, bool AX>
__device__ __forceinline__ void eu_stencil_slots(const KA<T>& a, int i, int c0, int py, int px, int W, int H,
                                                 const T* bread, T* bwrite, const Lanes<T, V>& yi,
                                                 Lanes<T, V>& acc, Lanes<T, V>& accA) {
    using VT = Lanes<T, V>;
    using S = Sten<KC>;
    constexpr int KH = KC / 2;
    constexpr int G = (KC < 8) ? KC : 8;   // slots whose loads are issued together
    const int d = a.d;
    // FP32: slots are visited in pairs, own slot m (the edge to an earlier
    // pixel, whose b this pixel stores) beside slot KC-1-m (the edge to a
    // later pixel, whose b that pixel stores at its slot m).  A pixel and
    // its later neighbour then read the shared b at the same point of their
    // loops, which keeps the second read in L2.  The sum over the slots
    // keeps the slot order: the later-pixel slots' weight and d - b are
    // held and added after the own slots.  FP64 (twice the registers per
    // value) visits the slots in order.
    constexpr bool kPair = sizeof(T) == 4;
    constexpr bool kHold = kPair && !AX;      // later-pixel slots held for the slot-order sum
    constexpr int GP = G / 2;                 // pairs whose loads are issued together
    static_assert(!kPair || KH % GP == 0, "pair groups must tile the own slots");
    auto slot_of = [&](int g, int h) {
        return kPair ? ((h < GP) ? g * GP + h : KC - 1 - (g * GP + h - GP)) : g * G + h;
    };
    T mw[KH];
    VT mdb[KH];
    auto group = [&](int g) {
        int jj[G];
        T ww[G];
        VT yj[G], bo[G];
        size_t ss[G];
#pragma unroll
        for (int h = 0; h < G; ++h) {
            const int kk = slot_of(g, h);
            const size_t sl = (size_t)kk * a.n + i;
            if constexpr (GEO) {
                const int yy = py + S::dy(kk), xx = px + S::dx(kk);
                jj[h] = (yy >= 0 && yy < H && xx >= 0 && xx < W) ? i + S::dy(kk) * W + S::dx(kk) : i;
            } else {
                jj[h] = a.scol[sl];
            }
            ww[h] = a.sw[sl];
            ss[h] = (kk < KH) ? sl : (size_t)(KC - 1 - kk) * a.n + jj[h];
            if (a.b_zero) {
#pragma unroll
                for (int u = 0; u < V; ++u) bo[h].v[u] = T(0);
            } else {
                bo[h] = ld_lanes<T, V>(bread + ss[h] * d + c0);
                if (kk >= KH) {
#pragma unroll
                    for (int u = 0; u < V; ++u) bo[h].v[u] = -bo[h].v[u];
                }
            }
        }
#pragma unroll
        for (int h = 0; h < G; ++h) yj[h] = ld_lanes<T, V>(a.Y + (size_t)jj[h] * d + c0);
#pragma unroll
        for (int h = 0; h < G; ++h) {
            const int kk = slot_of(g, h);
            VT bn, dn, db;
#pragma unroll
            for (int u = 0; u < V; ++u) {
                const T tv = fma_t(ww[h], yi.v[u] - yj[h].v[u], bo[h].v[u]);
                const T dv = shrink(tv, a.gamma);
                const T b1 = tv - dv;
                bn.v[u] = b1;
                dn.v[u] = dv;
                db.v[u] = dv - b1;
            }
            if constexpr (AX) {
                const T w2 = mul_t(ww[h], ww[h]);
#pragma unroll
                for (int u = 0; u < V; ++u) accA.v[u] = fma_t(w2, yj[h].v[u], accA.v[u]);
            }
            if (!kHold || kk < KH) {
#pragma unroll
                for (int u = 0; u < V; ++u) acc.v[u] = fma_t(ww[h], db.v[u], acc.v[u]);
            } else {
                mw[kk - KH] = ww[h];
                mdb[kk - KH] = db;
            }
            if (kk < KH) {
                st_lanes<T, V>(bwrite + ss[h] * d + c0, bn);
                if (a.keep_split) st_lanes<T, V>(a.ds + ss[h] * d + c0, dn);
            }
        }
    };
    if constexpr (AX) {
        // one group at a time (the caller's residual needs the registers that
        // unrolling the groups would take)
#pragma unroll 1
        for (int g = 0; g < KC / G; ++g) group(g);
    } else {
#pragma unroll
        for (int g = 0; g < KC / G; ++g) group(g);
    }
    if constexpr (kHold) {
#pragma unroll
        for (int m = 0; m < KH; ++m) {
#pragma unroll
            for (int u = 0; u < V; ++u) acc.v[u] = fma_t(mw[m], mdb[m].v[u], acc.v[u]);
        }
    }
}

// The slots of row i of the edge update on general layouts (ELL or CSR rows):
// b and d per slot, updated in place, Eqs. 9-10 per slot, acc += w (d - b) in
// slot order.  With AX the same loop also sums w^2 y_j in slot order (the
// residual kernel's order) for A y.
template <typename T, int V, bool AX>
__device__ __forceinline__ void eu_row_slots(const KA<T>& a, int i, int c0, const T* bread, T* bwrite,
                                             const Lanes<T, V>& yi, Lanes<T, V>& acc, Lanes<T, V>& accA) {
    using VT = Lanes<T, V>;
    const int d = a.d;
    int s0, cnt, st;
    row_slots<0>(a, i, s0, cnt, st);
    auto slot = [&](int sl, T w, const VT& yj, const VT& bo) {
        VT bn, dn;
#pragma unroll
        for (int u = 0; u < V; ++u) {
            const T tv = fma_t(w, yi.v[u] - yj.v[u], bo.v[u]);
            const T dv = shrink(tv, a.gamma);
            const T b1 = tv - dv;
            bn.v[u] = b1;
            dn.v[u] = dv;
            acc.v[u] = fma_t(w, dv - b1, acc.v[u]);
        }
        st_lanes<T, V>(bwrite + (size_t)sl * d + c0, bn);
        if (a.keep_split) st_lanes<T, V>(a.ds + (size_t)sl * d + c0, dn);
        if constexpr (AX) {
            const T w2 = mul_t(w, w);
#pragma unroll
            for (int u = 0; u < V; ++u) accA.v[u] = fma_t(w2, yj.v[u], accA.v[u]);
        }
    };
    // full groups of kRowGroup slots, then the rest one by one (slot order kept;
    // predicated last groups were slower)
    int k = 0;
    for (; k + kRowGroup <= cnt; k += kRowGroup) {
        T ww[kRowGroup];
        VT yj[kRowGroup], bo[kRowGroup];
#pragma unroll
        for (int g = 0; g < kRowGroup; ++g) {
            {
                const int sl = s0 + (k + g) * st;
                ww[g] = a.sw[sl];
                yj[g] = ld_lanes<T, V>(a.Y + (size_t)a.scol[sl] * d + c0);
                if (a.b_zero) {
#pragma unroll
                    for (int u = 0; u < V; ++u) bo[g].v[u] = T(0);
                } else {
                    bo[g] = ld_lanes<T, V>(bread + (size_t)sl * d + c0);
                }
            }
        }
#pragma unroll
        for (int g = 0; g < kRowGroup; ++g) slot(s0 + (k + g) * st, ww[g], yj[g], bo[g]);
    }
    for (; k < cnt; ++k) {
        const int sl = s0 + k * st;
        VT b1;
        if (a.b_zero) {
#pragma unroll
            for (int u = 0; u < V; ++u) b1.v[u] = T(0);
        } else {
            b1 = ld_lanes<T, V>(bread + (size_t)sl * d + c0);
        }
        slot(sl, a.sw[sl], ld_lanes<T, V>(a.Y + (size_t)a.scol[sl] * d + c0), b1);
    }
}

// Edge update, one thread per row (the
// PH_EU arithmetic without r0, element by element and in the same slot order):
// one thread per pixel and V consecutive columns, no LDS, one workgroup per
// kBlock / (d / V) pixels.  The edge update has no neighbour value shared by a
// recurrence, so it needs neither strips nor a co-resident grid: what bounds it
// is the number of independent loads in flight, which wide accesses and a full
// grid of small workgroups maximise.  With GEO (one image of W x H pixels) the
// neighbour of slot k is the stencil offset, and the slot columns are not read;
// otherwise (batches) they are.  KC = 0: general layouts (ELL or CSR rows), b
// and d stored per slot and updated in place, as in the row-chunk phase.
template <typename T, int KC, int V, bool GEO>
__global__ void __launch_bounds__(kBlock) k_eu_px(KA<T> a, int W, int H) {
    using VT = Lanes<T, V>;
    const int d = a.d, L = d / V, ppb = kBlock / L;
    const int q = threadIdx.x / L;
    const int64_t i64 = (int64_t)blockIdx.x * ppb + q;
    if (q >= ppb || i64 >= a.n) return;
    const int i = (int)i64;
    const int c0 = (threadIdx.x - q * L) * V;
    const size_t e = (size_t)i * d + c0;
    const T* bread = a.bsb[a.bpar & 1];
    T* bwrite = a.bsb[(a.bpar & 1) ^ 1];
    const VT yi = ld_lanes<T, V>(a.Y + e);
    VT acc;
#pragma unroll
    for (int u = 0; u < V; ++u) acc.v[u] = T(0);
    if constexpr (KC == 0) {
        // general layouts: the row's slots (ELL or CSR), b and d per slot, updated in place
        VT no_ax;
        eu_row_slots<T, V, false>(a, i, c0, bread, bwrite, yi, acc, no_ax);
    } else {
        int py = 0, px = 0;
        if constexpr (GEO) {
            py = i / W;
            px = i - py * W;
        }
        VT no_ax;
        eu_stencil_slots<T, KC, V, GEO, false>(a, i, c0, py, px, W, H, bread, bwrite, yi, acc, no_ax);
    }
    const T sq = a.sqrtD[i];
    VT pv = ld_lanes<T, V>(a.P + e);
    VT bv = ld_lanes<T, V>(a.B + e);
    VT rv;
#pragma unroll
    for (int u = 0; u < V; ++u) {
        const T split = mul_t(a.half_r, mul_t(sq, pv.v[u] - bv.v[u]));
        rv.v[u] = fma_t(a.c_off, acc.v[u], split);
    }
    st_lanes<T, V>(a.rhs + e, rv);
}

// ---------------------------------------------------------------------------
// Pixel launches (one image of a pixel-stencil layout, Jacobi PCG): the
// residual, w0 and each CG iteration as per-pixel kernels.  Logical workgroup
// lb owns the pixels [row0[lb], row0[lb + 1]) and walks them kBlock / (d / V)
// at a time, one thread per pixel and V consecutive columns (16-byte accesses
// where d allows); neighbour j of slot k is the stencil offset (slots leaving
// the image have weight 0 and point at the pixel itself, as in the slot
// layout).  The CG iteration runs in two passes, as on general layouts: the
// own-row updates storing u' = r' / diag(A) (k_px_ga), then w' = A u' gathering
// u' alone (k_px_gb); the neighbours' values come through L2 rather than an
// LDS ring.  The per-element arithmetic and slot order are those of the
// row-chunk phases.
// ---------------------------------------------------------------------------
// LDS of the pixel kernels: the finalisers' layout (partials of one column lane
// below 1024, the sums of up to seg_chunk() segments above); one or two
// workgroups per CU leave LDS to spare
constexpr int kPxSmemDoubles = kSmemDoubles;
static_assert(kBlock <= 1024, "the finalisers keep their sums at sh + 1024");

// neighbour of slot k of pixel i at (py, px) of a W x H image
template <int KC>
__device__ __forceinline__ int px_nb(int i, int py, int px, int W, int H, int k) {
    using S = Sten<KC>;
    const int yy = py + S::dy(k), xx = px + S::dx(k);
    return (yy >= 0 && yy < H && xx >= 0 && xx < W) ? i + S::dy(k) * W + S::dx(k) : i;
}

// per-thread FP64 accumulators of V columns -> the workgroup's partial of each
// (quantity, column) in part row qout[q]: one column lane u at a time, staged
// in LDS (pixel slot qp, thread lane l -> column l V + u), then one thread per
// column adds the workgroup's pixel slots in order
template <int NQ, int V>
__device__ __forceinline__ void block_partials_px(const double (&acc)[NQ][V], const int (&qout)[NQ], double* sh,
                                                  int d, double* part, int nblk, int lb) {
    const int t = threadIdx.x, L = d / V, ppb = kBlock / L;
    const int qp = t / L;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
#pragma unroll
        for (int u = 0; u < V; ++u) {
            if (qp < ppb) sh[t] = acc[q][u];
            __syncthreads();
            if (t < L) {
                double s = 0.0;
                for (int k = 0; k < ppb; ++k) s += sh[k * L + t];
                part[((size_t)qout[q] * nblk + lb) * d + t * V + u] = s;
            }
            __syncthreads();
        }
    }
}

// sum over the slots k of row i of w_k^2 v_j (slot order), V columns from c0:
// stencil offsets on pixel grids (KC > 0), the row's slot columns otherwise
// (ELL or CSR; loads in groups of kRowGroup slots, slot order kept)
template <typename T, int KC, int V>
__device__ __forceinline__ Lanes<T, V> px_nbsum(const KA<T>& a, const T* v, int i, int c0, int lb) {
    using VT = Lanes<T, V>;
    const int d = a.d;
    VT acc;
#pragma unroll
    for (int q = 0; q < V; ++q) acc.v[q] = T(0);
    if constexpr (KC > 0) {
        constexpr int G = (KC < 8) ? KC : 8;
        const int* gg = a.geo + 8 * lb;   // the workgroup's image: first row, width, height
        const int W = gg[1], H = gg[2];
        const int il = i - gg[0];
        const int py = il / W, px = il - py * W;
#pragma unroll
        for (int k0 = 0; k0 < KC; k0 += G) {
            T ww[G];
            VT vj[G];
#pragma unroll
            for (int k = 0; k < G; ++k) {
                ww[k] = a.sw[(size_t)(k0 + k) * a.n + i];
                vj[k] = ld_lanes<T, V>(v + (size_t)px_nb<KC>(i, py, px, W, H, k0 + k) * d + c0);
            }
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const T w2 = mul_t(ww[k], ww[k]);
#pragma unroll
                for (int q = 0; q < V; ++q) acc.v[q] = fma_t(w2, vj[k].v[q], acc.v[q]);
            }
        }
    } else {
        int s0, cnt, st;
        row_slots<0>(a, i, s0, cnt, st);
        int k = 0;
        for (; k + kRowGroup <= cnt; k += kRowGroup) {
            T ww[kRowGroup];
            VT vj[kRowGroup];
#pragma unroll
            for (int g = 0; g < kRowGroup; ++g) {
                const int sl = s0 + (k + g) * st;
                ww[g] = a.sw[sl];
                vj[g] = ld_lanes<T, V>(v + (size_t)a.scol[sl] * d + c0);
            }
#pragma unroll
            for (int g = 0; g < kRowGroup; ++g) {
                const T w2 = mul_t(ww[g], ww[g]);
#pragma unroll
                for (int q = 0; q < V; ++q) acc.v[q] = fma_t(w2, vj[g].v[q], acc.v[q]);
            }
        }
        for (; k < cnt; ++k) {
            const int sl = s0 + k * st;
            const T w2 = mul_t(a.sw[sl], a.sw[sl]);
            VT vj1 = ld_lanes<T, V>(v + (size_t)a.scol[sl] * d + c0);
#pragma unroll
            for (int q = 0; q < V; ++q) acc.v[q] = fma_t(w2, vj1.v[q], acc.v[q]);
        }
    }
    return acc;
}

// the pixels of logical workgroup lb, kBlock / (d / V) per step: f(i, e, c0)
// for each of this thread's pixels (element e = i d + c0).  The workgroups of
// an XCD band form a team that deals the band's steps out cyclically (chunks
// first + k stride of one step each), so the band is swept together and the
// neighbour rows one workgroup gathers were just read by the others of its XCD
template <int V, typename T, class F>
__device__ __forceinline__ void px_walk(const KA<T>& a, int lb, F&& f) {
    const int d = a.d, L = d / V, ppb = kBlock / L;
    const int qp = (int)threadIdx.x / L;
    if (qp >= ppb) return;
    const int c0 = ((int)threadIdx.x - qp * L) * V;
    const int first = a.bit[3 * lb], end = a.bit[3 * lb + 1], stride = a.bit[3 * lb + 2];
    for (int base = first; base < end; base += stride) {
        const int i = base + qp;
        if (i < end) f(i, (size_t)i * d + c0, c0);
    }
}

// residual r0 = rhs - A x (PH_E0: rhs = r/2 D^{1/2} (P - B), stored when
// store_rhs; PH_R0: the stored rhs), with u0 = r0 / diag(A) stored for w0;
// partials of rhs.rhs and r0.r0 (the st_res / ph_residual arithmetic)
template <typename T, int KC, int V>
__global__ void __launch_bounds__(kBlock) k_px_res(KA<T> a, int mode) {
    using VT = Lanes<T, V>;
    __shared__ double sh[kPxSmemDoubles];
    const int lb = logical_block(a.nblk);
    double acc[2][V] = {};
    px_walk<V>(a, lb, [&](int i, size_t e, int c0) {
        const VT accA = px_nbsum<T, KC, V>(a, a.x, i, c0, lb);
        VT rhs;
        if (mode == PH_R0) {
            rhs = ld_lanes<T, V>(a.rhs + e);
        } else {
            const T sq = a.sqrtD[i];
            VT pv = ld_lanes<T, V>(a.P + e);
            VT bv = ld_lanes<T, V>(a.B + e);
#pragma unroll
            for (int u = 0; u < V; ++u)
                rhs.v[u] = mul_t(a.half_r, mul_t(sq, pv.v[u] - bv.v[u]));
            if (a.store_rhs) st_lanes<T, V>(a.rhs + e, rhs);
        }
        const T dA = a.diagA[i], inv = a.invdiag[i];
        VT xi = ld_lanes<T, V>(a.x + e);
        VT rv, uv;
#pragma unroll
        for (int u = 0; u < V; ++u) {
            const T ax = fma_t(dA, xi.v[u], -mul_t(a.c_off, accA.v[u]));
            const T r = rhs.v[u] - ax;
            rv.v[u] = r;
            uv.v[u] = mul_t(inv, r);
            acc[0][u] += (double)rhs.v[u] * (double)rhs.v[u];
            acc[1][u] += (double)r * (double)r;
        }
        st_lanes<T, V>(a.rb[0] + e, rv);
        st_lanes<T, V>(a.zl + e, uv);
    });
    const int qo[2] = {0, 1};
    block_partials_px<2, V>(acc, qo, sh, a.d, a.part, a.nblk, lb);
    if (last_of_launch(a, 2, sh)) fin_res(a, sh, grouped_fin(a));
}

// The edge update of inner step l fused with the residual of solve l + 1, on
// pixel-stencil images or general layouts (KC = 0), per-row partition: Eqs.
// 9-10 per slot and the next right-hand side as in k_eu_px; then r0 = rhs - A x
// for the iterate that solve starts from (x = Y), out of the Y values the edge
// update has gathered, and u0 = r0 / diag(A); partials of rhs.rhs and r0.r0 and
// the finaliser as in k_px_res.  A x sums w^2 y_j in the slots' visiting order:
// the slot order in FP64 and on general layouts (r0 then equals k_px_res's
// bitwise), pairs of slots in FP32 on stencils (as does the right-hand side's
// sum here).  The right-hand side is stored only with store_rhs
// (factor-preconditioned solves, whose Jacobi fallback forms r0 from it
// again); a Jacobi solve reads only r0.
template <typename T, int KC, int V>
__global__ void __launch_bounds__(kBlock) k_eur_px(KA<T> a) {
    using VT = Lanes<T, V>;
    __shared__ double sh[kPxSmemDoubles];
    const int lb = logical_block(a.nblk);
    const T* bread = a.bsb[a.bpar & 1];
    T* bwrite = a.bsb[(a.bpar & 1) ^ 1];
    int row0 = 0, W = 0, H = 0;
    if constexpr (KC > 0) {
        const int* gg = a.geo + 8 * lb;   // the workgroup's image: first row, width, height
        row0 = gg[0];
        W = gg[1];
        H = gg[2];
    }
    double acc2[2][V] = {};
    px_walk<V>(a, lb, [&](int i, size_t e, int c0) {
        const VT yi = ld_lanes<T, V>(a.Y + e);
        VT acc, accA;
#pragma unroll
        for (int u = 0; u < V; ++u) acc.v[u] = accA.v[u] = T(0);
        if constexpr (KC > 0) {
            const int il = i - row0, py = il / W, px = il - py * W;
            eu_stencil_slots<T, KC, V, true, true>(a, i, c0, py, px, W, H, bread, bwrite, yi, acc, accA);
        } else {
            eu_row_slots<T, V, true>(a, i, c0, bread, bwrite, yi, acc, accA);
        }
        const T sq = a.sqrtD[i], dA = a.diagA[i], inv = a.invdiag[i];
        const VT pv = ld_lanes<T, V>(a.P + e);
        const VT bv = ld_lanes<T, V>(a.B + e);
        VT hv, rv, uv;
#pragma unroll
        for (int u = 0; u < V; ++u) {
            const T split = mul_t(a.half_r, mul_t(sq, pv.v[u] - bv.v[u]));
            const T rhs = fma_t(a.c_off, acc.v[u], split);
            const T ax = fma_t(dA, yi.v[u], -mul_t(a.c_off, accA.v[u]));
            const T r = rhs - ax;
            hv.v[u] = rhs;
            rv.v[u] = r;
            uv.v[u] = mul_t(inv, r);
            acc2[0][u] += (double)rhs * (double)rhs;
            acc2[1][u] += (double)r * (double)r;
        }
        if (a.store_rhs) st_lanes<T, V>(a.rhs + e, hv);
        st_lanes<T, V>(a.rb[0] + e, rv);
        st_lanes<T, V>(a.zl + e, uv);
    });
    const int qo[2] = {0, 1};
    block_partials_px<2, V>(acc2, qo, sh, a.d, a.part, a.nblk, lb);
    if (last_of_launch(a, 2, sh)) fin_res(a, sh, grouped_fin(a));
}

// w = A u for u in zl: the neighbours' u gathered, slot loads issued in groups
template <typename T, int KC, int V>
__device__ __forceinline__ Lanes<T, V> px_apply(const KA<T>& a, const T* u, int i, int c0,
                                                                const Lanes<T, V>& ui, int lb) {
    using VT = Lanes<T, V>;
    const VT accA = px_nbsum<T, KC, V>(a, u, i, c0, lb);
    const T dA = a.diagA[i];
    VT wv;
#pragma unroll
    for (int q = 0; q < V; ++q) wv.v[q] = fma_t(dA, ui.v[q], -mul_t(a.c_off, accA.v[q]));
    return wv;
}

// w0 = A u0 (u0 = r0 / diag(A) in zl); partials of r0.u0 and w0.u0 (the st_w0 arithmetic)
template <typename T, int KC, int V>
__global__ void __launch_bounds__(kBlock) k_px_w0(KA<T> a) {
    using VT = Lanes<T, V>;
    __shared__ double sh[kPxSmemDoubles];
    if (ld_flag(&a.S->done)) return;
    const int lb = logical_block(a.nblk);
    double acc[2][V] = {};
    px_walk<V>(a, lb, [&](int i, size_t e, int c0) {
        VT ui = ld_lanes<T, V>(a.zl + e);
        VT ri = ld_lanes<T, V>(a.rb[0] + e);
        VT wv = px_apply<T, KC, V>(a, a.zl, i, c0, ui, lb);
        st_lanes<T, V>(a.wb[0] + e, wv);
#pragma unroll
        for (int u = 0; u < V; ++u) {
            acc[0][u] += (double)ri.v[u] * (double)ui.v[u];
            acc[1][u] += (double)wv.v[u] * (double)ui.v[u];
        }
    });
    const int qo[2] = {0, 1};
    block_partials_px<2, V>(acc, qo, sh, a.d, a.part, a.nblk, lb);
    if (last_of_launch(a, 2, sh)) fin_w0(a, sh, grouped_fin(a));
}

// CG iteration, pass 1 (the ph_ga arithmetic, in place on buffer 0): p, s, x,
// r' = r - alpha s, u' = r' / diag(A) into zl; partials r'.u' (q0), r'.r' (q2)
template <typename T, int V>
__global__ void __launch_bounds__(kBlock) k_px_ga(KA<T> a) {
    using VT = Lanes<T, V>;
    __shared__ double sh[kPxSmemDoubles];
    if (ld_flag(&a.S->done)) return;
    const int lb = logical_block(a.nblk);
    const bool first = ld_flag(&a.S->it) == 0;
    const int d = a.d;
    double acc[2][V] = {};
    {
        const int L = d / V;
        const int c0 = ((int)threadIdx.x % L) * V;
        const int ci = a.blk_seg[lb] * d + c0;   // the workgroup's segment's column scalars
        T alpha[V], beta[V];
#pragma unroll
        for (int u = 0; u < V; ++u) {
            alpha[u] = (T)a.cs.alpha[ci + u];
            beta[u] = (T)a.cs.beta[ci + u];
        }
        px_walk<V>(a, lb, [&](int i, size_t e, int) {
            const T inv = a.invdiag[i];
            VT r = ld_lanes<T, V>(a.rb[0] + e);
            VT pold = ld_lanes<T, V>(a.p + e);
            VT sp = ld_lanes<T, V>(a.sb[0] + e);
            VT w = ld_lanes<T, V>(a.wb[0] + e);
            VT x = ld_lanes<T, V>(a.x + e);
            VT pn, sn, xn, rn, un;
#pragma unroll
            for (int u = 0; u < V; ++u) {
                const T ri = r.v[u];
                const T ui = mul_t(inv, ri);
                const T pi = first ? ui : fma_t(beta[u], pold.v[u], ui);
                const T si = cg_s(first, beta[u], sp.v[u], w.v[u]);
                const T rn_i = cg_r(alpha[u], si, ri);
                const T un_i = mul_t(inv, rn_i);
                pn.v[u] = pi;
                sn.v[u] = si;
                xn.v[u] = fma_t(alpha[u], pi, x.v[u]);
                rn.v[u] = rn_i;
                un.v[u] = un_i;
                acc[0][u] += (double)rn_i * (double)un_i;
                acc[1][u] += (double)rn_i * (double)rn_i;
            }
            st_lanes<T, V>(a.p + e, pn);
            st_lanes<T, V>(a.sb[0] + e, sn);
            st_lanes<T, V>(a.x + e, xn);
            st_lanes<T, V>(a.rb[0] + e, rn);
            st_lanes<T, V>(a.zl + e, un);
        });
    }
    const int qo[2] = {0, 2};
    block_partials_px<2, V>(acc, qo, sh, d, a.part, a.nblk, lb);
}

// CG iteration, pass 2 (the ph_gb arithmetic): w' = A u'; partial w'.u' (q1); finaliser
template <typename T, int KC, int V>
__global__ void __launch_bounds__(kBlock) k_px_gb(KA<T> a) {
    using VT = Lanes<T, V>;
    __shared__ double sh[kPxSmemDoubles];
    if (ld_flag(&a.S->done)) return;
    const int lb = logical_block(a.nblk);
    double acc[1][V] = {};
    px_walk<V>(a, lb, [&](int i, size_t e, int c0) {
        VT ui = ld_lanes<T, V>(a.zl + e);
        VT wv = px_apply<T, KC, V>(a, a.zl, i, c0, ui, lb);
        st_lanes<T, V>(a.wb[0] + e, wv);
#pragma unroll
        for (int u = 0; u < V; ++u) acc[0][u] += (double)wv.v[u] * (double)ui.v[u];
    });
    const int qo[1] = {1};
    block_partials_px<1, V>(acc, qo, sh, a.d, a.part, a.nblk, lb);
    if (last_of_launch(a, 3, sh)) {
        fin_it(a, sh, grouped_fin(a));
        if (threadIdx.x == 0 && a.S->done) solve_stats(a);
    }
}

// Factor-preconditioned PCG (M^{-1} = D_A^{-1/2} Gt^T Gt D_A^{-1/2}) by pixel
// launches on pixel grids, three passes per iteration with the st_la / st_lcd
// arithmetic; a neighbour's value is formed again from its loaded inputs where
// the strip kernels read it from an LDS ring:
//   k_pl_a: p = z + beta p, q = A p (neighbours' p from their z and old p);
//           partial p.q -> alpha
//   k_pl_c: x += alpha p, r' = r - alpha q (upd), y1 = Gt D_A^{-1/2} r' over the
//           lower slots (neighbours' r' from their r and q); y1 stored
//   k_pl_d: z = D_A^{-1/2} Gt^T y1 over the upper slots; partials r'.z, r'.r'
//           -> beta, convergence (initial: from the initial residual)
template <typename T, int KC, int V>
__global__ void __launch_bounds__(kBlock) k_pl_a(KA<T> a) {
    using VT = Lanes<T, V>;
    constexpr int G = (KC < 8) ? KC : 8;
    __shared__ double sh[kPxSmemDoubles];
    if (ld_flag(&a.S->done)) return;
    const int lb = logical_block(a.nblk);
    const int it = ld_flag(&a.S->it);
    const bool first = (it == 0);
    T* pnew = a.sb[it & 1];
    const T* pold = a.sb[(it & 1) ^ 1];
    const int d = a.d, L = d / V;
    const int ci = a.blk_seg[lb] * d + ((int)threadIdx.x % L) * V;
    T beta[V];
#pragma unroll
    for (int u = 0; u < V; ++u) beta[u] = (T)a.cs.beta[ci + u];
    const int* gg = a.geo + 8 * lb;
    const int W = gg[1], H = gg[2], r0g = gg[0];
    double acc[1][V] = {};
    auto p_of = [&](const VT& z, const VT& po) {
        VT p;
#pragma unroll
        for (int u = 0; u < V; ++u) p.v[u] = first ? z.v[u] : fma_t(beta[u], po.v[u], z.v[u]);
        return p;
    };
    px_walk<V>(a, lb, [&](int i, size_t e, int c0) {
        const int il = i - r0g, py = il / W, px = il - py * W;
        VT zero;
#pragma unroll
        for (int u = 0; u < V; ++u) zero.v[u] = T(0);
        const VT pi = p_of(ld_lanes<T, V>(a.zl + e), first ? zero : ld_lanes<T, V>(pold + e));
        VT accA = zero;
#pragma unroll
        for (int k0 = 0; k0 < KC; k0 += G) {
            T ww[G];
            VT pj[G];
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const size_t ej = (size_t)px_nb<KC>(i, py, px, W, H, k0 + k) * d + c0;
                ww[k] = a.sw[(size_t)(k0 + k) * a.n + i];
                pj[k] = p_of(ld_lanes<T, V>(a.zl + ej), first ? zero : ld_lanes<T, V>(pold + ej));
            }
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const T w2 = mul_t(ww[k], ww[k]);
#pragma unroll
                for (int u = 0; u < V; ++u) accA.v[u] = fma_t(w2, pj[k].v[u], accA.v[u]);
            }
        }
        const T dA = a.diagA[i];
        VT qi;
#pragma unroll
        for (int u = 0; u < V; ++u) {
            qi.v[u] = fma_t(dA, pi.v[u], -mul_t(a.c_off, accA.v[u]));
            acc[0][u] += (double)pi.v[u] * (double)qi.v[u];
        }
        st_lanes<T, V>(pnew + e, pi);
        st_lanes<T, V>(a.wb[0] + e, qi);
    });
    const int qo[1] = {0};
    block_partials_px<1, V>(acc, qo, sh, d, a.part, a.nblk, lb);
    if (last_of_launch(a, 1, sh)) fin_la(a, sh, grouped_fin(a));
}

template <typename T, int KC, int V>
__global__ void __launch_bounds__(kBlock) k_pl_c(KA<T> a, int upd) {
    using VT = Lanes<T, V>;
    constexpr int HS = KC / 2;
    if (ld_flag(&a.S->done)) return;
    const int lb = logical_block(a.nblk);
    const int it = upd ? ld_flag(&a.S->it) : 0;
    const T* r = a.rb[it & 1];
    T* rn = a.rb[(it & 1) ^ 1];
    const T* p = a.sb[it & 1];
    const T* q = a.wb[0];
    const int d = a.d, L = d / V;
    const int ci = a.blk_seg[lb] * d + ((int)threadIdx.x % L) * V;
    T alpha[V];
#pragma unroll
    for (int u = 0; u < V; ++u) alpha[u] = upd ? (T)a.cs.alpha[ci + u] : T(0);
    const int* gg = a.geo + 8 * lb;
    const int W = gg[1], H = gg[2], r0g = gg[0];
    // isq r' of element e of pixel j (r' = r - alpha q after the update)
    auto sr_of = [&](int j, size_t ej) {
        VT rv = ld_lanes<T, V>(r + ej);
        if (upd) {
            const VT qv = ld_lanes<T, V>(q + ej);
#pragma unroll
            for (int u = 0; u < V; ++u) rv.v[u] = fma_t(-alpha[u], qv.v[u], rv.v[u]);
        }
        return rv;
    };
    px_walk<V>(a, lb, [&](int i, size_t e, int c0) {
        const int il = i - r0g, py = il / W, px = il - py * W;
        const VT ri = sr_of(i, e);
        if (upd) {
            const VT pv = ld_lanes<T, V>(p + e);
            VT xv = ld_lanes<T, V>(a.x + e);
#pragma unroll
            for (int u = 0; u < V; ++u) xv.v[u] = fma_t(alpha[u], pv.v[u], xv.v[u]);
            st_lanes<T, V>(a.x + e, xv);
            st_lanes<T, V>(rn + e, ri);
        }
        const T gd = a.gdiag[i], si = a.isq[i];
        VT y;
#pragma unroll
        for (int u = 0; u < V; ++u) y.v[u] = mul_t(gd, mul_t(si, ri.v[u]));
        T gv[HS], sj[HS];
        VT rj[HS];
#pragma unroll
        for (int k = 0; k < HS; ++k) {
            const int j = px_nb<KC>(i, py, px, W, H, k);
            gv[k] = a.gval[(size_t)k * a.n + i];
            sj[k] = a.isq[j];
            rj[k] = sr_of(j, (size_t)j * d + c0);
        }
#pragma unroll
        for (int k = 0; k < HS; ++k) {
#pragma unroll
            for (int u = 0; u < V; ++u) y.v[u] = fma_t(gv[k], mul_t(sj[k], rj[k].v[u]), y.v[u]);
        }
        st_lanes<T, V>(a.y1 + e, y);
    });
}

template <typename T, int KC, int V>
__global__ void __launch_bounds__(kBlock) k_pl_d(KA<T> a, int initial) {
    using VT = Lanes<T, V>;
    constexpr int HS = KC / 2;
    __shared__ double sh[kPxSmemDoubles];
    if (ld_flag(&a.S->done)) return;
    const int lb = logical_block(a.nblk);
    const int it = initial ? 0 : ld_flag(&a.S->it);
    const T* rr = initial ? a.rb[0] : a.rb[(it & 1) ^ 1];
    const int d = a.d;
    const int* gg = a.geo + 8 * lb;
    const int W = gg[1], H = gg[2], r0g = gg[0];
    double acc[2][V] = {};
    px_walk<V>(a, lb, [&](int i, size_t e, int c0) {
        const int il = i - r0g, py = il / W, px = il - py * W;
        const T gd = a.gdiag[i];
        const VT yi = ld_lanes<T, V>(a.y1 + e);
        VT z;
#pragma unroll
        for (int u = 0; u < V; ++u) z.v[u] = mul_t(gd, yi.v[u]);
        T gv[KC - HS];
        VT yj[KC - HS];
#pragma unroll
        for (int k = HS; k < KC; ++k) {
            gv[k - HS] = a.gval[(size_t)k * a.n + i];
            yj[k - HS] = ld_lanes<T, V>(a.y1 + (size_t)px_nb<KC>(i, py, px, W, H, k) * d + c0);
        }
#pragma unroll
        for (int k = 0; k < KC - HS; ++k) {
#pragma unroll
            for (int u = 0; u < V; ++u) z.v[u] = fma_t(gv[k], yj[k].v[u], z.v[u]);
        }
        const T si = a.isq[i];
        const VT ri = ld_lanes<T, V>(rr + e);
#pragma unroll
        for (int u = 0; u < V; ++u) {
            z.v[u] = mul_t(si, z.v[u]);
            acc[0][u] += (double)ri.v[u] * (double)z.v[u];
            acc[1][u] += (double)ri.v[u] * (double)ri.v[u];
        }
        st_lanes<T, V>(a.zl + e, z);
    });
    const int qo[2] = {0, 1};
    block_partials_px<2, V>(acc, qo, sh, d, a.part, a.nblk, lb);
    if (last_of_launch(a, 2, sh)) {
        fin_ld(a, sh, initial != 0, grouped_fin(a));
        if (threadIdx.x == 0 && a.S->done) solve_stats(a);
    }
}

// learned-preconditioner PCG phases on strips
template <typename T, int KC>
__global__ void __launch_bounds__(kBlock) k_st_la(KA<T> a) {
    __shared__ double sh[kSmemDoubles];
    if (ld_flag(&a.S->done)) return;
    st_la<KC>(a, logical_block(a.nblk), sh);
    if (last_block(a.bar + kBarLast, a.nblk)) fin_la(a, sh);
}

template <typename T, int KC>
__global__ void __launch_bounds__(kBlock) k_st_lc(KA<T> a, int upd) {
    __shared__ double sh[kSmemDoubles];
    if (ld_flag(&a.S->done)) return;
    st_lc<KC>(a, logical_block(a.nblk), sh, upd);
}

template <typename T, int KC>
__global__ void __launch_bounds__(kBlock) k_st_ld(KA<T> a, int initial) {
    __shared__ double sh[kSmemDoubles];
    if (ld_flag(&a.S->done)) return;
    st_ld<KC>(a, logical_block(a.nblk), sh, initial);
    if (last_block(a.bar + kBarLast, a.nblk)) {
        fin_ld(a, sh, initial != 0);
        if (threadIdx.x == 0 && a.S->done) solve_stats(a);
    }
}

// LC and LD fused on strips with a two-radius halo
template <typename T, int KC>
__global__ void __launch_bounds__(kBlock) k_st_lcd(KA<T> a, int upd) {
    __shared__ double sh[kSmemDoubles];
    if (ld_flag(&a.S->done)) return;
    st_lcd<KC>(a, logical_block(a.nblk), sh, upd);
    if (last_block(a.bar + kBarLast, a.nblk)) {
        fin_ld(a, sh, upd == 0);
        if (threadIdx.x == 0 && a.S->done) solve_stats(a);
    }
}

// factor-preconditioned CG on strips, one kernel per iteration (mode 1) and
// one for u0, w0 before the first (mode 0)
template <typename T, int KC, int CPL>
__global__ void __launch_bounds__(kBlock) k_st_fcg(KA<T> a, int mode) {
    __shared__ double sh[FcgRings<KC, T, CPL>::doubles];
    if (ld_flag(&a.S->done)) return;
    st_fcg<KC, CPL>(a, logical_block(a.nblk), sh, mode);
    if (last_block(a.bar + kBarLast, a.nblk)) {
        if (mode == 0) {
            fin_w0(a, sh, false);
        } else {
            fin_it(a, sh, false);
            if (threadIdx.x == 0 && a.S->done) solve_stats(a);
        }
    }
}

// columns per lane of the one-pass factor CG: two (8-byte vector accesses,
// twice the pixels per strip) for FP32 and even d; one otherwise (the FP64
// rings of two columns per lane would not fit the LDS of a workgroup)
template <typename T>
constexpr int fcg_cpl(int d) { return (sizeof(T) == 4 && d % 2 == 0) ? 2 : 1; }

template <typename T>
const void* fcg_kernel(int ellK, int cpl) {
    const bool two = (cpl == 2 && sizeof(T) == 4);
#define PFE_FCG(K) (two ? reinterpret_cast<const void*>(&k_st_fcg<T, K, (sizeof(T) == 4 ? 2 : 1)>) \
                        : reinterpret_cast<const void*>(&k_st_fcg<T, K, 1>))
    switch (ellK) {
        case 4: return PFE_FCG(4);
        case 8: return PFE_FCG(8);
        case 24: return PFE_FCG(24);
        default: return nullptr;
    }
#undef PFE_FCG
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_cg_zero(KA<T> a) {
    ph_zero(a, logical_block(a.nblk), a.cs.zero);
}

template <typename T, int KC>
__global__ void __launch_bounds__(kBlock) k_lpcg_aq(KA<T> a) {
    __shared__ double sh[kSmemDoubles];
    if (ld_flag(&a.S->done)) return;
    const int lb = logical_block(a.nblk);
    ph_la<KC>(a, lb, sh);
    if (last_block(a.bar + kBarLast, a.nblk)) fin_la(a, sh);
}

template <typename T, int KC>
__global__ void __launch_bounds__(kBlock) k_lpcg_g(KA<T> a, int upd) {
    if (ld_flag(&a.S->done)) return;
    ph_lc<KC>(a, logical_block(a.nblk), upd);
}

template <typename T, int KC>
__global__ void __launch_bounds__(kBlock) k_lpcg_gt(KA<T> a, int initial) {
    __shared__ double sh[kSmemDoubles];
    if (ld_flag(&a.S->done)) return;
    const int lb = logical_block(a.nblk);
    ph_ld<KC>(a, lb, sh, initial);
    if (last_block(a.bar + kBarLast, a.nblk)) {
        fin_ld(a, sh, initial != 0);
        if (threadIdx.x == 0 && a.S->done) solve_stats(a);
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_gram(KA<T> a, int mode) {
    __shared__ double sh[kSmemDoubles];
    const int lb = logical_block(a.nblk);
    ph_gram(a, lb, mode, sh);
    // several segments: one workgroup per segment factors in k_factor
    if (a.nseg == 1 && last_block(a.bar + kBarLast, a.nblk)) seg_factor(a, 0, mode, sh, false, a.Tm, true);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_apply(KA<T> a, int mode) {
    __shared__ double sh[kSmemDoubles];
    if (!ld_flag(&a.S->ortho_ok)) return;
    const int lb = logical_block(a.nblk);
    ph_apply(a, lb, mode, sh, a.Tm + (size_t)a.blk_seg[lb] * kMaxD * kMaxD);
}

// P-update factors of a batch: workgroup sg reduces and factors segment sg
template <typename T>
__global__ void __launch_bounds__(kBlock) k_factor(KA<T> a, int mode) {
    __shared__ double sh[kSmemDoubles];
    const int sg = blockIdx.x;
    seg_factor(a, sg, mode, sh, false, a.Tm + (size_t)sg * kMaxD * kMaxD, true);
}

// statistics when a solve finished before its first iteration
template <typename T>
__global__ void k_stats_if_done(KA<T> a) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && a.S->done && a.S->it == 0) solve_stats(a);
}

// Status bookkeeping of a factor-preconditioned solve, which is judged on its
// own: the worst status met so far is set aside before it (save), cleared
// again before a Jacobi redo (clear), and combined with the status of the
// solve that stands afterwards (merge; a breakdown outranks maxit).
__device__ __forceinline__ int worse_status(int a, int b) {
    if (a == 0) return b;
    if (b == 0) return a;
    return (a == PFE_E_NOT_SPD || b == PFE_E_NOT_SPD) ? PFE_E_NOT_SPD : a;
}
__global__ void k_status_save(Scal* S) {
    if (threadIdx.x == 0) { S->saved_status = S->status; S->status = 0; }
}
__global__ void k_status_clear(Scal* S) {
    if (threadIdx.x == 0) S->status = 0;
}
// autotuner: every candidate launch shape is judged on its own run
__global__ void k_tune_reset(Scal* S) {
    if (threadIdx.x == 0) { S->status = 0; S->abort_flag = 0; S->ortho_ok = 1; }
}
__global__ void k_status_merge(Scal* S, int fallback) {
    if (threadIdx.x == 0) {
        S->status = worse_status(S->saved_status, S->status);
        if (fallback) S->fallbacks += 1;
    }
}

struct Plan {
    int l_begin;      // first inner index of the first SOC iteration
    int n_inner;      // inner iterations per SOC iteration
    int n_outer;      // SOC iterations to run
    int cache_np;     // chunks per workgroup held in the LDS row cache (LC kernels)
    int pupdate;      // 1: P- and B-update after the inner iterations; 0: Split Bregman alone
};

// Persistent path: whole SOC iterations in one cooperative launch.  One
// segment: the group leaders pre-reduce the partials of their XCD group.
// Several segments (a batch): the finalisers reduce every segment at once, and
// after the Gram phase every workgroup factors its own segment's Gram matrix
// (the same FP64 operations in the same order in each of them), so the
// P-update needs no further barrier.
template <typename T, int KC, bool LC>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1))) k_soc(KA<T> a, Plan plan) {
    __shared__ double sh[kSmemDoubles];
    __shared__ double Tsh[kMaxD * kMaxD];
    extern __shared__ __align__(16) unsigned char dyn_lds[];
    const int lb = logical_block(a.nblk);
    RowCache<T> rc;
    if constexpr (LC) rc = fill_row_cache<T, KC>(a, lb, dyn_lds, plan.cache_np);
    const unsigned nb = (unsigned)a.nblk;
    Scal* S = a.S;
    const int d = a.d;
    const int npair = d * (d + 1) / 2;
    const bool one = (a.nseg == 1);
    const int ncol = a.nseg * d;
    int l0 = plan.l_begin;
    unsigned nbar = 0;   // grid barriers passed in this launch
    if (one) {
        __shared__ LocState L;
        if (threadIdx.x == 0) L.status = 0;
        int par = 0;
        // the group partial buffer of the next barrier
        auto gbuf = [&]() { double* gp = a.gpart + (size_t)par * kGroupStride; par ^= 1; return gp; };
        for (int outer = 0; outer < plan.n_outer; ++outer) {
            for (int l = l0; l < plan.n_inner; ++l) {
                ph_residual<KC, 4, LC>(a, lb, (l == 0) ? PH_E0 : PH_EU, 1, (l == 1) ? 1 : 0, (l - 1) & 1, sh, rc);
                double* gp = gbuf();
                if (!grid_sync(a.bar, nb, S, nbar, [&](unsigned g) { group_reduce(a, g, d, 2, sh, gp); }, NoFin{})) return;
                lfin_res(a, L, gp, sh);
                if (!L.done) {
                    ph_w0<KC, 4, LC>(a, lb, sh, rc);
                    gp = gbuf();
                    if (!grid_sync(a.bar, nb, S, nbar, [&](unsigned g) { group_reduce(a, g, d, 2, sh, gp); }, NoFin{})) return;
                    lfin_w0(a, L, gp, sh);
                }
                while (!L.done) {
                    if constexpr (KC == 0) {
                        ph_ga(a, lb, sh, L.it, L.alpha, L.beta);
                        gbuf();
                        if (!grid_sync(a.bar, nb, S, nbar, NoFin{}, NoFin{})) return;
                        ph_gb(a, lb, sh);
                    } else {
                        ph_it<KC, 4, LC>(a, lb, sh, L.it, L.alpha, L.beta, rc);
                    }
                    gp = gbuf();
                    if (!grid_sync(a.bar, nb, S, nbar, [&](unsigned g) { group_reduce(a, g, d, 3, sh, gp); }, NoFin{})) return;
                    lfin_it(a, L, gp, sh);
                }
                if (lb == 0 && threadIdx.x == 0) solve_stats_loc(a, L);
                if (L.any_zero) {
                    // columns with a zero right-hand side: x_c = 0
                    ph_zero(a, lb, L.zero);
                    gbuf();
                    if (!grid_sync(a.bar, nb, S, nbar, NoFin{}, NoFin{})) return;
                }
            }
            l0 = 0;
            if (!plan.pupdate) continue;
            ph_gram(a, lb, 0, sh);
            double* gp = gbuf();
            if (!grid_sync(a.bar, nb, S, nbar, [&](unsigned g) { group_reduce(a, g, npair, 1, sh, gp); },
                           [&] { seg_factor(a, 0, 0, sh, true, a.Tm, true, gp); }))
                return;
            if (!ld_flag(&S->ortho_ok)) return;
            ph_apply(a, lb, 0, sh, a.Tm);
        }
        return;
    }
    for (int outer = 0; outer < plan.n_outer; ++outer) {
        for (int l = l0; l < plan.n_inner; ++l) {
            ph_residual<KC, 4, LC>(a, lb, (l == 0) ? PH_E0 : PH_EU, 1, (l == 1) ? 1 : 0, (l - 1) & 1, sh, rc);
            if (!grid_sync(a.bar, nb, S, nbar, NoFin{}, [&] { fin_res(a, sh, false); })) return;
            if (!ld_flag(&S->done)) {
                ph_w0<KC, 4, LC>(a, lb, sh, rc);
                if (!grid_sync(a.bar, nb, S, nbar, NoFin{}, [&] { fin_w0(a, sh, false); })) return;
            }
            while (!ld_flag(&S->done)) {
                if constexpr (KC == 0) {
                    ph_ga(a, lb, sh, ld_flag(&S->it), a.cs.alpha, a.cs.beta);
                    if (!grid_sync(a.bar, nb, S, nbar, NoFin{}, NoFin{})) return;
                    ph_gb(a, lb, sh);
                } else {
                    ph_it<KC, 4, LC>(a, lb, sh, ld_flag(&S->it), a.cs.alpha, a.cs.beta, rc);
                }
                if (!grid_sync(a.bar, nb, S, nbar, NoFin{}, [&] { fin_it(a, sh, false); })) return;
            }
            if (lb == 0 && threadIdx.x == 0) solve_stats(a);
            int any_zero = 0;
            for (int c = 0; c < ncol; ++c) any_zero |= a.cs.zero[c];
            if (any_zero) {
                // columns with a zero right-hand side: x_c = 0
                ph_zero(a, lb, a.cs.zero);
                if (!grid_sync(a.bar, nb, S, nbar, NoFin{}, NoFin{})) return;
            }
        }
        l0 = 0;
        if (!plan.pupdate) continue;
        ph_gram(a, lb, 0, sh);
        if (!grid_sync(a.bar, nb, S, nbar, NoFin{}, NoFin{})) return;
        const int sg = a.blk_seg[lb];
        // a segment whose Gram matrix is singular keeps its P and B; the
        // first workgroup of the segment records the failure
        if (seg_factor(a, sg, 0, sh, false, Tsh, lb == a.seg_blk0[sg])) ph_apply(a, lb, 0, sh, Tsh);
        // P and B of a row are written and read by the same workgroup; the
        // barrier after the next residual phase orders everything else.
    }
}

template <typename T, int KC>
__global__ void __launch_bounds__(kBlock) k_spmm(KA<T> a, const T* __restrict__ X, T* __restrict__ Q) {
    const int d = a.d, R = a.R, t = threadIdx.x;
    const int lb = blockIdx.x;
    const int rb = a.row0[lb], re = a.row0[lb + 1];
    if (t >= R * d) return;
    const int rl = t / d, c = t - rl * d;
    for (int i = rb + rl; i < re; i += R) {
        const size_t e = (size_t)i * d + c;
        int s0, cnt, st;
        row_slots<KC>(a, i, s0, cnt, st);
        T acc = T(0);
#pragma unroll kSlotUnroll<KC>
        for (int k = 0; k < cnt; ++k) {
            const int s = s0 + k * st;
            const T ww = a.sw[s];
            acc = fma_t(mul_t(ww, ww), X[(size_t)a.scol[s] * d + c], acc);
        }
        Q[e] = fma_t(a.diagA[i], X[e], -mul_t(a.c_off, acc));
    }
}

// diagonal of A = lambda/2 M^T M + r/2 D in FP64, and D^{+-1/2}
template <typename T>
__global__ void k_diag(int n, const double* __restrict__ degree, const double* __restrict__ wsq,
                       double half_lam, double half_r, T* diagA, T* invdiag, T* sqrtD, T* isqrtD, T* isq) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double da = half_lam * wsq[i] + half_r * degree[i];
    diagA[i] = (T)da;
    invdiag[i] = (T)(1.0 / da);
    isq[i] = (T)(1.0 / sqrt(da));
    sqrtD[i] = (T)sqrt(degree[i]);
    isqrtD[i] = (T)(1.0 / sqrt(degree[i]));
}

// per-slot state <-> per-undirected-edge blocks (orientation: lower index minus upper)
template <typename T>
__global__ void k_slots_to_edges(KA<T> a, const int* __restrict__ seid, const T* __restrict__ s,
                                 T* __restrict__ e) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int d = a.d;
    int s0, cnt, st;
    row_slots(a, i, s0, cnt, st);
    for (int k = 0; k < cnt; ++k) {
        int sl = s0 + k * st;
        int j = a.scol[sl];
        if (j <= i || seid[sl] < 0) continue;
        size_t eo = (size_t)seid[sl] * d, so = (size_t)sl * d;
        for (int c = 0; c < d; ++c) e[eo + c] = s[so + c];
    }
}

// per-edge storage (lower slots of the later pixel, orientation later minus
// earlier) <-> per-undirected-edge blocks (earlier minus later): a sign flip
template <typename T>
__global__ void k_half_to_edges(KA<T> a, const int* __restrict__ seid, const T* __restrict__ s, T* __restrict__ e) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int d = a.d;
    for (int k = 0; k < a.ell_K / 2; ++k) {
        const size_t sl = (size_t)k * a.n + i;
        if (seid[sl] < 0) continue;
        const size_t eo = (size_t)seid[sl] * d, so = sl * d;
        for (int c = 0; c < d; ++c) e[eo + c] = -s[so + c];
    }
}

template <typename T>
__global__ void k_edges_to_half(KA<T> a, const int* __restrict__ seid, const T* __restrict__ e, T* __restrict__ s) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int d = a.d;
    for (int k = 0; k < a.ell_K / 2; ++k) {
        const size_t sl = (size_t)k * a.n + i;
        const size_t so = sl * d;
        if (seid[sl] < 0) {
            for (int c = 0; c < d; ++c) s[so + c] = T(0);
            continue;
        }
        const size_t eo = (size_t)seid[sl] * d;
        for (int c = 0; c < d; ++c) s[so + c] = -e[eo + c];
    }
}

template <typename T>
__global__ void k_edges_to_slots(KA<T> a, const int* __restrict__ seid, const T* __restrict__ e,
                                 T* __restrict__ s) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int d = a.d;
    int s0, cnt, st;
    row_slots(a, i, s0, cnt, st);
    for (int k = 0; k < cnt; ++k) {
        int sl = s0 + k * st;
        size_t so = (size_t)sl * d;
        if (seid[sl] < 0) {
            for (int c = 0; c < d; ++c) s[so + c] = T(0);
            continue;
        }
        size_t eo = (size_t)seid[sl] * d;
        bool up = a.scol[sl] > i;
        for (int c = 0; c < d; ++c) s[so + c] = up ? e[eo + c] : -e[eo + c];
    }
}

// mask bit c set when column c (< 32) of rows [r0, r1) of Y has a nonzero
// entry: a bit mask per thread, OR-reduced in LDS, one atomic per workgroup
template <typename T>
__global__ void k_col_flags(const T* __restrict__ Y, int64_t r0, int64_t r1, int d, unsigned* __restrict__ mask) {
    __shared__ unsigned s_mask;
    if (threadIdx.x == 0) s_mask = 0u;
    __syncthreads();
    const size_t ne = (size_t)(r1 - r0) * d;
    unsigned m = 0u;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += (size_t)gridDim.x * blockDim.x)
        if (Y[(size_t)r0 * d + e] != T(0)) m |= 1u << (unsigned)(e % d);
    if (m) atomicOr(&s_mask, m);
    __syncthreads();
    if (threadIdx.x == 0 && s_mask) atomicOr(mask, s_mask);
}

template <typename T>
__global__ void k_fill(size_t n, T v, T* __restrict__ out) {
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) out[e] = v;
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
    const int nq = 3 + 2 * npair;
    const int rb = a.row0[lb], re = a.row0[lb + 1];
    double* pz = sh;
    double* yz = sh + kBlock;
    double obj = 0.0, spl = 0.0, pp = 0.0;
    double g1[2] = {0.0, 0.0}, g2[2] = {0.0, 0.0};
    int pa[2] = {0, 0}, pb[2] = {0, 0};
    for (int h = 0; h < 2; ++h) {
        int k = t + h * (int)blockDim.x;
        if (k < npair) pair_of(k, d, pa[h], pb[h]);
    }
    for (int base = rb; base < re; base += R) {
        int rows = min(R, re - base);
        if (t < rows * d) {
            int rl = t / d, c = t - rl * d;
            int i = base + rl;
            size_t e = (size_t)i * d + c;
            T yh = mul_t(a.isqrtD[i], a.P[e]);
            int s0, cnt, st;
            row_slots(a, i, s0, cnt, st);
            for (int k = 0; k < cnt; ++k) {
                int s = s0 + k * st;
                int j = a.scol[s];
                if (j <= i) continue;
                T yj = mul_t(a.isqrtD[j], a.P[(size_t)j * d + c]);
                obj += fabs((double)a.sw[s] * ((double)yh - (double)yj));
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
    if (last_block(a.bar + kBarLast, a.nblk)) {
        // per segment: its Gram matrices against I; sums over all segments
        double* tot = sh + 2048;
        double s_obj = 0.0, s_spl = 0.0, s_pp = 0.0, cmax = 0.0, omax = 0.0;
        for (int sg = 0; sg < a.nseg; ++sg) {
            reduce_range(a.part, 1, a.seg_blk0[sg], a.seg_blk0[sg + 1], nq, 1, tot, sh);  // part[b * nq + k]
            if (t == 0) {
                s_obj += tot[0];
                s_spl += tot[1];
                s_pp += tot[2];
                const int da = a.dact ? a.dact[sg] : d;
                for (int k = 0; k < npair; ++k) {
                    int r, cc;
                    pair_of(k, d, r, cc);
                    if (r >= da || cc >= da) continue;
                    double id = (r == cc) ? 1.0 : 0.0;
                    omax = fmax(omax, fabs(tot[3 + k] - id));
                    cmax = fmax(cmax, fabs(tot[3 + npair + k] - id));
                }
            }
            __syncthreads();
        }
        if (t == 0) {
            a.S->mon[0] = s_obj;
            a.S->mon[1] = cmax;
            a.S->mon[2] = sqrt(s_spl) / sqrt(s_pp);
            a.S->mon[3] = omax;
        }
    }
}

// |M Y| histogram passes for the exact order statistic (radix select on the
// bit pattern of the non-negative value).
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
        int s0, cnt, st;
        row_slots(a, i, s0, cnt, st);
        for (int k = 0; k < cnt; ++k) {
            int s = s0 + k * st;
            int j = a.scol[s];
            if (j <= i) continue;
            T v = fabs(mul_t(a.sw[s], yi - a.Y[(size_t)j * d + c]));
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

// ---------------------------------------------------------------------------
// FSAI factor (factorized sparse approximate inverse, Kolotilina and Yeremin):
// a non-learned factor of the learned one's form.  Row i of G lives on S_i =
// (the lower neighbours of i) + i and solves A[S_i, S_i] g = e_i, scaled so
// that (G A G^T)_ii = 1.  With A[S_i, S_i] = R R^T (Cholesky, R lower, i last)
// that row is the solution x of R^T x = e_last.  Pixel grids only: the
// stencil-ordered slots [0, K/2) of a row are its lower neighbours, and slot
// K-1-k of the neighbour behind slot k points back (symmetric stencil listed
// in lexicographic order).  A lower slot that leaves the image becomes an
// identity row and column of the local system (it decouples, its x is 0).
// One thread per row, FP64 throughout, A from the FP64 weights
// (A_jj = lambda/2 sum w^2 + r/2 deg_j, A_jk = -lambda/2 w_jk^2).  Stored
// like the learned factor: Gt = G D_A^{1/2} on both slots of every edge (the
// edge's lower-triangular entry) and on the diagonal.
// ---------------------------------------------------------------------------
// nonzero entries of the stored split variable d over the slots of real
// edges (each edge's two slots hold d and -d, so the fraction is per edge)
template <typename T>
__global__ void k_count_nonzero(int64_t nslot, int d, const int* __restrict__ seid, const T* __restrict__ ds,
                                unsigned long long* __restrict__ cnt) {
    __shared__ unsigned long long s_cnt;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    unsigned long long mine = 0;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nslot; s += (int64_t)gridDim.x * blockDim.x) {
        if (seid[s] < 0) continue;
        for (int c = 0; c < d; ++c) mine += (ds[(size_t)s * d + c] != T(0));
    }
    if (mine) atomicAdd(&s_cnt, mine);
    __syncthreads();
    if (threadIdx.x == 0 && s_cnt) atomicAdd(cnt, s_cnt);
}

struct FsaiArgs {
    int64_t n;
    const int* scol;
    const double* sw;
    const double* degree;
    const double* wsq;
    double hl, hr;       // lambda / 2, r / 2
    int* err;
};

// stencil offset of slot k (lexicographic (dy, dx) order of the 4-neighbour
// cross, the 3x3 window or the 5x5 window without its centre) and the slot of
// an offset (-1 outside the stencil)
template <int KC>
__host__ __device__ constexpr int sten_off(int k, bool want_dy) {
    if (KC == 4) {
        const int dy[4] = {-1, 0, 0, 1}, dx[4] = {0, -1, 1, 0};
        return want_dy ? dy[k] : dx[k];
    }
    const int R = (KC == 8) ? 1 : 2, w = 2 * R + 1, c = R * w + R;
    const int idx = (k < c) ? k : k + 1;
    return want_dy ? idx / w - R : idx % w - R;
}

template <int KC>
__host__ __device__ constexpr int sten_slot(int dy, int dx) {
    if (KC == 4) {
        if (dy == -1 && dx == 0) return 0;
        if (dy == 0 && dx == -1) return 1;
        if (dy == 0 && dx == 1) return 2;
        if (dy == 1 && dx == 0) return 3;
        return -1;
    }
    const int R = (KC == 8) ? 1 : 2, w = 2 * R + 1, c = R * w + R;
    if (dy < -R || dy > R || dx < -R || dx > R || (dy == 0 && dx == 0)) return -1;
    const int idx = (dy + R) * w + (dx + R);
    return idx < c ? idx : idx - 1;
}

// every slot maps back to itself, offsets ascend lexicographically, and slot
// K-1-k holds the negated offset of slot k
template <int KC>
constexpr bool sten_table_ok() {
    for (int k = 0; k < KC; ++k) {
        const int dy = sten_off<KC>(k, true), dx = sten_off<KC>(k, false);
        if (sten_slot<KC>(dy, dx) != k) return false;
        if (sten_off<KC>(KC - 1 - k, true) != -dy || sten_off<KC>(KC - 1 - k, false) != -dx) return false;
        if (k > 0) {
            const int py = sten_off<KC>(k - 1, true), px = sten_off<KC>(k - 1, false);
            if (!(py < dy || (py == dy && px < dx))) return false;
        }
    }
    return true;
}
static_assert(sten_table_ok<4>() && sten_table_ok<8>() && sten_table_ok<24>(), "stencil table");

// A_jk for the lower neighbours j (slot a of row i) and k (slot b): the slot of
// row j at offset off_b - off_a, if that offset is in the stencil and the slot
// points at k (both pixels are inside the image, so it does when they are
// neighbours)
template <int KC>
__device__ __forceinline__ double fsai_pair(const FsaiArgs& f, int a, int b, int j, int k) {
    const int q = sten_slot<KC>(sten_off<KC>(b, true) - sten_off<KC>(a, true),
                                sten_off<KC>(b, false) - sten_off<KC>(a, false));
    if (q < 0) return 0.0;
    const size_t s = (size_t)q * f.n + j;
    if (f.scol[s] != k) return 0.0;
    const double w = f.sw[s];
    return -f.hl * w * w;
}

template <typename T, int KC>
__global__ void __launch_bounds__(64) k_fsai(FsaiArgs f, T* __restrict__ gval, T* __restrict__ gdiag) {
    constexpr int H = KC / 2, MM = H + 1;
    const int64_t n = f.n;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int jj[MM];
    bool act[MM];
    double dA[MM];
#pragma unroll
    for (int a = 0; a < H; ++a) {
        const int j = f.scol[(size_t)a * n + i];
        jj[a] = j;
        act[a] = j < i;
        dA[a] = act[a] ? f.hl * f.wsq[j] + f.hr * f.degree[j] : 1.0;
    }
    jj[H] = (int)i;
    act[H] = true;
    dA[H] = f.hl * f.wsq[i] + f.hr * f.degree[i];
    double R[MM][MM];
#pragma unroll
    for (int a = 0; a < MM; ++a) {
#pragma unroll
        for (int b = 0; b < a; ++b) {
            double v = 0.0;
            if (act[a] && act[b]) {
                if (a == H) {
                    const double w = f.sw[(size_t)b * n + i];
                    v = -f.hl * w * w;
                } else {
                    v = fsai_pair<KC>(f, a, b, jj[a], jj[b]);
                }
            }
            R[a][b] = v;
        }
        R[a][a] = dA[a];
    }
    // Cholesky, lower, in place
    bool ok = true;
#pragma unroll
    for (int c = 0; c < MM; ++c) {
        double p = R[c][c];
#pragma unroll
        for (int k = 0; k < c; ++k) p -= R[c][k] * R[c][k];
        if (!(p > 0.0)) { ok = false; p = 1.0; }
        const double rc = sqrt(p), inv = 1.0 / rc;
        R[c][c] = rc;
#pragma unroll
        for (int a = c + 1; a < MM; ++a) {
            double v = R[a][c];
#pragma unroll
            for (int k = 0; k < c; ++k) v -= R[a][k] * R[c][k];
            R[a][c] = v * inv;
        }
    }
    if (!ok) atomicOr(f.err, 1);
    // R^T x = e_last
    double x[MM];
    x[H] = 1.0 / R[H][H];
#pragma unroll
    for (int k = H - 1; k >= 0; --k) {
        double v = 0.0;
#pragma unroll
        for (int l = k + 1; l < MM; ++l) v -= R[l][k] * x[l];
        x[k] = v / R[k][k];
    }
    gdiag[i] = (T)(x[H] * sqrt(dA[H]));
#pragma unroll
    for (int a = 0; a < H; ++a) {
        const T gv = act[a] ? (T)(x[a] * sqrt(dA[a])) : T(0);
        gval[(size_t)a * n + i] = gv;
        if (act[a]) {
            const size_t mirror = (size_t)(KC - 1 - a) * n + jj[a];
            if (f.scol[mirror] == (int)i) gval[mirror] = gv;
            else atomicOr(f.err, 2);
        }
    }
}

}  // namespace pfe

// ===========================================================================
// Host side
// ===========================================================================
using namespace pfe;

// Row partition of nblk logical workgroups over the segments (contiguous row
// ranges; every workgroup inside one segment).
struct Partition {
    int nblk = 0;
    int team = 1;             // workgroups per team (cyclic chunk ownership)
    int max_np = 0;           // largest number of R-row chunks of one workgroup
    int* row0 = nullptr;      // device, nblk + 1
    int* bit = nullptr;       // device, 3 nblk: first row, end row, stride
    int* blk_seg = nullptr;   // device, nblk
    int* seg_blk0 = nullptr;  // device, nseg + 1
    int* geo = nullptr;       // device, 8 nblk: strip geometry (strip partitions), or the image
                              // {row0, W, H} of each workgroup (pixel partitions of pixel grids)
};

struct pfe_ctx {
    pfe_graph* g = nullptr;
    pfe_params prm{};
    hipStream_t stream = nullptr;
    int device = 0;
    int esz = 4;
    int64_t n = 0, d = 0;
    int nseg = 1;
    int inner = 0;           // inner iterations done in the current SOC iteration
    Partition pm;            // multi-launch partition
    Partition pc;            // persistent partition (pc.nblk == 0: not available)
    Partition ps;            // strip partition of pixel grids (ps.nblk == 0: not available)
    Partition pl;            // strips with a two-radius halo (fused learned apply)
    Partition pf;            // strips with a three-radius halo (one-pass factor CG)
    Partition px[2];         // pixel launches: contiguous pixel (row) ranges, one / two workgroups
                             // per CU (nblk == 0: not available)
    int want_px = 0;         // Jacobi PCG by the per-pixel (per-row) kernels
                             // on px[want_px - 1] (0: not)
    int one_pass = 0;        // factor preconditioners on strips: one pass per CG iteration (0: two)
    int eu_px = 1;           // pixel stencils with b once per edge: the edge update by the per-pixel
                             // kernel (0: by the strip or row-chunk phase kernel)
    int eur_px = 1;          // per-row Jacobi PCG: edge updates that also form the next solve's residual
    int want_strips = 2;     // one launch per phase: residual, w0 and CG kernels on image strips sized
                             // for this many waves of co-resident strip workgroups (0: row chunks)
    int strip_slots = 0;     // co-resident strip workgroups on the device (0: no strip kernel)
    int fcg_slots = 0;       // co-resident workgroups of the one-pass factor CG kernel
    int fcg_cpl = 1;         // its columns per lane
    int ps_waves = 0;        // waves the strip partition was built for
    int part_blocks = 0;     // workgroups the partial-sum buffer holds
    void* Y = nullptr; void* P = nullptr; void* B = nullptr;
    void* bs = nullptr; void* ds = nullptr;
    void* bs2 = nullptr;     // second b buffer (per-edge storage: read one, write the other)
    int bhalf = 0;           // b, d once per undirected edge (pixel stencils), else per slot
    int64_t sslots = 0;      // storage slots of b and d
    void* rhs = nullptr; void* p = nullptr;
    void* rb[2] = {nullptr, nullptr};
    void* wb[2] = {nullptr, nullptr};
    void* sb[2] = {nullptr, nullptr};
    void* diagA = nullptr; void* invdiag = nullptr; void* sqrtD = nullptr; void* isqrtD = nullptr;
    void* isq = nullptr;       // D_A^{-1/2}
    void* gval = nullptr;      // learned factor per slot
    void* gdiag = nullptr;
    void* zl = nullptr;
    void* y1 = nullptr;
    void* xbak = nullptr;      // start of a factor-preconditioned solve (Jacobi fallback)
    int* dact = nullptr;       // per segment: active (leading) columns of Y0, when some segment has fewer than d
    std::vector<int> dact_h;
    int have_factor = 0;
    double* part = nullptr;
    double* gpart = nullptr;
    double* Tm = nullptr;
    double* colbuf = nullptr;
    int* colint = nullptr;
    int cache_np = 0;        // persistent kernel: LDS row cache chunks (0: no cache)
    int launched_coop = 0;   // the last advance ran the persistent kernel
    int fused_eur = 0;       // the last advance fused edge updates with the next residual
    // persistent launch shape
    std::vector<int64_t> seg_rows;
    int per_cu = 0;          // co-resident workgroups per CU
    int64_t coop = 0;        // persistent grid size (0: none)
    int team = 64;           // workgroups per team (cyclic chunk ownership)
    double second_weight = 1.0;   // persistent: rows of the second workgroup on each CU, relative
    int want_cache = 1;      // use the LDS row cache when the rows fit
    // one-launch-per-phase PCG replayed from a HIP graph of kCgChunk iterations
    hipGraphExec_t cg_exec = nullptr;
    std::vector<unsigned char> cg_key;   // kernel arguments the graph was built with
    ColState cs{};
    Scal* S = nullptr;
    unsigned* bar = nullptr;
    unsigned* hist = nullptr;
};

namespace {

#define PFE_TRY(x) do { pfe_status s__ = (x); if (s__ != PFE_OK) return s__; } while (0)

// Teams: runs of at most team_max consecutive logical workgroups of the same
// segment and the same XCD band (logical index / (nblk / 8) when nblk is a
// multiple of 8).  Member j of a team of m owning rows [b, e) takes the R-row
// chunks b + (j + k m) R.
static void team_iteration(const std::vector<int>& row0, const std::vector<int>& bseg, int R, int team_max,
                           std::vector<int>& bit) {
    const int nblk = (int)bseg.size();
    const int band = (nblk % kNumXcd == 0) ? nblk / kNumXcd : nblk;
    bit.assign(3 * (size_t)nblk, 0);
    int t0 = 0;
    while (t0 < nblk) {
        int t1 = t0 + 1;
        while (t1 < nblk && t1 - t0 < team_max && bseg[t1] == bseg[t0] && t1 / band == t0 / band) ++t1;
        const int m = t1 - t0;
        for (int j = 0; j < m; ++j) {
            bit[3 * (t0 + j)] = row0[t0] + j * R;
            bit[3 * (t0 + j) + 1] = row0[t1];
            bit[3 * (t0 + j) + 2] = m * R;
        }
        t0 = t1;
    }
}

// second_weight: share of rows, relative to the others, of the logical
// workgroups in the upper half of each XCD band (with two co-resident
// workgroups per CU and nblk a multiple of 16 these are the physical blocks
// nblk / 2 .. nblk - 1, the second workgroup placed on each CU); 1: equal rows
pfe_status make_partition(const std::vector<int64_t>& seg_rows, int want_blocks, int R, int team_max,
                          Partition& P, double second_weight = 1.0) {
    // workgroups per segment proportional to its rows (at least one each)
    const int nseg = (int)seg_rows.size();
    int64_t n = 0;
    for (auto r : seg_rows) n += r;
    std::vector<int> nb(nseg, 1);
    int total = nseg;
    if (want_blocks > nseg) {
        int extra = want_blocks - nseg;
        for (int s = 0; s < nseg; ++s) {
            int k = (int)((double)extra * (double)seg_rows[s] / (double)n);
            k = (int)std::min<int64_t>(k, std::max<int64_t>(0, seg_rows[s] - 1));
            nb[s] += k;
            total += k;
        }
        // top up to the requested count, largest rows-per-workgroup first
        while (total < want_blocks) {
            int best = -1;
            for (int q = 0; q < nseg; ++q)
                if (nb[q] < seg_rows[q] && (best < 0 || (double)seg_rows[q] / nb[q] > (double)seg_rows[best] / nb[best]))
                    best = q;
            if (best < 0) break;
            nb[best] += 1;
            ++total;
        }
    }
    std::vector<int> row0(total + 1), bseg(total), sb0(nseg + 1);
    const int band = (total % (2 * kNumXcd) == 0) ? total / kNumXcd : 0;
    auto weight = [&](int blk) { return (band > 0 && blk % band >= band / 2) ? second_weight : 1.0; };
    int b = 0;
    int64_t base = 0;
    for (int s = 0; s < nseg; ++s) {
        sb0[s] = b;
        double wsum = 0.0;
        for (int k = 0; k < nb[s]; ++k) wsum += weight(b + k);
        double acc = 0.0;
        for (int k = 0; k < nb[s]; ++k) {
            row0[b] = (int)(base + (int64_t)std::llround((double)seg_rows[s] * acc / wsum));
            acc += weight(b);
            bseg[b] = s;
            ++b;
        }
        base += seg_rows[s];
    }
    row0[total] = (int)base;
    sb0[nseg] = total;
    P.nblk = total;
    P.team = std::max(1, team_max);
    std::vector<int> bit;
    team_iteration(row0, bseg, R, P.team, bit);
    P.max_np = 0;
    for (int b = 0; b < total; ++b) {
        const int rb = bit[3 * b], re = bit[3 * b + 1], rs = bit[3 * b + 2];
        if (re > rb) P.max_np = std::max(P.max_np, (re - rb + rs - 1) / rs);
    }
    PFE_CHECK_HIP(dev_alloc((void**)&P.bit, sizeof(int) * bit.size()));
    PFE_CHECK_HIP(hipMemcpy(P.bit, bit.data(), sizeof(int) * bit.size(), hipMemcpyHostToDevice));
    PFE_CHECK_HIP(dev_alloc((void**)&P.row0, sizeof(int) * (total + 1)));
    PFE_CHECK_HIP(dev_alloc((void**)&P.blk_seg, sizeof(int) * total));
    PFE_CHECK_HIP(dev_alloc((void**)&P.seg_blk0, sizeof(int) * (nseg + 1)));
    PFE_CHECK_HIP(hipMemcpy(P.row0, row0.data(), sizeof(int) * (total + 1), hipMemcpyHostToDevice));
    PFE_CHECK_HIP(hipMemcpy(P.blk_seg, bseg.data(), sizeof(int) * total, hipMemcpyHostToDevice));
    PFE_CHECK_HIP(hipMemcpy(P.seg_blk0, sb0.data(), sizeof(int) * (nseg + 1), hipMemcpyHostToDevice));
    return PFE_OK;
}

void free_partition(Partition& P) {
    if (P.geo) (void)dev_free(P.geo);
    if (P.row0) (void)dev_free(P.row0);
    if (P.bit) (void)dev_free(P.bit);
    if (P.blk_seg) (void)dev_free(P.blk_seg);
    if (P.seg_blk0) (void)dev_free(P.seg_blk0);
    P = Partition{};
}

// Strip partition of a graph whose segments are pixel grids with a compiled
// stencil width (4, 8, 24 slots): image s is cut into nsx column strips of at
// most kBlock / d - 2 halos rho pixels (equal widths up to one pixel; halos = 1
// for the one-hop phases, 2 for the fused learned apply) and nsy bands
// of image rows (at least kStripMinRows rows each), the number of workgroups
// of each image proportional to its pixels.  Logical workgroups run in the
// order (image, band, strip), so the consecutive workgroups that one XCD holds
// are horizontally adjacent strips and share the cache lines at their borders.
// The count is padded to a multiple of the XCD count with empty workgroups.
constexpr int kStripMinRows = 16;

pfe_status make_strip_partition(const pfe_graph* g, int d, int want_blocks, int halos, Partition& P) {
    free_partition(P);
    int min_rows = kStripMinRows;
    if (const char* ev = getenv("PFE_STRIP_MINROWS")) min_rows = std::max(1, atoi(ev));   // launch-shape experiments
    const int K = g->ell_K;
    const int nseg = (int)g->seg_row0.size() - 1;
    if (!g->stencil || !(K == 4 || K == 8 || K == 24) || (int)g->seg_W.size() != nseg) return PFE_OK;
    for (int s = 0; s < nseg; ++s)
        if (g->seg_W[s] < 1 || g->seg_H[s] < 1) return PFE_OK;
    const int rho = (K == 24) ? 2 : 1;
    const int L = kBlock / d - 2 * halos * rho;   // a ring row spans halos stencil radii on each side
    if (L < 1) return PFE_OK;
    const double n = (double)g->n;
    std::vector<int> geo, bseg, sb0(nseg + 1);
    for (int s = 0; s < nseg; ++s) {
        const int W = g->seg_W[s], H = g->seg_H[s], row0 = (int)g->seg_row0[s];
        const int nsx = (W + L - 1) / L;
        const double ns = (double)W * H;
        int nsy = (int)std::llround((double)want_blocks * ns / (n * nsx));
        nsy = std::min(nsy, std::max(1, H / min_rows));
        nsy = std::max(1, std::min(nsy, H));
        sb0[s] = (int)bseg.size();
        for (int sy = 0; sy < nsy; ++sy) {
            const int y0 = (int)((int64_t)H * sy / nsy), y1 = (int)((int64_t)H * (sy + 1) / nsy);
            for (int sx = 0; sx < nsx; ++sx) {
                const int x0 = (int)((int64_t)W * sx / nsx), x1 = (int)((int64_t)W * (sx + 1) / nsx);
                const int gv[8] = {row0, W, H, x0, x1 - x0, y0, y1, 0};
                geo.insert(geo.end(), gv, gv + 8);
                bseg.push_back(s);
            }
        }
    }
    while (bseg.size() % kNumXcd) {
        const int s = nseg - 1;
        const int gv[8] = {(int)g->seg_row0[s], g->seg_W[s], g->seg_H[s], 0, 0, 0, 0, 0};
        geo.insert(geo.end(), gv, gv + 8);
        bseg.push_back(s);
    }
    const int total = (int)bseg.size();
    sb0[nseg] = total;
    std::vector<int> zeros(3 * (size_t)total + 1, 0);
    P.nblk = total;
    P.team = 1;
    P.max_np = 0;
    PFE_CHECK_HIP(dev_alloc((void**)&P.geo, sizeof(int) * geo.size()));
    PFE_CHECK_HIP(dev_alloc((void**)&P.bit, sizeof(int) * 3 * total));
    PFE_CHECK_HIP(dev_alloc((void**)&P.row0, sizeof(int) * (total + 1)));
    PFE_CHECK_HIP(dev_alloc((void**)&P.blk_seg, sizeof(int) * total));
    PFE_CHECK_HIP(dev_alloc((void**)&P.seg_blk0, sizeof(int) * (nseg + 1)));
    PFE_CHECK_HIP(hipMemcpy(P.geo, geo.data(), sizeof(int) * geo.size(), hipMemcpyHostToDevice));
    PFE_CHECK_HIP(hipMemcpy(P.bit, zeros.data(), sizeof(int) * 3 * total, hipMemcpyHostToDevice));
    PFE_CHECK_HIP(hipMemcpy(P.row0, zeros.data(), sizeof(int) * (total + 1), hipMemcpyHostToDevice));
    PFE_CHECK_HIP(hipMemcpy(P.blk_seg, bseg.data(), sizeof(int) * total, hipMemcpyHostToDevice));
    PFE_CHECK_HIP(hipMemcpy(P.seg_blk0, sb0.data(), sizeof(int) * (nseg + 1), hipMemcpyHostToDevice));
    return PFE_OK;
}

template <typename T>
KA<T> make_args(pfe_ctx* c, const Partition& pt) {
    KA<T> a{};
    a.n = (int)c->n;
    a.d = (int)c->d;
    a.R = kBlock / (int)c->d;
    a.nblk = pt.nblk;
    a.nseg = c->nseg;
    a.ell_K = c->g->ell_K;
    a.row0 = pt.row0;
    a.bit = pt.bit;
    a.blk_seg = pt.blk_seg;
    a.seg_blk0 = pt.seg_blk0;
    a.geo = pt.geo;
    a.rowptr = c->g->rowptr;
    a.scol = c->g->s_col;
    if (sizeof(T) == 4) a.sw = (const T*)c->g->s_w32; else a.sw = (const T*)c->g->s_w64;
    a.diagA = (const T*)c->diagA;
    a.invdiag = (const T*)c->invdiag;
    a.sqrtD = (const T*)c->sqrtD;
    a.isqrtD = (const T*)c->isqrtD;
    a.degree = c->g->degree;
    a.x = (T*)c->Y;
    a.Y = (T*)c->Y;
    a.P = (T*)c->P;
    a.B = (T*)c->B;
    a.bsb[0] = (T*)c->bs;
    a.bsb[1] = c->bs2 ? (T*)c->bs2 : (T*)c->bs;
    a.ds = (T*)c->ds;
    a.bhalf = c->bhalf;
    a.bpar = 0;
    a.rhs = (T*)c->rhs;
    for (int k = 0; k < 2; ++k) {
        a.rb[k] = (T*)c->rb[k];
        a.wb[k] = (T*)c->wb[k];
        a.sb[k] = (T*)c->sb[k];
    }
    a.p = (T*)c->p;
    a.gval = (const T*)c->gval;
    a.gdiag = (const T*)c->gdiag;
    a.isq = (const T*)c->isq;
    a.zl = (T*)c->zl;
    a.y1 = (T*)c->y1;
    a.part = c->part;
    a.gpart = c->gpart;
    a.Tm = c->Tm;
    a.cs = c->cs;
    a.S = c->S;
    a.bar = c->bar;
    a.c_off = (T)(0.5 * c->prm.lambda);
    a.gamma = (c->prm.lambda > 0.0) ? (T)(1.0 / c->prm.lambda) : (T)INFINITY;
    a.half_r = (T)(0.5 * c->prm.r);
    a.tol2 = c->prm.tol * c->prm.tol;
    a.maxit = c->prm.maxit;
    a.keep_split = c->prm.keep_split;
    a.store_rhs = 0;
    a.b_zero = 0;
    a.ortho = c->prm.ortho;
    a.sten = c->g->stencil;
    a.dact = c->dact;
    return a;
}

// launch kernel template K<T, KC> with KC the graph's ELL width when it has a
// specialisation (4, 8, 24), else the generic loops (KC = 0)
#define PFE_LAUNCH_KC(K, ellK, grid, stream, ...)                                                   \
    do {                                                                                           \
        switch (ellK) {                                                                            \
            case 4: hipLaunchKernelGGL((K<T, 4>), grid, dim3(kBlock), 0, stream, __VA_ARGS__); break; \
            case 8: hipLaunchKernelGGL((K<T, 8>), grid, dim3(kBlock), 0, stream, __VA_ARGS__); break; \
            case 24: hipLaunchKernelGGL((K<T, 24>), grid, dim3(kBlock), 0, stream, __VA_ARGS__); break; \
            default: hipLaunchKernelGGL((K<T, 0>), grid, dim3(kBlock), 0, stream, __VA_ARGS__); break; \
        }                                                                                          \
    } while (0)

// strip kernel K<T, KC> for the stencil width (strip partitions exist only for 4, 8, 24)
#define PFE_LAUNCH_ST(K, ellK, grid, stream, ...)                                                   \
    do {                                                                                           \
        switch (ellK) {                                                                            \
            case 4: hipLaunchKernelGGL((K<T, 4>), grid, dim3(kBlock), 0, stream, __VA_ARGS__); break; \
            case 8: hipLaunchKernelGGL((K<T, 8>), grid, dim3(kBlock), 0, stream, __VA_ARGS__); break; \
            case 24: hipLaunchKernelGGL((K<T, 24>), grid, dim3(kBlock), 0, stream, __VA_ARGS__); break; \
            default: set_error("strip kernels need a stencil of 4, 8 or 24 slots"); return PFE_E_STATE; \
        }                                                                                          \
    } while (0)

// pixel launch kernels of the ELL width K and V columns per thread
template <typename T, int V>
const void* px_kernel(int ph, int K) {
#define PFE_PXSEL(KN) switch (K) {                                                      \
        case 4: return reinterpret_cast<const void*>(&KN<T, 4, V>);                    \
        case 8: return reinterpret_cast<const void*>(&KN<T, 8, V>);                    \
        case 24: return reinterpret_cast<const void*>(&KN<T, 24, V>);                  \
        default: return reinterpret_cast<const void*>(&KN<T, 0, V>); }
#define PFE_PXSEL_ST(KN) switch (K) {                                                   \
        case 4: return reinterpret_cast<const void*>(&KN<T, 4, V>);                    \
        case 8: return reinterpret_cast<const void*>(&KN<T, 8, V>);                    \
        case 24: return reinterpret_cast<const void*>(&KN<T, 24, V>);                  \
        default: return nullptr; }
    switch (ph) {
        case PH_R0: PFE_PXSEL(k_px_res)
        case PH_W0: PFE_PXSEL(k_px_w0)
        case PH_IT: PFE_PXSEL(k_px_gb)
        case PH_GA: return reinterpret_cast<const void*>(&k_px_ga<T, V>);
        case PH_LA: PFE_PXSEL_ST(k_pl_a)
        case PH_LC: PFE_PXSEL_ST(k_pl_c)
        case PH_LD: PFE_PXSEL_ST(k_pl_d)
        default: return nullptr;
    }
#undef PFE_PXSEL
#undef PFE_PXSEL_ST
}

// columns per thread of the per-pixel kernels: 16-byte accesses where d allows
template <typename T>
int px_cols(int d) {
    static const int force = getenv("PFE_PX_COLS") ? atoi(getenv("PFE_PX_COLS")) : 0;   // launch-shape experiments
    if ((force == 1 || force == 2 || force == 4) && d % force == 0 && force * (int)sizeof(T) <= 16) return force;
    // (on the 64-image batch, d = 10, two columns per thread ran a SOC
    // iteration in 71.6 ms against 74.8 ms for one)
    return (sizeof(T) == 4) ? ((d % 4 == 0) ? 4 : ((d % 2 == 0) ? 2 : 1)) : ((d % 2 == 0) ? 2 : 1);
}

template <typename T>
const void* px_kernel_for(int ph, int K, int d) {
    const int V = px_cols<T>(d);
    if constexpr (sizeof(T) == 4) {
        if (V == 4) return px_kernel<T, 4>(ph, K);
    }
    if (V == 2) return px_kernel<T, 2>(ph, K);
    return px_kernel<T, 1>(ph, K);
}

template <typename T>
pfe_status launch_phase(pfe_ctx* c, const KA<T>& a, int ph, int mode, int do_r0) {
    const dim3 grid(a.nblk);
    hipStream_t st = c->stream;
    const int K = a.ell_K;
    if (a.pxl) {
        // pixel launch: the residual with r0, w0 and the CG iteration (two
        // kernels); stencil offsets on pixel grids, the slot columns otherwise
        const int KP = a.geo ? K : 0;
        KA<T> args = a;
        int pm = ph;
        void* kp1[] = {(void*)&args};
        void* kp2[] = {(void*)&args, (void*)&pm};
        const void* fn = nullptr;
        if ((ph == PH_E0 || ph == PH_R0) && do_r0) {
            fn = px_kernel_for<T>(PH_R0, KP, a.d);
            if (fn) { PFE_CHECK_HIP(hipLaunchKernel(fn, grid, dim3(kBlock), kp2, 0, st)); return PFE_OK; }
        } else if (ph == PH_W0) {
            fn = px_kernel_for<T>(PH_W0, KP, a.d);
            if (fn) { PFE_CHECK_HIP(hipLaunchKernel(fn, grid, dim3(kBlock), kp1, 0, st)); return PFE_OK; }
        } else if (ph == PH_IT) {
            const void* fa = px_kernel_for<T>(PH_GA, KP, a.d);
            fn = px_kernel_for<T>(PH_IT, KP, a.d);
            if (fa && fn) {
                PFE_CHECK_HIP(hipLaunchKernel(fa, grid, dim3(kBlock), kp1, 0, st));
                PFE_CHECK_HIP(hipLaunchKernel(fn, grid, dim3(kBlock), kp1, 0, st));
                return PFE_OK;
            }
        } else if (ph == PH_LA || ph == PH_LC || ph == PH_LD) {
            // factor-preconditioned PCG (pixel grids); PH_LC: mode = update, PH_LD: mode = initial
            fn = px_kernel_for<T>(ph, KP, a.d);
            pm = mode;
            if (fn) {
                PFE_CHECK_HIP(hipLaunchKernel(fn, grid, dim3(kBlock), ph == PH_LA ? kp1 : kp2, 0, st));
                return PFE_OK;
            }
        }
        set_error("phase %d has no pixel-launch kernel", ph);
        return PFE_E_STATE;
    }
    if (a.geo) {
        // strip partition: only the phases with a strip kernel
        switch (ph) {
            case PH_E0: case PH_R0:
                if (!do_r0) break;
                PFE_LAUNCH_ST(k_st_res, K, grid, st, a, ph);
                PFE_CHECK_HIP(hipGetLastError());
                return PFE_OK;
            case PH_EU:
                if (do_r0 || !a.store_rhs) break;
                PFE_LAUNCH_ST(k_st_eu, K, grid, st, a);
                PFE_CHECK_HIP(hipGetLastError());
                return PFE_OK;
            case PH_W0: PFE_LAUNCH_ST(k_st_w0, K, grid, st, a); PFE_CHECK_HIP(hipGetLastError()); return PFE_OK;
            case PH_LA: PFE_LAUNCH_ST(k_st_la, K, grid, st, a); PFE_CHECK_HIP(hipGetLastError()); return PFE_OK;
            case PH_LC: PFE_LAUNCH_ST(k_st_lc, K, grid, st, a, mode); PFE_CHECK_HIP(hipGetLastError()); return PFE_OK;
            case PH_LD: PFE_LAUNCH_ST(k_st_ld, K, grid, st, a, mode); PFE_CHECK_HIP(hipGetLastError()); return PFE_OK;
            case PH_LCD: PFE_LAUNCH_ST(k_st_lcd, K, grid, st, a, mode); PFE_CHECK_HIP(hipGetLastError()); return PFE_OK;
            case PH_FW0: case PH_FIT: {
                const void* fn = fcg_kernel<T>(K, c->fcg_cpl);
                if (!fn) break;
                KA<T> args = a;
                int fmode = (ph == PH_FIT) ? 1 : 0;
                void* kp[] = {(void*)&args, (void*)&fmode};
                PFE_CHECK_HIP(hipLaunchKernel(fn, grid, dim3(kBlock), kp, 0, st));
                return PFE_OK;
            }
            case PH_IT: PFE_LAUNCH_ST(k_st_it, K, grid, st, a); PFE_CHECK_HIP(hipGetLastError()); return PFE_OK;
            default: break;
        }
        set_error("phase %d has no strip kernel", ph);
        return PFE_E_STATE;
    }
    switch (ph) {
        case PH_E0: case PH_EU: case PH_R0: case PH_RHS: PFE_LAUNCH_KC(k_residual, K, grid, st, a, ph, do_r0); break;
        case PH_W0: PFE_LAUNCH_KC(k_cg_w0, K, grid, st, a); break;
        case PH_IT:
            if (K == 4 || K == 8 || K == 24) {
                PFE_LAUNCH_KC(k_cg_it, K, grid, st, a);
            } else {
                hipLaunchKernelGGL(k_cg_ga<T>, grid, dim3(kBlock), 0, st, a);
                hipLaunchKernelGGL(k_cg_gb<T>, grid, dim3(kBlock), 0, st, a);
            }
            break;
        case PH_ZERO: hipLaunchKernelGGL(k_cg_zero<T>, grid, dim3(kBlock), 0, st, a); break;
        case PH_LA: PFE_LAUNCH_KC(k_lpcg_aq, K, grid, st, a); break;
        case PH_LC: PFE_LAUNCH_KC(k_lpcg_g, K, grid, st, a, mode); break;
        case PH_LD: PFE_LAUNCH_KC(k_lpcg_gt, K, grid, st, a, mode); break;
        case PH_GRAM: hipLaunchKernelGGL(k_gram<T>, grid, dim3(kBlock), 0, st, a, mode); break;
        case PH_APPLY: hipLaunchKernelGGL(k_apply<T>, grid, dim3(kBlock), 0, st, a, mode); break;
        default: set_error("unknown phase %d", ph); return PFE_E_ARG;
    }
    PFE_CHECK_HIP(hipGetLastError());
    return PFE_OK;
}

// One-launch-per-phase PCG from a HIP graph: kCgChunk iterations (Jacobi: one
// kernel each; learned: the four phases each) as kernel nodes in sequence,
// replayed until the done flag is set (later nodes of a finished solve return
// at once).  Built with the graph API (no stream capture, so any stream works),
// cached per context and rebuilt when the kernel arguments change.
constexpr int kCgChunk = 8;

template <typename T>
const void* kernel_for(int which, int ellK, bool strip, int cpl = 1) {
    if (which == PH_FIT) return fcg_kernel<T>(ellK, cpl);
#define PFE_SSEL(K) switch (ellK) { \
        case 4: return reinterpret_cast<const void*>(&K<T, 4>); \
        case 8: return reinterpret_cast<const void*>(&K<T, 8>); \
        case 24: return reinterpret_cast<const void*>(&K<T, 24>); \
        default: return nullptr; }
    if (strip) {
        switch (which) {
            case PH_IT: PFE_SSEL(k_st_it)
            case PH_LA: PFE_SSEL(k_st_la)
            case PH_LC: PFE_SSEL(k_st_lc)
            case PH_LD: PFE_SSEL(k_st_ld)
            case PH_LCD: PFE_SSEL(k_st_lcd)
        }
        return nullptr;
    }
#undef PFE_SSEL
#define PFE_KSEL(K) switch (ellK) { \
        case 4: return reinterpret_cast<const void*>(&K<T, 4>); \
        case 8: return reinterpret_cast<const void*>(&K<T, 8>); \
        case 24: return reinterpret_cast<const void*>(&K<T, 24>); \
        default: return reinterpret_cast<const void*>(&K<T, 0>); }
    switch (which) {
        case PH_IT: PFE_KSEL(k_cg_it)
        case PH_LA: PFE_KSEL(k_lpcg_aq)
        case PH_LC: PFE_KSEL(k_lpcg_g)
        case PH_LD: PFE_KSEL(k_lpcg_gt)
    }
#undef PFE_KSEL
    return nullptr;
}

template <typename T>
pfe_status cg_chunk_graph(pfe_ctx* c, const KA<T>& a, bool learned, const KA<T>* al, hipGraphExec_t* out,
                          const KA<T>* af = nullptr) {
    // al: arguments of the fused learned apply (strips with a two-radius halo), or null;
    // af: arguments of the one-pass factor CG (strips with a three-radius halo), or null
    std::vector<unsigned char> key(3 * sizeof(KA<T>) + 2, 0);
    std::memcpy(key.data(), &a, sizeof(KA<T>));
    if (al) std::memcpy(key.data() + sizeof(KA<T>), al, sizeof(KA<T>));
    if (af) std::memcpy(key.data() + 2 * sizeof(KA<T>), af, sizeof(KA<T>));
    key[3 * sizeof(KA<T>)] = learned ? 1 : 0;
    key[3 * sizeof(KA<T>) + 1] = (unsigned char)sizeof(T);
    if (c->cg_exec && key == c->cg_key) { *out = c->cg_exec; return PFE_OK; }
    if (c->cg_exec) { (void)hipGraphExecDestroy(c->cg_exec); c->cg_exec = nullptr; }
    hipGraph_t g = nullptr;
    PFE_CHECK_HIP(hipGraphCreate(&g, 0));
    KA<T> args = a;
    KA<T> largs = al ? *al : a;
    KA<T> fargs = af ? *af : a;
    int initial = 0, upd = 1;
    void* p1[] = {(void*)&args};
    void* p2[] = {(void*)&args, (void*)&initial};
    void* p3[] = {(void*)&args, (void*)&upd};
    void* p4[] = {(void*)&largs, (void*)&upd};
    void* p5[] = {(void*)&fargs, (void*)&upd};
    hipGraphNode_t prev = nullptr;
    hipError_t e = hipSuccess;
    auto add = [&](const void* fn, void** kp, int nblk) {
        if (e != hipSuccess) return;
        if (!fn) { e = hipErrorInvalidDeviceFunction; return; }
        hipKernelNodeParams np{};
        np.func = const_cast<void*>(fn);
        np.gridDim = dim3(nblk);
        np.blockDim = dim3(kBlock);
        np.sharedMemBytes = 0;
        np.kernelParams = kp;
        np.extra = nullptr;
        hipGraphNode_t node = nullptr;
        e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &np);
        prev = node;
    };
    const int K = a.ell_K;
    const bool st = a.geo != nullptr;
    for (int k = 0; k < kCgChunk; ++k) {
        if (learned && af) {
            add(kernel_for<T>(PH_FIT, K, true, c->fcg_cpl), p5, af->nblk);
        } else if (learned && a.pxl) {
            add(px_kernel_for<T>(PH_LA, a.geo ? K : 0, a.d), p1, a.nblk);
            add(px_kernel_for<T>(PH_LC, a.geo ? K : 0, a.d), p3, a.nblk);
            add(px_kernel_for<T>(PH_LD, a.geo ? K : 0, a.d), p2, a.nblk);
        } else if (learned) {
            add(kernel_for<T>(PH_LA, K, st), p1, a.nblk);
            if (al) {
                add(kernel_for<T>(PH_LCD, K, true), p4, al->nblk);
            } else {
                add(kernel_for<T>(PH_LC, K, st), p3, a.nblk);
                add(kernel_for<T>(PH_LD, K, st), p2, a.nblk);
            }
        } else if (a.pxl) {
            add(px_kernel_for<T>(PH_GA, a.geo ? K : 0, a.d), p1, a.nblk);
            add(px_kernel_for<T>(PH_IT, a.geo ? K : 0, a.d), p1, a.nblk);
        } else if (!st && K != 4 && K != 8 && K != 24) {
            add(reinterpret_cast<const void*>(&k_cg_ga<T>), p1, a.nblk);
            add(reinterpret_cast<const void*>(&k_cg_gb<T>), p1, a.nblk);
        } else {
            add(kernel_for<T>(PH_IT, K, st), p1, a.nblk);
        }
    }
    hipGraphExec_t ex = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "PCG chunk graph", __FILE__, __LINE__);
    c->cg_exec = ex;
    c->cg_key = key;
    *out = ex;
    return PFE_OK;
}

// replay the chunk graph until the solve is done
template <typename T>
pfe_status pcg_replay(pfe_ctx* c, const KA<T>& a, bool learned, const KA<T>* al = nullptr,
                      const KA<T>* af = nullptr) {
    hipGraphExec_t ex = nullptr;
    PFE_TRY(cg_chunk_graph(c, a, learned, al, &ex, af));
    int it = 0, done = 0;
    while (true) {
        PFE_CHECK_HIP(hipGraphLaunch(ex, c->stream));
        it += kCgChunk;
        PFE_CHECK_HIP(hipMemcpyAsync(&done, &c->S->done, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        PFE_CHECK_HIP(hipStreamSynchronize(c->stream));
        if (done || it > c->prm.maxit + kCgChunk) break;
    }
    return PFE_OK;
}

// Multi-launch PCG after a residual phase (r0 in rb[0]); the host polls the
// done flag every few iterations; the iterate ends in a.x.  w0 and the
// iterations run on the arguments 'as' (the strip partition of a pixel grid,
// or 'a' itself).
template <typename T>
pfe_status pcg_loop_mk(pfe_ctx* c, const KA<T>& a, const KA<T>& as) {
    hipLaunchKernelGGL(k_stats_if_done<T>, dim3(1), dim3(64), 0, c->stream, a);
    PFE_TRY(launch_phase(c, as, PH_W0, 0, 0));
    if (c->prm.graphs) {
        PFE_TRY(pcg_replay(c, as, false));
        return launch_phase(c, a, PH_ZERO, 0, 0);
    }
    int it = 0;
    const int chunk = 4;
    int done = 0;
    while (true) {
        for (int k = 0; k < chunk; ++k) PFE_TRY(launch_phase(c, as, PH_IT, 0, 0));
        it += chunk;
        PFE_CHECK_HIP(hipMemcpyAsync(&done, &c->S->done, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        PFE_CHECK_HIP(hipStreamSynchronize(c->stream));
        if (done || it > c->prm.maxit + chunk) break;
    }
    PFE_TRY(launch_phase(c, a, PH_ZERO, 0, 0));
    return PFE_OK;
}

// Multi-launch PCG with the learned factor after a residual phase (r0 in rb[0]);
// the PCG phases run on the arguments 'as' (strips of a pixel grid, or 'a').
template <typename T>
pfe_status pcg_loop_learned_mk(pfe_ctx* c, const KA<T>& a, const KA<T>& as) {
    // on strips with a three-radius halo: one pass per iteration
    if (as.geo && !as.pxl && c->pf.nblk > 0 && c->one_pass) {
        KA<T> af = make_args<T>(c, c->pf);
        af.x = as.x;       // the iterate and rhs of this solve (a caller's buffers in pfe_pcg)
        af.rhs = as.rhs;
        hipLaunchKernelGGL(k_stats_if_done<T>, dim3(1), dim3(64), 0, c->stream, a);
        PFE_TRY(launch_phase(c, af, PH_FW0, 0, 0));
        if (c->prm.graphs) {
            PFE_TRY(pcg_replay<T>(c, as, true, nullptr, &af));
            return launch_phase(c, a, PH_ZERO, 0, 0);
        }
        int it = 0, done = 0;
        const int chunk = 4;
        while (true) {
            for (int k = 0; k < chunk; ++k) PFE_TRY(launch_phase(c, af, PH_FIT, 0, 0));
            it += chunk;
            PFE_CHECK_HIP(hipMemcpyAsync(&done, &c->S->done, sizeof(int), hipMemcpyDeviceToHost, c->stream));
            PFE_CHECK_HIP(hipStreamSynchronize(c->stream));
            if (done || it > c->prm.maxit + chunk) break;
        }
        return launch_phase(c, a, PH_ZERO, 0, 0);
    }
    // on strips the two factor products run as one kernel on strips with a
    // two-radius halo
    const bool fused = as.geo && !as.pxl && c->pl.nblk > 0;
    KA<T> al = as;
    if (fused) {
        al = make_args<T>(c, c->pl);
        al.x = as.x;       // the iterate and rhs of this solve (a caller's buffers in pfe_pcg)
        al.rhs = as.rhs;
    }
    hipLaunchKernelGGL(k_stats_if_done<T>, dim3(1), dim3(64), 0, c->stream, a);
    if (fused) {
        PFE_TRY(launch_phase(c, al, PH_LCD, 0, 0));    // z and r.z from the initial residual
    } else {
        PFE_TRY(launch_phase(c, as, PH_LC, 0, 0));     // y1 from the initial residual
        PFE_TRY(launch_phase(c, as, PH_LD, 1, 0));     // initial r.z
    }
    if (c->prm.graphs) {
        PFE_TRY(pcg_replay(c, as, true, fused ? &al : nullptr));
        return launch_phase(c, a, PH_ZERO, 0, 0);
    }
    int it = 0;
    const int chunk = 4;
    int done = 0;
    while (true) {
        for (int k = 0; k < chunk; ++k) {
            PFE_TRY(launch_phase(c, as, PH_LA, 0, 0));
            if (fused) {
                PFE_TRY(launch_phase(c, al, PH_LCD, 1, 0));
            } else {
                PFE_TRY(launch_phase(c, as, PH_LC, 1, 0));
                PFE_TRY(launch_phase(c, as, PH_LD, 0, 0));
            }
        }
        it += chunk;
        PFE_CHECK_HIP(hipMemcpyAsync(&done, &c->S->done, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        PFE_CHECK_HIP(hipStreamSynchronize(c->stream));
        if (done || it > c->prm.maxit + chunk) break;
    }
    PFE_TRY(launch_phase(c, a, PH_ZERO, 0, 0));
    return PFE_OK;
}

// One PCG solve of Eq. 13, one launch per phase: the residual phase res_ph
// (PH_E0 / PH_R0, r0 = rhs - A x), then the iterations.  With a factor
// preconditioner (learned or FSAI) Jacobi-PCG stays the fallback: the solve's
// starting x is kept, and when the factor PCG breaks down (PFE_E_NOT_SPD: a
// non-positive or non-finite scalar) or reaches maxit (PFE_E_NOCONV), x is
// restored and the same solve is redone with Jacobi from the same start;
// fallbacks counts such solves, and the status reported is the redo's.
template <typename T>
pfe_status pcg_solve_mk(pfe_ctx* c, const KA<T>& a, const KA<T>& as, int res_ph, bool r0_ready = false) {
    // r0_ready: the previous edge update formed r0, u0 and the CG state (k_eur_px)
    if (c->prm.precond == PFE_JACOBI) {
        if (!r0_ready) PFE_TRY(launch_phase(c, as, res_ph, 0, 1));
        return pcg_loop_mk(c, a, as);
    }
    const size_t bytes = (size_t)c->n * c->d * sizeof(T);
    if (!c->xbak) PFE_CHECK_HIP(dev_alloc(&c->xbak, (size_t)c->n * c->d * 8));
    PFE_CHECK_HIP(hipMemcpyAsync(c->xbak, a.x, bytes, hipMemcpyDeviceToDevice, c->stream));
    hipLaunchKernelGGL(k_status_save, dim3(1), dim3(64), 0, c->stream, c->S);
    if (!r0_ready) PFE_TRY(launch_phase(c, as, res_ph, 0, 1));
    PFE_TRY(pcg_loop_learned_mk(c, a, as));
    int st = 0;
    PFE_CHECK_HIP(hipMemcpyAsync(&st, &c->S->status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    PFE_CHECK_HIP(hipStreamSynchronize(c->stream));
    const bool redo = (st == PFE_E_NOT_SPD || st == PFE_E_NOCONV);
    if (redo) {
        PFE_CHECK_HIP(hipMemcpyAsync(a.x, c->xbak, bytes, hipMemcpyDeviceToDevice, c->stream));
        hipLaunchKernelGGL(k_status_clear, dim3(1), dim3(64), 0, c->stream, c->S);
        PFE_TRY(launch_phase(c, as, res_ph, 0, 1));
        PFE_TRY(pcg_loop_mk(c, a, as));
    }
    hipLaunchKernelGGL(k_status_merge, dim3(1), dim3(64), 0, c->stream, c->S, redo ? 1 : 0);
    PFE_CHECK_HIP(hipGetLastError());
    return PFE_OK;
}

// the strip partition is used in the one-launch-per-phase path when the graph
// has one and the context wants it
inline bool use_strips(const pfe_ctx* c) { return c->want_strips > 0 && c->ps.nblk > 0; }

// pixel launches: PCG by the per-row kernels (Jacobi on any layout, the factor
// preconditioners on pixel grids), when the context wants them
inline bool use_px(const pfe_ctx* c) {
    if (c->want_px <= 0 || c->want_px > 2) return false;
    const Partition& P = c->px[c->want_px - 1];
    // the factor preconditioners' pixel kernels exist for pixel grids only
    return P.nblk > 0 && (c->prm.precond == PFE_JACOBI || P.geo != nullptr);
}

// arguments of the PCG phases (residual, w0, iterations) for the iterate and
// right-hand side of a: pixel launches, strips or row chunks
template <typename T>
KA<T> pcg_args(pfe_ctx* c, const KA<T>& a) {
    if (use_px(c)) {
        KA<T> ap = make_args<T>(c, c->px[c->want_px - 1]);
        ap.x = a.x;
        ap.rhs = a.rhs;
        ap.pxl = 1;
        return ap;
    }
    if (use_strips(c)) {
        KA<T> as = make_args<T>(c, c->ps);
        as.x = a.x;
        as.rhs = a.rhs;
        return as;
    }
    return a;
}

// (re)build the strip partition for the wanted number of waves
pfe_status setup_strips(pfe_ctx* c) {
    if (c->want_strips <= 0 || c->strip_slots <= 0 || c->ps_waves == c->want_strips) return PFE_OK;
    int want = c->want_strips * c->strip_slots;
    if (const char* ev = getenv("PFE_STRIP_WG")) want = std::max(1, atoi(ev));   // launch-shape experiments
    PFE_TRY(make_strip_partition(c->g, (int)c->d, want, 1, c->ps));
    PFE_TRY(make_strip_partition(c->g, (int)c->d, want, 2, c->pl));
    {
        // one-pass factor CG: strips of CPL columns per lane, as many as its own
        // co-resident workgroups for the wanted waves
        const int cpl = c->fcg_cpl;
        int want_f = c->want_strips * (c->fcg_slots > 0 ? c->fcg_slots : c->strip_slots);
        if (const char* ev = getenv("PFE_STRIP_WG")) want_f = std::max(1, atoi(ev));
        PFE_TRY(make_strip_partition(c->g, (int)c->d / cpl, want_f, 3, c->pf));
    }
    c->ps_waves = c->want_strips;
    if (c->part_blocks > 0 && std::max(std::max(c->ps.nblk, c->pl.nblk), c->pf.nblk) > c->part_blocks) {
        free_partition(c->ps);
        free_partition(c->pl);
        free_partition(c->pf);
        c->ps_waves = 0;
        set_error("strip partition of %d workgroups exceeds the partial-sum buffer", c->ps.nblk);
        return PFE_E_STATE;
    }
    return PFE_OK;
}

// the per-pixel edge update (k_eu_px): pixel stencils of 4, 8 or 24 slots with b
// once per undirected edge, and general layouts (ELL or CSR) with b per slot
inline bool eu_px_ok(const pfe_ctx* c) {
    const int K = c->g->ell_K;
    if (!c->eu_px) return false;
    if (!c->g->stencil) return !c->bhalf;    // general layouts: b per slot
    return c->bhalf && (K == 4 || K == 8 || K == 24);
}

template <typename T, int KC, int V>
pfe_status launch_eu_px_v(pfe_ctx* c, const KA<T>& a, dim3 grid, bool geo, int W, int H) {
    if constexpr (KC > 0) {
        if (geo) hipLaunchKernelGGL((k_eu_px<T, KC, V, true>), grid, dim3(kBlock), 0, c->stream, a, W, H);
        else hipLaunchKernelGGL((k_eu_px<T, KC, V, false>), grid, dim3(kBlock), 0, c->stream, a, W, H);
    } else {
        hipLaunchKernelGGL((k_eu_px<T, 0, V, false>), grid, dim3(kBlock), 0, c->stream, a, W, H);
    }
    PFE_CHECK_HIP(hipGetLastError());
    return PFE_OK;
}

template <typename T, int V>
pfe_status launch_eu_px_k(pfe_ctx* c, const KA<T>& a, dim3 grid, bool geo, int W, int H) {
    switch (c->g->stencil ? c->g->ell_K : 0) {
        case 0: return launch_eu_px_v<T, 0, V>(c, a, grid, false, W, H);
        case 4: return launch_eu_px_v<T, 4, V>(c, a, grid, geo, W, H);
        case 8: return launch_eu_px_v<T, 8, V>(c, a, grid, geo, W, H);
        case 24: return launch_eu_px_v<T, 24, V>(c, a, grid, geo, W, H);
        default: set_error("the per-pixel edge update needs a stencil of 4, 8 or 24 slots"); return PFE_E_STATE;
    }
}

// columns per thread as in the per-row passes: the widest access of up to 16
// bytes that d allows
template <typename T>
pfe_status launch_eu_px(pfe_ctx* c, const KA<T>& a) {
    const int d = (int)c->d;
    const int V = px_cols<T>(d);
    const int ppb = kBlock / (d / V);
    const dim3 grid((unsigned)((c->n + ppb - 1) / ppb));
    // one image: neighbours from the stencil offsets; batches read the slot columns
    const pfe_graph* g = c->g;
    const bool geo = c->nseg == 1 && g->seg_W.size() == 1 && g->seg_W[0] > 0 && g->seg_H[0] > 0 &&
                     (int64_t)g->seg_W[0] * g->seg_H[0] == c->n;
    const int W = geo ? g->seg_W[0] : 0, H = geo ? g->seg_H[0] : 0;
    if constexpr (sizeof(T) == 4) {
        if (V == 4) return launch_eu_px_k<T, 4>(c, a, grid, geo, W, H);
    }
    if (V == 2) return launch_eu_px_k<T, 2>(c, a, grid, geo, W, H);
    return launch_eu_px_k<T, 1>(c, a, grid, geo, W, H);
}

// the edge update fused with the next solve's residual (k_eur_px): PCG by
// per-row launches (pixel stencils or general layouts) or on strips of
// pixel-stencil images, warm starts (the iterate is Y).  f: the kernel's arguments on a per-row partition (the
// solve's own with per-row launches; with strips, whose w0 kernel reads r0
// alone, the partition of two workgroups per CU).  False when the shape does
// not allow it.
template <typename T>
bool eur_px_args(pfe_ctx* c, const KA<T>& a, const KA<T>& as, KA<T>& f) {
    const int K = c->g->ell_K;
    const bool sten = c->g->stencil;
    if (!c->eur_px || c->prm.cold_start || !eu_px_ok(c) || (sten && !(K == 4 || K == 8 || K == 24)) || a.x != a.Y)
        return false;
    if (as.pxl) {
        f = as;
    } else if (sten && use_strips(c) && as.geo != nullptr && c->px[0].nblk > 0) {
        // two workgroups per CU where built (64-image batch, d = 10: 58.1 ms per
        // SOC iteration against 60.2 with one, and 60.2 unfused)
        f = make_args<T>(c, c->px[c->px[1].nblk > 0 ? 1 : 0]);
        f.x = a.x;
        f.rhs = a.rhs;
        f.pxl = 1;
    } else {
        return false;
    }
    return !sten || f.geo != nullptr;   // stencils take the workgroups' image geometry
}

template <typename T, int V>
pfe_status launch_eur_px_v(pfe_ctx* c, const KA<T>& f) {
    const dim3 grid(f.nblk);
    switch (c->g->stencil ? c->g->ell_K : 0) {
        case 0: hipLaunchKernelGGL((k_eur_px<T, 0, V>), grid, dim3(kBlock), 0, c->stream, f); break;
        case 4: hipLaunchKernelGGL((k_eur_px<T, 4, V>), grid, dim3(kBlock), 0, c->stream, f); break;
        case 8: hipLaunchKernelGGL((k_eur_px<T, 8, V>), grid, dim3(kBlock), 0, c->stream, f); break;
        case 24: hipLaunchKernelGGL((k_eur_px<T, 24, V>), grid, dim3(kBlock), 0, c->stream, f); break;
        default: set_error("the fused edge update needs a stencil of 4, 8 or 24 slots or a general layout"); return PFE_E_STATE;
    }
    PFE_CHECK_HIP(hipGetLastError());
    c->fused_eur = 1;
    return PFE_OK;
}

template <typename T>
pfe_status launch_eur_px(pfe_ctx* c, const KA<T>& f) {
    const int V = px_cols<T>((int)c->d);
    if constexpr (sizeof(T) == 4) {
        if (V == 4) return launch_eur_px_v<T, 4>(c, f);
    }
    if (V == 2) return launch_eur_px_v<T, 2>(c, f);
    return launch_eur_px_v<T, 1>(c, f);
}

// inner iteration l of a Split-Bregman run (l = 0: b = d = 0), one launch per
// phase.  next: inner iteration l + 1 follows in the same call, so its residual
// may be formed by this edge update (*fused is then set); r0_ready: the previous
// inner iteration's edge update formed this solve's residual.
template <typename T>
pfe_status inner_at(pfe_ctx* c, int l, bool next = false, bool r0_ready = false, bool* fused = nullptr) {
    KA<T> a = make_args<T>(c, c->pm);
    const KA<T> as = pcg_args<T>(c, a);
    // cold start: the solve begins from Y = 0 (the right-hand side does not
    // depend on Y; the previous edge update has already consumed it)
    if (c->prm.cold_start) PFE_CHECK_HIP(hipMemsetAsync(c->Y, 0, (size_t)c->n * c->d * sizeof(T), c->stream));
    PFE_TRY(pcg_solve_mk(c, a, as, (l == 0) ? PH_E0 : PH_R0, r0_ready && l > 0));
    // edge update of this inner step and rhs of the next one (on strips when
    // the slot data are loaded one image row ahead, widths up to 8)
    KA<T> b = (as.geo && !as.pxl && c->g->ell_K <= 8) ? as : a;
    b.store_rhs = 1;
    b.b_zero = (l == 0);
    b.bpar = l & 1;
    KA<T> f;
    if (next && fused && eur_px_args(c, a, as, f)) {
        f.b_zero = b.b_zero;
        f.bpar = b.bpar;
        // the factor path's Jacobi fallback forms r0 again from the stored rhs
        f.store_rhs = c->prm.precond != PFE_JACOBI;
        *fused = true;
        return launch_eur_px(c, f);
    }
    if (eu_px_ok(c)) return launch_eu_px(c, b);
    PFE_TRY(launch_phase(c, b, PH_EU, 0, 0));
    return PFE_OK;
}

template <typename T>
pfe_status inner_mk(pfe_ctx* c) {
    PFE_TRY(inner_at<T>(c, c->inner));
    c->inner += 1;
    return PFE_OK;
}

template <typename T>
pfe_status ortho_mk(pfe_ctx* c, int mode) {
    KA<T> a = make_args<T>(c, c->pm);
    PFE_TRY(launch_phase(c, a, PH_GRAM, mode, 0));
    if (a.nseg > 1) {
        hipLaunchKernelGGL(k_factor<T>, dim3(a.nseg), dim3(kBlock), 0, c->stream, a, mode);
        PFE_CHECK_HIP(hipGetLastError());
    }
    PFE_TRY(launch_phase(c, a, PH_APPLY, mode, 0));
    return PFE_OK;
}

template <typename T>
pfe_status outer_mk(pfe_ctx* c) {
    // the remaining inner iterations run back to back: each edge update but the
    // last may form the next solve's residual
    bool r0 = false;
    while (c->inner < c->prm.n_inner) {
        bool fused = false;
        PFE_TRY(inner_at<T>(c, c->inner, c->inner + 1 < c->prm.n_inner, r0, &fused));
        r0 = fused;
        c->inner += 1;
    }
    PFE_TRY(ortho_mk<T>(c, 0));
    c->inner = 0;
    return PFE_OK;
}

// persistent kernel specialised for the graph's ELL width (0: generic loops),
// with or without the LDS row cache
template <typename T>
const void* soc_kernel(int ell_K, bool lc) {
    switch (ell_K) {
        case 4: return lc ? reinterpret_cast<const void*>(&k_soc<T, 4, true>) : reinterpret_cast<const void*>(&k_soc<T, 4, false>);
        case 8: return lc ? reinterpret_cast<const void*>(&k_soc<T, 8, true>) : reinterpret_cast<const void*>(&k_soc<T, 8, false>);
        case 24: return lc ? reinterpret_cast<const void*>(&k_soc<T, 24, true>) : reinterpret_cast<const void*>(&k_soc<T, 24, false>);
        default: return reinterpret_cast<const void*>(&k_soc<T, 0, false>);
    }
}

// one cooperative launch of the persistent kernel: n_outer runs of n_inner
// Split-Bregman iterations, each followed by the P- and B-update when pupdate
template <typename T>
pfe_status launch_soc(pfe_ctx* c, int n_inner, int n_outer, int pupdate) {
    KA<T> a = make_args<T>(c, c->pc);
    const bool lc = c->cache_np > 0;
    Plan plan{0, n_inner, n_outer, lc ? c->cache_np : 0, pupdate};
    const size_t dyn = lc ? row_cache_bytes<T>(c->cache_np, a.R, c->g->ell_K) : 0;
    PFE_CHECK_HIP(hipMemsetAsync(c->bar, 0, 512 * sizeof(unsigned), c->stream));
    void* args[] = {(void*)&a, (void*)&plan};
    PFE_CHECK_HIP(hipLaunchCooperativeKernel(soc_kernel<T>(c->g->ell_K, lc), dim3(a.nblk), dim3(kBlock), args, dyn,
                                             c->stream));
    c->launched_coop = 1;
    return PFE_OK;
}

template <typename T>
pfe_status outer_coop(pfe_ctx* c, int n_outer) {
    if (c->inner > 0) {
        // finish the current SOC iteration one phase per launch
        PFE_TRY(outer_mk<T>(c));
        if (--n_outer == 0) return PFE_OK;
    }
    PFE_TRY(launch_soc<T>(c, c->prm.n_inner, n_outer, 1));
    c->inner = 0;
    return PFE_OK;
}

// Stage II: n_iter Split-Bregman iterations from b = d = 0 with P and B fixed,
// in one persistent launch when the context runs that way, else one launch per
// phase; the context stays between SOC iterations (inner index 0)
template <typename T>
pfe_status split_bregman_run(pfe_ctx* c, int n_iter) {
    if (c->prm.persistent && c->pc.nblk > 0 && c->prm.precond == PFE_JACOBI && !c->prm.cold_start)
        return launch_soc<T>(c, n_iter, 1, 0);
    bool r0 = false;
    for (int l = 0; l < n_iter; ++l) {
        bool fused = false;
        PFE_TRY(inner_at<T>(c, l, l + 1 < n_iter, r0, &fused));
        r0 = fused;
    }
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
        info->workgroups = c->launched_coop ? c->pc.nblk : 0;
        const bool px = !c->launched_coop && use_px(c);
        info->flags = ((c->launched_coop && c->cache_np > 0) ? 1 : 0) |
                      ((!c->launched_coop && !px && use_strips(c)) ? 2 : 0) | (px ? 4 : 0) |
                      (c->fused_eur ? 8 : 0);
    }
    if (h.status != 0) {
        set_error("%s", pfe_status_string((pfe_status)h.status));
        return (pfe_status)h.status;
    }
    return PFE_OK;
}

pfe_status reset_stats(pfe_ctx* c) {
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
                       (T*)c->isqrtD, (T*)c->isq);
    PFE_CHECK_HIP(hipGetLastError());
    return PFE_OK;
}

void free_ctx(pfe_ctx* c) {
    void* bufs[] = {c->Y, c->P, c->B, c->bs, c->bs2, c->ds, c->rhs, c->p, c->rb[0], c->rb[1], c->wb[0], c->wb[1],
                    c->sb[0], c->sb[1], c->diagA, c->invdiag, c->sqrtD, c->isqrtD, c->isq, c->gval, c->gdiag,
                    c->zl, c->y1, c->xbak, c->dact, c->part, c->gpart,
                    c->Tm, c->colbuf, c->colint, c->S, c->bar, c->hist};
    for (void* p : bufs)
        if (p) (void)dev_free(p);
    free_partition(c->pm);
    free_partition(c->pc);
    free_partition(c->ps);
    free_partition(c->pl);
    free_partition(c->pf);
    free_partition(c->px[0]);
    free_partition(c->px[1]);
    if (c->cg_exec) (void)hipGraphExecDestroy(c->cg_exec);
    c->cg_exec = nullptr;
}

bool params_ok(const pfe_params* p, int64_t n) {
    if (p->d < 1 || p->d > kMaxD || p->d >= n) { set_error("d must be in [1, %d] and below n", kMaxD); return false; }
    if (!(p->lambda >= 0.0) || !std::isfinite(p->lambda)) { set_error("lambda must be >= 0"); return false; }
    if (!(p->r > 0.0) || !std::isfinite(p->r)) { set_error("r must be > 0"); return false; }
    if (p->n_inner < 1) { set_error("n_inner must be >= 1"); return false; }
    if (!(p->tol > 0.0) || p->maxit < 1) { set_error("tol must be > 0 and maxit >= 1"); return false; }
    if (p->precond != PFE_JACOBI && p->precond != PFE_LEARNED && p->precond != PFE_FSAI) { set_error("unknown preconditioner"); return false; }
    if (p->ortho != PFE_POLAR && p->ortho != PFE_CHOL) { set_error("unknown ortho mode"); return false; }
    if (p->dtype != PFE_FP32 && p->dtype != PFE_FP64) { set_error("unknown dtype"); return false; }
    return true;
}

// Per segment, the active columns of Y0: a segment whose Y0 has trailing
// all-zero columns is embedded in that many fewer dimensions (its zero columns
// stay zero: zero right-hand sides, zero edge differences, and a P-update on
// the leading block of its Gram matrix).  This is how one launch carries
// problems of several d (the largest d, the others padded with zero columns).
// A zero column before a nonzero one is a rank deficiency.
template <typename T>
pfe_status active_dims(pfe_ctx* c) {
    const int nseg = c->nseg, d = (int)c->d;
    unsigned* flags = nullptr;
    PFE_CHECK_HIP(dev_alloc((void**)&flags, sizeof(unsigned) * (size_t)nseg));
    pfe_status st = PFE_OK;
    std::vector<unsigned> h((size_t)nseg, 0u);
    do {
        if (hipMemsetAsync(flags, 0, sizeof(unsigned) * h.size(), c->stream) != hipSuccess) { st = PFE_E_HIP; break; }
        for (int sg = 0; sg < nseg; ++sg) {
            const int64_t r0 = c->g->seg_row0[sg], r1 = c->g->seg_row0[sg + 1];
            const unsigned grid = (unsigned)std::min<int64_t>(((r1 - r0) * d + 255) / 256, 1024);
            hipLaunchKernelGGL(k_col_flags<T>, dim3(std::max(1u, grid)), dim3(256), 0, c->stream, (const T*)c->Y, r0,
                               r1, d, flags + sg);
        }
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(h.data(), flags, sizeof(unsigned) * h.size(), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess) {
            st = PFE_E_HIP;
            break;
        }
    } while (0);
    (void)dev_free(flags);
    if (st != PFE_OK) { set_error("pfe_init: column scan of Y0 failed"); return st; }
    c->dact_h.assign(nseg, d);
    bool padded = false;
    for (int sg = 0; sg < nseg; ++sg) {
        int da = 0;
        for (int col = 0; col < d; ++col)
            if ((h[sg] >> col) & 1u) da = col + 1;
        for (int col = 0; col < da; ++col)
            if (!((h[sg] >> col) & 1u)) {
                set_error("pfe_init: Y0 has a zero column %d before a nonzero one on segment %d", col, sg);
                return PFE_E_RANK;
            }
        if (da == 0) {
            set_error("pfe_init: Y0 is zero on segment %d", sg);
            return PFE_E_RANK;
        }
        c->dact_h[sg] = da;
        padded = padded || da < d;
    }
    if (!padded) { c->dact_h.clear(); return PFE_OK; }
    PFE_CHECK_HIP(dev_alloc((void**)&c->dact, sizeof(int) * nseg));
    PFE_CHECK_HIP(hipMemcpy(c->dact, c->dact_h.data(), sizeof(int) * nseg, hipMemcpyHostToDevice));
    return PFE_OK;
}

template <typename T>
pfe_status monitor_impl(pfe_ctx* c, pfe_monitors* out) {
    KA<T> a = make_args<T>(c, c->pm);
    hipLaunchKernelGGL(k_monitor<T>, dim3(a.nblk), dim3(kBlock), 0, c->stream, a);
    PFE_CHECK_HIP(hipGetLastError());
    double mon[4];
    PFE_CHECK_HIP(hipMemcpyAsync(mon, c->S->mon, sizeof(mon), hipMemcpyDeviceToHost, c->stream));
    PFE_CHECK_HIP(hipStreamSynchronize(c->stream));
    out->objective = mon[0];
    out->constraint = mon[1];
    out->split = mon[2];
    out->orthogonality = mon[3];
    out->split_nonzero = -1.0;
    if (c->ds && c->g->n_edges > 0) {
        unsigned long long* cnt = reinterpret_cast<unsigned long long*>(c->hist);
        PFE_CHECK_HIP(hipMemsetAsync(cnt, 0, sizeof(unsigned long long), c->stream));
        const int64_t ns = c->sslots;
        const unsigned grid = (unsigned)std::min<int64_t>((ns + 255) / 256, 2048);
        hipLaunchKernelGGL(k_count_nonzero<T>, dim3(grid), dim3(256), 0, c->stream, ns, (int)c->d, c->g->s_eid,
                           (const T*)c->ds, cnt);
        PFE_CHECK_HIP(hipGetLastError());
        unsigned long long h = 0;
        PFE_CHECK_HIP(hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, c->stream));
        PFE_CHECK_HIP(hipStreamSynchronize(c->stream));
        // out of the entries of each segment's active columns (each edge stored
        // once per direction with per-slot storage, once with per-edge storage)
        const double per_edge = c->bhalf ? 1.0 : 2.0;
        double entries = per_edge * (double)c->g->n_edges * (double)c->d;
        if (!c->dact_h.empty()) {
            entries = 0.0;
            for (int sg = 0; sg < c->nseg; ++sg)
                entries += per_edge * (double)(c->g->seg_edge0[sg + 1] - c->g->seg_edge0[sg]) * (double)c->dact_h[sg];
        }
        out->split_nonzero = (double)h / entries;
    }
    return PFE_OK;
}

template <typename T>
pfe_status quantile_impl(pfe_ctx* c, double q, double* out) {
    typedef typename Bits<T>::U U;
    KA<T> a = make_args<T>(c, c->pm);
    const int W = Bits<T>::W;
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
    }
    // with FP64 the lowest 16 bits stay unresolved: the value is the bin's lower edge
    U u = (U)(prefix << (W - consumed));
    T v;
    memcpy(&v, &u, sizeof(T));
    *out = (double)v;
    return PFE_OK;
}

template <typename T>
pfe_status split_to_edges(pfe_ctx* c, const void* src, void* dst) {
    KA<T> a = make_args<T>(c, c->pm);
    const int n = (int)c->n;
    if (c->bhalf)
        hipLaunchKernelGGL(k_half_to_edges<T>, dim3((n + 255) / 256), dim3(256), 0, c->stream, a, c->g->s_eid,
                           (const T*)src, (T*)dst);
    else
        hipLaunchKernelGGL(k_slots_to_edges<T>, dim3((n + 255) / 256), dim3(256), 0, c->stream, a, c->g->s_eid,
                           (const T*)src, (T*)dst);
    PFE_CHECK_HIP(hipGetLastError());
    return PFE_OK;
}

template <typename T>
pfe_status edges_to_split(pfe_ctx* c, const void* src, void* dst) {
    KA<T> a = make_args<T>(c, c->pm);
    const int n = (int)c->n;
    if (c->bhalf)
        hipLaunchKernelGGL(k_edges_to_half<T>, dim3((n + 255) / 256), dim3(256), 0, c->stream, a, c->g->s_eid,
                           (const T*)src, (T*)dst);
    else
        hipLaunchKernelGGL(k_edges_to_slots<T>, dim3((n + 255) / 256), dim3(256), 0, c->stream, a, c->g->s_eid,
                           (const T*)src, (T*)dst);
    PFE_CHECK_HIP(hipGetLastError());
    return PFE_OK;
}

template <typename T>
pfe_status launch_spmm(pfe_ctx* c, const KA<T>& a, const T* X, T* Q) {
    switch (c->g->ell_K) {
        case 4: hipLaunchKernelGGL((k_spmm<T, 4>), dim3(a.nblk), dim3(kBlock), 0, c->stream, a, X, Q); break;
        case 8: hipLaunchKernelGGL((k_spmm<T, 8>), dim3(a.nblk), dim3(kBlock), 0, c->stream, a, X, Q); break;
        case 24: hipLaunchKernelGGL((k_spmm<T, 24>), dim3(a.nblk), dim3(kBlock), 0, c->stream, a, X, Q); break;
        default: hipLaunchKernelGGL((k_spmm<T, 0>), dim3(a.nblk), dim3(kBlock), 0, c->stream, a, X, Q); break;
    }
    PFE_CHECK_HIP(hipGetLastError());
    return PFE_OK;
}

// Gt = I (Jacobi) until a network is evaluated on the context
template <typename T>
pfe_status identity_factor(pfe_ctx* c) {
    const size_t ns = (size_t)c->g->nslot + 1, n = (size_t)c->n;
    hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, c->stream, ns, T(0), (T*)c->gval);
    hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, n, T(1), (T*)c->gdiag);
    PFE_CHECK_HIP(hipGetLastError());
    c->have_factor = 0;
    return PFE_OK;
}

template <typename T>
pfe_status fsai_factor(pfe_ctx* c) {
    const pfe_graph* g = c->g;
    const int64_t n = c->n;
    int* err = nullptr;
    PFE_CHECK_HIP(dev_alloc((void**)&err, sizeof(int)));
    PFE_CHECK_HIP(hipMemsetAsync(err, 0, sizeof(int), c->stream));
    const size_t ns = (size_t)g->nslot + 1;
    hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, c->stream, ns, T(0), (T*)c->gval);
    FsaiArgs f{n, g->s_col, g->s_w64, g->degree, g->wsq, 0.5 * c->prm.lambda, 0.5 * c->prm.r, err};
    const dim3 grid((unsigned)((n + 63) / 64));
    switch (g->ell_K) {
        case 4: hipLaunchKernelGGL((k_fsai<T, 4>), grid, dim3(64), 0, c->stream, f, (T*)c->gval, (T*)c->gdiag); break;
        case 8: hipLaunchKernelGGL((k_fsai<T, 8>), grid, dim3(64), 0, c->stream, f, (T*)c->gval, (T*)c->gdiag); break;
        default: hipLaunchKernelGGL((k_fsai<T, 24>), grid, dim3(64), 0, c->stream, f, (T*)c->gval, (T*)c->gdiag); break;
    }
    hipError_t e = hipGetLastError();
    int h = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, err, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)dev_free(err);
    if (e != hipSuccess) return hip_fail(e, "FSAI factor", __FILE__, __LINE__);
    if (h) {
        set_error("pfe_set_fsai: %s", (h & 2) ? "slot layout is not a symmetric stencil" : "local system not positive definite");
        return PFE_E_STATE;
    }
    return PFE_OK;
}

NetGraph net_graph(const pfe_ctx* c) {
    NetGraph ng;
    ng.n = c->n;
    ng.nslot = c->g->nslot;
    ng.ell_K = c->g->ell_K;
    ng.deg_max = c->g->max_deg;
    ng.rowptr = c->g->rowptr;
    ng.scol = c->g->s_col;
    ng.seid = c->g->s_eid;
    ng.sw64 = c->g->s_w64;
    ng.degree = c->g->degree;
    ng.wsq = c->g->wsq;
    ng.lambda = c->prm.lambda;
    ng.r = c->prm.r;
    return ng;
}

template <typename T>
pfe_status residual_to(pfe_ctx* c, void* dst) {
    KA<T> a = make_args<T>(c, c->pm);
    PFE_TRY(launch_phase(c, a, (c->inner == 0) ? PH_E0 : PH_R0, 0, 1));
    PFE_CHECK_HIP(hipMemcpyAsync(dst, c->rb[0], (size_t)c->n * c->d * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
    return PFE_OK;
}

template <typename T>
pfe_status factor_to_edges(pfe_ctx* c, void* edge_vals, void* diag) {
    KA<T> a = make_args<T>(c, c->pm);
    a.d = 1;
    const int n = (int)c->n;
    if (edge_vals)
        hipLaunchKernelGGL(k_slots_to_edges<T>, dim3((n + 255) / 256), dim3(256), 0, c->stream, a, c->g->s_eid,
                           (const T*)c->gval, (T*)edge_vals);
    if (diag) PFE_CHECK_HIP(hipMemcpyAsync(diag, c->gdiag, sizeof(T) * n, hipMemcpyDeviceToDevice, c->stream));
    PFE_CHECK_HIP(hipGetLastError());
    return PFE_OK;
}

template <typename T>
pfe_status rebuild_rhs(pfe_ctx* c) {
    KA<T> a = make_args<T>(c, c->pm);
    a.bpar = c->inner & 1;     // the buffer holding b after c->inner edge updates
    return launch_phase(c, a, PH_RHS, 0, 0);
}

// the b buffer holding the current b (after c->inner edge updates)
inline void* current_b(pfe_ctx* c) { return ((c->inner & 1) && c->bs2) ? c->bs2 : c->bs; }

// n_outer SOC iterations in the context's current launch shape
template <typename T>
pfe_status run_outer(pfe_ctx* c, int n_outer) {
    if (c->prm.persistent && c->pc.nblk > 0 && c->prm.precond == PFE_JACOBI && !c->prm.cold_start)
        return outer_coop<T>(c, n_outer);
    for (int k = 0; k < n_outer; ++k) PFE_TRY(outer_mk<T>(c));
    return PFE_OK;
}

// (Re)build the persistent partition for the context's launch shape (team
// size, row cache) and decide whether the LDS row cache fits.
pfe_status setup_persistent(pfe_ctx* c) {
    free_partition(c->pc);
    c->cache_np = 0;
    if (c->coop < kNumXcd) return PFE_OK;
    const int R = kBlock / (int)c->d;
    const int K = c->g->ell_K;
    PFE_TRY(make_partition(c->seg_rows, (int)c->coop, R, c->team, c->pc, c->per_cu == 2 ? c->second_weight : 1.0));
    hipDeviceProp_t prop;
    PFE_CHECK_HIP(hipGetDeviceProperties(&prop, c->device));
    if (c->pc.nblk % kNumXcd != 0 || c->pc.nblk > c->per_cu * prop.multiProcessorCount) {
        free_partition(c->pc);
        return PFE_OK;
    }
    if (c->want_cache && (K == 4 || K == 8 || K == 24)) {
        // LDS row cache when the persistent workgroups' rows fit without
        // lowering their co-residency
        const bool f64 = c->prm.dtype == PFE_FP64;
        const size_t bytes = f64 ? row_cache_bytes<double>(c->pc.max_np, R, K) : row_cache_bytes<float>(c->pc.max_np, R, K);
        int occ_lc = 0;
        if (bytes <= 48 * 1024 &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_lc, f64 ? soc_kernel<double>(K, true) : soc_kernel<float>(K, true),
                                                         kBlock, bytes) == hipSuccess &&
            occ_lc >= c->per_cu)
            c->cache_np = c->pc.max_np;
    }
    return PFE_OK;
}

}  // namespace

extern "C" {

// the image {row0, W, H} of each workgroup of a pixel partition of pixel-grid
// segments (the workgroups of make_partition lie in one segment each)
pfe_status set_px_geo(pfe_ctx* c, Partition& P) {
    const pfe_graph* g = c->g;
    std::vector<int> bseg(P.nblk), geo((size_t)8 * P.nblk, 0);
    PFE_CHECK_HIP(hipMemcpy(bseg.data(), P.blk_seg, sizeof(int) * P.nblk, hipMemcpyDeviceToHost));
    for (int b = 0; b < P.nblk; ++b) {
        const int sg = bseg[b];
        geo[8 * (size_t)b] = (int)g->seg_row0[sg];
        geo[8 * (size_t)b + 1] = g->seg_W[sg];
        geo[8 * (size_t)b + 2] = g->seg_H[sg];
    }
    PFE_CHECK_HIP(dev_alloc((void**)&P.geo, sizeof(int) * geo.size()));
    PFE_CHECK_HIP(hipMemcpy(P.geo, geo.data(), sizeof(int) * geo.size(), hipMemcpyHostToDevice));
    return PFE_OK;
}

pfe_status pfe_init(pfe_graph* g, const pfe_params* p, const void* Y0, hipStream_t stream, pfe_ctx** out) {
    if (!g || !p || !Y0 || !out) { set_error("pfe_init: null argument"); return PFE_E_ARG; }
    *out = nullptr;
    if (!params_ok(p, g->n)) return PFE_E_ARG;
    pfe_ctx* c = new pfe_ctx();
    c->g = g;
    c->prm = *p;
    c->stream = stream;
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; set_error("hipGetDevice failed"); return PFE_E_HIP; }
    c->esz = (p->dtype == PFE_FP64) ? 8 : 4;
    c->n = g->n;
    c->d = p->d;
    c->nseg = (int)g->seg_row0.size() - 1;
    std::vector<int64_t> seg_rows(c->nseg);
    for (int sg = 0; sg < c->nseg; ++sg) {
        seg_rows[sg] = g->seg_row0[sg + 1] - g->seg_row0[sg];
        if (seg_rows[sg] <= p->d) {
            delete c;
            set_error("pfe_init: graph %d of the batch has %lld vertices, not more than d = %d", sg,
                      (long long)seg_rows[sg], p->d);
            return PFE_E_ARG;
        }
    }
    const size_t nd = (size_t)c->n * c->d * c->esz;
    // b and d once per undirected edge on pixel stencils (lower slots), else per slot
    c->bhalf = (g->stencil && (g->ell_K == 4 || g->ell_K == 8 || g->ell_K == 24)) ? 1 : 0;
    if (const char* ev = getenv("PFE_SPLIT_PER_SLOT")) if (atoi(ev)) c->bhalf = 0;   // layout experiments
    c->sslots = c->bhalf ? (int64_t)(g->ell_K / 2) * g->n : g->nslot;
    const size_t sd = (size_t)(c->sslots + 1) * c->d * c->esz;
    const size_t nv = (size_t)c->n * c->esz;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) { delete c; set_error("hipGetDeviceProperties failed"); return PFE_E_HIP; }
    const int ncu = prop.multiProcessorCount;
    const int R = kBlock / (int)c->d;
    const int64_t want = (c->n + R - 1) / R;
    int occ = 0;
    hipError_t oe = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &occ, (p->dtype == PFE_FP64) ? soc_kernel<double>(g->ell_K, false) : soc_kernel<float>(g->ell_K, false), kBlock, 0);
    if (oe != hipSuccess) occ = 0;
    c->per_cu = std::max(0, std::min(occ, 2));
    c->seg_rows = seg_rows;
    if (const char* ev = getenv("PFE_TEAM")) c->team = std::max(1, atoi(ev));   // launch-shape experiments
    if (const char* ev = getenv("PFE_ROWCACHE")) c->want_cache = atoi(ev) != 0;
    if (const char* ev = getenv("PFE_SECOND_WEIGHT")) c->second_weight = std::min(1.0, std::max(0.25, atof(ev)));
    pfe_status s = make_partition(seg_rows, (int)std::min<int64_t>(want, 2048), R, c->team, c->pm);
    // persistent grid: every co-resident workgroup (at most one per R rows), a
    // multiple of the XCD count; built even when the context starts in the
    // one-launch-per-phase mode, so that the autotuner can try it
    c->coop = (int64_t)c->per_cu * ncu;
    if (const char* ev = getenv("PFE_PERSISTENT_WG")) {
        // launch-shape experiments: cap the persistent grid (never above co-residency)
        int64_t cap = atoll(ev);
        if (cap > 0 && cap < c->coop) c->coop = cap;
    }
    if (c->coop > want) c->coop = want;
    c->coop -= c->coop % kNumXcd;
    if (s == PFE_OK) s = setup_persistent(c);
    if (const char* ev = getenv("PFE_STRIPS")) c->want_strips = std::max(0, atoi(ev));   // launch-shape experiments
    if (const char* ev = getenv("PFE_ONE_PASS")) c->one_pass = atoi(ev) != 0;
    if (const char* ev = getenv("PFE_EU_PX")) c->eu_px = atoi(ev) != 0;     // launch-shape experiments
    if (const char* ev = getenv("PFE_EUR_PX")) c->eur_px = atoi(ev) != 0;   // launch-shape experiments
    if (s == PFE_OK) {
        // strip partition: built first for the most waves any later shape asks
        // for (it has the most workgroups), then for the wanted count
        int occ_st = 0;
        const void* kst = nullptr;
        switch (g->ell_K) {
            case 4: kst = (p->dtype == PFE_FP64) ? (const void*)&k_st_it<double, 4> : (const void*)&k_st_it<float, 4>; break;
            case 8: kst = (p->dtype == PFE_FP64) ? (const void*)&k_st_it<double, 8> : (const void*)&k_st_it<float, 8>; break;
            case 24: kst = (p->dtype == PFE_FP64) ? (const void*)&k_st_it<double, 24> : (const void*)&k_st_it<float, 24>; break;
            default: break;
        }
        if (kst && hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_st, kst, kBlock, 0) != hipSuccess) occ_st = 0;
        c->strip_slots = kst ? std::max(1, occ_st) * ncu : 0;
        c->fcg_cpl = (p->dtype == PFE_FP64) ? fcg_cpl<double>((int)c->d) : fcg_cpl<float>((int)c->d);
        if (const char* ev = getenv("PFE_FCG_CPL")) c->fcg_cpl = (atoi(ev) == 2 && c->fcg_cpl == 2) ? 2 : 1;
        const void* kf = (p->dtype == PFE_FP64) ? fcg_kernel<double>(g->ell_K, c->fcg_cpl)
                                                : fcg_kernel<float>(g->ell_K, c->fcg_cpl);
        int occ_f = 0;
        if (kf && hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_f, kf, kBlock, 0) != hipSuccess) occ_f = 0;
        c->fcg_slots = kf ? std::max(1, occ_f) * ncu : 0;
        const int want = c->want_strips;
        c->want_strips = std::max(want, 2);
        s = setup_strips(c);
        c->want_strips = want;
    }
    bool px_grid = g->stencil && (g->ell_K == 4 || g->ell_K == 8 || g->ell_K == 24) &&
                   (int)g->seg_W.size() == c->nseg;
    for (int sg = 0; px_grid && sg < c->nseg; ++sg)
        px_grid = g->seg_W[sg] > 0 && g->seg_H[sg] > 0 && (int64_t)g->seg_W[sg] * g->seg_H[sg] == seg_rows[sg];
    if (s == PFE_OK && (px_grid || !g->stencil)) {
        // pixel (per-row) launches of pixel-grid images (one or a batch) or of a
        // general layout: one workgroup per CU, each a contiguous pixel (row)
        // range of one segment (on
        // the 1024 x 1024 window graph 256 workgroups ran a SOC iteration in
        // 20.3 ms, 512 in 21.5, 768 in 22.4, 1024 in 23.0, 2048 in 25.9)
        const int V = (p->dtype == PFE_FP64) ? px_cols<double>((int)c->d) : px_cols<float>((int)c->d);
        const int ppb = kBlock / ((int)c->d / V);
        const int64_t steps = (c->n + ppb - 1) / ppb;
        for (int k = 0; k < 2 && s == PFE_OK; ++k) {
            int want_px = (k + 1) * ncu;
            if (const char* ev = getenv("PFE_PX_BLOCKS")) want_px = std::max(kNumXcd, atoi(ev));   // launch-shape experiments
            want_px = (int)std::min<int64_t>(want_px, steps);
            if (want_px >= kNumXcd) want_px -= want_px % kNumXcd;   // whole XCD groups where there are enough
            if (k == 1 && want_px <= c->px[0].nblk) break;          // no second size
            int team_px = 64;   // the whole XCD band sweeps together (team_iteration caps at the band)
            if (const char* ev = getenv("PFE_PX_TEAM")) team_px = std::max(1, atoi(ev));   // launch-shape experiments
            s = make_partition(seg_rows, std::max(1, want_px), ppb, team_px, c->px[k]);
            if (s == PFE_OK && px_grid) s = set_px_geo(c, c->px[k]);
        }
    }
    if (const char* ev = getenv("PFE_PIXEL")) c->want_px = std::min(2, std::max(0, atoi(ev)));   // launch-shape experiments
    if (s != PFE_OK) { free_ctx(c); delete c; return s; }
    const int nblk_max = std::max(std::max(std::max(std::max(c->pm.nblk, c->pc.nblk), std::max(c->ps.nblk, c->pl.nblk)),
                                  c->pf.nblk), std::max(c->px[0].nblk, c->px[1].nblk));
    c->part_blocks = nblk_max;
    if (s == PFE_OK) s = setup_strips(c);
    if (s != PFE_OK) { free_ctx(c); delete c; return s; }
    const int npair = (int)(c->d * (c->d + 1) / 2);
    const size_t part_doubles = (size_t)nblk_max * std::max<int64_t>(3 * c->d, 3 + 2 * npair) + 64;
    const size_t ncol = (size_t)c->nseg * c->d;
    hipError_t e = hipSuccess;
#define ALLOC(ptr, bytes) do { if (e == hipSuccess) e = dev_alloc((void**)&(ptr), (bytes)); } while (0)
    ALLOC(c->Y, nd); ALLOC(c->P, nd); ALLOC(c->B, nd);
    ALLOC(c->bs, sd);
    if (c->bhalf) ALLOC(c->bs2, sd);
    if (p->keep_split) ALLOC(c->ds, sd);
    ALLOC(c->rhs, nd); ALLOC(c->p, nd);
    for (int k = 0; k < 2; ++k) { ALLOC(c->rb[k], nd); ALLOC(c->wb[k], nd); ALLOC(c->sb[k], nd); }
    ALLOC(c->diagA, nv); ALLOC(c->invdiag, nv); ALLOC(c->sqrtD, nv); ALLOC(c->isqrtD, nv); ALLOC(c->isq, nv);
    ALLOC(c->gval, (size_t)(g->nslot + 1) * c->esz); ALLOC(c->gdiag, nv); ALLOC(c->zl, nd); ALLOC(c->y1, nd);
    ALLOC(c->part, sizeof(double) * part_doubles);
    ALLOC(c->gpart, sizeof(double) * 2 * kGroupStride);
    ALLOC(c->Tm, sizeof(double) * c->nseg * kMaxD * kMaxD);
    ALLOC(c->colbuf, sizeof(double) * ncol * 5);
    ALLOC(c->colint, sizeof(int) * ncol * 3);
    ALLOC(c->S, sizeof(Scal));
    ALLOC(c->bar, 512 * sizeof(unsigned));
    ALLOC(c->hist, 4096 * sizeof(unsigned));
#undef ALLOC
    if (e != hipSuccess) {
        free_ctx(c);
        delete c;
        return hip_fail(e, "device allocation (context)", __FILE__, __LINE__);
    }
    c->cs.gamma = c->colbuf;
    c->cs.alpha = c->colbuf + ncol;
    c->cs.beta = c->colbuf + 2 * ncol;
    c->cs.bnorm2 = c->colbuf + 3 * ncol;
    c->cs.rr = c->colbuf + 4 * ncol;
    c->cs.iters = c->colint;
    c->cs.active = c->colint + ncol;
    c->cs.zero = c->colint + 2 * ncol;
    do {
        if (hipMemsetAsync(c->S, 0, sizeof(Scal), stream) != hipSuccess ||
            hipMemsetAsync(c->bar, 0, 512 * sizeof(unsigned), stream) != hipSuccess ||
            hipMemsetAsync(c->bs, 0, sd, stream) != hipSuccess ||
            (c->bs2 && hipMemsetAsync(c->bs2, 0, sd, stream) != hipSuccess) ||
            hipMemsetAsync(c->p, 0, nd, stream) != hipSuccess ||
            // vectors start at zero (every phase then reads defined values,
            // whatever launch shape ran before)
            hipMemsetAsync(c->rhs, 0, nd, stream) != hipSuccess ||
            hipMemsetAsync(c->rb[0], 0, nd, stream) != hipSuccess || hipMemsetAsync(c->rb[1], 0, nd, stream) != hipSuccess ||
            hipMemsetAsync(c->wb[0], 0, nd, stream) != hipSuccess || hipMemsetAsync(c->wb[1], 0, nd, stream) != hipSuccess ||
            hipMemsetAsync(c->sb[0], 0, nd, stream) != hipSuccess || hipMemsetAsync(c->sb[1], 0, nd, stream) != hipSuccess ||
            hipMemsetAsync(c->colbuf, 0, sizeof(double) * ncol * 5, stream) != hipSuccess ||
            hipMemsetAsync(c->colint, 0, sizeof(int) * ncol * 3, stream) != hipSuccess ||
            (c->ds && hipMemsetAsync(c->ds, 0, sd, stream) != hipSuccess) ||
            hipMemcpyAsync(c->Y, Y0, nd, hipMemcpyDeviceToDevice, stream) != hipSuccess) {
            s = hip_fail(hipGetLastError(), "context initialisation", __FILE__, __LINE__);
            break;
        }
        s = (p->dtype == PFE_FP64) ? set_diag<double>(c) : set_diag<float>(c);
        if (s != PFE_OK) break;
        s = (p->dtype == PFE_FP64) ? identity_factor<double>(c) : identity_factor<float>(c);
        if (s != PFE_OK) break;
        s = (p->dtype == PFE_FP64) ? active_dims<double>(c) : active_dims<float>(c);
        if (s != PFE_OK) break;
        if (p->init_ortho) {
            s = (p->dtype == PFE_FP64) ? ortho_mk<double>(c, 1) : ortho_mk<float>(c, 1);
        } else {
            // P = D^{1/2} Y, B = 0 through the same apply pass with T = I
            std::vector<double> I((size_t)c->nseg * kMaxD * kMaxD, 0.0);
            for (int sg = 0; sg < c->nseg; ++sg)
                for (int k = 0; k < c->d; ++k) I[(size_t)sg * kMaxD * kMaxD + k * kMaxD + k] = 1.0;
            int one = 1;
            if (hipMemcpyAsync(c->Tm, I.data(), sizeof(double) * I.size(), hipMemcpyHostToDevice, stream) != hipSuccess ||
                hipMemcpyAsync(&c->S->ortho_ok, &one, sizeof(int), hipMemcpyHostToDevice, stream) != hipSuccess) {
                s = PFE_E_HIP; break;
            }
            if (p->dtype == PFE_FP64) { KA<double> ad = make_args<double>(c, c->pm); s = launch_phase(c, ad, PH_APPLY, 1, 0); }
            else { KA<float> af = make_args<float>(c, c->pm); s = launch_phase(c, af, PH_APPLY, 1, 0); }
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
    c->launched_coop = 0;
    c->fused_eur = 0;
    if (info) PFE_TRY(reset_stats(c));
    pfe_status s;
    const bool f64 = c->prm.dtype == PFE_FP64;
    if (granularity == PFE_INNER) {
        if (c->inner >= c->prm.n_inner) { set_error("all inner iterations done; call pfe_step(PFE_OUTER)"); return PFE_E_STATE; }
        s = f64 ? inner_mk<double>(c) : inner_mk<float>(c);
    } else if (granularity == PFE_OUTER) {
        if (c->prm.persistent && c->pc.nblk > 0 && c->inner == 0 && c->prm.precond == PFE_JACOBI && !c->prm.cold_start)
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
    c->launched_coop = 0;
    c->fused_eur = 0;
    if (info) PFE_TRY(reset_stats(c));
    const bool f64 = c->prm.dtype == PFE_FP64;
    if (c->prm.persistent && c->pc.nblk > 0 && n_outer > 0 && c->prm.precond == PFE_JACOBI && !c->prm.cold_start) {
        PFE_TRY(f64 ? outer_coop<double>(c, n_outer) : outer_coop<float>(c, n_outer));
    } else {
        for (int k = 0; k < n_outer; ++k) PFE_TRY(f64 ? outer_mk<double>(c) : outer_mk<float>(c));
    }
    if (info) return read_info(c, info);
    return PFE_OK;
}

pfe_status pfe_split_bregman(pfe_ctx* c, int n_iter, pfe_step_info* info) {
    if (!c || n_iter < 0) { set_error("pfe_split_bregman: bad argument"); return PFE_E_ARG; }
    if (c->inner != 0) { set_error("pfe_split_bregman: call between SOC iterations (inner index 0)"); return PFE_E_STATE; }
    c->launched_coop = 0;
    c->fused_eur = 0;
    if (info) PFE_TRY(reset_stats(c));
    if (n_iter > 0) PFE_TRY(c->prm.dtype == PFE_FP64 ? split_bregman_run<double>(c, n_iter) : split_bregman_run<float>(c, n_iter));
    if (info) return read_info(c, info);
    return PFE_OK;
}

pfe_status pfe_autotune(pfe_ctx* c, int trials, pfe_tune_result* results, int max_results, int* n_results) {
    if (!c || trials < 1 || max_results < 0 || (max_results > 0 && !results)) {
        set_error("pfe_autotune: bad argument");
        return PFE_E_ARG;
    }
    if (c->inner != 0) { set_error("pfe_autotune: call between SOC iterations (inner index 0)"); return PFE_E_STATE; }
    if (n_results) *n_results = 0;
    const bool f64 = c->prm.dtype == PFE_FP64;
    const size_t nd = (size_t)c->n * c->d * c->esz;
    struct Shape { int persistent, team, cache, strips; double w2; int one_pass, pixel; };
    const Shape shapes[] = {{1, 64, 1, 0, 1.0, 0, 0}, {1, 64, 0, 0, 1.0, 0, 0}, {1, 1, 1, 0, 1.0, 0, 0},
                            {1, 1, 0, 0, 1.0, 0, 0}, {1, 1, 1, 0, 0.9, 0, 0}, {1, 1, 0, 0, 0.9, 0, 0},
                            {1, 1, 1, 0, 0.85, 0, 0}, {1, 1, 0, 0, 0.85, 0, 0}, {1, 1, 1, 0, 0.8, 0, 0},
                            {1, 1, 0, 0, 0.8, 0, 0},
                            {0, c->team, 0, 0, 1.0, 0, 0}, {0, c->team, 0, 1, 1.0, 0, 0}, {0, c->team, 0, 2, 1.0, 0, 0},
                            {0, c->team, 0, 1, 1.0, 1, 0}, {0, c->team, 0, 2, 1.0, 1, 0},
                            {0, c->team, 0, 0, 1.0, 0, 1}, {0, c->team, 0, 0, 1.0, 0, 2}};
    const Shape orig{c->prm.persistent, c->team, c->want_cache, c->want_strips, c->second_weight, c->one_pass,
                     c->want_px};
    char* save = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    pfe_status st = PFE_OK;
    // the state (Y, P, B) and the solver flags as they were before the call:
    // a candidate that ends in a breakdown or a barrier time-out leaves no
    // trace in the next candidate's run or in later calls
    auto restore = [&]() -> pfe_status {
        PFE_CHECK_HIP(hipMemcpyAsync(c->Y, save, nd, hipMemcpyDeviceToDevice, c->stream));
        PFE_CHECK_HIP(hipMemcpyAsync(c->P, save + nd, nd, hipMemcpyDeviceToDevice, c->stream));
        PFE_CHECK_HIP(hipMemcpyAsync(c->B, save + 2 * nd, nd, hipMemcpyDeviceToDevice, c->stream));
        hipLaunchKernelGGL(k_tune_reset, dim3(1), dim3(64), 0, c->stream, c->S);
        PFE_CHECK_HIP(hipGetLastError());
        c->inner = 0;
        return PFE_OK;
    };
    int timeouts = 0;
    int best = -1, count = 0;
    double best_ms = 0.0;
    std::vector<pfe_tune_result> found;
    Scal h_flags;
    do {
        if (dev_alloc((void**)&save, 3 * nd) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
            hipEventCreate(&e1) != hipSuccess) {
            st = hip_fail(hipGetLastError(), "pfe_autotune set-up", __FILE__, __LINE__);
            break;
        }
        if (hipMemcpyAsync(save, c->Y, nd, hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
            hipMemcpyAsync(save + nd, c->P, nd, hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
            hipMemcpyAsync(save + 2 * nd, c->B, nd, hipMemcpyDeviceToDevice, c->stream) != hipSuccess) {
            st = hip_fail(hipGetLastError(), "pfe_autotune save", __FILE__, __LINE__);
            break;
        }
        for (int k = 0; k < (int)(sizeof(shapes) / sizeof(shapes[0])) && st == PFE_OK; ++k) {
            const Shape& sh = shapes[k];
            if (sh.persistent && (c->coop < kNumXcd || c->prm.precond != PFE_JACOBI || c->prm.cold_start)) continue;
            if (sh.strips && c->strip_slots == 0) continue;
            if (sh.w2 != 1.0 && c->per_cu != 2) continue;
            if (sh.one_pass && (c->prm.precond == PFE_JACOBI || c->fcg_slots == 0)) continue;
            if (sh.pixel && (c->px[sh.pixel - 1].nblk == 0 ||
                             (c->prm.precond != PFE_JACOBI && c->px[sh.pixel - 1].geo == nullptr)))
                continue;
            c->one_pass = sh.one_pass;
            c->want_px = sh.pixel;
            c->prm.persistent = sh.persistent;
            c->team = sh.team;
            c->want_cache = sh.cache;
            c->want_strips = sh.strips;
            c->second_weight = sh.w2;
            if ((st = setup_strips(c)) != PFE_OK) break;
            if (sh.strips && c->ps.nblk == 0) continue;
            if (sh.one_pass && c->pf.nblk == 0) continue;
            if (sh.persistent) {
                if ((st = setup_persistent(c)) != PFE_OK) break;
                if (c->pc.nblk == 0 || (sh.cache && c->cache_np == 0)) continue;
            }
            // one untimed SOC iteration (code loading, caches), then the timed ones
            hipLaunchKernelGGL(k_tune_reset, dim3(1), dim3(64), 0, c->stream, c->S);
            st = f64 ? run_outer<double>(c, 1) : run_outer<float>(c, 1);
            if (st == PFE_OK) st = restore();
            if (st == PFE_OK && hipEventRecord(e0, c->stream) != hipSuccess) st = PFE_E_HIP;
            if (st == PFE_OK) st = f64 ? run_outer<double>(c, trials) : run_outer<float>(c, trials);
            if (st == PFE_OK && hipEventRecord(e1, c->stream) != hipSuccess) st = PFE_E_HIP;
            if (st == PFE_OK && hipEventSynchronize(e1) != hipSuccess) st = PFE_E_HIP;
            float ms = 0.f;
            if (st == PFE_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = PFE_E_HIP;
            if (st == PFE_OK && hipMemcpy(&h_flags, c->S, sizeof(Scal), hipMemcpyDeviceToHost) != hipSuccess)
                st = PFE_E_HIP;
            if (st == PFE_OK) st = restore();
            if (st != PFE_OK) break;
            // flags of the timed run (restore() above resets them after the copy)
            if (hipStreamSynchronize(c->stream) != hipSuccess) { st = PFE_E_HIP; break; }
            if (h_flags.abort_flag) ++timeouts;
            if (h_flags.abort_flag || (h_flags.status != 0 && h_flags.status != PFE_E_NOCONV)) continue;
            pfe_tune_result r{};
            r.persistent = sh.persistent;
            r.team = sh.team;
            r.row_cache = sh.persistent ? (c->cache_np > 0) : 0;
            r.strips = sh.strips;
            r.second_weight = sh.persistent ? sh.w2 : 1.0;
            r.one_pass = sh.one_pass;
            r.pixel = sh.pixel;
            r.workgroups = sh.persistent ? c->pc.nblk
                                         : (sh.pixel ? c->px[sh.pixel - 1].nblk
                                                     : (sh.one_pass ? c->pf.nblk : (sh.strips ? c->ps.nblk : c->pm.nblk)));
            r.ms = ms / trials;
            found.push_back(r);
            if (best < 0 || r.ms < best_ms) { best = (int)found.size() - 1; best_ms = r.ms; }
        }
    } while (0);
    // keep the fastest shape (the original one if nothing was measured)
    if (best >= 0) {
        c->prm.persistent = found[best].persistent;
        c->team = found[best].persistent ? found[best].team : orig.team;
        c->want_cache = found[best].persistent ? found[best].row_cache : orig.cache;
        c->want_strips = found[best].persistent ? orig.strips : found[best].strips;
        c->second_weight = found[best].persistent ? found[best].second_weight : orig.w2;
        c->one_pass = found[best].persistent ? orig.one_pass : found[best].one_pass;
        c->want_px = found[best].persistent ? orig.pixel : found[best].pixel;
        found[best].chosen = 1;
    } else {
        c->prm.persistent = orig.persistent;
        c->team = orig.team;
        c->want_cache = orig.cache;
        c->want_strips = orig.strips;
        c->second_weight = orig.w2;
        c->one_pass = orig.one_pass;
        c->want_px = orig.pixel;
    }
    pfe_status s2 = setup_persistent(c);
    if (s2 == PFE_OK) s2 = setup_strips(c);
    if (st == PFE_OK) st = s2;
    if (save && st == PFE_OK) st = restore();
    (void)hipStreamSynchronize(c->stream);
    if (save) (void)dev_free(save);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st == PFE_OK) st = reset_stats(c);
    if (st == PFE_OK && timeouts > 0) {
        // the shapes that ran normally were still measured and the fastest kept
        set_error("pfe_autotune: a grid barrier timed out in %d candidate launch shape(s); they were skipped",
                  timeouts);
        st = PFE_E_HIP;
    }
    for (size_t k = 0; k < found.size() && (int)k < max_results; ++k) results[k] = found[k];
    if (n_results) *n_results = (int)std::min<size_t>(found.size(), (size_t)max_results);
    return st;
}

pfe_status pfe_set_launch_shape(pfe_ctx* c, const pfe_tune_result* sh) {
    if (!c || !sh) { set_error("pfe_set_launch_shape: null argument"); return PFE_E_ARG; }
    if (c->inner != 0) { set_error("pfe_set_launch_shape: call between SOC iterations (inner index 0)"); return PFE_E_STATE; }
    if (sh->team < 1 || sh->team > 64 || sh->strips < 0 || sh->strips > 2 || !(sh->second_weight > 0.0) ||
        sh->second_weight > 1.0) {
        set_error("pfe_set_launch_shape: team in [1, 64], strips in [0, 2], second_weight in (0, 1]");
        return PFE_E_ARG;
    }
    if (sh->persistent && c->coop < kNumXcd) {
        set_error("pfe_set_launch_shape: no persistent launch on this context");
        return PFE_E_ARG;
    }
    if (!sh->persistent && sh->strips > 0 && c->strip_slots == 0) {
        set_error("pfe_set_launch_shape: image strips need a pixel-grid graph with 4, 8 or 24 slots");
        return PFE_E_ARG;
    }
    if (!sh->persistent && sh->one_pass && (sh->strips == 0 || c->fcg_slots == 0)) {
        set_error("pfe_set_launch_shape: the one-pass factor CG runs on image strips of a pixel-grid graph");
        return PFE_E_ARG;
    }
    if (!sh->persistent && (sh->pixel < 0 || sh->pixel > 2 || (sh->pixel > 0 && c->px[sh->pixel - 1].nblk == 0))) {
        set_error("pfe_set_launch_shape: pixel launches take 1 or 2 workgroups per CU (2: a graph with more "
                  "pixel steps than CUs)");
        return PFE_E_ARG;
    }
    c->prm.persistent = sh->persistent ? 1 : 0;
    if (sh->persistent) {
        c->team = sh->team;
        c->want_cache = sh->row_cache ? 1 : 0;
        c->second_weight = c->per_cu == 2 ? sh->second_weight : 1.0;
    } else {
        c->want_strips = sh->strips;
        c->one_pass = sh->one_pass ? 1 : 0;
        c->want_px = sh->pixel;
    }
    PFE_TRY(setup_persistent(c));
    PFE_TRY(setup_strips(c));
    if (sh->persistent && c->pc.nblk == 0) {
        set_error("pfe_set_launch_shape: the persistent partition does not fit this device");
        return PFE_E_ARG;
    }
    if (!sh->persistent && sh->strips > 0 && c->ps.nblk == 0) {
        set_error("pfe_set_launch_shape: no strip partition for this graph and d");
        return PFE_E_ARG;
    }
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
    const int d = (int)c->d;
    switch (which) {
        case PFE_Y: PFE_CHECK_HIP(hipMemcpyAsync(dst, c->Y, nd, hipMemcpyDeviceToDevice, st)); break;
        case PFE_P: PFE_CHECK_HIP(hipMemcpyAsync(dst, c->P, nd, hipMemcpyDeviceToDevice, st)); break;
        case PFE_B: PFE_CHECK_HIP(hipMemcpyAsync(dst, c->B, nd, hipMemcpyDeviceToDevice, st)); break;
        case PFE_RHS: PFE_CHECK_HIP(hipMemcpyAsync(dst, c->rhs, nd, hipMemcpyDeviceToDevice, st)); break;
        case PFE_RESID: PFE_TRY(c->esz == 8 ? residual_to<double>(c, dst) : residual_to<float>(c, dst)); break;
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
            void* src = (which == PFE_BSPLIT) ? current_b(c) : c->ds;
            if (!src) { set_error("pfe_get: split variable d not kept (keep_split = 0)"); return PFE_E_STATE; }
            if (c->inner == 0) {
                // b and d restart from zero at every SOC iteration
                PFE_CHECK_HIP(hipMemsetAsync(dst, 0, (size_t)c->g->n_edges * d * c->esz, st));
                break;
            }
            PFE_TRY(c->esz == 8 ? split_to_edges<double>(c, src, dst) : split_to_edges<float>(c, src, dst));
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
    switch (which) {
        case PFE_Y: PFE_CHECK_HIP(hipMemcpyAsync(c->Y, src, nd, hipMemcpyDeviceToDevice, st)); break;
        case PFE_P: PFE_CHECK_HIP(hipMemcpyAsync(c->P, src, nd, hipMemcpyDeviceToDevice, st)); break;
        case PFE_B: PFE_CHECK_HIP(hipMemcpyAsync(c->B, src, nd, hipMemcpyDeviceToDevice, st)); break;
        case PFE_BSPLIT:
        case PFE_DSPLIT: {
            void* dstp = (which == PFE_BSPLIT) ? current_b(c) : c->ds;
            if (!dstp) { set_error("pfe_set: split variable d not kept (keep_split = 0)"); return PFE_E_STATE; }
            PFE_TRY(c->esz == 8 ? edges_to_split<double>(c, src, dstp) : edges_to_split<float>(c, src, dstp));
            break;
        }
        default: set_error("pfe_set: block %d cannot be set", which); return PFE_E_ARG;
    }
    // the stored rhs follows the state when mid-way through a SOC iteration
    if (c->inner > 0 && c->ds) PFE_TRY(c->esz == 8 ? rebuild_rhs<double>(c) : rebuild_rhs<float>(c));
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
    if (inner_index > 0 && c->bs2 && ((inner_index ^ c->inner) & 1)) {
        // the b buffer of the new position holds the current b
        const size_t sd = (size_t)(c->sslots + 1) * c->d * c->esz;
        void* from = current_b(c);
        void* to = (from == c->bs) ? c->bs2 : c->bs;
        PFE_CHECK_HIP(hipMemcpyAsync(to, from, sd, hipMemcpyDeviceToDevice, c->stream));
    }
    c->inner = inner_index;
    if (inner_index == 0) {
        const size_t sd = (size_t)(c->sslots + 1) * c->d * c->esz;
        PFE_CHECK_HIP(hipMemsetAsync(c->bs, 0, sd, c->stream));
        if (c->bs2) PFE_CHECK_HIP(hipMemsetAsync(c->bs2, 0, sd, c->stream));
        if (c->ds) PFE_CHECK_HIP(hipMemsetAsync(c->ds, 0, sd, c->stream));
    } else {
        PFE_TRY(c->esz == 8 ? rebuild_rhs<double>(c) : rebuild_rhs<float>(c));
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
        KA<double> a = make_args<double>(c, c->pm);
        PFE_TRY(launch_spmm<double>(c, a, (const double*)X, (double*)Q));
    } else {
        KA<float> a = make_args<float>(c, c->pm);
        PFE_TRY(launch_spmm<float>(c, a, (const float*)X, (float*)Q));
    }
    PFE_CHECK_HIP(hipGetLastError());
    PFE_CHECK_HIP(hipStreamSynchronize(c->stream));
    return PFE_OK;
}

pfe_status pfe_pcg(pfe_ctx* c, const void* RHS, void* X, int32_t* iters, pfe_step_info* info) {
    if (!c || !RHS || !X) { set_error("pfe_pcg: null argument"); return PFE_E_ARG; }
    PFE_TRY(reset_stats(c));
    if (c->esz == 8) {
        KA<double> a = make_args<double>(c, c->pm);
        a.x = (double*)X;
        a.rhs = (double*)RHS;
        const KA<double> as = pcg_args<double>(c, a);
        PFE_TRY(pcg_solve_mk(c, a, as, PH_R0));
    } else {
        KA<float> a = make_args<float>(c, c->pm);
        a.x = (float*)X;
        a.rhs = (float*)RHS;
        const KA<float> as = pcg_args<float>(c, a);
        PFE_TRY(pcg_solve_mk(c, a, as, PH_R0));
    }
    if (iters) {
        // per column, the largest count over the segments of a batch
        std::vector<int> all((size_t)c->nseg * c->d);
        PFE_CHECK_HIP(hipMemcpyAsync(all.data(), c->cs.iters, sizeof(int) * all.size(), hipMemcpyDeviceToHost,
                                     c->stream));
        PFE_CHECK_HIP(hipStreamSynchronize(c->stream));
        for (int col = 0; col < c->d; ++col) {
            int m = 0;
            for (int sg = 0; sg < c->nseg; ++sg) m = std::max(m, all[(size_t)sg * c->d + col]);
            iters[col] = m;
        }
    }
    return read_info(c, info);
}

pfe_status pfe_set_learned(pfe_ctx* c, pfe_mpnn* net) {
    if (!c || !net) { set_error("pfe_set_learned: null argument"); return PFE_E_ARG; }
    PFE_TRY(mpnn_factor(net, net_graph(c), c->gval, c->gdiag, c->esz, c->stream));
    PFE_CHECK_HIP(hipStreamSynchronize(c->stream));
    c->have_factor = 1;
    c->prm.precond = PFE_LEARNED;
    return PFE_OK;
}


pfe_status pfe_set_fsai(pfe_ctx* c) {
    if (!c) { set_error("pfe_set_fsai: null context"); return PFE_E_ARG; }
    const int K = c->g->ell_K;
    if (!c->g->stencil || (K != 4 && K != 8 && K != 24)) {
        set_error("pfe_set_fsai: needs a pixel-grid graph (stencil slot layout with 4, 8 or 24 slots)");
        return PFE_E_ARG;
    }
    PFE_TRY(c->esz == 8 ? fsai_factor<double>(c) : fsai_factor<float>(c));
    c->have_factor = 1;
    c->prm.precond = PFE_FSAI;
    return PFE_OK;
}

pfe_status pfe_set_preconditioner(pfe_ctx* c, int precond) {
    if (!c) { set_error("null context"); return PFE_E_ARG; }
    if (precond != PFE_JACOBI && precond != PFE_LEARNED && precond != PFE_FSAI) { set_error("unknown preconditioner"); return PFE_E_ARG; }
    c->prm.precond = precond;
    return PFE_OK;
}

pfe_status pfe_get_factor(pfe_ctx* c, void* edge_vals, void* diag) {
    if (!c) { set_error("pfe_get_factor: null context"); return PFE_E_ARG; }
    PFE_TRY(c->esz == 8 ? factor_to_edges<double>(c, edge_vals, diag) : factor_to_edges<float>(c, edge_vals, diag));
    PFE_CHECK_HIP(hipStreamSynchronize(c->stream));
    return PFE_OK;
}

pfe_status pfe_mpnn_train_step(pfe_mpnn* net, pfe_ctx* c, const void* samples, int k, float lr, double* loss) {
    if (!net || !c || !samples || k < 1 || k > 32 || !(lr >= 0.f)) {
        set_error("pfe_mpnn_train_step: bad argument (1 <= k <= 32, lr >= 0)");
        return PFE_E_ARG;
    }
    PFE_TRY(mpnn_train_step(net, net_graph(c), samples, c->esz, k, lr, loss, c->stream));
    PFE_CHECK_HIP(hipStreamSynchronize(c->stream));
    return PFE_OK;
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
