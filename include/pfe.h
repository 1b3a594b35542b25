/*
 * pfe.h — C ABI of libpfe, the MI355X (gfx950) implementation of the
 * piecewise-flat-embedding (PFE) hot path of Meinhold, Hayes and Cahill,
 * "Efficiently Computing Piecewise Flat Embeddings for Data Clustering and
 * Image Segmentation".
 *
 * The library runs the nested Bregman iteration of the paper on the GPU:
 *   - the SOC outer loop (Algorithm 1): Y-update, P-update, B-update;
 *   - the Y-update by Split Bregman (Algorithm 2) in the compact n x d form of
 *     Sec. III: the least-squares step as the d systems of Eq. (13),
 *         [lambda/2 M^T M + r/2 D] Y = lambda/2 M^T (d - b) + r/2 D^{1/2} (P - B),
 *     solved together by preconditioned conjugate gradient (Sec. III, last
 *     paragraph), then the shrink of Eq. (9) and the Bregman update of Eq. (10);
 *   - the P-update, argmin ||P - (D^{1/2} Y + B)|| s.t. P^T P = I, from an FP64
 *     d x d Gram matrix and its Cholesky factor.
 *
 * Sign convention: Eq. (13) prints Q2 = B - P; the library uses P - B, which
 * is the stationarity condition of Algorithm 2's least-squares objective.
 *
 * Conventions for every entry point
 *   - All functions return a pfe_status; on failure a message is available from
 *     pfe_last_error() (thread-local, valid until the next call on the thread).
 *     No C++ exception crosses this boundary.
 *   - Matrices are row-major.  n x d blocks (Y, P, B, right-hand sides) hold d
 *     consecutive values per vertex.  Per-edge blocks (the split variables b and
 *     d) hold d values per undirected edge, edges ordered by (i, j), i < j,
 *     lexicographically — the row order of M in Sec. II.
 *   - Element type of n x d and per-edge blocks is float for PFE_FP32 contexts
 *     and double for PFE_FP64 contexts.
 *   - "device" pointers are HIP device allocations on the current device; the
 *     caller keeps ownership of every buffer it passes, and the library never
 *     keeps a caller pointer after the call returns.  Library objects
 *     (pfe_graph, pfe_ctx) own their device memory until destroyed.
 *   - Work is enqueued on the stream given at creation; functions that return
 *     host-side results (info structs, scalars) synchronise that stream.
 */
#ifndef PFE_H
#define PFE_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PFE_OK = 0,
    PFE_E_ARG = -1,      /* invalid argument (null pointer, size, parameter range) */
    PFE_E_GRAPH = -2,    /* invalid graph: isolated vertex, bad/duplicate edge, non-finite weight */
    PFE_E_HIP = -3,      /* a HIP runtime call failed */
    PFE_E_NOMEM = -4,    /* device allocation failed */
    PFE_E_NOT_SPD = -5,  /* CG breakdown: p^T A p <= 0 or non-finite scalar */
    PFE_E_RANK = -6,     /* Gram matrix not positive definite (rank-deficient embedding) */
    PFE_E_NOCONV = -7,   /* CG reached maxit; the state was still updated */
    PFE_E_STATE = -8     /* request not valid in the context's current state */
} pfe_status;

/* graph kinds */
enum { PFE_GRID = 0, PFE_EDGES = 1 };
/* preconditioners */
enum { PFE_JACOBI = 0, PFE_LEARNED = 1, PFE_FSAI = 2 };
/* P-update */
enum { PFE_POLAR = 0, PFE_CHOL = 1 };
/* element type of the vector state */
enum { PFE_FP32 = 0, PFE_FP64 = 1 };
/* pfe_step granularity */
enum { PFE_INNER = 0, PFE_OUTER = 1 };
/* state blocks for pfe_get / pfe_set */
enum {
    PFE_Y = 0,      /* n x d, the current Y */
    PFE_P = 1,      /* n x d */
    PFE_B = 2,      /* n x d, SOC Bregman variable */
    PFE_YHAT = 3,   /* n x d, D^{-1/2} P (feasible embedding, Yhat^T D Yhat = I); get only */
    PFE_BSPLIT = 4, /* |E| x d, Split-Bregman variable b */
    PFE_DSPLIT = 5, /* |E| x d, Split-Bregman variable d (needs keep_split on get) */
    PFE_RHS = 6,    /* n x d, right-hand side of the next least-squares solve; get only */
    PFE_RESID = 7   /* n x d, initial residual rhs - A Y of the next least-squares solve; get only */
};

typedef struct pfe_graph pfe_graph;
typedef struct pfe_ctx pfe_ctx;

/*
 * Graph description (Sec. II).  Edge weights are the heat kernel
 * w_ij = exp(-||x_i - x_j||^2 / (2 sigma^2)), evaluated in FP64.
 *
 * PFE_GRID: one vertex per pixel, index y*W + x; feat is H*W x m (row-major,
 *   float); stencil 4 or 8 selects the 4-/8-neighbourhood, a negative value -R
 *   the (2R+1)^2 window minus its centre.
 * PFE_EDGES: n vertices and n_edges undirected edges (src[e], dst[e]) with
 *   squared feature distances dist2[e]; each unordered pair at most once, no
 *   self loops.
 * on_device: 1 if feat/src/dst/dist2 are device pointers, 0 if host pointers.
 */
typedef struct {
    int kind;
    int H, W, m;
    const float* feat;
    int stencil;
    int64_t n;
    int64_t n_edges;
    const int32_t* src;
    const int32_t* dst;
    const double* dist2;
    double sigma;
    int on_device;
} pfe_graph_desc;

/*
 * Solver parameters.
 *   d          embedding dimension, 1 <= d <= 32, d < n
 *   lambda     Split-Bregman penalty (Algorithm 2), >= 0; shrink threshold 1/lambda
 *   r          SOC penalty (Algorithm 1), > 0
 *   n_inner    Split-Bregman iterations per SOC iteration, >= 1
 *   tol        PCG stop: ||r_c|| <= tol ||rhs_c|| for every column c
 *   maxit      PCG iteration cap per solve
 *   precond    PFE_JACOBI, or PFE_LEARNED / PFE_FSAI (both apply the context's sparse
 *              factor, set by pfe_set_learned or pfe_set_fsai; Gt = I until then).
 *              Jacobi-PCG stays the fallback of the factor preconditioners: a
 *              solve whose factor PCG breaks down (PFE_E_NOT_SPD) or reaches maxit
 *              (PFE_E_NOCONV) is redone with Jacobi from the same starting point,
 *              counted in pfe_step_info.fallbacks
 *   ortho      PFE_POLAR (exact argmin, default) or PFE_CHOL (Cholesky QR)
 *   dtype      PFE_FP32 (vectors, SpMM, shrink in float; CG scalars and Gram
 *              in double) or PFE_FP64 (everything in double)
 *   init_ortho 1: D-orthonormalise Y0 (Y0 <- Y0 R^{-1}, R^T R = Y0^T D Y0); 0: use Y0 as is
 *   keep_split 1: also store the split variable d (needed by pfe_get(PFE_DSPLIT))
 *   persistent 1: run each SOC iteration as one cooperative launch with grid
 *              barriers; 0: one launch per phase with stream-ordered phases
 *   graphs     1: in the one-launch-per-phase mode (and for the learned
 *              preconditioner), replay the PCG iterations from a HIP graph of 8
 *              iterations instead of launching each kernel from the host
 *   cold_start 0 (default): every PCG solve of Eq. (13) starts from the current
 *              Y (warm start); 1: from zero (runs one launch per phase)
 */
typedef struct {
    int d;
    double lambda;
    double r;
    int n_inner;
    double tol;
    int maxit;
    int precond;
    int ortho;
    int dtype;
    int init_ortho;
    int keep_split;
    int persistent;
    int graphs;
    int cold_start;
} pfe_params;

/* Per-call solver statistics (filled when a non-null pointer is passed). */
typedef struct {
    int64_t solves;          /* PCG solves performed by the call */
    int64_t cg_iters_total;  /* sum over solves of the iterations of the slowest column */
    int32_t cg_iters_max;    /* largest iteration count of a single solve */
    int32_t cg_iters_last;   /* iteration count of the last solve */
    double rel_res_max;      /* largest final ||r_c||/||rhs_c|| (recursive residual) */
    int32_t status;          /* worst pfe_status met (PFE_E_NOCONV, PFE_E_NOT_SPD, ...) */
    int32_t fallbacks;       /* factor-preconditioned (PFE_LEARNED / PFE_FSAI) solves redone
                                with Jacobi-PCG from the same start after the factor PCG broke
                                down or reached maxit (the redo's status is reported) */
    int32_t workgroups;      /* workgroups of the persistent launch (0: one launch per phase) */
    int32_t flags;           /* bit 0: persistent launch with the rows' slot data held in LDS;
                                bit 1: one launch per phase on image strips;
                                bit 2: Jacobi PCG by pixel launches (pfe_tune_result.pixel);
                                bit 3: edge updates that also formed the next solve's
                                residual (PCG by pixel launches or on strips of a pixel
                                grid, inner iterations run in one call) */
} pfe_step_info;

/* Monitors of the current state (Eq. 1, Eq. 2). */
typedef struct {
    double objective;        /* ||M Yhat||_1, each undirected edge once */
    double constraint;       /* max |Yhat^T D Yhat - I| */
    double split;            /* ||D^{1/2} Y - P||_F / ||P||_F */
    double orthogonality;    /* max |P^T P - I| */
    double split_nonzero;    /* fraction of nonzero entries of the split variable d
                                as last stored (keep_split = 1; -1 otherwise): the
                                share of edge differences the shrink left active */
} pfe_monitors;

/* ---- graph ------------------------------------------------------------ */

/* Build the graph of Sec. II on the device: CSR adjacency with both directions
 * of every edge (columns ascending per row), FP64 heat-kernel weights stored in
 * FP32 and FP64, degrees d_i = sum_j w_ij (Algorithm 1, D = diag(W 1)).
 * Errors: PFE_E_ARG for bad sizes/pointers, PFE_E_GRAPH for an isolated vertex
 * (degree below FLT_MIN), a self loop, a duplicate or out-of-range edge, or a
 * non-finite weight. */
pfe_status pfe_build_graph(const pfe_graph_desc* desc, hipStream_t stream, pfe_graph** out);

/* Sizes: vertices, undirected edges, CSR nonzeros of A (n + 2|E|). */
pfe_status pfe_graph_info(const pfe_graph* g, int64_t* n, int64_t* n_edges, int64_t* nnz_A);

/* Copy the CSR adjacency to caller device buffers (any may be null):
 * rowptr[n+1], col[2|E|], w[2|E|] (float), degree[n] (double). */
pfe_status pfe_graph_csr(const pfe_graph* g, int32_t* rowptr, int32_t* col, float* w,
                         double* degree);

/* Block-diagonal union of count graphs, for running a batch of independent
 * problems (one PFE per part, Algorithms 1 and 2 applied to each) as one
 * graph.  Vertex v of part p becomes vertex off_p + v with off_p the number of
 * vertices in parts 0..p-1; its edges are renumbered the same way, so the
 * per-edge blocks of the union are the parts' blocks one after another.  Each
 * part becomes one segment (a part that is itself a union contributes its
 * segments); a solver on the union keeps separate CG scalars, convergence and
 * P-update (Gram matrix, constraint Yhat^T D Yhat = I) per segment.  The parts
 * are only read (they may be destroyed afterwards) and must live on the
 * current device.  The pixel-stencil slot layout is kept when every part has
 * the same stencil.  Errors: PFE_E_ARG for a null part, count < 1, another
 * device, or a union above 2^30 vertices / 2^31 slots. */
pfe_status pfe_graph_union(const pfe_graph* const* parts, int count, hipStream_t stream, pfe_graph** out);

/* Segments of a graph: *count (1 for a graph built by pfe_build_graph), and
 * if non-null the host arrays row0[count + 1] (first vertex of each segment,
 * then n) and edge0[count + 1] (first undirected edge, then |E|). */
pfe_status pfe_graph_segments(const pfe_graph* g, int* count, int64_t* row0, int64_t* edge0);

void pfe_destroy_graph(pfe_graph* g);

/* ---- solver context ------------------------------------------------------ */

/* Create a solver for graph g (which must outlive the context): builds
 * A = lambda/2 M^T M + r/2 D (Eq. 13) implicitly (its diagonal and Jacobi
 * inverse), copies Y0 (device, n x d, dtype of params) and sets
 * P = D^{1/2} Y, B = 0 (Algorithm 1 initialisation), after D-orthonormalising
 * Y0 when init_ortho is set.  PFE_E_RANK if Y0 is rank deficient. */
pfe_status pfe_init(pfe_graph* g, const pfe_params* p, const void* Y0, hipStream_t stream,
                    pfe_ctx** out);

/* Change lambda and r (recomputes the diagonal of A); the state is kept. */
pfe_status pfe_set_penalties(pfe_ctx* c, double lambda, double r);

/* Advance the iteration.
 * PFE_INNER: one Split-Bregman iteration (Algorithm 2): least-squares solve
 *   of Eq. (13) by PCG warm-started from the current Y, then the shrink of
 *   Eq. (9) and Bregman update of Eq. (10); b and d start from zero at the first
 *   inner iteration of each SOC iteration.
 * PFE_OUTER: complete the current SOC iteration (Algorithm 1): the remaining
 *   inner iterations (n_inner in total), the P-update and the B-update.
 * Returns PFE_E_NOCONV if some solve hit maxit (state updated), PFE_E_NOT_SPD
 * or PFE_E_RANK on breakdown. */
pfe_status pfe_step(pfe_ctx* c, int granularity, pfe_step_info* info);

/* n_outer calls of pfe_step(PFE_OUTER) (Algorithm 1 for a fixed count). */
pfe_status pfe_solve(pfe_ctx* c, int n_outer, pfe_step_info* info);

/* Stage II of the paper's two-stage procedure (Sec. IV, experiments): after
 * the SOC iterations, the orthogonality constraint is relaxed and only
 * Split-Bregman iterations run.  Here: n_iter >= 0 iterations of Algorithm 2
 * from b = d = 0 with P and B held at their current values (each a PCG solve
 * of Eq. (13) warm-started from the current Y, then Eqs. (9) and (10)), in the
 * context's launch shape.  On return Y (device state) holds the iterate of the
 * last solve; P and B are unchanged; b and d are not part of the result (the
 * context stays between SOC iterations, so a later SOC iteration starts them
 * from zero).  PFE_E_STATE inside a SOC iteration (inner index > 0); solver
 * statuses as for pfe_step. */
pfe_status pfe_split_bregman(pfe_ctx* c, int n_iter, pfe_step_info* info);

/* Launch shape of the solver (how the same arithmetic is mapped on the GPU):
 * persistent (one cooperative launch per SOC iteration) or one launch per
 * phase; team = workgroups that deal an XCD band's row chunks out cyclically
 * (1: contiguous row ranges); row_cache = slot data of the workgroups' rows
 * held in LDS; second_weight = share of rows of the workgroup dispatched second
 * onto each CU (its waves are issued after the first's, so it may be given
 * fewer rows); strips = one launch per phase with the residual, w0 and CG
 * kernels of a pixel-grid graph on image strips (each workgroup walks a strip
 * row by row, neighbour values from an LDS ring).  The results are identical
 * up to the summation order of the FP64 reductions. */
typedef struct {
    int32_t persistent;
    int32_t team;
    int32_t row_cache;
    int32_t workgroups;      /* persistent launch: its workgroups; one launch per phase: the CG kernels' */
    double ms;               /* measured milliseconds per SOC iteration */
    int32_t chosen;          /* 1 for the shape kept */
    int32_t strips;          /* one launch per phase on image strips sized for this many waves of
                                co-resident workgroups (0: row chunks) */
    double second_weight;    /* persistent, teams of 1: rows of the second workgroup placed on each CU
                                relative to the first (1: equal) */
    int32_t one_pass;        /* factor preconditioners (learned, FSAI) on image strips: 1 = one pass
                                per CG iteration (Chronopoulos-Gear form, M^{-1} r and A M^{-1} r
                                through three LDS rings over a three-radius halo), 0 = two passes
                                (A p, then the factor apply with the x, r update) */
    int32_t pixel;           /* one launch per phase, Jacobi PCG by per-row kernels on 1 or 2 workgroups
                                per CU (0: not), each a row range of one segment (image or graph):
                                the residual, w0 and each CG iteration in two passes (the own-row
                                updates storing u' = r'/diag(A), then w' = A u' gathering u'), one
                                thread per row (pixel) and 1, 2 or 4 columns, neighbours through L2
                                from the stencil offsets (pixel grids) or the slot columns (flags
                                bit 2 of pfe_step_info) */
} pfe_tune_result;

/* Autotune the launch shape on this context's graph: from the current state
 * (between SOC iterations) run one untimed and `trials` timed SOC iterations
 * per candidate shape, restore the state after each, and keep the fastest for
 * later pfe_step / pfe_solve calls.  Candidates: persistent with teams of 64
 * or 1, each with and without the LDS row cache (when the rows fit), teams of 1
 * also with second_weight 0.9, 0.85 and 0.8, and one
 * launch per phase on row chunks and (pixel grids) on image strips sized for
 * one or two waves of co-resident workgroups (with a factor preconditioner,
 * strips with one and with two passes per CG iteration).  results (host, may be null when max_results is 0)
 * receives up to max_results measured shapes, *n_results their number.
 * Allocates a temporary copy of Y, P, B.  Each candidate starts from the
 * saved state with the solver flags cleared, so a shape that breaks down is
 * skipped without affecting the others.  PFE_E_STATE inside a SOC iteration;
 * PFE_E_HIP if a grid barrier timed out in some candidate (that candidate is
 * skipped, the fastest of the others is still kept). */
pfe_status pfe_autotune(pfe_ctx* c, int trials, pfe_tune_result* results, int max_results, int* n_results);

/* Use a launch shape in the form pfe_autotune reports it: persistent, team,
 * row_cache and second_weight for the persistent launch, strips (0: row chunks,
 * 1 or 2: image strips sized for that many waves) for one launch per phase;
 * the other fields are ignored.  For running a shape measured on another
 * context of the same graph, or a chosen shape in tests.  Only the summation
 * order of the FP64 reductions differs between shapes.  The persistent launch
 * still applies only to Jacobi-PCG with warm starts.  PFE_E_ARG for a shape
 * this context cannot run (persistent grid that does not fit, strips on a
 * graph without a pixel layout, fields out of range); PFE_E_STATE inside a
 * SOC iteration. */
pfe_status pfe_set_launch_shape(pfe_ctx* c, const pfe_tune_result* shape);

/* Statistics accumulated since the last reset (pfe_step / pfe_solve with a
 * non-null info reset them first).  reset != 0 clears them after reading.
 * Synchronises the stream; returns the worst solver status met (as in info). */
pfe_status pfe_stats(pfe_ctx* c, pfe_step_info* out, int reset);

/* Copy a state block to / from a caller device buffer (layouts above).
 * pfe_set(PFE_BSPLIT / PFE_DSPLIT) also rebuilds the right-hand side of the
 * next inner solve.  PFE_E_STATE for PFE_DSPLIT when keep_split is 0. */
pfe_status pfe_get(pfe_ctx* c, int which, void* dst);
pfe_status pfe_set(pfe_ctx* c, int which, const void* src);

/* Position inside the current SOC iteration: number of inner iterations done
 * (0 .. n_inner-1).  Setting it to 0 clears b and d. */
pfe_status pfe_get_inner_index(pfe_ctx* c, int* inner_index);
pfe_status pfe_set_inner_index(pfe_ctx* c, int inner_index);

/* Objective, constraint and split residuals of the current state. */
pfe_status pfe_monitor(pfe_ctx* c, pfe_monitors* out);

/* Q = A X for caller device blocks X, Q (n x d, context dtype): the operator
 * of Eq. (13). */
pfe_status pfe_apply_A(pfe_ctx* c, const void* X, void* Q);

/* Solve A X = RHS by the context's PCG, X (device) holds the initial guess on
 * entry and the solution on return.  iters (host, may be null) receives the
 * per-column iteration counts (d ints; for a batch, the largest over its
 * segments). */
pfe_status pfe_pcg(pfe_ctx* c, const void* RHS, void* X, int32_t* iters, pfe_step_info* info);

/* ---- learned preconditioner ---------------------------------------------------
 * Not part of the paper (which preconditions with incomplete Cholesky, Sec. III):
 * M^{-1} = G^T G, G = Gt D_A^{-1/2}, Gt lower triangular on the pattern of A with
 * a positive (softplus) diagonal, so M^{-1} is SPD for any weights and Gt = I is
 * Jacobi.  Gt comes from a two-layer message-passing network of width 16 on the
 * scaled matrix D_A^{-1/2} A D_A^{-1/2}; its dense layers run on MFMA with bf16
 * weights and fp32 accumulation.  Parameters: PFE_MPNN_NPARAMS floats in the
 * order W1s (16x4), W1m (16x4), b1 (16), W2s (16x16), W2m (16x16), b2 (16),
 * u (16), v (16), q (16), c, bd. */
#define PFE_MPNN_NPARAMS 722
typedef struct pfe_mpnn pfe_mpnn;

/* Create a network from host parameters, or the identity network (Gt = I)
 * when params is null.  Weights and Adam state live on the current device. */
pfe_status pfe_mpnn_create(const float* params, pfe_mpnn** out);
/* Copy the parameters and/or the gradient of the last training step to host
 * arrays of PFE_MPNN_NPARAMS floats (either may be null). */
pfe_status pfe_mpnn_get_params(pfe_mpnn* net, float* params, float* grad);
/* Replace the parameters (host array) and reset the Adam state. */
pfe_status pfe_mpnn_set_params(pfe_mpnn* net, const float* params);
void pfe_mpnn_destroy(pfe_mpnn* net);
/* Save the parameters to a network file / create a network from one (host
 * path): an 8-byte magic "PFEMPNN1", a uint32 count (PFE_MPNN_NPARAMS), then
 * the parameters as little-endian float32.  pfe_mpnn_load rejects a file of
 * another size, magic or count, or with non-finite values (PFE_E_ARG) before
 * any device memory is taken. */
pfe_status pfe_mpnn_save(pfe_mpnn* net, const char* path);
pfe_status pfe_mpnn_load(const char* path, pfe_mpnn** out);

/* One training step on the context's system: samples are k residual vectors
 * (device, n x k row-major, context element type, 1 <= k <= 32), scaled to
 * rho = D_A^{-1/2} r / ||D_A^{-1/2} r||; loss = mean_k ||At Gt^T Gt rho_k - rho_k||^2
 * with At = D_A^{-1/2} A D_A^{-1/2}.  lr > 0 applies one Adam step (lr = 0 only
 * computes the gradient).  loss (host, may be null) receives the loss before
 * the update. */
pfe_status pfe_mpnn_train_step(pfe_mpnn* net, pfe_ctx* c, const void* samples, int k, float lr,
                               double* loss);

/* Evaluate the network on the context's A and switch its PCG to
 * M^{-1} = G^T G (PFE_LEARNED).  The factor is kept until the next call;
 * pfe_set_penalties recomputes A but not the factor. */
pfe_status pfe_set_learned(pfe_ctx* c, pfe_mpnn* net);
/* Non-learned factor of the same form, for comparison: the factorized sparse
 * approximate inverse (FSAI, Kolotilina and Yeremin; not in the paper, which
 * uses incomplete Cholesky, Sec. III) on the lower pattern of A: row i of G
 * solves A[S_i, S_i] g = e_i over S_i = {i} and the lower neighbours of i,
 * scaled so that (G A G^T)_ii = 1; M^{-1} = G^T G, stored as Gt = G D_A^{1/2}
 * like the learned factor (pfe_get_factor reads it back).  Computed on the
 * device in FP64 from the context's A (one thread per row, a Cholesky
 * factorisation of the local system) and switches the PCG to PFE_FSAI.
 * Pixel-grid graphs only (4, 8 or 24 stencil slots): PFE_E_ARG otherwise.
 * pfe_set_penalties recomputes A but not the factor. */
pfe_status pfe_set_fsai(pfe_ctx* c);
/* Switch between PFE_JACOBI and the factor preconditioners PFE_LEARNED and
 * PFE_FSAI (the latter two apply whatever factor was set last). */
pfe_status pfe_set_preconditioner(pfe_ctx* c, int precond);
/* Copy the current factor: per undirected edge (lexicographic (i, j), i < j)
 * the entry Gt_ji, and the diagonal (device buffers, context element type). */
pfe_status pfe_get_factor(pfe_ctx* c, void* edge_vals, void* diag);

/* q-quantile of |M Y| over all |E| x d entries for the current Y (the order
 * statistic of rank floor(q (N - 1)) among the N values, computed in the
 * context dtype).  Used to place the shrink threshold. */
pfe_status pfe_edge_quantile(pfe_ctx* c, double q, double* out);

void pfe_destroy_ctx(pfe_ctx* c);

/* ---- Laplacian-eigenmap initialisation ----------------------------------------
 * The spectral embedding the method starts from (Sec. I): the solutions of the
 * generalised eigenproblem (D - W) y = mu D y with the d smallest nonzero mu,
 * computed on the device in FP64 for a graph built by pfe_build_graph (a single
 * graph, not a union).  Chebyshev-filtered subspace iteration on the normalised
 * adjacency D^{-1/2} W D^{-1/2} with a block of k vectors (d <= k <= 32; more
 * guard vectors than d speed up clustered spectra), the trivial solution
 * (mu = 0) projected out exactly, Rayleigh-Ritz by Jacobi rotations.
 *   X0       device, n x k doubles row-major: the starting block (the caller's
 *            random draw), must have full rank after removing the trivial vector
 *   tol      stop when every one of the d wanted Ritz pairs has
 *            ||N x - theta x|| <= tol (x = D^{1/2} y with unit norm)
 *   Y        device, n x d doubles: y_i with y_i^T D y_i = 1, ordered by
 *            increasing mu, each column's entry of largest magnitude (lowest
 *            row on ties) positive
 *   mu       host, d doubles (may be null)
 * PFE_E_NOCONV after max_iter outer iterations without reaching tol (Y and mu
 * hold the last iterate); PFE_E_RANK if the block loses rank; PFE_E_ARG for
 * bad sizes.  Allocates its work space (about 3 n k doubles) for the call and
 * synchronises the stream. */
typedef struct {
    int32_t iterations;      /* outer (filter + Rayleigh-Ritz) iterations run */
    int32_t degree;          /* Chebyshev degree of the last filter */
    double residual;         /* largest ||N x - theta x|| over the d wanted pairs */
    int32_t converged;
} pfe_le_info;
pfe_status pfe_le_init(const pfe_graph* g, int d, const double* X0, int k, double tol, int max_iter, double* Y,
                       double* mu, pfe_le_info* info, hipStream_t stream);

/* ---- k-means on an embedding ----------------------------------------------------
 * The segmentation experiment (Sec. IV) clusters the embedding by k-means.
 * Lloyd iterations on the n rows of Y (device, n x d row-major, dtype
 * PFE_FP32 or PFE_FP64; for the embedding, pfe_get(PFE_YHAT)) from the
 * initial centroids C0 (device, K x d doubles; choosing them is the caller's
 * random draw).  One iteration assigns each row to its nearest centroid (the
 * squared Euclidean distance summed over the coordinates in order in FP64,
 * each product and sum rounded on its own; ties to the lowest index) and then
 * moves each centroid to the mean of its rows (a centroid without rows stays).
 * Stops after max_iter iterations or after one in which no label changed.
 * labels (device, n int32) and centroids (device, K x d doubles; may be C0)
 * receive the result, iters (host, may be null) the iterations run.
 * 1 <= d <= 32, 1 <= K <= 256, K d <= 8000, n < 2^31.  Synchronises the
 * stream: iterations are launched in groups of 8 and the host reads the
 * convergence state after each group (iterations after convergence return
 * at once on the device). */
pfe_status pfe_kmeans(const void* Y, int64_t n, int d, int dtype, const double* C0, int K, int max_iter,
                      int32_t* labels, double* centroids, int32_t* iters, hipStream_t stream);

/* The same as pfe_kmeans, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): it calls no hipMalloc, hipFree or other allocating routine.  Its
 * scratch (the change counters and the K x S x (d + 1) FP64 slice sums, S <= 64
 * row slices) lives in a static device array of the library, 4,227,328 bytes on
 * each GPU it runs on, held until the process ends; its device address is
 * looked up on the first call on a device.  Every argument limit of pfe_kmeans
 * applies (they keep the scratch within the array; a larger need would be
 * rejected with PFE_E_ARG).  All calls on one GPU share that array and leave
 * it holding the last call's values (each call clears what must start at
 * zero): calls that overlap on one GPU, from several threads or streams, race
 * and must be serialised by the caller.  Labels, centroids and iteration
 * counts are identical to pfe_kmeans's. */
pfe_status pfe_kmeans_noalloc(const void* Y, int64_t n, int d, int dtype, const double* C0, int K, int max_iter,
                              int32_t* labels, double* centroids, int32_t* iters, hipStream_t stream);

/* ---- device memory ------------------------------------------------------------
 * Graphs, contexts, networks and the temporaries of a call take device memory
 * from hipMalloc / hipFree unless the caller routes it through its own
 * allocator (for example a caching allocator that owns the process's device
 * memory): alloc(bytes, device, user) returns at least `bytes` bytes of device
 * memory on `device` (256-byte aligned) or null on failure (the library call
 * then returns PFE_E_HIP); release(ptr, device, user) takes it back, called
 * after the device has finished with it.  Both functions or neither (null,
 * null: back to hipMalloc).  Only while no library allocation is live
 * (PFE_E_STATE otherwise); not thread-safe against concurrent library calls. */
typedef void* (*pfe_alloc_fn)(size_t bytes, int device, void* user);
typedef void (*pfe_free_fn)(void* ptr, int device, void* user);
pfe_status pfe_set_allocator(pfe_alloc_fn alloc, pfe_free_fn release, void* user);
/* Device allocations of the library currently live (from either allocator). */
int64_t pfe_live_allocations(void);

/* ---- diagnostics ----------------------------------------------------------- */

/* Plain device copy dst[0..bytes) = src[0..bytes) with 16-byte vector loads and
 * stores (bytes a multiple of 16, both pointers 16-byte aligned), enqueued on
 * stream.  Measures the achievable HBM bandwidth and calibrates traffic
 * counters; it is no part of the embedding method. */
pfe_status pfe_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t stream);

const char* pfe_status_string(pfe_status s);
const char* pfe_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PFE_H */
