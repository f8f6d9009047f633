/*
 * podcg.h -- C ABI of libpodcg, the GPU (MI355X, gfx950) hot path of the
 * POD-augmented conjugate-gradient method for a sequence of SPD systems
 *
 *     A_j x_j = b_j,  j = 1, 2, ...           (Eq. (sequence), Section 2)
 *
 * solved to ||b_j - A_j x_j||_2 <= rtol * ||b_j||_2 (Eq. (sequenceInexact) with
 * a relative forcing term).  Each solve runs Stage 1 (Alg. 2: Galerkin
 * projection onto the augmenting basis W_j) followed by augmented PCG
 * (Alg. 1 with Y = W_j and a Jacobi preconditioner M_j = diag(A_j)); this is
 * Stage 3 of Section 4 with an empty Stage 2.  After a solve the caller
 * pushes the centred solution x_j - xbar_j as a snapshot, and the next basis
 * W_{j+1} is the POD of the last omega snapshots in the metric A_j with
 * inverse-distance weights 2^{1-i} (Alg. pod_evd, Appendix A; weights of
 * Section 3.3; metric choice Theta = A of Section 3.3).
 *
 * Conventions for every entry point:
 *   - Pointers named "device" are HIP device pointers; "host" pointers are
 *     ordinary host memory.  The library never keeps a caller pointer after
 *     the call returns: what it needs later (matrix, snapshots) it copies.
 *   - All device work is ordered on the HIP stream passed to podcg_create
 *     (NULL = the legacy default stream).  Calls that must read a result back
 *     (pattern ingest, status of a factorisation, convergence, statistics)
 *     synchronise that stream before returning; no call synchronises the
 *     whole device.
 *   - Return value: 0 = success, > 0 = warning (result usable), < 0 = error.
 *     No C++ exception crosses this boundary.  podcg_strerror() turns a code
 *     into text; podcg_last_error() gives the context's last detailed message.
 *   - A context is not thread-safe; use one context per host thread.
 *   - Sizes: n < 2^31, nnz < 2^31, basis and snapshot counts <= PODCG_MAX_BASIS.
 */
#ifndef PODCG_H
#define PODCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PODCG_MAX_BASIS 32

/* status codes */
#define PODCG_OK                0
#define PODCG_NOT_CONVERGED     1   /* iteration cap reached; x holds the last iterate       */
#define PODCG_RANK_REDUCED      2   /* basis truncated at a small Cholesky pivot (still solved) */
#define PODCG_ERR_INVALID_ARG  (-1)
#define PODCG_ERR_HIP          (-2)
#define PODCG_ERR_OOM          (-3)
#define PODCG_ERR_NOT_SPD      (-4) /* non-positive diagonal or (A p, p) <= 0                 */
#define PODCG_ERR_NONFINITE    (-5) /* NaN/Inf in b, xbar, the matrix or an iterate            */
#define PODCG_ERR_NO_MATRIX    (-6)
#define PODCG_ERR_SIZE         (-7)

typedef struct podcg_ctx podcg_ctx;

typedef struct {
    int32_t omega;        /* snapshot memory: the last omega snapshots feed the POD (1..32)   */
    int32_t rank_max;     /* largest POD dimension y (0..32); 0 turns recycling off          */
    int32_t maxit;        /* iteration cap of one solve (>= 0)                                */
    int32_t check_every;  /* the host reads the convergence flag every this many iterations  */
    int32_t weights;      /* snapshot weights: 0 = inverse distance 2^{1-i}, 1 = all ones     */
    int32_t timing;       /* > 0: time the three loop kernels with HIP events on every
                             timing-th iteration (statistics only; 0 = off)                   */
    double  rank_rtol;    /* POD keeps eigenvalues lam_i > rank_rtol * lam_1                  */
    double  energy;       /* POD energy criterion in (0, 1); >= 1 disables it                 */
    int32_t precision;    /* 0: FP64 throughout.  1: the augmented PCG runs in FP32 (matrix,
                             vectors and basis stored in FP32, sums in FP64) as the inner solve
                             of FP64 iterative refinement; A W, W^T A W, its Cholesky factor,
                             the POD and the refinement residuals b - A x stay FP64          */
    int32_t max_refine;   /* refinement steps cap when precision = 1                         */
    double  inner_rtol;   /* relative tolerance of each FP32 inner solve (precision = 1)      */
    int32_t spmv_grid;    /* workgroups of the loop SpMV (0 = default 1024; at most 4096)     */
    int32_t update_grid;  /* workgroups of the residual-update kernel (0 = default: for the
                             implicit form one per 2048 rows, rounded up to a multiple of 256
                             and kept within [512, 1024]; 512 otherwise; at most 4096)        */
    int32_t dir_grid;     /* workgroups of the direction kernel (0 = default 1024; <= 4096)   */
    int32_t projection;   /* form of the direction recurrence of Alg. 1 in FP64 solves:
                             0 explicit: p = z + beta p - W mu is formed every iteration;
                             1 implicit: the loop keeps pt = z + beta pt and the coefficients
                               nu of p = pt - W nu (nu = mu + beta nu), forms A p as
                               A pt - (A W) nu inside the residual update and x as
                               xt - W xi once at exit, so W is not read in the loop.  The
                               iterates are the same in exact arithmetic.  Batched solves
                               follow each member's setting; mixed precision
                               (precision = 1) and plain PCG always use the explicit form. */
    int32_t lds_solve;    /* 1: systems of at most 1024 unknowns (slices at most 8 entries
                             wide, basis of at most 5 columns, precision 0) are solved by one
                             workgroup in a single launch, with every vector in registers and
                             the search direction in LDS (explicit direction form); 0: always
                             the multi-kernel loop.  Same arithmetic steps either way.        */
} podcg_options;

typedef struct {
    int32_t iters;          /* search directions used = preconditioner applications in the loop */
    int32_t matvecs;        /* products with A in this solve, setup included                    */
    int32_t rank;           /* dimension of the augmenting basis used                            */
    int32_t status;         /* the solve's return code                                           */
    double  stage1_relres;  /* ||r|| / ||b|| after Stage 1                                       */
    double  relres;         /* recursive ||r|| / ||b|| at exit                                   */
    double  true_relres;    /* ||b - A x|| / ||b|| at exit                                      */
    double  bnorm;          /* ||b||_2                                                           */
    double  cond_G;         /* condition number of W^T A W (1 when there is no basis)            */
    double  setup_ms;       /* A W, W^T A W, its factorisation (GPU time, 0 if reused)           */
    double  solve_ms;       /* Stage 1 + loop + true residual (GPU time)                         */
    int32_t timed_iters;    /* iterations whose kernels were timed (options.timing)              */
    int32_t polls;          /* host reads of the convergence flag                                */
    double  spmv_ms;        /* summed durations of the timed SpMV launches                       */
    double  update_ms;      /* ... of the timed update/reduction launches                        */
    double  dir_ms;         /* ... of the timed direction-update launches                        */
    int32_t refine_steps;   /* FP32 inner solves performed (precision = 1; 0 otherwise)          */
    int32_t path;           /* 1: solved by the one-workgroup kernel (lds_solve), 0: multi-kernel loop */
    double  first_inner_relres; /* ||b - A x|| / ||b|| in FP64 after the first FP32 inner solve */
} podcg_stats;

/* Fill *opt with defaults: omega 20, rank_max 10, maxit 10000, check_every 16,
 * inverse-distance weights, no timing, rank_rtol 1e-12, energy 1 (off),
 * precision 0 (FP64), max_refine 20, inner_rtol 1e-6, default loop grids,
 * projection 1 (implicit), lds_solve 1. */
void podcg_default_options(podcg_options* opt);

/* Create a context for systems of size n.  opt may be NULL (defaults).
 * hip_stream is a hipStream_t (NULL = default stream).  On success *out owns
 * all device state; free it with podcg_destroy.
 * Errors: INVALID_ARG (n < 1, options out of range), OOM, HIP. */
int podcg_create(podcg_ctx** out, int64_t n, const podcg_options* opt, void* hip_stream);

/* Release every resource of the context (NULL is accepted). */
int podcg_destroy(podcg_ctx* ctx);

/* Set the current matrix A_j (Section 2: sparse SPD, n x n) from CSR arrays
 * in device memory: rowptr[n + 1] (int32, rowptr[0] = 0, rowptr[n] = nnz,
 * non-decreasing), colind[nnz] (int32, 0 <= col < n), vals[nnz] (float64).
 * The matrix is copied into the library's SELL-64 layout.  Passing rowptr
 * and colind as NULL reuses the pattern of the previous call (values-only
 * update, the usual case inside a sequence).  The Jacobi preconditioner
 * diag(A_j)^{-1} is formed here.  Any stored basis stays but its products
 * with the matrix are recomputed at the next solve.
 * Errors: INVALID_ARG (bad pattern), NOT_SPD (missing or non-positive
 * diagonal), NONFINITE (NaN/Inf value), NO_MATRIX (NULL pattern on first
 * call), SIZE (nnz differs from the cached pattern), OOM, HIP. */
int podcg_set_matrix(podcg_ctx* ctx, int64_t nnz, const int32_t* rowptr,
                     const int32_t* colind, const double* vals);

/* Append a snapshot s (device, n float64) to the memory of the last omega
 * snapshots; the oldest is overwritten once omega are stored.  In a sequence
 * s = x_j - xbar_j (the centred solution, Section 3.2).  Copied.
 * Errors: INVALID_ARG, HIP. */
int podcg_push_snapshot(podcg_ctx* ctx, const double* s);

/* Forget all stored snapshots (the basis is kept). */
int podcg_reset_snapshots(podcg_ctx* ctx);

/* Build the next augmenting basis W = POD of the stored snapshots in the
 * metric of the current matrix (Alg. pod_evd): Gram diag(w) S^T A S diag(w),
 * symmetric eigen-decomposition, dimension y = #{lam_i > rank_rtol lam_1}
 * capped by rank_max and the energy criterion, W = S diag(w) V_y Sigma_y^{-1}
 * (so W^T A W = I for the current A).  *rank_out (host, may be NULL)
 * receives y, which makes the call wait for the GPU.  With rank_out NULL the
 * call only enqueues the work on the context's stream (the basis is formed
 * with the rank chosen on the device) and returns; the next call that needs
 * the rank on the host (a solve, the basis or spectrum getters, set_basis,
 * another build) waits for it then.  With no snapshots the basis becomes
 * empty.  Errors: NO_MATRIX, HIP. */
int podcg_build_pod(podcg_ctx* ctx, int32_t* rank_out);

/* Replace the augmenting basis with W (device, n x y, column-major with
 * leading dimension n, y <= PODCG_MAX_BASIS; y = 0 clears it).  Copied.
 * Lets a caller supply any basis to Alg. 1 (the paper's Y). */
int podcg_set_basis(podcg_ctx* ctx, const double* W, int32_t y);

/* Copy the current basis into W (device, n x y column-major, ld n, room for
 * rank_max columns).  *rank (host) receives y. */
int podcg_get_basis(podcg_ctx* ctx, double* W, int32_t* rank);

/* Copy the reduced matrix G = W^T A W of the last setup and its inverse (both
 * row-major y x y, host buffers of PODCG_MAX_BASIS^2 doubles, either may be
 * NULL); *rank (host) receives y.  Runs the setup if it is stale. */
int podcg_get_reduced(podcg_ctx* ctx, double* G, double* Ginv, int32_t* rank);

/* Copy the eigenvalues of the last POD Gram matrix (decreasing) into lam
 * (host, PODCG_MAX_BASIS doubles); *count (host) receives how many. */
int podcg_get_pod_spectrum(podcg_ctx* ctx, double* lam, int32_t* count);

/* How the current matrix pattern is stored (the sliced layout of the SpMV
 * that multiplies by A_j every iteration, Alg. 1): counts (host, 5 int64)
 * receives the number of 64-row slices whose columns are stored as
 * [0] int32 indices, [1] 16-bit offsets col - row, [2] one offset table per
 * slice (rows drawing on at most 8 common offsets, as stencils do); [3] the
 * stored value slots (nonzeros plus padding); [4] the bytes of column data
 * one product reads (4 or 2 per slot, 32 per table slice).  Returns
 * PODCG_ERR_NO_MATRIX before the first pattern. */
int podcg_get_format(podcg_ctx* ctx, int64_t* counts);

/* Solve A_j x = b (Stage 1 + augmented PCG, Alg. 2 then Alg. 1 with the
 * current basis; plain Jacobi PCG when the basis is empty).
 * b: device, n float64.  x: device, n float64, holds xbar_j on entry and x_j
 * on return.  rtol >= 0.  st (host, may be NULL) receives statistics.
 * With precision = 1 the solve is FP64 iterative refinement: r = b - A x in
 * FP64; Stage 1 on r in FP64; an FP32 augmented PCG for the correction to
 * relative tolerance inner_rtol (but no further than half the outer target
 * rtol ||b||), its steps added to x in FP64; repeated until the FP64
 * residual meets rtol or max_refine steps were made; maxit caps each inner
 * solve and iters counts all of them.
 * Returns OK, NOT_CONVERGED (x = last iterate), RANK_REDUCED, or an error:
 * NO_MATRIX, INVALID_ARG, NOT_SPD, NONFINITE, HIP. */
int podcg_solve(podcg_ctx* ctx, const double* b, double* x, double rtol, podcg_stats* st);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): podcg_solve
 * on a small system, with no allocation of any kind in the call.  Same
 * arguments, arithmetic and return codes as podcg_solve taking its
 * one-workgroup path (the basis setup is redone on every call), but the
 * device state, A W, W^T A W with its factor and inverse, and the setup
 * kernel's partial sums and counters live in one static device array of the
 * library (about 46 KB per GPU, held until the process ends) instead of the
 * context's buffers; the call reads the context's matrix, Jacobi inverse and
 * basis and writes only x, *st and that array.
 * Limit: precision 0, n <= 1024, slices at most 8 entries wide, a basis of at
 * most 5 columns; anything larger returns PODCG_ERR_SIZE (see
 * podcg_last_error) and runs nothing.  All calls on one GPU share the array:
 * calls that overlap on one GPU (several host threads, or several streams
 * without ordering between them) race; calls ordered on one stream are safe.
 * Synchronises the context stream before returning, like podcg_solve. */
int podcg_solve_noalloc(podcg_ctx* ctx, const double* b, double* x, double rtol, podcg_stats* st);

/* Plain Jacobi PCG on the current matrix, ignoring the basis (the baseline
 * of the comparison; Eq. (KrylovSolve)).  Same arguments and codes. */
int podcg_solve_plain(podcg_ctx* ctx, const double* b, double* x, double rtol, podcg_stats* st);

/* y = A_j x for device vectors of length n (x and y must not overlap). */
int podcg_matvec(podcg_ctx* ctx, const double* x, double* y);

/* out_vals[e] = scale * u[row(e)] * v[col(e)] for every stored entry e of the
 * current CSR pattern, in the caller's CSR order (device, nnz float64).
 * u, v: device, n float64.  With u = lambda (the adjoint solution, Section 2's
 * output functional q = C x differentiated through A x = b), v = x and
 * scale = -1, this is the gradient of lambda^T (b - A x) with respect to the
 * matrix values, i.e. the matrix part of the adjoint of a solve.
 * Errors: NO_MATRIX, INVALID_ARG, HIP. */
int podcg_pattern_outer(podcg_ctx* ctx, const double* u, const double* v, double scale,
                        double* out_vals);

/* Bandwidth probe for the roofline: c[i] = a[i] + s * b[i] over n float64
 * device elements (a, b, c 16-byte aligned, else PODCG_ERR_INVALID_ARG), launched
 * `reps` times on the context stream; *ms (host) receives the mean GPU time
 * of one launch.  Not part of the method. */
int podcg_stream_triad(podcg_ctx* ctx, const double* a, const double* b, double* c,
                       int64_t n, double s, int32_t reps, double* ms);

/* ------------------------------------------------------------- batches
 * Many independent sequences advanced together.  A batch groups existing
 * contexts (its members, each with its own matrix, snapshots and basis, all on
 * one device, precision 0); every member still follows the sequence
 * semantics above (set_matrix / solve / push_snapshot / build_pod on the
 * member itself, or podcg_batch_set_values / podcg_batch_push_build for all
 * members at once).  podcg_batch_solve replaces the members' podcg_solve calls
 * for one system each: every member gets its basis setup and Stage 1
 * (Alg. 2), then the loop of augmented PCG (Alg. 1) runs for all members at
 * once -- per iteration one launch of each loop kernel over a work list of row
 * ranges of the members still running, blocks of graph_iters iterations
 * replayed from a HIP graph.  Per member the arithmetic is that of
 * podcg_solve; only the grouping of partial sums differs (deterministic for
 * fixed options).
 *
 * The batch uses its own HIP stream, ordered after each member's stream at
 * the start of a call; podcg_batch_solve and podcg_batch_tune synchronise it
 * before returning.  Members must outlive the batch and must not be used
 * from another thread during a batch call. */
typedef struct podcg_batch podcg_batch;

typedef struct {
    int32_t slices_per_item;  /* SELL slices (64 rows each) per SpMV work item (>= 1)           */
    int32_t rows_per_item;    /* rows per work item of the vector kernels (>= 256, multiple of 64) */
    int32_t grid;             /* workgroups per loop-kernel launch (1..65536)                  */
    int32_t graph_iters;      /* iterations per captured HIP graph; 0 = direct launches          */
    int32_t check_every;      /* iterations between polls when graph_iters = 0 (>= 1)           */
} podcg_batch_options;

/* Defaults: 8 slices, 2048 rows, grid 1024, graph_iters 16, check_every 16. */
void podcg_batch_default_options(podcg_batch_options* opt);

/* members: host array of `count` (1..1024) distinct contexts.  opt may be NULL.
 * Errors: INVALID_ARG (count, duplicate member, mixed devices, a member with
 * precision 1, options out of range), OOM, HIP. */
int podcg_batch_create(podcg_batch** out, int32_t count, podcg_ctx* const* members,
                       const podcg_batch_options* opt);
int podcg_batch_destroy(podcg_batch* batch);
int podcg_batch_set_options(podcg_batch* batch, const podcg_batch_options* opt);
int podcg_batch_get_options(podcg_batch* batch, podcg_batch_options* opt);

/* One system per member: b[m] (device, n_m float64) and x[m] (device, in:
 * xbar, out: x) are host arrays of device pointers, rtol[m] host doubles;
 * plain != 0 solves with plain Jacobi PCG (no basis).  stats (host, count
 * entries, may be NULL) receives each member's statistics; its status field
 * holds the member's code.  The return value is the most severe member
 * code (an error, else NOT_CONVERGED, else RANK_REDUCED, else OK). */
int podcg_batch_solve(podcg_batch* batch, const double* const* b, double* const* x,
                      const double* rtol, int32_t plain, podcg_stats* stats);

/* New matrix values for every member, with each member's cached pattern:
 * the values-only podcg_set_matrix of all members at once (one ingest launch
 * over all members, one synchronisation).  nnz: host array of `count` entry
 * counts; vals: host array of `count` device pointers (member m's CSR values,
 * nnz[m] float64).  Returns OK, or the first of NONFINITE / NOT_SPD found
 * (that member keeps no matrix and names the cause in its own last error; the
 * others take their values), or INVALID_ARG (a null pointer), NO_MATRIX (a
 * member without a pattern), SIZE (nnz[m] differs from the member's pattern);
 * after INVALID_ARG, NO_MATRIX or SIZE no member changed. */
int podcg_batch_set_values(podcg_batch* batch, const int64_t* nnz, const double* const* vals);

/* After a solve of every member (Section 3.3, Alg. pod_evd): push s[m]
 * (device, n_m float64) as member m's newest snapshot and build its next basis,
 * as podcg_push_snapshot + podcg_build_pod(rank_out = NULL) on each member,
 * with the copies, the Grams S^T A S, the eigen-solves and the bases W = S T
 * each one launch over all members.  Returns without waiting; a member's rank
 * is taken when a later call needs it.  Errors: INVALID_ARG (a null pointer),
 * NO_MATRIX, HIP. */
int podcg_batch_push_build(podcg_batch* batch, const double* const* s);

/* Autotuner: times `iters` loop iterations of all members (Stage 1 first,
 * tolerance 0 so that no member stops early) for candidate work-item sizes and
 * grids, by coordinate descent (SpMV item, vector item, grid), keeps the
 * fastest options in the batch and returns them in *chosen (host, may be
 * NULL) with the time of `iters` iterations in *best_ms.  Each candidate is
 * timed three times (the fastest run counts) and replaces the current choice
 * only when it is at least 1% faster.  x[m] is used as
 * scratch and overwritten.  Errors as podcg_batch_solve. */
int podcg_batch_tune(podcg_batch* batch, const double* const* b, double* const* x, int32_t iters,
                     podcg_batch_options* chosen, double* best_ms);

const char* podcg_batch_last_error(podcg_batch* batch);

/* ------------------------------------------------- three-stage method
 * The paper's full method (Alg. 3, Section 4) with the non-iterative Stage 3
 * (Section 4.3, phi = 0) or the iterative one (Section 4.3.1, phi = 1).  The
 * context keeps an accumulated basis Y (m <= cap columns,
 * device memory) and a stage-1 basis W made of columns of Y.  One
 * podcg_ts_solve runs, for the current matrix A_j:
 *   Stage 1 (Alg. 2)       the direct Galerkin solve over W from x (= xbar);
 *   Stage 2 (Section 4.2)  augmented CG with M = I on Y^T A_j Y (never formed:
 *                          each step is Y p, one SpMV and Y^T q), augmented by
 *                          W, to the stage-2 tolerance
 *                          max(stage2_factor * rtol * ||b||, 1e-6 ||Y^T r||),
 *                          at most min(stage2_maxit, 32 - w) steps;
 *   Stage 3 (Section 4.3)  augmented PCG (Alg. 1, Jacobi) from the Stage-2
 *                          solution over [W, X] (X: the Stage-2 directions)
 *                          with the reused factor blockdiag(R, sqrt(Gammahat))
 *                          (stage3_gram = 0) or the computed and factored Gram
 *                          (stage3_gram = 1), to ||b - A x|| <= rtol ||b||;
 *   Stage 3, phi = 1       augmented PCG from the Stage-2 solution with all of Y
 *                          as the augmenting basis: each projection
 *                          Y^T A Y mu = Y^T A z is solved by augmented CG on the
 *                          reduced matrix against the reduced stage-1 columns,
 *                          the stage-2 directions and the directions of earlier
 *                          projection solves (block-diagonal factor), started
 *                          from the Galerkin solution over them, to inner_rtol
 *                          (default: 1e-2 of the solve's rtol -- the error an
 *                          inexact projection leaves in range(Y) is never
 *                          corrected);
 *                          Stage 2 then runs to stage2_factor rtol ||b|| (floor
 *                          1e-13 of ||Y^T r||, at most min(stage2_maxit, m - w)
 *                          steps), and directions formed from a residual below
 *                          1e-6 of their solve's initial one are not kept;
 * then the Stage-3 directions, scaled to unit A_j-norm, are appended to Y.
 * If Y then has more than ybar columns it is replaced by its POD (metric A_j,
 * weights: RBF 2^{1-i} over the systems since the last truncation or the
 * previous weights, Section 3.3.2; at most y_trunc vectors, energy_y) and W by
 * its leading vectors (w_max, energy_w); otherwise W gains the new vectors the
 * rho rule selects (rho = 0 none, rho = 1 all, else gamma_k / sum gamma > rho),
 * up to w_cap columns.  Directions beyond `cap - m` are not recorded.
 * The three-stage calls leave the context's own basis (podcg_set_basis /
 * podcg_build_pod / podcg_solve) untouched.  Precision 0 only. */
typedef struct {
    int32_t ybar;          /* truncate when Y would exceed ybar columns (1 <= ybar < cap)  */
    int32_t y_trunc;       /* POD dimension after a truncation (1..ybar)                    */
    int32_t w_max;         /* stage-1 dimension after a truncation (0..min(32, y_trunc))    */
    int32_t w_cap;         /* largest stage-1 dimension between truncations (0..32)         */
    int32_t stage2_maxit;  /* Stage-2 step cap (0..32)                                      */
    int32_t cap;           /* column capacity of Y (2..512)                                 */
    int32_t weights;       /* 0 = RBF weights, 1 = previous weights                          */
    int32_t stage3_gram;   /* 0 = reused block-diagonal factor, 1 = computed Gram            */
    double energy_y;       /* energy criterion of the truncated basis, (0, 1], 1 = off       */
    double energy_w;       /* energy criterion of the stage-1 basis, (0, 1], 1 = off         */
    double rho;            /* new-vector rule, [0, 1]                                        */
    double stage2_factor;  /* stage-2 tolerance relative to rtol ||b|| (>= 0)                */
    int32_t phi;           /* Stage 3 over [W, X] (0, Section 4.3) or over all of Y (1, the
                              iterative Stage 3 of Section 4.3.1)                            */
    int32_t inner_maxit;   /* phi = 1: step cap of each projection solve (>= 0)               */
    double inner_rtol;     /* phi = 1: tolerance of each projection solve relative to the norm
                              of its right-hand side Y^T A z (< 1); <= 0: 1e-2 of the solve's
                              rtol                                                            */
} podcg_ts_options;

typedef struct {
    int32_t w, m;          /* stage-1 dimension used, dim Y at the start                     */
    int32_t k2, k3;        /* Stage-2 steps, Stage-3 iterations (preconditioner applications) */
    int32_t matvecs;
    int32_t truncated;     /* 1 if Y was truncated after this solve                          */
    int32_t m_next, w_next;
    int32_t status;
    int32_t jacobi_sweeps; /* sweeps of the truncation's eigen-solver                        */
    double stage1_relres, stage2_relres, relres, true_relres, bnorm;
    double stage12_ms, stage3_ms, accum_ms;
    int32_t k_in;          /* phi = 1: steps of all projection solves                        */
    int32_t projections;   /* phi = 1: projection solves (one per Stage-3 direction)         */
} podcg_ts_stats;

/* Defaults: ybar 200, y_trunc 100, w_max 5, w_cap 16, stage2_maxit 24, cap 512,
 * RBF weights, reused factor, energies 1, rho 0, stage2_factor 1e-4, phi 0,
 * inner_maxit 256, inner_rtol 0 (1e-2 of the solve's rtol). */
void podcg_ts_default_options(podcg_ts_options* opt);

/* Turns the three-stage mode on (or resets it) with an empty Y; allocates two
 * n x cap blocks.  opt may be NULL.  Errors: INVALID_ARG, OOM, HIP. */
int podcg_ts_enable(podcg_ctx* ctx, const podcg_ts_options* opt);

/* One system of Alg. 3 with the current matrix.  b, x: device, n float64
 * (x: in xbar, out x_j).  stats (host) may be NULL.  Returns the Stage-3
 * status (OK, NOT_CONVERGED) or an error (NOT_SPD, NONFINITE, NO_MATRIX,
 * INVALID_ARG, HIP). */
int podcg_ts_solve(podcg_ctx* ctx, const double* b, double* x, double rtol, podcg_ts_stats* stats);

/* Y (device, n x m column-major, may be NULL) and the stage-1 columns sel
 * (host, w entries, may be NULL). */
int podcg_ts_get_state(podcg_ctx* ctx, double* Y, int32_t* m, int32_t* sel, int32_t* w);

/* Replaces Y (device, n x m column-major, m <= ybar), the stage-1 columns
 * (host, w entries, each < m) and the RBF weight accumulator (host, m
 * entries, NULL = zeros).  For tests and restarts. */
int podcg_ts_set_state(podcg_ctx* ctx, const double* Y, int32_t m, const int32_t* sel, int32_t w,
                       const double* eta_acc);

/* Text of a status code (static storage). */
const char* podcg_strerror(int code);

/* Detailed message of the last error in this context (static until the next call). */
const char* podcg_last_error(podcg_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* PODCG_H */
