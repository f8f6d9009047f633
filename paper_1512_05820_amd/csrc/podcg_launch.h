// Launchers of libpodcg's kernels, shared by the host translation units.  Not
// a public header.
#pragma once

#include "podcg_device.h"

namespace podcg {

// SELL kernels (k_sell.hip)
hipError_t launch_validate_csr(int n, int64_t nnz, const int32_t* rowptr, const int32_t* colind,
                               int* flag, hipStream_t s);
hipError_t launch_slice_widths(int n, int nslices, const int32_t* rowptr, int64_t* sptr, hipStream_t s);
hipError_t launch_scan_slices(int nslices, int64_t* sptr, hipStream_t s);
hipError_t launch_fill_pattern(int n, int nslices, const int32_t* rowptr, const int32_t* colind,
                               const int64_t* sptr, int* cols, int* map, hipStream_t s);
// cols16 / sflag from cols: a slice gets 16-bit offsets when every entry of
// its rows < n has |col - row| <= 32767 (padding slots have col = row).
// Per-slice offset tables (flag 2) for the slices whose rows all draw on one
// list of at most kTabMax offsets, exactly as many as the slice is wide; their
// slots are re-laid out in table order (cols and map follow).  Other slices
// get flag 0, and launch_fill_offsets16 then decides between 0 and 1.
hipError_t launch_fill_table(int n, int nslices, const int32_t* rowptr, const int64_t* sptr, int* cols,
                             int* map, int* soff, uint8_t* sflag, hipStream_t s);
hipError_t launch_fill_offsets16(int n, int nslices, const int64_t* sptr, const int* cols, int16_t* cols16,
                                 uint8_t* sflag, hipStream_t s);
// The per-slice metadata records read by the loop SpMV (after the flags are final).
hipError_t launch_fill_meta(int nslices, const int64_t* sptr, const uint8_t* sflag, const int* soff, int* smeta,
                            hipStream_t s);
hipError_t launch_fill_values(int n, int nslices, const int64_t* sptr, const int* cols,
                              const int* map, const uint8_t* sflag, const int* soff, const double* csr_vals,
                              double* vals, double* dinv, int* flag, hipStream_t s);
hipError_t launch_pattern_outer(int n, int nslices, const int64_t* sptr, const int* cols, const int* map,
                                const double* u, const double* v, double scale, double* out,
                                hipStream_t s);
// The loop launchers take optional start/stop events that the dispatch itself
// records (hipExtLaunchKernel): the kernel time without event-marker overhead.
// pairs: use the two-rows-a-lane kernel (matrices stored mostly as offset-table
// slices); otherwise, and for vectors not 16-byte aligned, one row a lane.
hipError_t launch_spmv_gamma(const DevBufs& B, const double* p, double* q, int k, bool pairs, hipStream_t s,
                             hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_spmv_gamma32(const DevBufs& B, const float* p, float* q, int k, hipStream_t s,
                               hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_matvec(const DevBufs& B, const double* x, double* y, hipStream_t s);
hipError_t launch_resid(const DevBufs& B, int yb, int y, const double* b, const double* x,
                        double* r, const double* W, bool store, bool stage1, hipStream_t s);
// AX = A X (stored when `store`) and G = X^T A X (row-major k x k), FP64 MFMA.
hipError_t launch_spmm_gram(const DevBufs& B, int k, const double* X, double* AX, bool store, double* G,
                            hipStream_t s);

// AX = A X for k <= kYMax columns, stored, no Gram (k_gram.hip).
hipError_t launch_spmm(const DevBufs& B, int k, const double* X, double* AX, hipStream_t s);

// Tall-skinny products on the FP64 matrix cores (k_gemm.hip).  X, Y, Out are
// column-major with leading dimension ld.
//   Partial Grams of row chunks: P_c = X(chunk c)^T Y(chunk c), M x N row-major
//   at P + c pstride with row stride ldp; `chunks` is a request (the launch
//   rounds the chunk height to whole panels: gemm_tn_chunks gives the count);
//   sym (M = N, a symmetric product) computes only the tiles on and above the
//   diagonal.  launch_gram_sum adds the chunks in order (mirroring with sym)
//   into G (row stride ldg).
int gemm_tn_chunks(int n, int chunks);
hipError_t launch_gemm_tn_parts(int n, size_t ld, const double* X, int M, const double* Y, int N, int chunks,
                                bool sym, double* P, size_t pstride, int ldp, hipStream_t s);
hipError_t launch_gram_sum(const double* P, int nparts, size_t pstride, int M, int N, int ldp, bool sym,
                           double* G, int ldg, hipStream_t s);
//   Out (n x Ny) = X (n x M) T (M x Ny, column-major, leading dimension ldt).
hipError_t launch_gemm_nn(int n, size_t ld, const double* X, int M, const double* T, int ldt, int Ny,
                          double* Out, hipStream_t s);

// Streaming vector kernels (k_vec.hip)
int basis_tier(int y);   // smallest compiled register tier >= y
// Loop kernels of iteration k (0, 1, ...): each is a no-op once k >= stop.
// The update kernel sums the SpMV's (A p, p) partials itself and forms alpha;
// the direction kernel sums the update's group partials itself and forms beta,
// mu and the convergence decision (workgroup 0 records them in the state).
int spmv_blocks(const DevBufs& B);     // launch grid of the loop SpMV
int update_blocks(const DevBufs& B);   // launch grid of the update kernels
hipError_t launch_update(const DevBufs& B, int yb, int y, double* r, double* z, const double* q,
                         const double* AW, int k, hipStream_t s, hipEvent_t e0 = nullptr,
                         hipEvent_t e1 = nullptr);
// init: the first direction (k unused); otherwise iteration k
hipError_t launch_dir(const DevBufs& B, int yb, int y, double* p, double* x, const double* z,
                      const double* W, bool init, int k, hipStream_t s, hipEvent_t e0 = nullptr,
                      hipEvent_t e1 = nullptr);
hipError_t launch_stage1_apply(const DevBufs& B, int yb, int y, double* x, double* r, double* z,
                               const double* W, const double* AW, hipStream_t s);
// Implicit form of the direction (state flag `implicit`): the loop keeps
// pt = z + beta pt and the coefficients nu of p = pt - W nu, so the direction
// kernel runs with no basis columns and the update kernel forms
// A p = A pt - (A W) nu from the columns of A W it already streams.  The
// solution accumulates x = xt - W xi; launch_implicit_finish applies W xi once.
// AWt: A W in 64-row tiles, element (i, j) at (i / 64) 64 y + 64 j + i mod 64
// (launch_tile_columns), so that the y columns a wave reads are one
// contiguous block of 512 y bytes.
hipError_t launch_update_implicit(const DevBufs& B, int yb, int y, double* r, double* z, const double* qt,
                                  const double* AWt, int k, hipStream_t s, hipEvent_t e0 = nullptr,
                                  hipEvent_t e1 = nullptr);
// dst = the y columns of src (column-major, leading dimension ld, a multiple
// of 64) in 64-row tiles, as read by the implicit update.
hipError_t launch_tile_columns(const double* src, size_t ld, int y, double* dst, hipStream_t s);
// iteration k of the implicit form: x += alpha pt, pt = z + beta pt, and the
// coefficient recurrences (yb, y: the update's basis tier and rank)
hipError_t launch_dir_implicit(const DevBufs& B, int yb, int y, double* p, double* x, const double* z, int k,
                               hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_implicit_finish(const DevBufs& B, int yb, int y, double* x, const double* W, hipStream_t s);
// FP32 loop kernels of the mixed-precision inner solve (same state machine).
hipError_t launch_update32(const DevBufs& B, int yb, int y, float* r, float* z, const float* q,
                           const float* AW, int k, hipStream_t s, hipEvent_t e0 = nullptr,
                           hipEvent_t e1 = nullptr);
hipError_t launch_dir32(const DevBufs& B, int yb, int y, float* p, double* x, const float* z,
                        const float* W, bool init, int k, hipStream_t s, hipEvent_t e0 = nullptr,
                        hipEvent_t e1 = nullptr);
// Mixed-precision Stage 1 of one refinement step: from the FP64 residual r64
// (and what = G^{-1} W^T r64 in the state), x64 += W what, r = r64 - (A W) what
// in FP64, then r32 = r, z32 = M^{-1} r32, sums (r, z), (r, r), (A W)^T z; the
// inner tolerance is max(inner_rtol^2 (r, r), (rtol ||b|| / 2)^2).
hipError_t launch_stage1_mixed(const DevBufs& B, int yb, int y, double* x64, const double* r64,
                               float* r32, float* z32, const double* W, const double* AW,
                               const float* AW32, double inner_rtol, hipStream_t s);
hipError_t launch_to_float(const double* src, float* dst, size_t n, hipStream_t s);
hipError_t launch_pod_form(int n, size_t ld, const double* S, int count, const double* T, int ymax,
                           const int* ydev, double* W, hipStream_t s);
hipError_t launch_copy(const double* src, double* dst, size_t n, hipStream_t s);
hipError_t launch_triad(const double* a, const double* b, double* c, size_t n, double sc,
                        hipStream_t s);
hipError_t launch_state_init(DevState* st, int maxit, double tol2, int y, hipStream_t s,
                             bool implicit = false);

// Batched loop kernels (k_batch.hip).  `counts` holds the lengths of the
// compacted SpMV and vector lists; `active` the number of members still
// iterating.
int batch_tier(int y);   // smallest compiled batched tier >= y
hipError_t launch_batch_compact(const BatchMember* mem, int count, const BatchItem* spmv_full,
                                const BatchItem* vec_full, BatchItem* spmv, BatchItem* vec,
                                int* counts, int* active, hipStream_t s);
hipError_t launch_batch_spmv(const BatchMember* mem, const BatchItem* items, const int* counts,
                             int* active, int grid, hipStream_t s);
hipError_t launch_batch_update(int yb, const BatchMember* mem, const BatchItem* items,
                               const int* counts, int* active, int grid, hipStream_t s);
hipError_t launch_batch_dir(int yb, const BatchMember* mem, const BatchItem* items, const int* counts,
                            int grid, hipStream_t s);
hipError_t launch_batch_gather(const BatchMember* mem, int count, PollBlock* out, hipStream_t s);

// Per-member inputs of the batched basis setup and Stage 1 (index = member,
// parallel to the BatchMember table).
struct BatchSetup {
    const double* b;     // right-hand side of this solve
    double tol2;         // rtol^2 (the Stage-1 kernel scales it by ||b||^2)
    double* G;           // W^T A W (ynom x ynom), its Cholesky factor R, inverse, eigenvalues
    double* R;
    double* Ginv;
    double* lamG;
    double* AWt;         // A W in 64-row tiles for the implicit update, or null
    double* report;      // kept rank, largest and smallest kept eigenvalue (3 doubles)
    int maxit;
    int setup;           // 1: A W, W^T A W and its factor are formed in this solve
    int ynom;            // columns of W before the factor's pivot cut
    int pad;
};

// Per-member inputs of the batched value ingest and POD build.
struct BatchAux {
    const double* src;     // CSR values (ingest) or the new snapshot (POD build)
    const int* map;        // SELL slot -> CSR entry
    double* vals;          // SELL values and 1 / diag, written by the ingest
    double* dinv;
    int* flag;             // ingest flags: 4 diagonal missing or not positive, 8 non-finite value
    double* S;             // snapshot ring, column-major, leading dimension ld
    double* Gs;            // S^T A S (count x count)
    double* T;             // POD coefficients (count x y)
    double* lam;           // POD spectrum
    int* yout;             // POD rank (the member's)
    int* rank;             // the batch's copy of it
    double* W;             // the member's basis
    int slot;              // ring slot of the new snapshot
    int count;             // snapshots in the POD (0: no POD built)
    int rank_max;
    int pad;
    double rank_rtol, energy;
    double w[kYMax];       // weight of each ring slot
};

// Batched value ingest over the SpMV items (k_sell.hip); batched snapshot
// copy and POD form over the vector items (k_vec.hip); the POD eigen-solves,
// one workgroup per listed member (k_small.hip).  The POD Gram S^T A S runs
// through launch_batch_spmm_gram with W = S and no A X store.
hipError_t launch_batch_fill_values(const BatchMember* mem, const BatchAux* aux, const BatchItem* items,
                                    int nitems, int grid, hipStream_t s);
hipError_t launch_batch_push(const BatchMember* mem, const BatchAux* aux, const BatchItem* items, int nitems,
                             int grid, hipStream_t s);
hipError_t launch_batch_pod_coeffs(const BatchAux* aux, const int* list, int nlist, hipStream_t s);
hipError_t launch_batch_pod_form(int kb, const BatchMember* mem, const BatchAux* aux, const BatchItem* items,
                                 int nitems, int grid, hipStream_t s);

// Batched basis setup (k_gram.hip, k_small.hip, k_batch.hip): A W and
// W^T A W over the SpMV items of the members with `setup` set (ks >= their
// ynom), then one workgroup per listed member for the factor, inverse and
// eigenvalues, then the tiled copy of A W over the vector items.
hipError_t launch_batch_spmm_gram(int ks, const BatchMember* mem, const BatchSetup* su, const BatchItem* items,
                                  int nitems, int grid, hipStream_t s);
hipError_t launch_batch_reduced_factor(const BatchMember* mem, const BatchSetup* su, const int* list, int nlist,
                                       hipStream_t s);
hipError_t launch_batch_tile_aw(int yb, const BatchMember* mem, const BatchSetup* su, const BatchItem* items,
                                int nitems, int grid, hipStream_t s);
// Batched Stage 1 (Alg. 2) and the first direction of every member (k_batch.hip).
hipError_t launch_batch_state_init(const BatchMember* mem, const BatchSetup* su, int count, hipStream_t s);
hipError_t launch_batch_resid(int yb, const BatchMember* mem, const BatchSetup* su, const BatchItem* items,
                              int nitems, int grid, hipStream_t s);
hipError_t launch_batch_stage1(int yb, const BatchMember* mem, const BatchItem* items, int nitems, int grid,
                               hipStream_t s);
hipError_t launch_batch_dir_init(int yb, const BatchMember* mem, const BatchItem* items, int nitems, int grid,
                                 hipStream_t s);

hipError_t launch_dir_rec(const DevBufs& B, int yb, int y, double* p, double* x, const double* z,
                          const double* W, double* V, size_t ldv, int cap, double* gamma,
                          double* alpha, int k, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_gemv_n(int n, size_t ld, const double* Y, int m, const double* c, double* out,
                         double sign, bool accumulate, hipStream_t s);
// out = Y^T v through kTsChunks row chunks (part: kTsChunks x m scratch).
hipError_t launch_gemv_t(int n, size_t ld, const double* Y, int m, const double* v, double* part,
                         double* out, hipStream_t s);
hipError_t launch_ts_s2_init(TsDev* T, const DevState* st, int m, const int* sel, int w,
                             const double* GinvW, double tau_rel, double floor_rel, int k2max,
                             hipStream_t s);
// One Stage-2 step; aug (iterative Stage 3, else NULL) receives the kept directions.
hipError_t launch_ts_s2_step(TsDev* T, int m, const int* sel, int w, const double* GinvW, double* aug,
                             hipStream_t s);
// T->gh = Ghat T->ph with Ghat = Y^T A Y formed (row-major m x m).
hipError_t launch_ts_ghat_mv(TsDev* T, const double* Ghat, int m, hipStream_t s);
// A projection solve of the iterative Stage 3 (Section 4.3.1), right-hand side
// in T->cin, in one launch: the Galerkin start over the kept directions, then
// steps with Ghat = Y^T A Y (row-major m x m, formed beforehand) to the
// tolerance rel ||c|| or kinmax steps; acc[0] += steps, acc[1] += 1.
hipError_t launch_ts_in_solve(TsDev* T, double* aug, int m, const int* sel, int w, const double* GinvW,
                              const double* Ghat, double rel, int kinmax, int* acc, hipStream_t s);
hipError_t launch_ts_ginv_blockdiag(const double* GinvW, int w, const TsDev* T, int k2, double* GinvB,
                                    hipStream_t s);
hipError_t launch_ts_eta(TsDev* T, int m, int kr, hipStream_t s);
hipError_t launch_ts_gather(const double* Y, size_t ld, int n, const int* sel, int w, double* B,
                            hipStream_t s);
hipError_t launch_ts_weight_sym(double* G, int M, const double* eta, hipStream_t s);
// Cyclic Jacobi eigen-solver of a symmetric M x M matrix (row-major): init
// (V = I), sweeps over two alternating buffers (each ends with the
// convergence flag), finish (sorted eigenvalues, eigenvectors as columns of
// the current buffer).
hipError_t launch_ts_jacobi_init(double* V, int M, hipStream_t s);
hipError_t launch_ts_jacobi_sweep(double** A, double** A2, double* V, int M, int* flag, hipStream_t s);
hipError_t launch_ts_jacobi_offnorm(const double* A, int M, int* flag, hipStream_t s);
hipError_t launch_ts_jacobi_finish(double* A, int M, double* V, double* lam, hipStream_t s);
hipError_t launch_ts_pod_coeffs(const double* Vs, int M, const double* lam, const double* eta, int y,
                                double* T, hipStream_t s);

// One-workgroup solve of a small system (k_lds.hip): Stage 1 (Alg. 2) and the
// loop of Alg. 1 in one launch of kLdsThreads threads, one row per thread, for
// n <= kLdsThreads, slices at most kLdsWidth wide and a basis of at most
// kLdsYMax columns.  It reads the kept rank (st->y), maxit and the relative
// tolerance (st->tol2) from the state set up by launch_state_init (and the
// factor kernel), and writes the poll block fields as a finished solve does.
int lds_tier(int n, int y);   // y if the one-workgroup solve covers (n, y), else -1
hipError_t launch_lds_solve(const DevBufs& B, int yb, const double* b, double* x, const double* W,
                            const double* AW, hipStream_t s);

// Single-workgroup dense kernels (k_small.hip)
// G (m x m row-major, symmetrised here) -> R, Ginv = G^{-1} on the accepted
// leading block, kept rank written to st->y, eigenvalues of G to lam (cond).
hipError_t launch_reduced_factor(double* G, int m, double* R, double* Ginv, double* lam,
                                 DevState* st, hipStream_t s);
// POD coefficients: Gram (count x count, unweighted S^T A S) -> weighted,
// symmetrised, eigen-decomposed; writes T (count x y row-major) with
// W = S T, lam (count), and y to *y_out.
hipError_t launch_pod_coeffs(const double* Gs, int count, const double* w, int rank_max,
                             double rank_rtol, double energy, double* T, double* lam, int* y_out,
                             hipStream_t s);

}  // namespace podcg
