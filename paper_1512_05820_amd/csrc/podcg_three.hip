// The three-stage method of Alg. 3 (the podcg_ts_* calls of include/podcg.h),
// with the non-iterative Stage 3 of Section 4.3.
//
// Per system: Stage 1 (Alg. 2) over the stage-1 basis W = columns `sel` of the
// accumulated basis Y; Stage 2 (Section 4.2) -- augmented CG on the reduced
// matrix Y^T A Y, never formed: every step is Y p, one SpMV and Y^T q; Stage 3 --
// augmented PCG over [W, X] (X = the Stage-2 directions in full space) from the
// Stage-2 solution, recording its directions V and gamma_k = p_k^T A p_k.  Then
// Z = [Y, V Gamma^{-1/2}] becomes the next Y, or is truncated by POD (metric
// A_j, previous or RBF weights, Section 3.3.2) when it exceeds ybar.
//
// All of it runs in the library's kernels, the two dense products of a
// truncation (Z^T (A Z) and Z T) on the FP64 matrix cores (k_gemm.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "podcg.h"
#include "podcg_launch.h"
#include "podcg_host.h"

using namespace podcg;
using namespace podcg_host;

namespace podcg_host {

struct TsHost {
    podcg_ts_options opt{};
    int m = 0;                   // columns of Y
    std::vector<int> sel;        // columns of Y forming W
    int j = 0, jc = 0;           // systems solved, latest truncation
    double *d_Y = nullptr, *d_AZ = nullptr, *d_B = nullptr, *d_AB = nullptr;
    double *d_part = nullptr, *d_G = nullptr, *d_R = nullptr, *d_GinvW = nullptr, *d_GinvB = nullptr;
    double *d_lamG = nullptr, *d_Gbig = nullptr, *d_Vbig = nullptr, *d_lam = nullptr, *d_T = nullptr;
    int* d_sel = nullptr;
    int* d_info = nullptr;
    double* d_Gbig2 = nullptr;   // second buffer of the Jacobi rounds
    double* d_Gparts = nullptr;  // partial Grams of the row chunks
    double* d_aug = nullptr;     // iterative Stage 3: kept reduced directions and Ghat times them
    int* d_acc = nullptr;        // iterative Stage 3: projection steps and solves of the current system
    TsDev* d_ts = nullptr;
    double* h_dbl = nullptr;     // pinned, kTsCap + 8
    int* h_int = nullptr;        // pinned, kYMax + 8
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
};

void ts_release(podcg_ctx* ctx) {
    TsHost* T = ctx->ts;
    if (!T) return;
    void* dev[] = {T->d_Y, T->d_AZ, T->d_B, T->d_AB, T->d_part, T->d_G, T->d_R, T->d_GinvW, T->d_GinvB,
                   T->d_lamG, T->d_Gbig, T->d_Vbig, T->d_lam, T->d_T, T->d_sel, T->d_info, T->d_ts,
                   T->d_Gbig2, T->d_Gparts, T->d_aug, T->d_acc};
    for (void* p : dev)
        if (p) (void)hipFree(p);
    if (T->h_dbl) (void)hipHostFree(T->h_dbl);
    if (T->h_int) (void)hipHostFree(T->h_int);
    for (hipEvent_t e : T->ev)
        if (e) (void)hipEventDestroy(e);
    delete T;
    ctx->ts = nullptr;
}

}  // namespace podcg_host

namespace {

constexpr double kStage2Floor = 1e-6;   // stage-2 tolerance floor, relative to ||Y^T r||
// Iterative Stage 3 (phi = 1): floor of Stage 2 and of the projection solves,
// relative to their initial residual (rounding level)
constexpr double kRoundingFloor = 1e-13;
// Iterative Stage 3: default projection-solve tolerance relative to the solve's rtol
constexpr double kInnerMargin = 1e-2;
constexpr int kJacobiMaxSweeps = 60;
constexpr int kGramChunks = 64;         // row chunks of the truncation Gram

template <class M>
M* ts_field(TsDev* base, size_t offset) {
    return reinterpret_cast<M*>(reinterpret_cast<char*>(base) + offset);
}
#define TSF(T, field) ts_field<double>((T)->d_ts, offsetof(TsDev, field))

void check_ts_opts(podcg_ctx* ctx, const podcg_ts_options& o) {
    const bool ok = o.cap >= 2 && o.cap <= kTsCap && o.ybar >= 1 && o.ybar < o.cap && o.y_trunc >= 1 &&
                    o.y_trunc <= o.ybar && o.w_max >= 0 && o.w_max <= kYMax && o.w_max <= o.y_trunc &&
                    o.w_cap >= 0 && o.w_cap <= kYMax && o.stage2_maxit >= 0 &&
                    o.stage2_maxit <= (o.phi == 1 ? kTsCap : kYMax) && (o.phi == 0 || o.phi == 1) &&
                    o.inner_maxit >= 0 && o.inner_rtol < 1.0 &&
                    (o.weights == 0 || o.weights == 1) && (o.stage3_gram == 0 || o.stage3_gram == 1) &&
                    o.energy_y > 0.0 && o.energy_y <= 1.0 && o.energy_w > 0.0 && o.energy_w <= 1.0 &&
                    o.rho >= 0.0 && o.rho <= 1.0 && o.stage2_factor >= 0.0;
    if (!ok) fail(ctx, PODCG_ERR_INVALID_ARG, "three-stage options out of range");
}

// Smallest count reaching the energy fraction of the eigenvalues lam (all of
// them count towards the total), capped by y (Sections 3.3.4 and 4.5).
int energy_count(const double* lam, int M, int y, double energy) {
    if (!(energy > 0.0 && energy < 1.0) || y <= 0) return y;
    double tot = 0.0, acc = 0.0;
    for (int i = 0; i < M; ++i)
        if (lam[i] > 0.0) tot += lam[i];
    for (int i = 0; i < y; ++i) {
        acc += lam[i];
        if (acc >= energy * tot) return i + 1;
    }
    return y;
}

// POD truncation of the M accumulated vectors in Y (metric A_j, weights eta).
void truncate(podcg_ctx* ctx, TsHost* T, int M, podcg_ts_stats& S) {
    hipStream_t s = ctx->stream;
    DevBufs D = bufs(ctx);
    const size_t ld = ctx->ld;
    const int n = (int)ctx->n;
    for (int c0 = 0; c0 < M; c0 += kYMax) {
        const int kc = std::min(kYMax, M - c0);
        HIPCHECK(launch_spmm(D, kc, T->d_Y + c0 * ld, T->d_AZ + c0 * ld, s));
    }
    // Z^T (A Z): partial Grams of row chunks on the matrix cores (tiles on and
    // above the diagonal only: the product is symmetric), summed in chunk
    // order; one M x M output alone would leave most of the GPU idle
    const size_t pstride = (size_t)kTsCap * kTsCap;
    HIPCHECK(launch_gemm_tn_parts(n, ld, T->d_Y, M, T->d_AZ, M, kGramChunks, true, T->d_Gparts, pstride, M, s));
    HIPCHECK(launch_gram_sum(T->d_Gparts, gemm_tn_chunks(n, kGramChunks), pstride, M, M, M, true, T->d_Gbig, M, s));
    const double* eta = T->opt.weights == 0 ? TSF(T, eta_acc) : TSF(T, eta_prev);
    HIPCHECK(launch_ts_weight_sym(T->d_Gbig, M, eta, s));
    // Jacobi sweeps until the off-diagonal norm is <= 1e-15 of the Frobenius norm
    HIPCHECK(launch_ts_jacobi_init(T->d_Vbig, M, s));
    HIPCHECK(launch_ts_jacobi_offnorm(T->d_Gbig, M, T->d_info, s));
    double* cur = T->d_Gbig;
    double* other = T->d_Gbig2;
    int sweeps = 0;
    for (;;) {
        HIPCHECK(hipMemcpyAsync(T->h_int, T->d_info, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        if (T->h_int[0] || sweeps >= kJacobiMaxSweeps) break;
        HIPCHECK(launch_ts_jacobi_sweep(&cur, &other, T->d_Vbig, M, T->d_info, s));
        ++sweeps;
    }
    HIPCHECK(launch_ts_jacobi_finish(cur, M, T->d_Vbig, T->d_lam, s));
    HIPCHECK(hipMemcpyAsync(T->h_dbl, T->d_lam, sizeof(double) * M, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    const double* lam = T->h_dbl;
    S.jacobi_sweeps = sweeps;
    int y = 0;
    if (lam[0] > 0.0)
        for (int i = 0; i < M; ++i)
            if (lam[i] > ctx->opt.rank_rtol * lam[0]) y = i + 1;
    y = std::min(y, T->opt.y_trunc);
    y = energy_count(lam, M, y, T->opt.energy_y);
    int w = std::min(T->opt.w_max, y);
    w = energy_count(lam, M, w, T->opt.energy_w);
    if (y > 0) {
        HIPCHECK(launch_ts_pod_coeffs(cur, M, T->d_lam, eta, y, T->d_T, s));
        HIPCHECK(launch_gemm_nn(n, ld, T->d_Y, M, T->d_T, M, y, T->d_AZ, s));
        std::swap(T->d_Y, T->d_AZ);
    }
    T->m = y;
    T->sel.clear();
    for (int i = 0; i < w; ++i) T->sel.push_back(i);
    HIPCHECK(hipMemsetAsync(TSF(T, eta_acc), 0, sizeof(double) * kTsCap, s));
    T->jc = T->j;
    S.truncated = 1;
}

// Accumulation (Alg. 3): Z = [Y, V Gamma^{-1/2}], weights, truncation or the
// rho rule; then the timings and the statistics.  Shared by both Stage 3s.
int ts_finish(podcg_ctx* ctx, TsHost* T, int m, int k3, int code, podcg_ts_stats& S, podcg_ts_stats* out) {
    hipStream_t s = ctx->stream;
    const int cap_rec = T->opt.cap - m;
    if (code >= 0) {
        const int kr = std::min(k3, cap_rec);
        HIPCHECK(launch_ts_eta(T->d_ts, m, kr, s));
        const int M = m + kr;
        if (M > T->opt.ybar) {
            truncate(ctx, T, M, S);
        } else {
            T->m = M;
            std::vector<int> pick;
            if (T->opt.rho >= 1.0) {
                for (int k = 0; k < kr; ++k) pick.push_back(m + k);
            } else if (T->opt.rho > 0.0 && kr > 0) {
                HIPCHECK(hipMemcpyAsync(T->h_dbl, TSF(T, gam3), sizeof(double) * kr, hipMemcpyDeviceToHost, s));
                HIPCHECK(hipStreamSynchronize(s));
                double tot = 0.0;
                for (int k = 0; k < kr; ++k) tot += T->h_dbl[k];
                for (int k = 0; k < kr; ++k)
                    if (T->h_dbl[k] / tot > T->opt.rho) pick.push_back(m + k);
            }
            for (int c : pick)
                if ((int)T->sel.size() < T->opt.w_cap) T->sel.push_back(c);
        }
    }
    HIPCHECK(hipEventRecord(T->ev[3], s));
    HIPCHECK(hipStreamSynchronize(s));
    float a = 0.f, b3 = 0.f, c = 0.f;
    HIPCHECK(hipEventElapsedTime(&a, T->ev[0], T->ev[1]));
    HIPCHECK(hipEventElapsedTime(&b3, T->ev[1], T->ev[2]));
    HIPCHECK(hipEventElapsedTime(&c, T->ev[2], T->ev[3]));
    S.stage12_ms = a;
    S.stage3_ms = b3;
    S.accum_ms = c;
    S.m_next = T->m;
    S.w_next = (int)T->sel.size();
    if (out) *out = S;
    return code;
}

// Stage 3 with phi = 1 (Section 4.3.1): augmented PCG (Alg. 1, Jacobi) from
// the Stage-2 solution with all of Y as the augmenting basis.  The loop
// kernels run with no basis (p = z + beta p); each projection
// Y^T A Y mu = Y^T A z is a projection solve (k_three.hip) whose products
// with Ghat are Y^T (A (Y ph)), and then p -= Y mu.  The host reads the
// convergence flag after every iteration and the projection solve's flag
// after every step of it.
int ts_stage3_iterative(podcg_ctx* ctx, TsHost* T, const double* b, double* x, double rtol, int m, int w, int k2,
                        podcg_ts_stats& S, podcg_ts_stats* out) {
    hipStream_t s = ctx->stream;
    DevBufs D = bufs(ctx);
    const size_t ld = ctx->ld;
    const int n = (int)ctx->n;
    const int maxit = ctx->opt.maxit;
    // the projection solves' tolerance: inner_rtol, or a margin below the
    // solve's own rtol (the error a projection leaves in range(Y) stays)
    const double rel = std::max(T->opt.inner_rtol > 0.0 ? T->opt.inner_rtol : kInnerMargin * rtol, kRoundingFloor);
    // Ghat = Y^T A Y and A Y (in T->d_Gbig2 and T->d_AZ) were formed before Stage 2
    HIPCHECK(hipMemsetAsync(T->d_acc, 0, 2 * sizeof(int), s));
    // T->muin = Ghat^{-1} Y^T A v, iteratively; Y^T A v = (A Y)^T v from the
    // block A Y formed above (A symmetric), with no product with A
    auto project = [&](const double* v) {
        HIPCHECK(launch_gemv_t(n, ld, T->d_AZ, m, v, T->d_part, TSF(T, cin), s));
        HIPCHECK(launch_ts_in_solve(T->d_ts, T->d_aug, m, T->d_sel, w, T->d_GinvW, T->d_Gbig2, rel,
                                    T->opt.inner_maxit, T->d_acc, s));
    };
    HIPCHECK(hipEventRecord(T->ev[1], s));
    HIPCHECK(launch_state_init(ctx->d_st, maxit, rtol * rtol, 0, s));
    // r = b - A x0 (no projection of x0), z = M^{-1} r, and the test before the loop
    HIPCHECK(launch_resid(D, 0, 0, b, x, ctx->d_r, nullptr, true, true, s));
    HIPCHECK(launch_stage1_apply(D, 0, 0, x, ctx->d_r, ctx->d_z, nullptr, nullptr, s));
    poll(ctx);
    const int cap_rec = T->opt.cap - m;
    double* vrec = T->d_Y + (size_t)m * ld;
    if (ctx->h_poll->done == kRunning) {
        project(ctx->d_z);
        HIPCHECK(launch_dir(D, 0, 0, ctx->d_p, x, ctx->d_z, nullptr, true, -1, s));        // p = z
        HIPCHECK(launch_gemv_n(n, ld, T->d_Y, m, TSF(T, muin), ctx->d_p, -1.0, true, s));  // p -= Y mu
        for (int k = 0; k < maxit; ++k) {
            HIPCHECK(launch_spmv_gamma(D, ctx->d_p, ctx->d_q, k, ctx->spmv_pairs, s));
            HIPCHECK(launch_update(D, 0, 0, ctx->d_r, ctx->d_z, ctx->d_q, nullptr, k, s));
            // x += alpha p, p recorded, p = z + beta p, convergence and cap
            HIPCHECK(launch_dir_rec(D, 0, 0, ctx->d_p, x, ctx->d_z, nullptr, vrec, ld, cap_rec, TSF(T, gam3),
                                    TSF(T, alp3), k, s));
            poll(ctx);
            if (ctx->h_poll->done != kRunning) break;
            project(ctx->d_z);
            HIPCHECK(launch_gemv_n(n, ld, T->d_Y, m, TSF(T, muin), ctx->d_p, -1.0, true, s));
        }
    }
    HIPCHECK(launch_resid(D, 0, 0, b, x, nullptr, nullptr, false, false, s));
    int* hacc = T->h_int + kYMax;
    HIPCHECK(hipMemcpyAsync(hacc, T->d_acc, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    poll(ctx);
    const int kin = hacc[0], nproj = hacc[1];
    const PollBlock P = *ctx->h_poll;
    HIPCHECK(hipEventRecord(T->ev[2], s));
    const double bn = S.bnorm;
    const int k3 = P.iter;
    S.k3 = k3;
    S.k_in = kin;
    S.projections = nproj;
    S.relres = bn > 0 ? std::sqrt(P.rr) / bn : std::sqrt(P.rr);
    S.true_relres = bn > 0 ? std::sqrt(P.true_rr) / bn : std::sqrt(P.true_rr);
    // products with A: Stage 1, r0, the loop, A Y for Ghat, the true residual
    // (Stage 2 and the projection solves apply Ghat)
    S.matvecs = w + 1 + 1 + k3 + m + 1;
    const int code = P.done == kFailed ? fail_code(ctx, P) : P.status;
    S.status = code;
    return ts_finish(ctx, T, m, k3, code, S, out);
}

int ts_solve_impl(podcg_ctx* ctx, const double* b, double* x, double rtol, podcg_ts_stats* out) {
    TsHost* T = ctx->ts;
    if (!T) fail(ctx, PODCG_ERR_INVALID_ARG, "three-stage mode is not enabled");
    if (!ctx->has_values) fail(ctx, PODCG_ERR_NO_MATRIX, "no matrix set");
    if (!b || !x || !(rtol >= 0.0)) fail(ctx, PODCG_ERR_INVALID_ARG, "bad solve arguments");
    podcg_ts_stats S{};
    hipStream_t s = ctx->stream;
    DevBufs D = bufs(ctx);
    const size_t ld = ctx->ld;
    const int n = (int)ctx->n;
    const int maxit = ctx->opt.maxit;
    T->j += 1;
    S.m = T->m;
    HIPCHECK(hipEventRecord(T->ev[0], s));

    // ---- Stage 1 (Alg. 2) over W = Y(:, sel)
    int w = (int)T->sel.size();
    if (w > 0) {
        for (int i = 0; i < w; ++i) T->h_int[i] = T->sel[i];
        HIPCHECK(hipMemcpyAsync(T->d_sel, T->h_int, sizeof(int) * w, hipMemcpyHostToDevice, s));
        HIPCHECK(launch_ts_gather(T->d_Y, ld, n, T->d_sel, w, T->d_B, s));
        HIPCHECK(launch_spmm_gram(D, w, T->d_B, T->d_AB, true, T->d_G, s));
        HIPCHECK(launch_reduced_factor(T->d_G, w, T->d_R, T->d_GinvW, T->d_lamG, ctx->d_st, s));
        poll(ctx);
        const int kept = ctx->h_poll->y;
        if (kept < w) {
            w = kept;
            T->sel.resize(w);
        }
    }
    S.w = w;
    D.Ginv = T->d_GinvW;
    HIPCHECK(launch_state_init(ctx->d_st, maxit, rtol * rtol, w, s));
    HIPCHECK(launch_resid(D, basis_tier(w), w, b, x, ctx->d_r, T->d_B, true, true, s));
    if (w > 0) HIPCHECK(launch_stage1_apply(D, basis_tier(w), w, x, ctx->d_r, ctx->d_z, T->d_B, T->d_AB, s));
    poll(ctx);
    const double bn = std::sqrt(ctx->h_poll->bnorm2);
    S.bnorm = bn;
    {
        const double r1 = w > 0 ? ctx->h_poll->rr0 : ctx->h_poll->true_rr;
        S.stage1_relres = bn > 0 ? std::sqrt(r1) / bn : std::sqrt(r1);
    }

    // ---- Stage 2 (Section 4.2) over Y
    int k2 = 0;
    const int m = T->m;
    // phi = 1: the stage-2 directions join the reduced augmentation of the
    // projection solves instead of a [W, X] basis of at most kYMax columns, and
    // Stage 2 runs to its tolerance with a rounding-level floor only (Alg. 1
    // over all of Y never corrects the error it leaves in range(Y))
    const bool iter3 = T->opt.phi == 1 && m > 0;
    if (iter3) {
        // Ghat = Y^T A Y, formed once for the system: A Y in blocks of up to
        // kYMax columns (into the truncation's block, free until the
        // truncation, and kept for the right-hand sides of the projection
        // solves), then the MFMA Gram of the row chunks.  Stage 2 and the
        // projection solves then need Ghat p only, an m x m product, instead
        // of two passes over the tall Y and a matvec per step.
        for (int c0 = 0; c0 < m; c0 += kYMax) {
            const int kc = std::min(kYMax, m - c0);
            HIPCHECK(launch_spmm(D, kc, T->d_Y + c0 * ld, T->d_AZ + c0 * ld, s));
        }
        const size_t pstride = (size_t)kTsCap * kTsCap;
        HIPCHECK(launch_gemm_tn_parts(n, ld, T->d_Y, m, T->d_AZ, m, kGramChunks, true, T->d_Gparts, pstride, m, s));
        HIPCHECK(launch_gram_sum(T->d_Gparts, gemm_tn_chunks(n, kGramChunks), pstride, m, m, m, true, T->d_Gbig2, m,
                                 s));
    }
    if (m > 0) {
        const int k2max = iter3 ? std::min(T->opt.stage2_maxit, m - w) : std::min(T->opt.stage2_maxit, kYMax - w);
        for (int i = 0; i < w; ++i)
            HIPCHECK(launch_gemv_t(n, ld, T->d_Y, m, T->d_AB + i * ld, T->d_part, TSF(T, wtgy) + (size_t)i * m, s));
        HIPCHECK(launch_gemv_t(n, ld, T->d_Y, m, ctx->d_r, T->d_part, TSF(T, rh), s));
        HIPCHECK(launch_ts_s2_init(T->d_ts, ctx->d_st, m, T->d_sel, w, T->d_GinvW, T->opt.stage2_factor * rtol,
                                   iter3 ? kRoundingFloor : kStage2Floor, k2max, s));
        int* h = T->h_int + kYMax;
        for (int k = 0;; ++k) {
            HIPCHECK(hipMemcpyAsync(h, ts_field<int>(T->d_ts, offsetof(TsDev, k2)), 2 * sizeof(int),
                                    hipMemcpyDeviceToHost, s));
            HIPCHECK(hipStreamSynchronize(s));
            if (h[1] || k >= k2max) break;   // h = {k2, done2}
            // u = Y p and q = A u become columns of [W, X] (phi = 0); with
            // phi = 1 the step needs Ghat p only
            if (iter3) {
                HIPCHECK(launch_ts_ghat_mv(T->d_ts, T->d_Gbig2, m, s));
            } else {
                double* u = T->d_B + (size_t)(w + k) * ld;
                double* q = T->d_AB + (size_t)(w + k) * ld;
                HIPCHECK(launch_gemv_n(n, ld, T->d_Y, m, TSF(T, ph), u, 1.0, false, s));
                HIPCHECK(launch_matvec(D, u, q, s));
                HIPCHECK(launch_gemv_t(n, ld, T->d_Y, m, q, T->d_part, TSF(T, gh), s));
            }
            HIPCHECK(launch_ts_s2_step(T->d_ts, m, T->d_sel, w, T->d_GinvW, iter3 ? T->d_aug : nullptr, s));
        }
        k2 = h[0];
        HIPCHECK(hipMemcpyAsync(T->h_dbl, TSF(T, rn), sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        S.stage2_relres = bn > 0 ? T->h_dbl[0] / bn : T->h_dbl[0];
        // x = xbar + Y xhat: Stage 1 already added W what, Stage 2 adds sum_k alpha_k Y p_k
        if (k2 > 0) {
            if (iter3) HIPCHECK(launch_gemv_n(n, ld, T->d_Y, m, TSF(T, xinc), x, 1.0, true, s));
            else HIPCHECK(launch_gemv_n(n, ld, T->d_B + (size_t)w * ld, k2, TSF(T, alp2), x, 1.0, true, s));
        }
    }
    S.k2 = k2;
    if (iter3) return ts_stage3_iterative(ctx, T, b, x, rtol, m, w, k2, S, out);

    // ---- Stage 3 (Section 4.3): augmented PCG over [W, X] from the Stage-2 solution
    int y = w + k2;
    if (y > 0) {
        if (T->opt.stage3_gram == 1) {
            HIPCHECK(launch_spmm_gram(D, y, T->d_B, T->d_AB, true, T->d_G, s));
            HIPCHECK(launch_reduced_factor(T->d_G, y, T->d_R, T->d_GinvB, T->d_lamG, ctx->d_st, s));
            poll(ctx);
            y = ctx->h_poll->y;
        } else {
            HIPCHECK(launch_ts_ginv_blockdiag(T->d_GinvW, w, T->d_ts, k2, T->d_GinvB, s));
        }
    }
    D.Ginv = T->d_GinvB;
    const int yb = basis_tier(y);
    HIPCHECK(hipEventRecord(T->ev[1], s));
    HIPCHECK(launch_state_init(ctx->d_st, maxit, rtol * rtol, y, s));
    // r = b - A x0, with no projection of x0 (what stays zero)
    HIPCHECK(launch_resid(D, 0, 0, b, x, ctx->d_r, nullptr, true, true, s));
    HIPCHECK(launch_stage1_apply(D, yb, y, x, ctx->d_r, ctx->d_z, T->d_B, T->d_AB, s));
    HIPCHECK(launch_dir(D, yb, y, ctx->d_p, x, ctx->d_z, T->d_B, true, -1, s));
    const int cap_rec = T->opt.cap - m;
    double* vrec = T->d_Y + (size_t)m * ld;
    int polls = 0;
    (void)run_loop(ctx, 0, &polls, [&](bool, hipEvent_t*, int k) {
        HIPCHECK(launch_spmv_gamma(D, ctx->d_p, ctx->d_q, k, ctx->spmv_pairs, s));
        HIPCHECK(launch_update(D, yb, y, ctx->d_r, ctx->d_z, ctx->d_q, T->d_AB, k, s));
        HIPCHECK(launch_dir_rec(D, yb, y, ctx->d_p, x, ctx->d_z, T->d_B, vrec, ld, cap_rec, TSF(T, gam3),
                                TSF(T, alp3), k, s));
    });
    HIPCHECK(launch_resid(D, 0, 0, b, x, nullptr, nullptr, false, false, s));
    poll(ctx);
    const PollBlock P = *ctx->h_poll;
    ctx->prev_iters[0] = P.iter;
    HIPCHECK(hipEventRecord(T->ev[2], s));
    const int k3 = P.iter;
    S.k3 = k3;
    S.relres = bn > 0 ? std::sqrt(P.rr) / bn : std::sqrt(P.rr);
    S.true_relres = bn > 0 ? std::sqrt(P.true_rr) / bn : std::sqrt(P.true_rr);
    S.matvecs = w + 1 + k2 + (T->opt.stage3_gram == 1 ? w + k2 : 0) + 1 + k3 + 1;
    int code = P.done == kFailed ? fail_code(ctx, P) : P.status;
    S.status = code;

    return ts_finish(ctx, T, m, k3, code, S, out);
}

}  // namespace

extern "C" {

void podcg_ts_default_options(podcg_ts_options* o) {
    if (!o) return;
    o->ybar = 200;
    o->y_trunc = 100;
    o->w_max = 5;
    o->w_cap = 16;
    o->stage2_maxit = 24;
    o->cap = kTsCap;
    o->weights = 0;
    o->stage3_gram = 0;
    o->energy_y = 1.0;
    o->energy_w = 1.0;
    o->rho = 0.0;
    o->stage2_factor = 1e-4;
    o->phi = 0;
    o->inner_maxit = 256;
    o->inner_rtol = 0.0;
}

int podcg_ts_enable(podcg_ctx* ctx, const podcg_ts_options* opt) {
    return guarded(ctx, [&]() {
        podcg_ts_options o;
        podcg_ts_default_options(&o);
        if (opt) o = *opt;
        check_ts_opts(ctx, o);
        if (ctx->opt.precision != 0) fail(ctx, PODCG_ERR_INVALID_ARG, "three-stage mode needs precision 0");
        ts_release(ctx);
        TsHost* T = new TsHost();
        ctx->ts = T;
        T->opt = o;
        const size_t ld = ctx->ld;
        hipStream_t s = ctx->stream;
        dalloc(ctx, &T->d_Y, ld * (size_t)o.cap);
        dalloc(ctx, &T->d_AZ, ld * (size_t)o.cap);
        dalloc(ctx, &T->d_B, ld * (size_t)kYMax);
        dalloc(ctx, &T->d_AB, ld * (size_t)kYMax);
        dalloc(ctx, &T->d_part, (size_t)kTsChunks * kTsCap);
        dalloc(ctx, &T->d_G, kYMax * kYMax);
        dalloc(ctx, &T->d_R, kYMax * kYMax);
        dalloc(ctx, &T->d_GinvW, kYMax * kYMax);
        dalloc(ctx, &T->d_GinvB, kYMax * kYMax);
        dalloc(ctx, &T->d_lamG, kYMax);
        dalloc(ctx, &T->d_Gbig, (size_t)kTsCap * kTsCap);
        dalloc(ctx, &T->d_Vbig, (size_t)kTsCap * kTsCap);
        dalloc(ctx, &T->d_lam, kTsCap);
        dalloc(ctx, &T->d_T, (size_t)kTsCap * kTsCap);
        dalloc(ctx, &T->d_sel, kYMax);
        dalloc(ctx, &T->d_info, 4);
        dalloc(ctx, &T->d_Gbig2, (size_t)kTsCap * kTsCap);
        dalloc(ctx, &T->d_acc, 2);
        dalloc(ctx, &T->d_Gparts, (size_t)(kGramChunks + 1) * kTsCap * kTsCap);
        if (o.phi == 1) dalloc(ctx, &T->d_aug, kTsAugDoubles);
        dalloc(ctx, &T->d_ts, 1);
        HIPCHECK(hipMemsetAsync(T->d_Y, 0, sizeof(double) * ld * (size_t)o.cap, s));
        HIPCHECK(hipMemsetAsync(T->d_AZ, 0, sizeof(double) * ld * (size_t)o.cap, s));
        HIPCHECK(hipMemsetAsync(T->d_B, 0, sizeof(double) * ld * kYMax, s));
        HIPCHECK(hipMemsetAsync(T->d_AB, 0, sizeof(double) * ld * kYMax, s));
        HIPCHECK(hipMemsetAsync(T->d_ts, 0, sizeof(TsDev), s));
        HIPCHECK(hipHostMalloc((void**)&T->h_dbl, sizeof(double) * (kTsCap + 8), hipHostMallocDefault));
        HIPCHECK(hipHostMalloc((void**)&T->h_int, sizeof(int) * (kYMax + 8), hipHostMallocDefault));
        for (auto& e : T->ev) HIPCHECK(hipEventCreate(&e));
        sync(ctx);
        return PODCG_OK;
    });
}

int podcg_ts_solve(podcg_ctx* ctx, const double* b, double* x, double rtol, podcg_ts_stats* stats) {
    return guarded(ctx, [&]() { return ts_solve_impl(ctx, b, x, rtol, stats); });
}

int podcg_ts_get_state(podcg_ctx* ctx, double* Y, int32_t* m, int32_t* sel, int32_t* w) {
    return guarded(ctx, [&]() {
        TsHost* T = ctx->ts;
        if (!T) fail(ctx, PODCG_ERR_INVALID_ARG, "three-stage mode is not enabled");
        if (m) *m = T->m;
        if (w) *w = (int)T->sel.size();
        if (sel)
            for (size_t i = 0; i < T->sel.size(); ++i) sel[i] = T->sel[i];
        if (Y)
            for (int k = 0; k < T->m; ++k)
                HIPCHECK(launch_copy(T->d_Y + (size_t)k * ctx->ld, Y + (size_t)k * ctx->n, (size_t)ctx->n,
                                     ctx->stream));
        sync(ctx);
        return PODCG_OK;
    });
}

int podcg_ts_set_state(podcg_ctx* ctx, const double* Y, int32_t m, const int32_t* sel, int32_t w,
                       const double* eta_acc) {
    return guarded(ctx, [&]() {
        TsHost* T = ctx->ts;
        if (!T) fail(ctx, PODCG_ERR_INVALID_ARG, "three-stage mode is not enabled");
        if (m < 0 || m > T->opt.ybar || (m > 0 && !Y) || w < 0 || w > kYMax || (w > 0 && !sel))
            fail(ctx, PODCG_ERR_INVALID_ARG, "bad three-stage state");
        for (int i = 0; i < w; ++i)
            if (sel[i] < 0 || sel[i] >= m) fail(ctx, PODCG_ERR_INVALID_ARG, "selected column out of range");
        for (int k = 0; k < m; ++k)
            HIPCHECK(launch_copy(Y + (size_t)k * ctx->n, T->d_Y + (size_t)k * ctx->ld, (size_t)ctx->n,
                                 ctx->stream));
        HIPCHECK(hipMemsetAsync(TSF(T, eta_acc), 0, sizeof(double) * kTsCap, ctx->stream));
        if (eta_acc && m > 0) {
            std::memcpy(T->h_dbl, eta_acc, sizeof(double) * m);
            HIPCHECK(hipMemcpyAsync(TSF(T, eta_acc), T->h_dbl, sizeof(double) * m, hipMemcpyHostToDevice,
                                    ctx->stream));
        }
        T->m = m;
        T->sel.assign(sel, sel + w);
        sync(ctx);
        return PODCG_OK;
    });
}

}  // extern "C"
