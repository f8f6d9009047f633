// Host side of libpodcg: the C ABI declared in include/podcg.h.
//
// A context owns the SELL copy of the current matrix, the Jacobi inverse, the
// augmenting basis W with A W and the factor of W^T A W, the snapshot ring,
// the CG vectors and the device scalar state.  Every entry point validates its
// arguments, enqueues kernels on the context stream and converts failures to
// status codes; no C++ exception leaves this file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
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

DevBufs bufs(podcg_ctx* ctx) {
    DevBufs B;
    B.n = (int)ctx->n;
    B.nslices = ctx->nslices;
    B.ld = ctx->ld;
    B.sptr = ctx->d_sptr;
    B.cols = ctx->d_cols;
    B.cols16 = ctx->d_cols16;
    B.sflag = ctx->d_sflag;
    B.soff = ctx->d_soff;
    B.smeta = ctx->d_smeta;
    B.vals = ctx->d_vals;
    B.dinv = ctx->d_dinv;
    B.st = ctx->d_st;
    B.part = ctx->d_part;
    B.counter = ctx->d_counter;
    B.gpart = ctx->d_gpart;
    B.Ginv = ctx->d_Ginv;
    B.vals32 = ctx->d_vals32;
    B.dinv32 = ctx->d_dinv32;
    B.spmv_grid = ctx->opt.spmv_grid > 0 ? ctx->opt.spmv_grid : kSpmvGrid;
    B.update_grid = ctx->opt.update_grid > 0 ? ctx->opt.update_grid : kUpdateGrid;
    B.dir_grid = ctx->opt.dir_grid > 0 ? ctx->opt.dir_grid : kDirGrid;
    return B;
}

void sync(podcg_ctx* ctx) { HIPCHECK(hipStreamSynchronize(ctx->stream)); }

void pod_resolve(podcg_ctx* ctx) {
    if (!ctx->y_pending) return;
    HIPCHECK(hipEventSynchronize(ctx->ev_ext ? ctx->ev_ext : ctx->ev_pod));
    ctx->y = ctx->rank_ext ? *ctx->rank_ext : *ctx->h_rank;
    ctx->y_pending = false;
    ctx->rank_ext = nullptr;
    ctx->ev_ext = nullptr;
}

void pod_slot_weights(const podcg_ctx* ctx, double* w) {
    for (int slot = 0; slot < ctx->count; ++slot) {
        const int age = (ctx->head - 1 - slot + ctx->opt.omega) % ctx->opt.omega;   // 0 = newest
        w[slot] = ctx->opt.weights == 0 ? std::ldexp(1.0, -age) : 1.0;
    }
}

void poll(podcg_ctx* ctx) {
    HIPCHECK(hipMemcpyAsync(ctx->h_poll, ctx->d_st, sizeof(PollBlock), hipMemcpyDeviceToHost,
                            ctx->stream));
    sync(ctx);
}

void check_opts(const podcg_options& o) {
    if (o.omega < 1 || o.omega > PODCG_MAX_BASIS || o.rank_max < 0 || o.rank_max > PODCG_MAX_BASIS ||
        o.maxit < 0 || o.check_every < 1 || (o.weights != 0 && o.weights != 1) || o.timing < 0 ||
        !(o.rank_rtol >= 0.0) || !(o.energy > 0.0) || (o.precision != 0 && o.precision != 1) ||
        o.max_refine < 1 || !(o.inner_rtol > 0.0 && o.inner_rtol < 1.0) || o.spmv_grid < 0 ||
        o.spmv_grid > kLoopGridMax || o.update_grid < 0 || o.update_grid > kLoopGridMax || o.dir_grid < 0 ||
        o.dir_grid > kLoopGridMax || (o.projection != 0 && o.projection != 1) ||
        (o.lds_solve != 0 && o.lds_solve != 1))
        throw Fail{PODCG_ERR_INVALID_ARG};
}

// A W, G = W^T A W, factor and inverse; sync to read the kept rank.
void setup_basis(podcg_ctx* ctx) {
    if (ctx->y == 0) {
        ctx->y_kept = 0;
        ctx->setup_valid = true;
        ctx->cond_G = 1.0;
        ctx->rank_reduced = false;
        return;
    }
    DevBufs B = bufs(ctx);
    HIPCHECK(launch_spmm_gram(B, ctx->y, ctx->d_W, ctx->d_AW, true, ctx->d_G, ctx->stream));
    HIPCHECK(launch_reduced_factor(ctx->d_G, ctx->y, ctx->d_R, ctx->d_Ginv, ctx->d_lamG, ctx->d_st,
                                   ctx->stream));
    // the kept rank and the eigenvalues of G (for its condition number) come
    // back under one synchronisation
    HIPCHECK(hipMemcpyAsync(ctx->h_poll, ctx->d_st, sizeof(PollBlock), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHECK(hipMemcpyAsync(ctx->h_dbl, ctx->d_lamG, sizeof(double) * ctx->y, hipMemcpyDeviceToHost,
                            ctx->stream));
    sync(ctx);
    const int kept = ctx->h_poll->y;
    ctx->y_kept = kept;
    ctx->rank_reduced = kept < ctx->y;
    if (kept > 0) {
        const double lmax = ctx->h_dbl[0], lmin = ctx->h_dbl[kept - 1];
        ctx->cond_G = lmin > 0.0 ? lmax / lmin : INFINITY;
    } else {
        ctx->cond_G = 1.0;
    }
    if (ctx->opt.precision == 1 && kept > 0) {
        HIPCHECK(launch_to_float(ctx->d_W, ctx->d_W32, ctx->ld * (size_t)kept, ctx->stream));
        HIPCHECK(launch_to_float(ctx->d_AW, ctx->d_AW32, ctx->ld * (size_t)kept, ctx->stream));
    }
    if (ctx->opt.precision == 0 && ctx->opt.projection == 1 && kept > 0)   // the implicit update's tiled copy of A W
        HIPCHECK(launch_tile_columns(ctx->d_AW, ctx->ld, kept, ctx->d_AWt, ctx->stream));
    ctx->setup_valid = true;
}

void record(podcg_ctx* ctx, hipEvent_t e) { HIPCHECK(hipEventRecord(e, ctx->stream)); }

// Add the event-timed kernel durations of the first `iters` iterations.
void add_timing(podcg_ctx* ctx, const std::vector<int>& timed, int iters, podcg_stats& S) {
    for (size_t k = 0; k < timed.size(); ++k) {
        if (timed[k] >= iters) break;
        float a = 0, b = 0, c = 0;
        HIPCHECK(hipEventElapsedTime(&a, ctx->tev[6 * k + 0], ctx->tev[6 * k + 1]));
        HIPCHECK(hipEventElapsedTime(&b, ctx->tev[6 * k + 2], ctx->tev[6 * k + 3]));
        HIPCHECK(hipEventElapsedTime(&c, ctx->tev[6 * k + 4], ctx->tev[6 * k + 5]));
        S.spmv_ms += a;
        S.update_ms += b;
        S.dir_ms += c;
        S.timed_iters += 1;
    }
}

int fail_code(podcg_ctx* ctx, const PollBlock& P) {
    ctx->last_error = P.status == PODCG_ERR_NOT_SPD ? "(A p, p) <= 0: matrix not SPD"
                                                    : "non-finite value in the iteration";
    return P.status;
}

// FP64 iterative refinement around FP32 augmented PCG (precision = 1).
int solve_mixed(podcg_ctx* ctx, const double* b, double* x, double rtol, podcg_stats& S, bool plain,
                int y, bool did_setup) {
    const int yb = basis_tier(y);
    DevBufs B = bufs(ctx);
    hipStream_t s = ctx->stream;
    const int slot = plain ? 1 : 0;
    int polls = 0, total = 0, steps = 0, code = PODCG_NOT_CONVERGED;
    double bn2 = 0.0, rr64 = 0.0;
    std::vector<int> timed_all;
    for (int step = 0;; ++step) {
        HIPCHECK(launch_state_init(ctx->d_st, ctx->opt.maxit, rtol * rtol, y, s));
        // FP64 residual r = b - A x, with what = G^{-1} W^T r for Stage 1
        HIPCHECK(launch_resid(B, yb, y, b, x, ctx->d_r, ctx->d_W, true, true, s));
        poll(ctx);
        ++polls;
        const PollBlock R = *ctx->h_poll;
        if (R.done == kFailed) return fail_code(ctx, R);
        bn2 = R.bnorm2;
        rr64 = R.true_rr;
        if (step == 1) S.first_inner_relres = bn2 > 0 ? std::sqrt(rr64 / bn2) : std::sqrt(rr64);
        if (rr64 <= rtol * rtol * bn2) {
            code = PODCG_OK;
            break;
        }
        if (step >= ctx->opt.max_refine) break;
        // Stage 1 in FP64, then the FP32 augmented PCG on the correction
        HIPCHECK(launch_stage1_mixed(B, yb, y, x, ctx->d_r, ctx->d_r32, ctx->d_z32, ctx->d_W,
                                     ctx->d_AW, ctx->d_AW32, ctx->opt.inner_rtol, s));
        HIPCHECK(launch_dir32(B, yb, y, ctx->d_p32, x, ctx->d_z32, ctx->d_W32, true, -1, s));
        std::vector<int> timed = run_loop(ctx, slot, &polls, [&](bool t, hipEvent_t* ev, int k) {
            hipEvent_t none[6] = {};
            hipEvent_t* e = t ? ev : none;
            HIPCHECK(launch_spmv_gamma32(B, ctx->d_p32, ctx->d_q32, k, s, e[0], e[1]));
            HIPCHECK(launch_update32(B, yb, y, ctx->d_r32, ctx->d_z32, ctx->d_q32, ctx->d_AW32, k, s, e[2], e[3]));
            HIPCHECK(launch_dir32(B, yb, y, ctx->d_p32, x, ctx->d_z32, ctx->d_W32, false, k, s, e[4], e[5]));
        });
        poll(ctx);
        const PollBlock P = *ctx->h_poll;
        if (P.done == kFailed) return fail_code(ctx, P);
        if (step == 0) S.stage1_relres = bn2 > 0 ? std::sqrt(P.rr0 / bn2) : std::sqrt(P.rr0);
        add_timing(ctx, timed, P.iter, S);
        ctx->prev_iters[slot] = P.iter;
        total += P.iter;
        ++steps;
    }
    const double bn = std::sqrt(bn2);
    S.bnorm = bn;
    S.iters = total;
    S.refine_steps = steps;
    S.relres = S.true_relres = bn > 0 ? std::sqrt(rr64) / bn : std::sqrt(rr64);
    if (steps == 0) S.stage1_relres = S.relres;
    S.matvecs = total + steps + 1 + (did_setup ? ctx->y : 0);
    S.polls = polls;
    S.rank = y;
    S.cond_G = y > 0 ? ctx->cond_G : 1.0;
    return code;
}

// Whether the one-workgroup solve takes this system: FP64, at most
// kLdsThreads unknowns, slices at most kLdsWidth wide and a basis (its
// uncut dimension, an upper bound of the kept rank) within the register tiers.
bool lds_path(podcg_ctx* ctx, bool plain) {
    if (ctx->opt.precision != 0 || ctx->opt.lds_solve == 0) return false;
    if (ctx->max_width < 0 || ctx->max_width > kLdsWidth) return false;
    return lds_tier((int)ctx->n, plain ? 0 : ctx->y) >= 0;
}

// Stage 1 + augmented PCG of a small system in one launch (k_lds.hip), after
// the setup kernels when the basis products are stale.  The kept rank goes
// from the factor kernel to the solve through the device state, so the host
// synchronises once, at the end, for the statistics.
int solve_lds(podcg_ctx* ctx, const double* b, double* x, double rtol, podcg_stats& S, bool plain) {
    hipStream_t s = ctx->stream;
    DevBufs B = bufs(ctx);
    const bool setup = !plain && !ctx->setup_valid && ctx->y > 0;
    const int y0 = plain ? 0 : (ctx->setup_valid ? ctx->y_kept : ctx->y);
    HIPCHECK(hipEventRecord(ctx->ev_a, s));
    HIPCHECK(launch_state_init(ctx->d_st, ctx->opt.maxit, rtol * rtol, y0, s));
    if (setup) {
        HIPCHECK(launch_spmm_gram(B, ctx->y, ctx->d_W, ctx->d_AW, true, ctx->d_G, s));
        HIPCHECK(launch_reduced_factor(ctx->d_G, ctx->y, ctx->d_R, ctx->d_Ginv, ctx->d_lamG, ctx->d_st, s));
    }
    HIPCHECK(hipEventRecord(ctx->ev_b, s));
    HIPCHECK(launch_lds_solve(B, plain ? 0 : ctx->y, b, x, ctx->d_W, ctx->d_AW, s));
    HIPCHECK(hipEventRecord(ctx->ev_c, s));
    HIPCHECK(hipMemcpyAsync(ctx->h_poll, ctx->d_st, sizeof(PollBlock), hipMemcpyDeviceToHost, s));
    if (setup)
        HIPCHECK(hipMemcpyAsync(ctx->h_dbl, ctx->d_lamG, sizeof(double) * ctx->y, hipMemcpyDeviceToHost, s));
    sync(ctx);
    const PollBlock P = *ctx->h_poll;
    if (setup) {
        const int kept = P.y;
        ctx->y_kept = kept;
        ctx->rank_reduced = kept < ctx->y;
        const double lmax = kept > 0 ? ctx->h_dbl[0] : 1.0, lmin = kept > 0 ? ctx->h_dbl[kept - 1] : 1.0;
        ctx->cond_G = kept > 0 ? (lmin > 0.0 ? lmax / lmin : INFINITY) : 1.0;
        ctx->setup_valid = true;
    }
    const int y = plain ? 0 : P.y;
    const double bn = std::sqrt(P.bnorm2);
    S.iters = P.iter;
    S.rank = y;
    S.bnorm = bn;
    S.stage1_relres = bn > 0 ? std::sqrt(P.rr0) / bn : std::sqrt(P.rr0);
    S.relres = bn > 0 ? std::sqrt(P.rr) / bn : std::sqrt(P.rr);
    S.true_relres = bn > 0 ? std::sqrt(P.true_rr) / bn : std::sqrt(P.true_rr);
    S.cond_G = y > 0 ? ctx->cond_G : 1.0;
    S.matvecs = P.iter + 2 + (setup ? ctx->y : 0);
    S.polls = 1;
    S.path = 1;
    float ms = 0.f;
    HIPCHECK(hipEventElapsedTime(&ms, ctx->ev_a, ctx->ev_b));
    S.setup_ms = setup ? ms : 0.0;
    HIPCHECK(hipEventElapsedTime(&ms, ctx->ev_b, ctx->ev_c));
    S.solve_ms = ms;
    int code = P.done == kFailed ? fail_code(ctx, P) : P.status;
    if (code == PODCG_OK && !plain && ctx->rank_reduced) code = PODCG_RANK_REDUCED;
    S.status = code;
    return code;
}

int solve_impl(podcg_ctx* ctx, const double* b, double* x, double rtol, podcg_stats* st, bool plain) {
    if (!ctx->has_values) fail(ctx, PODCG_ERR_NO_MATRIX, "no matrix set");
    pod_resolve(ctx);
    if (!b || !x || !(rtol >= 0.0)) fail(ctx, PODCG_ERR_INVALID_ARG, "bad solve arguments");
    podcg_stats S{};
    float ms = 0.f;
    if (lds_path(ctx, plain)) {
        const int code = solve_lds(ctx, b, x, rtol, S, plain);
        if (st) *st = S;
        return code;
    }

    HIPCHECK(hipEventRecord(ctx->ev_a, ctx->stream));
    bool did_setup = false;
    if (!plain && !ctx->setup_valid) {   // also resets the kept rank when the basis is empty
        setup_basis(ctx);
        did_setup = ctx->y > 0;
    }
    HIPCHECK(hipEventRecord(ctx->ev_b, ctx->stream));
    const int y = plain ? 0 : ctx->y_kept;
    const int yb = basis_tier(y);
    DevBufs B = bufs(ctx);
    hipStream_t s = ctx->stream;
    int code;

    if (ctx->opt.precision == 1) {
        code = solve_mixed(ctx, b, x, rtol, S, plain, y, did_setup);
        HIPCHECK(hipEventRecord(ctx->ev_c, s));
        sync(ctx);
    } else {
        // implicit form: d_p holds pt and the direction kernel carries no basis
        const bool imp = y > 0 && ctx->opt.projection == 1;
        const int dyb = imp ? 0 : yb, dy = imp ? 0 : y;
        // the implicit update by default: about sixteen rows a thread (one
        // workgroup per 4096 rows, a multiple of 256, between 512 and 1024;
        // 512 at 128^3, where it took 27.8 against 29.6 us at 1024 once the
        // update stored z alone)
        if (imp && ctx->opt.update_grid == 0)
            B.update_grid = (int)std::min<int64_t>(kUpdateGridImplicit,
                std::max<int64_t>(kUpdateGrid, ((ctx->n + 4095) / 4096 + 255) / 256 * 256));
        HIPCHECK(launch_state_init(ctx->d_st, ctx->opt.maxit, rtol * rtol, y, s, imp));
        // Stage 1: rbar = b - A xbar, what = G^{-1} W^T rbar
        HIPCHECK(launch_resid(B, yb, y, b, x, ctx->d_r, ctx->d_W, true, true, s));
        // x = xbar + W what, r = rbar - (A W) what, z = M^{-1} r, mu = G^{-1} (A W)^T z
        HIPCHECK(launch_stage1_apply(B, yb, y, x, ctx->d_r, ctx->d_z, ctx->d_W, ctx->d_AW, s));
        // p = z - W mu (explicit), pt = z (implicit)
        HIPCHECK(launch_dir(B, dyb, dy, ctx->d_p, x, ctx->d_z, ctx->d_W, true, -1, s));
        int polls = 0;
        std::vector<int> timed = run_loop(ctx, plain ? 1 : 0, &polls, [&](bool t, hipEvent_t* ev, int k) {
            hipEvent_t none[6] = {};
            hipEvent_t* e = t ? ev : none;
            HIPCHECK(launch_spmv_gamma(B, ctx->d_p, ctx->d_q, k, ctx->spmv_pairs, s, e[0], e[1]));
            if (imp) {
                HIPCHECK(launch_update_implicit(B, yb, y, ctx->d_r, ctx->d_z, ctx->d_q, ctx->d_AWt, k, s, e[2], e[3]));
                HIPCHECK(launch_dir_implicit(B, yb, y, ctx->d_p, x, ctx->d_z, k, s, e[4], e[5]));
            } else {
                HIPCHECK(launch_update(B, yb, y, ctx->d_r, ctx->d_z, ctx->d_q, ctx->d_AW, k, s, e[2], e[3]));
                HIPCHECK(launch_dir(B, yb, y, ctx->d_p, x, ctx->d_z, ctx->d_W, false, k, s, e[4], e[5]));
            }
        });
        if (imp) HIPCHECK(launch_implicit_finish(B, yb, y, x, ctx->d_W, s));   // x = xt - W xi
        // true residual ||b - A x||
        HIPCHECK(launch_resid(B, 0, 0, b, x, nullptr, nullptr, false, false, s));
        HIPCHECK(hipEventRecord(ctx->ev_c, s));
        poll(ctx);
        const PollBlock P = *ctx->h_poll;
        S.iters = P.iter;
        ctx->prev_iters[plain ? 1 : 0] = P.iter;
        S.rank = y;
        const double bn = std::sqrt(P.bnorm2);
        S.bnorm = bn;
        S.stage1_relres = bn > 0 ? std::sqrt(P.rr0) / bn : std::sqrt(P.rr0);
        S.relres = bn > 0 ? std::sqrt(P.rr) / bn : std::sqrt(P.rr);
        S.true_relres = bn > 0 ? std::sqrt(P.true_rr) / bn : std::sqrt(P.true_rr);
        S.cond_G = y > 0 ? ctx->cond_G : 1.0;
        S.matvecs = P.iter + 2 + (did_setup ? ctx->y : 0);
        S.polls = polls;
        add_timing(ctx, timed, P.iter, S);
        code = P.done == kFailed ? fail_code(ctx, P) : P.status;
    }
    HIPCHECK(hipEventElapsedTime(&ms, ctx->ev_a, ctx->ev_b));
    S.setup_ms = did_setup ? ms : 0.0;
    HIPCHECK(hipEventElapsedTime(&ms, ctx->ev_b, ctx->ev_c));
    S.solve_ms = ms;
    if (code == PODCG_OK && !plain && ctx->rank_reduced) code = PODCG_RANK_REDUCED;
    S.status = code;
    if (st) *st = S;
    return code;
}

}  // namespace podcg_host

namespace {

void release(podcg_ctx* ctx) {
    ts_release(ctx);
    void* dev[] = {ctx->d_sptr, ctx->d_cols, ctx->d_cols16, ctx->d_sflag, ctx->d_soff, ctx->d_smeta, ctx->d_map, ctx->d_vals, ctx->d_dinv, ctx->d_r,
                   ctx->d_z, ctx->d_p, ctx->d_q, ctx->d_W, ctx->d_AW, ctx->d_AWt, ctx->d_G, ctx->d_R,
                   ctx->d_Ginv, ctx->d_lamG, ctx->d_S, ctx->d_Gs, ctx->d_T,
                   ctx->d_lamS, ctx->d_yout, ctx->d_st, ctx->d_part, ctx->d_counter, ctx->d_gpart, ctx->d_flag,
                   ctx->d_vals32, ctx->d_dinv32, ctx->d_W32, ctx->d_AW32, ctx->d_r32, ctx->d_z32,
                   ctx->d_p32, ctx->d_q32};
    for (void* p : dev)
        if (p) (void)hipFree(p);
    if (ctx->h_poll) (void)hipHostFree(ctx->h_poll);
    if (ctx->h_int) (void)hipHostFree(ctx->h_int);
    if (ctx->h_dbl) (void)hipHostFree(ctx->h_dbl);
    if (ctx->h_rank) (void)hipHostFree(ctx->h_rank);
    if (ctx->ev_pod) (void)hipEventDestroy(ctx->ev_pod);
    hipEvent_t evs[] = {ctx->ev_a, ctx->ev_b, ctx->ev_c, ctx->ev_d};
    for (hipEvent_t e : evs)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->tev) (void)hipEventDestroy(e);
}

}  // namespace

// ====================================================================== ABI

extern "C" {

void podcg_default_options(podcg_options* o) {
    if (!o) return;
    o->omega = 20;
    o->rank_max = 10;
    o->maxit = 10000;
    o->check_every = 16;
    o->weights = 0;
    o->timing = 0;
    o->rank_rtol = 1e-12;
    o->energy = 1.0;
    o->precision = 0;
    o->max_refine = 20;
    o->inner_rtol = 1e-6;
    o->spmv_grid = 0;
    o->update_grid = 0;
    o->dir_grid = 0;
    o->projection = 1;
    o->lds_solve = 1;
}

const char* podcg_strerror(int code) {
    switch (code) {
        case PODCG_OK: return "success";
        case PODCG_NOT_CONVERGED: return "iteration cap reached before the tolerance";
        case PODCG_RANK_REDUCED: return "augmenting basis truncated at a small Cholesky pivot";
        case PODCG_ERR_INVALID_ARG: return "invalid argument";
        case PODCG_ERR_HIP: return "HIP runtime error";
        case PODCG_ERR_OOM: return "out of device memory";
        case PODCG_ERR_NOT_SPD: return "matrix is not symmetric positive definite";
        case PODCG_ERR_NONFINITE: return "non-finite value";
        case PODCG_ERR_NO_MATRIX: return "no matrix has been set";
        case PODCG_ERR_SIZE: return "size mismatch";
        default: return "unknown status";
    }
}

const char* podcg_last_error(podcg_ctx* ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }

int podcg_create(podcg_ctx** out, int64_t n, const podcg_options* opt, void* hip_stream) {
    if (!out) return PODCG_ERR_INVALID_ARG;
    *out = nullptr;
    if (n < 1 || n > (int64_t)0x7fffffff - 64) return PODCG_ERR_INVALID_ARG;
    podcg_options o;
    podcg_default_options(&o);
    if (opt) o = *opt;
    try {
        check_opts(o);
    } catch (const Fail& e) {
        return e.code;
    }
    podcg_ctx* ctx = new (std::nothrow) podcg_ctx();
    if (!ctx) return PODCG_ERR_OOM;
    ctx->n = n;
    ctx->opt = o;
    ctx->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&ctx->device) != hipSuccess) {
        delete ctx;
        return PODCG_ERR_HIP;
    }
    ctx->nslices = (int)((n + kSlice - 1) / kSlice);
    // leading dimension of the vectors and column blocks: the slices, plus one
    // padding slice for large systems with an even slice count, so that the
    // stride between columns of W, A W, S and Y is an odd multiple of 512
    // bytes -- at a multiple of 8 KB (n = 2^21, say) every column's rows map
    // to the same L1 set and the multi-column gathers stall on tag conflicts
    ctx->ld = (size_t)(ctx->nslices + (ctx->nslices >= 1024 && ctx->nslices % 2 == 0 ? 1 : 0)) * kSlice;
    int rc = guarded(ctx, [&]() {
        const int src = noalloc_init(ctx->device, &ctx->last_error);
        if (src != PODCG_OK) throw Fail{src};
        const size_t ld = ctx->ld;
        dalloc(ctx, &ctx->d_sptr, (size_t)ctx->nslices + 1);
        dalloc(ctx, &ctx->d_sflag, (size_t)ctx->nslices);
        dalloc(ctx, &ctx->d_soff, (size_t)ctx->nslices * kTabMax);
        dalloc(ctx, &ctx->d_smeta, (size_t)ctx->nslices * kMetaWords);
        dalloc(ctx, &ctx->d_dinv, ld);
        dalloc(ctx, &ctx->d_r, ld);
        dalloc(ctx, &ctx->d_z, ld);
        dalloc(ctx, &ctx->d_p, ld);
        dalloc(ctx, &ctx->d_q, ld);
        dalloc(ctx, &ctx->d_W, ld * (size_t)std::max(1, o.rank_max));
        dalloc(ctx, &ctx->d_AW, ld * (size_t)std::max(1, o.rank_max));
        dalloc(ctx, &ctx->d_AWt, ld * (size_t)std::max(1, o.rank_max));
        dalloc(ctx, &ctx->d_S, ld * (size_t)o.omega);
        if (o.precision == 1) {
            dalloc(ctx, &ctx->d_dinv32, ld);
            dalloc(ctx, &ctx->d_r32, ld);
            dalloc(ctx, &ctx->d_z32, ld);
            dalloc(ctx, &ctx->d_p32, ld);
            dalloc(ctx, &ctx->d_q32, ld);
            dalloc(ctx, &ctx->d_W32, ld * (size_t)std::max(1, o.rank_max));
            dalloc(ctx, &ctx->d_AW32, ld * (size_t)std::max(1, o.rank_max));
            HIPCHECK(hipMemsetAsync(ctx->d_p32, 0, ld * sizeof(float), ctx->stream));
            HIPCHECK(hipMemsetAsync(ctx->d_q32, 0, ld * sizeof(float), ctx->stream));
        }
        dalloc(ctx, &ctx->d_G, kYMax * kYMax);
        dalloc(ctx, &ctx->d_R, kYMax * kYMax);
        dalloc(ctx, &ctx->d_Ginv, kYMax * kYMax);
        dalloc(ctx, &ctx->d_lamG, kYMax);
        dalloc(ctx, &ctx->d_Gs, kYMax * kYMax);
        dalloc(ctx, &ctx->d_T, kYMax * kYMax);
        dalloc(ctx, &ctx->d_lamS, kYMax);
        dalloc(ctx, &ctx->d_yout, 4);
        dalloc(ctx, &ctx->d_st, 1);
        dalloc(ctx, &ctx->d_part, kPartials);
        dalloc(ctx, &ctx->d_counter, kCounters);
        dalloc(ctx, &ctx->d_gpart, kLoopGridMax);
        dalloc(ctx, &ctx->d_flag, 4);
        HIPCHECK(hipMemsetAsync(ctx->d_counter, 0, kCounters * sizeof(unsigned), ctx->stream));
        HIPCHECK(hipMemsetAsync(ctx->d_r, 0, ld * sizeof(double), ctx->stream));
        HIPCHECK(hipMemsetAsync(ctx->d_z, 0, ld * sizeof(double), ctx->stream));
        HIPCHECK(hipMemsetAsync(ctx->d_p, 0, ld * sizeof(double), ctx->stream));
        HIPCHECK(hipMemsetAsync(ctx->d_q, 0, ld * sizeof(double), ctx->stream));
        HIPCHECK(hipMemsetAsync(ctx->d_Ginv, 0, kYMax * kYMax * sizeof(double), ctx->stream));
        HIPCHECK(hipHostMalloc((void**)&ctx->h_poll, sizeof(PollBlock), hipHostMallocDefault));
        HIPCHECK(hipHostMalloc((void**)&ctx->h_int, 64 * sizeof(int), hipHostMallocDefault));
        HIPCHECK(hipHostMalloc((void**)&ctx->h_dbl, 64 * sizeof(double), hipHostMallocDefault));
        HIPCHECK(hipHostMalloc((void**)&ctx->h_rank, sizeof(int), hipHostMallocDefault));
        HIPCHECK(hipEventCreateWithFlags(&ctx->ev_pod, hipEventDisableTiming));
        HIPCHECK(hipEventCreate(&ctx->ev_a));
        HIPCHECK(hipEventCreate(&ctx->ev_b));
        HIPCHECK(hipEventCreate(&ctx->ev_c));
        HIPCHECK(hipEventCreate(&ctx->ev_d));
        sync(ctx);
        return PODCG_OK;
    });
    if (rc != PODCG_OK) {
        release(ctx);
        delete ctx;
        return rc;
    }
    *out = ctx;
    return PODCG_OK;
}

int podcg_destroy(podcg_ctx* ctx) {
    if (!ctx) return PODCG_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    release(ctx);
    delete ctx;
    return PODCG_OK;
}

int podcg_set_matrix(podcg_ctx* ctx, int64_t nnz, const int32_t* rowptr, const int32_t* colind,
                     const double* vals) {
    return guarded(ctx, [&]() {
        if (!vals || nnz < 1 || nnz > (int64_t)0x7fffffff) fail(ctx, PODCG_ERR_INVALID_ARG, "bad nnz or vals");
        if ((rowptr == nullptr) != (colind == nullptr))
            fail(ctx, PODCG_ERR_INVALID_ARG, "rowptr and colind must both be given or both be NULL");
        hipStream_t s = ctx->stream;
        const int n = (int)ctx->n;
        if (rowptr) {
            HIPCHECK(hipMemsetAsync(ctx->d_flag, 0, sizeof(int), s));
            HIPCHECK(launch_validate_csr(n, nnz, rowptr, colind, ctx->d_flag, s));
            HIPCHECK(hipMemcpyAsync(ctx->h_int, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
            sync(ctx);
            if (ctx->h_int[0]) {
                ctx->has_pattern = ctx->has_values = false;
                fail(ctx, PODCG_ERR_INVALID_ARG,
                     (ctx->h_int[0] & 1) ? "rowptr is not a valid CSR offset array"
                                         : "column index out of range");
            }
            HIPCHECK(launch_slice_widths(n, ctx->nslices, rowptr, ctx->d_sptr, s));
            HIPCHECK(launch_scan_slices(ctx->nslices, ctx->d_sptr, s));
            // the total slot count; for systems the one-workgroup solve may take,
            // every slice offset (their widest slice decides)
            const bool small = n <= kLdsThreads;
            const int nsp = small ? ctx->nslices + 1 : 1;
            HIPCHECK(hipMemcpyAsync(ctx->h_dbl, ctx->d_sptr + (small ? 0 : ctx->nslices),
                                    nsp * sizeof(int64_t), hipMemcpyDeviceToHost, s));
            sync(ctx);
            int64_t nsell = 0;
            std::memcpy(&nsell, ctx->h_dbl + (nsp - 1), sizeof(int64_t));
            ctx->max_width = -1;
            if (small) {
                int64_t sp[kLdsThreads / kSlice + 1];
                std::memcpy(sp, ctx->h_dbl, nsp * sizeof(int64_t));
                int wmax = 0;
                for (int i = 0; i < ctx->nslices; ++i) wmax = std::max<int>(wmax, (int)((sp[i + 1] - sp[i]) / kSlice));
                ctx->max_width = wmax;
            }
            if (nsell > ctx->sell_cap) {
                ctx->has_pattern = ctx->has_values = false;
                dalloc(ctx, &ctx->d_cols, (size_t)nsell);
                dalloc(ctx, &ctx->d_cols16, (size_t)nsell);
                dalloc(ctx, &ctx->d_map, (size_t)nsell);
                dalloc(ctx, &ctx->d_vals, (size_t)nsell);
                if (ctx->opt.precision == 1) dalloc(ctx, &ctx->d_vals32, (size_t)nsell);
                ctx->sell_cap = nsell;
            }
            ctx->nsell = nsell;
            HIPCHECK(launch_fill_pattern(n, ctx->nslices, rowptr, colind, ctx->d_sptr, ctx->d_cols,
                                         ctx->d_map, s));
            HIPCHECK(launch_fill_table(n, ctx->nslices, rowptr, ctx->d_sptr, ctx->d_cols, ctx->d_map,
                                       ctx->d_soff, ctx->d_sflag, s));
            HIPCHECK(launch_fill_offsets16(n, ctx->nslices, ctx->d_sptr, ctx->d_cols, ctx->d_cols16,
                                           ctx->d_sflag, s));
            HIPCHECK(launch_fill_meta(ctx->nslices, ctx->d_sptr, ctx->d_sflag, ctx->d_soff, ctx->d_smeta, s));
            // the loop SpMV takes two rows a lane where the slices have tables
            {
                std::vector<uint8_t> f((size_t)ctx->nslices);
                HIPCHECK(hipMemcpyAsync(f.data(), ctx->d_sflag, f.size(), hipMemcpyDeviceToHost, s));
                sync(ctx);
                int64_t tabled = 0;
                for (uint8_t v : f) tabled += v == 2;
                ctx->spmv_pairs = tabled * 10 >= (int64_t)ctx->nslices * 9;
            }
            ctx->has_pattern = true;
            ctx->nnz = nnz;
        } else {
            if (!ctx->has_pattern) fail(ctx, PODCG_ERR_NO_MATRIX, "values-only update before any pattern");
            if (nnz != ctx->nnz) fail(ctx, PODCG_ERR_SIZE, "nnz differs from the cached pattern");
        }
        HIPCHECK(hipMemsetAsync(ctx->d_flag, 0, sizeof(int), s));
        HIPCHECK(launch_fill_values(n, ctx->nslices, ctx->d_sptr, ctx->d_cols, ctx->d_map, ctx->d_sflag,
                                    ctx->d_soff, vals, ctx->d_vals, ctx->d_dinv, ctx->d_flag, s));
        HIPCHECK(hipMemcpyAsync(ctx->h_int, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
        sync(ctx);
        ctx->setup_valid = false;
        if (ctx->h_int[0] & 8) {
            ctx->has_values = false;
            fail(ctx, PODCG_ERR_NONFINITE, "non-finite matrix value");
        }
        if (ctx->h_int[0] & 4) {
            ctx->has_values = false;
            fail(ctx, PODCG_ERR_NOT_SPD, "missing or non-positive diagonal entry");
        }
        if (ctx->opt.precision == 1) {
            HIPCHECK(launch_to_float(ctx->d_vals, ctx->d_vals32, (size_t)ctx->nsell, s));
            HIPCHECK(launch_to_float(ctx->d_dinv, ctx->d_dinv32, ctx->ld, s));
        }
        ctx->has_values = true;
        return PODCG_OK;
    });
}

int podcg_push_snapshot(podcg_ctx* ctx, const double* x) {
    return guarded(ctx, [&]() {
        if (!x) fail(ctx, PODCG_ERR_INVALID_ARG, "null snapshot");
        HIPCHECK(launch_copy(x, ctx->d_S + (size_t)ctx->head * ctx->ld, (size_t)ctx->n, ctx->stream));
        ctx->head = (ctx->head + 1) % ctx->opt.omega;
        ctx->count = std::min(ctx->count + 1, ctx->opt.omega);
        return PODCG_OK;
    });
}

int podcg_reset_snapshots(podcg_ctx* ctx) {
    return guarded(ctx, [&]() {
        ctx->head = 0;
        ctx->count = 0;
        return PODCG_OK;
    });
}

int podcg_build_pod(podcg_ctx* ctx, int32_t* rank_out) {
    return guarded(ctx, [&]() {
        if (!ctx->has_values) fail(ctx, PODCG_ERR_NO_MATRIX, "no matrix set");
        pod_resolve(ctx);
        const int count = ctx->count;
        if (count == 0 || ctx->opt.rank_max == 0) {
            ctx->y = 0;
            ctx->pod_count = 0;
            ctx->setup_valid = false;
            if (rank_out) *rank_out = 0;
            return PODCG_OK;
        }
        hipStream_t s = ctx->stream;
        DevBufs B = bufs(ctx);
        // the used snapshots are ring slots 0..count-1; weight by age
        double w[kYMax];
        pod_slot_weights(ctx, w);
        HIPCHECK(launch_spmm_gram(B, count, ctx->d_S, nullptr, false, ctx->d_Gs, s));
        HIPCHECK(launch_pod_coeffs(ctx->d_Gs, count, w, ctx->opt.rank_max, ctx->opt.rank_rtol,
                                   ctx->opt.energy, ctx->d_T, ctx->d_lamS, ctx->d_yout, s));
        // W = S T with the rank the eigen-solve chose, read on the device
        HIPCHECK(launch_pod_form((int)ctx->n, ctx->ld, ctx->d_S, count, ctx->d_T, std::min(count, ctx->opt.rank_max),
                                 ctx->d_yout, ctx->d_W, s));
        HIPCHECK(hipMemcpyAsync(ctx->h_rank, ctx->d_yout, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHECK(hipEventRecord(ctx->ev_pod, s));
        ctx->y_pending = true;
        ctx->pod_count = count;
        ctx->setup_valid = false;
        if (rank_out) {
            pod_resolve(ctx);
            *rank_out = ctx->y;
        }
        return PODCG_OK;
    });
}

int podcg_set_basis(podcg_ctx* ctx, const double* W, int32_t y) {
    return guarded(ctx, [&]() {
        pod_resolve(ctx);
        if (y < 0 || y > ctx->opt.rank_max || (y > 0 && !W))
            fail(ctx, PODCG_ERR_INVALID_ARG, "basis dimension out of range");
        for (int k = 0; k < y; ++k)
            HIPCHECK(launch_copy(W + (size_t)k * ctx->n, ctx->d_W + (size_t)k * ctx->ld, (size_t)ctx->n,
                                 ctx->stream));
        ctx->y = y;
        ctx->setup_valid = false;
        return PODCG_OK;
    });
}

int podcg_get_basis(podcg_ctx* ctx, double* W, int32_t* rank) {
    return guarded(ctx, [&]() {
        pod_resolve(ctx);
        if (rank) *rank = ctx->y;
        if (ctx->y > 0 && !W) fail(ctx, PODCG_ERR_INVALID_ARG, "null output");
        for (int k = 0; k < ctx->y; ++k)
            HIPCHECK(launch_copy(ctx->d_W + (size_t)k * ctx->ld, W + (size_t)k * ctx->n, (size_t)ctx->n,
                                 ctx->stream));
        sync(ctx);
        return PODCG_OK;
    });
}

int podcg_get_reduced(podcg_ctx* ctx, double* G, double* Ginv, int32_t* rank) {
    return guarded(ctx, [&]() {
        pod_resolve(ctx);
        if (!ctx->has_values) fail(ctx, PODCG_ERR_NO_MATRIX, "no matrix set");
        if (!ctx->setup_valid) setup_basis(ctx);
        const int y = ctx->y_kept;
        if (rank) *rank = y;
        // copies ordered on the context stream, then that stream alone is awaited
        std::vector<double> g((size_t)kYMax * kYMax);
        if (G && ctx->y > 0)
            HIPCHECK(hipMemcpyAsync(g.data(), ctx->d_G, sizeof(double) * ctx->y * ctx->y, hipMemcpyDeviceToHost,
                                    ctx->stream));
        if (Ginv && y > 0)
            HIPCHECK(hipMemcpyAsync(Ginv, ctx->d_Ginv, sizeof(double) * y * y, hipMemcpyDeviceToHost, ctx->stream));
        sync(ctx);
        if (G && ctx->y > 0)
            for (int i = 0; i < y; ++i)
                for (int j = 0; j < y; ++j) G[i * y + j] = g[(size_t)i * ctx->y + j];
        return PODCG_OK;
    });
}

int podcg_get_pod_spectrum(podcg_ctx* ctx, double* lam, int32_t* count) {
    return guarded(ctx, [&]() {
        pod_resolve(ctx);
        if (count) *count = ctx->pod_count;
        if (lam && ctx->pod_count > 0) {
            HIPCHECK(hipMemcpyAsync(lam, ctx->d_lamS, sizeof(double) * ctx->pod_count, hipMemcpyDeviceToHost,
                                    ctx->stream));
            sync(ctx);
        }
        return PODCG_OK;
    });
}

int podcg_get_format(podcg_ctx* ctx, int64_t* counts) {
    return guarded(ctx, [&]() {
        if (!counts) fail(ctx, PODCG_ERR_INVALID_ARG, "counts is NULL");
        if (!ctx->has_pattern) fail(ctx, PODCG_ERR_NO_MATRIX, "no matrix pattern set");
        std::vector<uint8_t> f((size_t)ctx->nslices);
        std::vector<int64_t> sp((size_t)ctx->nslices + 1);
        HIPCHECK(hipMemcpyAsync(f.data(), ctx->d_sflag, f.size(), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHECK(hipMemcpyAsync(sp.data(), ctx->d_sptr, sp.size() * sizeof(int64_t), hipMemcpyDeviceToHost,
                                ctx->stream));
        sync(ctx);
        for (int k = 0; k < 5; ++k) counts[k] = 0;
        for (size_t s = 0; s < f.size(); ++s) {
            const int kind = f[s] <= 2 ? f[s] : 0;
            const int64_t slots = sp[s + 1] - sp[s];
            counts[kind] += 1;
            counts[3] += slots;
            counts[4] += kind == 2 ? 4 * kTabMax : (kind == 1 ? 2 : 4) * slots;
        }
        return PODCG_OK;
    });
}

int podcg_solve(podcg_ctx* ctx, const double* b, double* x, double rtol, podcg_stats* st) {
    return guarded(ctx, [&]() { return solve_impl(ctx, b, x, rtol, st, false); });
}

int podcg_solve_plain(podcg_ctx* ctx, const double* b, double* x, double rtol, podcg_stats* st) {
    return guarded(ctx, [&]() { return solve_impl(ctx, b, x, rtol, st, true); });
}

int podcg_matvec(podcg_ctx* ctx, const double* x, double* y) {
    return guarded(ctx, [&]() {
        if (!ctx->has_values) fail(ctx, PODCG_ERR_NO_MATRIX, "no matrix set");
        if (!x || !y || x == y) fail(ctx, PODCG_ERR_INVALID_ARG, "bad vectors");
        HIPCHECK(launch_matvec(bufs(ctx), x, y, ctx->stream));
        return PODCG_OK;
    });
}

int podcg_pattern_outer(podcg_ctx* ctx, const double* u, const double* v, double scale,
                        double* out_vals) {
    return guarded(ctx, [&]() {
        if (!ctx->has_pattern) fail(ctx, PODCG_ERR_NO_MATRIX, "no matrix pattern set");
        if (!u || !v || !out_vals) fail(ctx, PODCG_ERR_INVALID_ARG, "bad vectors");
        HIPCHECK(launch_pattern_outer((int)ctx->n, ctx->nslices, ctx->d_sptr, ctx->d_cols, ctx->d_map, u,
                                      v, scale, out_vals, ctx->stream));
        return PODCG_OK;
    });
}

int podcg_stream_triad(podcg_ctx* ctx, const double* a, const double* b, double* c, int64_t n,
                       double s, int32_t reps, double* ms) {
    return guarded(ctx, [&]() {
        if (!a || !b || !c || n < 1 || reps < 1) fail(ctx, PODCG_ERR_INVALID_ARG, "bad triad arguments");
        if (((uintptr_t)a | (uintptr_t)b | (uintptr_t)c) & 15)
            fail(ctx, PODCG_ERR_INVALID_ARG, "triad arrays must be 16-byte aligned");
        HIPCHECK(launch_triad(a, b, c, (size_t)n, s, ctx->stream));   // warm-up
        HIPCHECK(hipEventRecord(ctx->ev_a, ctx->stream));
        for (int r = 0; r < reps; ++r) HIPCHECK(launch_triad(a, b, c, (size_t)n, s, ctx->stream));
        HIPCHECK(hipEventRecord(ctx->ev_b, ctx->stream));
        sync(ctx);
        float t = 0.f;
        HIPCHECK(hipEventElapsedTime(&t, ctx->ev_a, ctx->ev_b));
        if (ms) *ms = t / reps;
        return PODCG_OK;
    });
}

}  // extern "C"
