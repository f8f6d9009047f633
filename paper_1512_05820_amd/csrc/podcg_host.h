// Internal host-side declarations of libpodcg shared by the ABI translation
// units: the context structure and the error-handling helpers.  Not a public
// header.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "podcg.h"
#include "podcg_launch.h"

namespace podcg_host {

struct Fail {
    int code;
};

}  // namespace podcg_host

namespace podcg_host {
struct TsHost;   // three-stage state (podcg_three.hip)
}

struct podcg_ctx {
    int64_t n = 0;
    int nslices = 0;
    size_t ld = 0;
    podcg_options opt{};
    hipStream_t stream = nullptr;
    int device = 0;

    // matrix
    bool has_pattern = false, has_values = false;
    bool spmv_pairs = false;   // at least 90% of the slices are offset-table slices
    int64_t nnz = 0, nsell = 0, sell_cap = 0;
    int max_width = -1;                     // widest slice when n <= kLdsThreads (else -1)
    int64_t* d_sptr = nullptr;
    int* d_cols = nullptr;
    int16_t* d_cols16 = nullptr;
    uint8_t* d_sflag = nullptr;
    int* d_soff = nullptr;                  // per-slice offset tables, kTabMax each
    int* d_smeta = nullptr;                 // per-slice metadata records of the loop SpMV
    int* d_map = nullptr;
    double* d_vals = nullptr;
    double* d_dinv = nullptr;

    // CG vectors (length ld)
    double *d_r = nullptr, *d_z = nullptr, *d_p = nullptr, *d_q = nullptr;
    // mixed precision: FP32 copies of the matrix, Jacobi inverse, basis and
    // the inner-solve vectors (the solution itself stays FP64)
    float *d_vals32 = nullptr, *d_dinv32 = nullptr, *d_W32 = nullptr, *d_AW32 = nullptr;
    float *d_r32 = nullptr, *d_z32 = nullptr, *d_p32 = nullptr, *d_q32 = nullptr;

    // basis
    double *d_W = nullptr, *d_AW = nullptr;
    double* d_AWt = nullptr;                // A W in 64-row tiles (read by the implicit update)
    int y = 0;                 // columns of W
    int y_kept = 0;            // columns accepted by the last factorisation
    bool setup_valid = false;
    bool rank_reduced = false;
    double cond_G = 1.0;
    double *d_G = nullptr, *d_R = nullptr, *d_Ginv = nullptr, *d_lamG = nullptr;

    // snapshots
    double *d_S = nullptr, *d_Gs = nullptr, *d_T = nullptr, *d_lamS = nullptr;
    int head = 0, count = 0, pod_count = 0;
    int* d_yout = nullptr;
    // a POD built without waiting: its rank arrives in h_rank (pinned) when
    // ev_pod completes; calls that need the rank on the host wait for it first.
    // A batched build points rank_ext / ev_ext at the batch's copy instead.
    bool y_pending = false;
    int* h_rank = nullptr;
    hipEvent_t ev_pod = nullptr;
    const int* rank_ext = nullptr;
    hipEvent_t ev_ext = nullptr;

    // scalar state and scratch
    podcg::DevState* d_st = nullptr;
    double* d_part = nullptr;
    unsigned* d_counter = nullptr;
    double* d_gpart = nullptr;              // SpMV partials of (A p, p), one per workgroup
    int* d_flag = nullptr;
    podcg::PollBlock* h_poll = nullptr;     // pinned
    int* h_int = nullptr;            // pinned scratch ints
    double* h_dbl = nullptr;         // pinned scratch doubles

    hipEvent_t ev_a = nullptr, ev_b = nullptr, ev_c = nullptr, ev_d = nullptr;
    std::vector<hipEvent_t> tev;     // per-iteration kernel timing events
    int prev_iters[2] = {0, 0};      // iterations of the last augmented / plain solve

    podcg_host::TsHost* ts = nullptr;    // three-stage mode, when enabled

    std::string last_error;
};

#define HIPCHECK(expr)                                                                              \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) {                                                                     \
            ctx->last_error = std::string(#expr) + ": " + hipGetErrorString(e_);                    \
            throw podcg_host::Fail{e_ == hipErrorOutOfMemory ? PODCG_ERR_OOM : PODCG_ERR_HIP};      \
        }                                                                                           \
    } while (0)

namespace podcg_host {

template <class C>
[[noreturn]] void fail(C* ctx, int code, const std::string& msg) {
    ctx->last_error = msg;
    throw Fail{code};
}

template <class C, class T>
void dalloc(C* ctx, T** p, size_t count) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    if (count == 0) count = 1;
    HIPCHECK(hipMalloc((void**)p, count * sizeof(T)));
}

// Runs f() with the context's device current and converts failures to codes.
template <class C, class F>
int guarded(C* ctx, F&& f) {
    if (!ctx) return PODCG_ERR_INVALID_ARG;
    try {
        if (hipSetDevice(ctx->device) != hipSuccess) return PODCG_ERR_HIP;
        return f();
    } catch (const Fail& e) {
        if (ctx->last_error.empty()) ctx->last_error = podcg_strerror(e.code);
        return e.code;
    } catch (const std::bad_alloc&) {
        ctx->last_error = "host allocation failed";
        return PODCG_ERR_OOM;
    } catch (...) {
        ctx->last_error = "unexpected exception";
        return PODCG_ERR_HIP;
    }
}

podcg::DevBufs bufs(podcg_ctx* ctx);
void sync(podcg_ctx* ctx);
void poll(podcg_ctx* ctx);
// A W, G = W^T A W, its factor and inverse, the kept rank (synchronises).
void setup_basis(podcg_ctx* ctx);
// Takes the rank of a POD built without waiting (no-op when none is pending).
void pod_resolve(podcg_ctx* ctx);
// POD weight of each ring slot (inverse distance 2^{-age}, newest 1, or all
// ones), slots 0..count-1.
void pod_slot_weights(const podcg_ctx* ctx, double* w);
int fail_code(podcg_ctx* ctx, const podcg::PollBlock& P);
void record(podcg_ctx* ctx, hipEvent_t e);
// Launch loop iterations in batches until the device reports that the solve
// finished, or maxit iterations were launched.  `iter3(t, ev, k)` enqueues
// iteration k (SpMV, update, direction); when t, ev[2j], ev[2j + 1] are the
// start/stop events of kernel j, recorded by the dispatches themselves.  The first convergence check comes after most of the previous
// solve's iteration count (kernels after convergence are no-ops), then every
// check_every iterations.  Returns the iteration indices that were timed.
template <class F>
std::vector<int> run_loop(podcg_ctx* ctx, int slot, int* polls, F&& iter3) {
    const int timing = ctx->opt.timing;
    std::vector<int> timed;
    int launched = 0;
    ctx->h_poll->done = podcg::kRunning;   // the loop kernels are no-ops once Stage 1 has finished
    int first = (int)(0.85 * ctx->prev_iters[slot]);
    first = std::max(first, ctx->opt.check_every);
    while (ctx->h_poll->done == podcg::kRunning && launched < ctx->opt.maxit) {
        const int want = launched == 0 ? first : ctx->opt.check_every;
        const int batch = std::min(want, ctx->opt.maxit - launched);
        for (int k = 0; k < batch; ++k, ++launched) {
            const bool t = timing > 0 && (launched % timing) == 0;
            hipEvent_t* ev = nullptr;
            if (t) {
                const size_t base = timed.size() * 6;
                while (ctx->tev.size() < base + 6) {
                    hipEvent_t e;
                    HIPCHECK(hipEventCreate(&e));
                    ctx->tev.push_back(e);
                }
                timed.push_back(launched);
                ev = &ctx->tev[base];
            }
            iter3(t, ev, launched);
        }
        poll(ctx);
        ++*polls;
    }
    return timed;
}

void ts_release(podcg_ctx* ctx);
// Sets up this device's address of the scratch array of podcg_solve_noalloc
// (podcg_noalloc.hip); the device must be current.  Once per device.
int noalloc_init(int device, std::string* err);

}  // namespace podcg_host
