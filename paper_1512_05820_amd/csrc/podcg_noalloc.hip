// podcg_solve_noalloc: the small-system solve of podcg_solve (Stage 1 and the
// augmented PCG loop in one workgroup, with the basis setup ahead of it) for
// callers that cannot allocate device memory.  Its kernels take their scratch
// -- the device state block, A W, the reduced matrix W^T A W with its factor,
// inverse and eigenvalues, and the setup kernel's partial sums and arrival
// counters -- from one file-scope device array instead of the context's
// buffers; the call itself allocates nothing.
//
// The array exists once per GPU (each device holds its own copy at its own
// address) and lives until the process ends.  Host code never uses the
// array's name as an address: at set-up (podcg_create, once per device, with
// that device current) hipGetSymbolAddress gives the device address, which is
// kept per device and passed to the kernels.  Every call on one GPU shares the
// array, so calls that overlap on one GPU race (from several host threads or
// on several streams); calls ordered on one stream, or separated by a
// synchronisation, are safe, and each call clears the counters it needs.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "podcg.h"
#include "podcg_launch.h"
#include "podcg_host.h"

using namespace podcg;
using namespace podcg_host;

namespace {

// Layout of the scratch array, in doubles; each part starts on a 256-byte
// boundary (a multiple of 32 doubles).
constexpr size_t round32(size_t v) { return (v + 31) / 32 * 32; }
constexpr size_t kStateDoubles = round32((sizeof(DevState) + sizeof(double) - 1) / sizeof(double));
constexpr size_t kAWDoubles = round32((size_t)kLdsThreads * kLdsYMax);    // A W, ld <= kLdsThreads
constexpr size_t kSmallDoubles = round32((size_t)kLdsYMax * kLdsYMax);   // G, R, Ginv (row-major y x y)
constexpr size_t kLamDoubles = 32;                                       // eigenvalues of G
// partial sums of the fused SpMM + Gram kernel: y^2 per workgroup and per
// group of workgroups; at most (kLdsThreads / kSlice + 3) / 4 = 4 workgroups
constexpr int kGramBlocks = (kLdsThreads / kSlice + kWavesPerBlock - 1) / kWavesPerBlock;
constexpr size_t kPartDoubles = round32((size_t)kLdsYMax * kLdsYMax * (kGramBlocks + 1));
constexpr size_t kCounterWords = 64;                                     // arrival counters (uint32)

constexpr size_t kOffState = 0;
constexpr size_t kOffAW = kOffState + kStateDoubles;
constexpr size_t kOffG = kOffAW + kAWDoubles;
constexpr size_t kOffR = kOffG + kSmallDoubles;
constexpr size_t kOffGinv = kOffR + kSmallDoubles;
constexpr size_t kOffLam = kOffGinv + kSmallDoubles;
constexpr size_t kOffPart = kOffLam + kLamDoubles;
constexpr size_t kOffCounter = kOffPart + kPartDoubles;
constexpr size_t kScratchDoubles = kOffCounter + kCounterWords / 2;
static_assert(kScratchDoubles * sizeof(double) <= 64 * 1024, "scratch is meant to stay small");

}  // namespace

// The scratch of podcg_solve_noalloc (one copy per GPU).  Host code reaches it
// only through the address hipGetSymbolAddress returns.
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

__global__ void k_zero_words(unsigned* p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0u;
}

}  // namespace

namespace podcg_host {

// The device address of this device's scratch array (the device must be
// current).  Called by podcg_create, so that the entry point finds it set.
int noalloc_init(int device, std::string* err) {
    if (device < 0 || device >= kMaxDevices) {
        if (err) *err = "device index beyond the scratch table";
        return PODCG_ERR_HIP;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[device]) return PODCG_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        if (err) *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        return PODCG_ERR_HIP;
    }
    g_scratch[device] = static_cast<double*>(p);
    return PODCG_OK;
}

}  // namespace podcg_host

extern "C" int podcg_solve_noalloc(podcg_ctx* ctx, const double* b, double* x, double rtol, podcg_stats* st) {
    return guarded(ctx, [&]() {
        if (!ctx->has_values) fail(ctx, PODCG_ERR_NO_MATRIX, "no matrix set");
        if (!b || !x || !(rtol >= 0.0)) fail(ctx, PODCG_ERR_INVALID_ARG, "bad solve arguments");
        pod_resolve(ctx);
        const int y = ctx->y;
        if (ctx->opt.precision != 0 || ctx->max_width < 0 || ctx->max_width > kLdsWidth ||
            lds_tier((int)ctx->n, y) < 0)
            fail(ctx, PODCG_ERR_SIZE,
                 "podcg_solve_noalloc takes FP64 systems of at most " + std::to_string(kLdsThreads) +
                     " unknowns with slices at most " + std::to_string(kLdsWidth) +
                     " entries wide and a basis of at most " + std::to_string(kLdsYMax) + " columns");
        double* base = nullptr;
        {
            std::lock_guard<std::mutex> lock(g_scratch_mu);
            base = g_scratch[ctx->device];
        }
        if (!base) fail(ctx, PODCG_ERR_HIP, "scratch address not set up for this device");
        DevState* dst = reinterpret_cast<DevState*>(base + kOffState);
        double* AW = base + kOffAW;
        double* G = base + kOffG;
        double* R = base + kOffR;
        double* Ginv = base + kOffGinv;
        double* lam = base + kOffLam;
        unsigned* counter = reinterpret_cast<unsigned*>(base + kOffCounter);
        // the context's matrix and basis, the scratch for everything else
        DevBufs B = bufs(ctx);
        B.st = dst;
        B.part = base + kOffPart;
        B.counter = counter;
        B.Ginv = Ginv;
        const int groups = (ctx->nslices + kWavesPerBlock - 1) / kWavesPerBlock;
        if (groups > kGramBlocks || (size_t)y * y * (groups + 1) > kPartDoubles || (size_t)ctx->ld > (size_t)kLdsThreads)
            fail(ctx, PODCG_ERR_SIZE, "system exceeds the scratch array");
        hipStream_t s = ctx->stream;
        HIPCHECK(hipEventRecord(ctx->ev_a, s));
        hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(kCounterWords), 0, s, counter, (int)kCounterWords);
        HIPCHECK(hipGetLastError());
        HIPCHECK(launch_state_init(dst, ctx->opt.maxit, rtol * rtol, y, s));
        if (y > 0) {
            HIPCHECK(launch_spmm_gram(B, y, ctx->d_W, AW, true, G, s));
            HIPCHECK(launch_reduced_factor(G, y, R, Ginv, lam, dst, s));
        }
        HIPCHECK(hipEventRecord(ctx->ev_b, s));
        HIPCHECK(launch_lds_solve(B, y, b, x, ctx->d_W, AW, s));
        HIPCHECK(hipEventRecord(ctx->ev_c, s));
        HIPCHECK(hipMemcpyAsync(ctx->h_poll, dst, sizeof(PollBlock), hipMemcpyDeviceToHost, s));
        if (y > 0) HIPCHECK(hipMemcpyAsync(ctx->h_dbl, lam, sizeof(double) * y, hipMemcpyDeviceToHost, s));
        sync(ctx);
        const PollBlock P = *ctx->h_poll;
        podcg_stats S{};
        const int kept = P.y;
        const double bn = std::sqrt(P.bnorm2);
        S.iters = P.iter;
        S.rank = kept;
        S.bnorm = bn;
        S.stage1_relres = bn > 0 ? std::sqrt(P.rr0) / bn : std::sqrt(P.rr0);
        S.relres = bn > 0 ? std::sqrt(P.rr) / bn : std::sqrt(P.rr);
        S.true_relres = bn > 0 ? std::sqrt(P.true_rr) / bn : std::sqrt(P.true_rr);
        if (kept > 0) {
            const double lmax = ctx->h_dbl[0], lmin = ctx->h_dbl[kept - 1];
            S.cond_G = lmin > 0.0 ? lmax / lmin : INFINITY;
        } else {
            S.cond_G = 1.0;
        }
        S.matvecs = P.iter + 2 + y;
        S.polls = 1;
        S.path = 1;
        float ms = 0.f;
        HIPCHECK(hipEventElapsedTime(&ms, ctx->ev_a, ctx->ev_b));
        S.setup_ms = y > 0 ? ms : 0.0;
        HIPCHECK(hipEventElapsedTime(&ms, ctx->ev_b, ctx->ev_c));
        S.solve_ms = ms;
        int code = P.done == kFailed ? fail_code(ctx, P) : P.status;
        if (code == PODCG_OK && kept < y) code = PODCG_RANK_REDUCED;
        S.status = code;
        if (st) *st = S;
        return code;
    });
}
