// One-workgroup solve of a small system: Stage 1 (Alg. 2) and augmented PCG
// (Alg. 1 with the Jacobi preconditioner and the explicit direction
// recurrence p = z + beta p - W mu) in a single launch of 1024 threads.
//
// For a few thousand unknowns the multi-kernel loop is bound by launch and
// synchronisation latency (three dependent launches per iteration, each
// finishing a grid reduction).  Here one workgroup of 16 wavefronts keeps the
// whole solve on one compute unit: each thread owns R rows (row 64 s + lane
// of slice s = wave + 16 r, the SELL layout's own mapping) and holds that
// row's matrix entries, x, r, z, p, the Jacobi inverse and the rows of W and
// A W in registers for the whole solve; only the search direction, which the
// product A p gathers across rows, is shared through LDS.  Reductions are
// wavefront butterflies followed by a fixed-order sum of the 16 wave
// partials, so results are bitwise repeatable.  Per iteration: one gathered
// product, two reductions and four workgroup barriers, and no memory round
// trip at all (the matrix rows stay in registers).
//
// The basis products (A W, W^T A W and its factor, Alg. 2) come from the
// setup kernels of the multi-kernel path, launched ahead of this kernel on the
// same stream; the kept rank is read from the device state, so the host does
// not wait for the factorisation.
#include "podcg_launch.h"

namespace podcg {

constexpr int kLdsWaves = kLdsThreads / kWave;   // 16

// Wave sums of NV values, stored by lane 0 of each wave at red[wave * NV + k].
template <int NV>
__device__ __forceinline__ void lds_wave_partials(double (&v)[NV], double* red) {
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) red[wid * NV + k] = v[k];
    }
}

// Lane t of the calling wave: the total of value t (t < NV), the 16 wave
// partials added in wave order.
template <int NV>
__device__ __forceinline__ double lds_total(const double* red) {
    const int t = threadIdx.x & (kWave - 1);
    double s = 0.0;
    if (t < NV) {
        s = red[t];
#pragma unroll
        for (int w = 1; w < kLdsWaves; ++w) s += red[w * NV + t];
    }
    return s;
}

// In wave 0: out[i] = sum_j Ginv[i y + j] tot_{2 + j} for i < y, where lane l
// holds tot_l.  Every lane takes part in the shuffles.
template <int YB>
__device__ __forceinline__ void lds_project(double tot, const double* sginv, int y, double* out) {
    const int t = threadIdx.x & (kWave - 1);
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < YB; ++j) {
        const double c = __shfl(tot, 2 + j, kWave);
        if (t < y && j < y) s += sginv[t * YB + j] * c;
    }
    if (t < y) out[t] = s;
}

// Shared scalars of the solve.
struct LdsShared {
    double tol2, rho, beta, rz, rr;
    int state;   // kRunning, kFinished or kFailed
    int status;
};

template <int YB>
__global__ __launch_bounds__(kLdsThreads) void k_lds_solve(DevBufs B, const double* __restrict__ b,
                                                           double* __restrict__ x,
                                                           const double* __restrict__ W,
                                                           const double* __restrict__ AW) {
    constexpr int NV = 2 + YB;
    __shared__ double sp[kLdsThreads];            // the vector the product gathers from
    __shared__ double red[kLdsWaves * NV];        // wave partials of the vector sums
    __shared__ double redg[kLdsWaves];            // wave partials of (A p, p) and of ||b - A x||^2
    __shared__ double sginv[YB > 0 ? YB * YB : 1];
    __shared__ double smu[YB > 0 ? YB : 1];       // what in Stage 1, then mu
    __shared__ LdsShared sh;
    DevState* st = B.st;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int n = B.n;
    const int y = YB > 0 ? min(st->y, YB) : 0;
    const int maxit = st->maxit;

    // ---- this thread's row (row 64 s + lane of slice s = wave): matrix
    // entries, vectors, basis rows
    const int row = wid * kSlice + lane;
    const bool in = row < n;
    int mw = 0;
    double av[kLdsWidth];
    int ac[kLdsWidth];
    if (wid < B.nslices) {
        // slice bounds, width and column storage are wave-uniform
        const int s = __builtin_amdgcn_readfirstlane(wid);
        const int64_t base = B.sptr[s];
        mw = (int)((B.sptr[s + 1] - base) / kSlice);
        const int flag = B.sflag[s];
        const int rb = in ? row : 0;
#pragma unroll
        for (int j = 0; j < kLdsWidth; ++j) {
            av[j] = 0.0;
            ac[j] = rb;
            if (j < mw) {
                const size_t e = (size_t)base + (size_t)j * kSlice + lane;
                int c;
                if (flag == 2) c = row + B.soff[(size_t)s * kTabMax + j];
                else if (flag == 1) c = rb + (int)B.cols16[e];
                else c = B.cols[e];
                ac[j] = c < 0 ? 0 : (c < n ? c : n - 1);
                av[j] = B.vals[e];
            }
        }
    }
    const double bi = in ? b[row] : 0.0;
    double xi = in ? x[row] : 0.0;
    const double di = in ? B.dinv[row] : 0.0;
    double ri, zi = 0.0, pi = 0.0;
    double wr[YB > 0 ? YB : 1], awr[YB > 0 ? YB : 1];
#pragma unroll
    for (int k = 0; k < YB; ++k) {
        wr[k] = in && k < y ? W[(size_t)k * B.ld + row] : 0.0;
        awr[k] = in && k < y ? AW[(size_t)k * B.ld + row] : 0.0;
    }
    if (YB > 0)
        for (int e = threadIdx.x; e < y * y; e += kLdsThreads) sginv[(e / y) * YB + e % y] = B.Ginv[e];
    // (A v)_row, v gathered from sp
    auto product = [&]() {
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < kLdsWidth; ++j)
            if (j < mw) acc = fma(av[j], sp[ac[j]], acc);
        return acc;
    };

    // ---- Stage 1 (Alg. 2): rbar = b - A xbar, (b, b), (rbar, rbar), W^T rbar
    sp[row] = xi;
    __syncthreads();
    {
        ri = in ? bi - product() : 0.0;
        double v[NV];
        v[0] = bi * bi;
        v[1] = ri * ri;
#pragma unroll
        for (int k = 0; k < YB; ++k) v[2 + k] = wr[k] * ri;
        lds_wave_partials<NV>(v, red);
        __syncthreads();
        if (wid == 0) {
            const double tot = lds_total<NV>(red);
            lds_project<YB>(tot, sginv, y, smu);   // what = G^{-1} W^T rbar
            const double bb = __shfl(tot, 0, kWave), rb2 = __shfl(tot, 1, kWave);
            if (lane == 0) {
                sh.tol2 = st->tol2 * bb;
                st->tol2 = sh.tol2;
                st->bnorm2 = bb;
                const bool ok = is_finite(bb) && is_finite(rb2);
                sh.state = ok ? kRunning : kFailed;
                sh.status = ok ? kStNotConverged : kStNonfinite;
                sh.rho = sh.beta = 0.0;
            }
        }
        __syncthreads();
    }
    const double tol2 = sh.tol2;
    int iters = 0;
    double rr_last = 0.0, alpha = 0.0, gamma = 0.0;
    if (sh.state == kRunning) {
        // x = xbar + W what, r = rbar - (A W) what, z = M^{-1} r,
        // sums (r, z), (r, r), c = (A W)^T z; mu = G^{-1} c
        {
            if (YB > 0) {
                double wx = 0.0, awx = 0.0;
#pragma unroll
                for (int k = 0; k < YB; ++k) {
                    const double wh = k < y ? smu[k] : 0.0;
                    wx += wr[k] * wh;
                    awx += awr[k] * wh;
                }
                xi += wx;
                ri -= awx;
            }
            zi = di * ri;
            double v[NV];
            v[0] = ri * zi;
            v[1] = ri * ri;
#pragma unroll
            for (int k = 0; k < YB; ++k) v[2 + k] = awr[k] * zi;
            lds_wave_partials<NV>(v, red);
        }
        __syncthreads();
        if (wid == 0) {
            const double tot = lds_total<NV>(red);
            lds_project<YB>(tot, sginv, y, smu);
            const double rz = __shfl(tot, 0, kWave), rr = __shfl(tot, 1, kWave);
            if (lane == 0) {
                sh.rho = rz;
                sh.rr = rr;
                st->rr0 = rr;
                if (!is_finite(rr) || !is_finite(rz)) {
                    sh.state = kFailed;
                    sh.status = kStNonfinite;
                } else if (rr <= tol2) {
                    sh.state = kFinished;
                    sh.status = kStOk;
                } else if (maxit <= 0) {
                    sh.state = kFinished;
                    sh.status = kStNotConverged;
                }
            }
        }
        __syncthreads();
        rr_last = sh.rr;
        double rho = sh.rho;
        // the first direction p = z - W mu
        {
            double s = zi;
#pragma unroll
            for (int k = 0; k < YB; ++k) s -= wr[k] * (k < y ? smu[k] : 0.0);
            pi = s;
        }
        // ---- the loop of Alg. 1
        while (sh.state == kRunning) {
            sp[row] = pi;
            __syncthreads();
            // q = A p, gamma = (A p, p)
            const double q = in ? product() : 0.0;
            double g[1] = {q * pi};
            lds_wave_partials<1>(g, redg);
            __syncthreads();
            gamma = redg[0];
#pragma unroll
            for (int w = 1; w < kLdsWaves; ++w) gamma += redg[w];
            if (!(gamma > 0.0 && is_finite(gamma))) {   // gamma is the same in every thread
                if (threadIdx.x == 0) {
                    sh.state = kFailed;
                    sh.status = is_finite(gamma) ? kStNotSpd : kStNonfinite;
                }
                break;
            }
            alpha = rho / gamma;
            // x += alpha p, r -= alpha q, z = M^{-1} r; (r, z), (r, r), (A W)^T z
            xi = xi + alpha * pi;
            ri = ri - alpha * q;
            zi = di * ri;
            {
                double v[NV];
                v[0] = ri * zi;
                v[1] = ri * ri;
#pragma unroll
                for (int k = 0; k < YB; ++k) v[2 + k] = awr[k] * zi;
                lds_wave_partials<NV>(v, red);
            }
            __syncthreads();
            ++iters;
            if (wid == 0) {
                const double tot = lds_total<NV>(red);
                lds_project<YB>(tot, sginv, y, smu);   // mu = G^{-1} (A W)^T z
                const double rz = __shfl(tot, 0, kWave), rr = __shfl(tot, 1, kWave);
                if (lane == 0) {
                    sh.rz = rz;
                    sh.rr = rr;
                    if (!is_finite(rr) || !is_finite(rz)) {
                        sh.state = kFailed;
                        sh.status = kStNonfinite;
                    } else if (rr <= tol2 || iters >= maxit) {
                        sh.state = kFinished;
                        sh.status = rr <= tol2 ? kStOk : kStNotConverged;
                    }
                }
            }
            __syncthreads();
            rr_last = sh.rr;
            if (sh.state != kRunning) break;
            // p = z + beta p - W mu, beta = (r', z') / (r, z)
            const double rz = sh.rz;
            const double beta = rz / rho;
            rho = rz;
            double s = zi + beta * pi;
#pragma unroll
            for (int k = 0; k < YB; ++k) s -= wr[k] * (k < y ? smu[k] : 0.0);
            pi = s;
            if (threadIdx.x == 0) sh.beta = beta;
        }
        if (threadIdx.x == 0) sh.rho = rho;
    }
    // ---- the true residual ||b - A x|| and the solution
    __syncthreads();
    sp[row] = xi;
    __syncthreads();
    double t[1] = {0.0};
    if (in) {
        const double rt = bi - product();
        t[0] = rt * rt;
        x[row] = xi;
    }
    lds_wave_partials<1>(t, redg);
    __syncthreads();
    if (threadIdx.x == 0) {
        double trr = redg[0];
        for (int w = 1; w < kLdsWaves; ++w) trr += redg[w];
        st->true_rr = trr;
        st->iter = iters;
        st->rr = rr_last;
        st->status = sh.status;
        st->done = sh.state == kFailed ? kFailed : kFinished;
        st->stop = iters;
        st->y = y;
        st->rho = sh.rho;
        st->alpha = alpha;
        st->beta = sh.beta;
        st->gamma = gamma;
    }
}

// Basis dimensions of the one-workgroup solve: up to kLdsYMax, where the
// registers of 16 wavefronts per compute unit (128 per lane) still hold the
// rows of W and A W without spilling.
int lds_tier(int n, int y) { return n >= 1 && n <= kLdsThreads && y >= 0 && y <= kLdsYMax ? y : -1; }

hipError_t launch_lds_solve(const DevBufs& B, int yb, const double* b, double* x, const double* W,
                            const double* AW, hipStream_t s) {
    if (lds_tier(B.n, yb) != yb || B.nslices > kLdsWaves) return hipErrorInvalidValue;
    const dim3 g(1), t(kLdsThreads);
    switch (yb) {
#define CASE(T) case T: hipLaunchKernelGGL((k_lds_solve<T>), g, t, 0, s, B, b, x, W, AW); break;
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace podcg
