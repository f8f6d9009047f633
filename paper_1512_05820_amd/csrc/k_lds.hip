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
// product, two reductions and three workgroup barriers, and no memory round
// trip at all (the matrix rows stay in registers).  Wave sums use DPP row
// operations (VALU lane moves) rather than LDS permutes, and every wavefront
// finishes each reduction itself from the 16 wave partials (same values in
// the same order, so every wave reaches the same decisions) instead of waiting
// behind a barrier for one wave to do it.
//
// The basis products (A W, W^T A W and its factor, Alg. 2) come from the
// setup kernels of the multi-kernel path, launched ahead of this kernel on the
// same stream; the kept rank is read from the device state, so the host does
// not wait for the factorisation.
#include "podcg_launch.h"

namespace podcg {

constexpr int kLdsWaves = kLdsThreads / kWave;   // 16

// One DPP lane move of a double (two 32-bit moves); lanes the row and bank
// masks leave out, or whose source lane does not exist, receive 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave in a fixed order; the total lands in lane
// 63.  Within each row of 16 lanes: swap neighbours, swap pairs, rotate by 4
// and by 8 (every lane then holds its row's sum); then lane 15 of rows 0 and 2
// is added into rows 1 and 3, and lane 31 into rows 2 and 3.
__device__ __forceinline__ double wave_sum_to_last(double v) {
    v += dpp_move<0xb1, 0xf>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_move<0x4e, 0xf>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_move<0x124, 0xf>(v);   // row_ror 4
    v += dpp_move<0x128, 0xf>(v);   // row_ror 8
    v += dpp_move<0x142, 0xa>(v);   // row_bcast 15 into rows 1 and 3
    v += dpp_move<0x143, 0xc>(v);   // row_bcast 31 into rows 2 and 3
    return v;
}

// Lane `l` (wave-uniform) of v, as a scalar.
__device__ __forceinline__ double lane_value(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// Wave sums of NV values, stored by lane 63 of each wave at red[wave * NV + k].
template <int NV>
__device__ __forceinline__ void lds_wave_partials(double (&v)[NV], double* red) {
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum_to_last(v[k]);
    if (lane == kWave - 1) {
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
    double rr_last = 0.0, alpha = 0.0, gamma = 0.0, rho_last = 0.0, beta_last = 0.0;
    int state = sh.state, status = sh.status;
    if (state == kRunning) {
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
        state = sh.state;
        status = sh.status;
        // ---- the loop of Alg. 1; every thread keeps the same state, so no
        // barrier is needed to share the decisions
        while (state == kRunning) {
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
            if (!(gamma > 0.0 && is_finite(gamma))) {
                state = kFailed;
                status = is_finite(gamma) ? kStNotSpd : kStNonfinite;
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
            // every wave sums the 16 wave partials itself: lane t < NV holds
            // total t, read back as scalars
            double tot = 0.0;
            if (lane < NV) {
                tot = red[lane];
#pragma unroll
                for (int w = 1; w < kLdsWaves; ++w) tot += red[w * NV + lane];
            }
            const double rz = lane_value(tot, 0), rr = lane_value(tot, 1);
            rr_last = rr;
            if (!is_finite(rr) || !is_finite(rz)) {
                state = kFailed;
                status = kStNonfinite;
                break;
            }
            if (rr <= tol2 || iters >= maxit) {
                state = kFinished;
                status = rr <= tol2 ? kStOk : kStNotConverged;
                break;
            }
            // mu = G^{-1} (A W)^T z: lane k < y forms mu_k
            double muk = 0.0;
            {
                const int kl = lane < YB ? lane : 0;
#pragma unroll
                for (int j = 0; j < YB; ++j) {
                    const double cj = lane_value(tot, 2 + j);
                    if (lane < y && j < y) muk += sginv[kl * YB + j] * cj;
                }
            }
            // p = z + beta p - W mu, beta = (r', z') / (r, z)
            const double beta = rz / rho;
            rho = rz;
            beta_last = beta;
            double s = zi + beta * pi;
#pragma unroll
            for (int k = 0; k < YB; ++k) s -= wr[k] * (k < y ? lane_value(muk, k) : 0.0);
            pi = s;
        }
        rho_last = rho;
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
        st->status = status;
        st->done = state == kFailed ? kFailed : kFinished;
        st->stop = iters;
        st->y = y;
        st->rho = rho_last;
        st->alpha = alpha;
        st->beta = beta_last;
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
