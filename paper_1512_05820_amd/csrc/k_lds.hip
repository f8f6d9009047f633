// One-workgroup solve of a small system: Stage 1 (Alg. 2) and augmented PCG
// (Alg. 1 with the Jacobi preconditioner and the explicit direction
// recurrence p = z + beta p - W mu) in a single launch of 512 threads.
//
// For a few thousand unknowns the multi-kernel loop is bound by launch and
// synchronisation latency (three dependent launches per iteration, each
// finishing a grid reduction).  Here one workgroup of 8 wavefronts keeps the
// whole solve on one compute unit: each thread owns two rows (row 64 s + lane
// of slices s = wave and wave + 8, the SELL layout's own mapping) and holds
// their matrix entries, x, r, z, p, the Jacobi inverse and the rows of W and
// A W in registers for the whole solve; only the search direction, which the
// product A p gathers across rows, is shared through LDS.  Per iteration: one
// gathered product, two reductions and three workgroup barriers, and no
// memory round trip at all (the matrix rows stay in registers).  A reduction
// adds the thread's two rows, sums each wave with DPP row operations (VALU
// lane moves rather than LDS permutes), and then every wavefront sums the 8
// wave partials itself (same values in the same order, so every wave reaches
// the same decisions) instead of waiting behind a barrier for one wave to do
// it; results are bitwise repeatable.  Two rows a thread halve the reduction
// work each SIMD issues per iteration (two wavefronts a SIMD instead of four).
//
// The basis products (A W, W^T A W and its factor, Alg. 2) come from the
// setup kernels of the multi-kernel path, launched ahead of this kernel on the
// same stream; the kept rank is read from the device state, so the host does
// not wait for the factorisation.
#include "podcg_launch.h"

namespace podcg {

constexpr int kLdsRows = 2;                       // rows per thread
constexpr int kLdsBlock = kLdsThreads / kLdsRows; // 512 threads
constexpr int kLdsWaves = kLdsBlock / kWave;      // 8

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

// Lane t of the calling wave: the total of value t (t < NV), the wave
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
__global__ __launch_bounds__(kLdsBlock) void k_lds_solve(DevBufs B, const double* __restrict__ b,
                                                         double* __restrict__ x,
                                                         const double* __restrict__ W,
                                                         const double* __restrict__ AW) {
    constexpr int NV = 2 + YB;
    constexpr int R = kLdsRows;
    __shared__ double sp[kLdsThreads];            // the vector the product gathers from
    __shared__ double red[kLdsWaves * NV];        // wave partials of the vector sums
    __shared__ double redg[kLdsWaves];            // wave partials of (A p, p) and of ||b - A x||^2
    __shared__ double sginv[YB > 0 ? YB * YB : 1];
    __shared__ double smu[YB > 0 ? YB : 1];       // what in Stage 1
    __shared__ LdsShared sh;
    DevState* st = B.st;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int n = B.n;
    const int y = YB > 0 ? min(st->y, YB) : 0;
    const int maxit = st->maxit;

    // ---- this thread's rows (row 64 s + lane of slices s = wave + 8 q):
    // matrix entries, vectors, basis rows
    int row[R], mw[R];
    bool in[R];
    double av[R][kLdsWidth];
    int ac[R][kLdsWidth];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int sl = wid + kLdsWaves * q;
        row[q] = sl * kSlice + lane;
        in[q] = row[q] < n;
        mw[q] = 0;
        const int rb = in[q] ? row[q] : 0;
#pragma unroll
        for (int j = 0; j < kLdsWidth; ++j) {
            av[q][j] = 0.0;
            ac[q][j] = rb;
        }
        if (sl < B.nslices) {
            // slice bounds, width and column storage are wave-uniform
            const int s = __builtin_amdgcn_readfirstlane(sl);
            const int64_t base = B.sptr[s];
            mw[q] = (int)((B.sptr[s + 1] - base) / kSlice);
            const int flag = B.sflag[s];
#pragma unroll
            for (int j = 0; j < kLdsWidth; ++j) {
                if (j < mw[q]) {
                    const size_t e = (size_t)base + (size_t)j * kSlice + lane;
                    int c;
                    if (flag == 2) c = row[q] + B.soff[(size_t)s * kTabMax + j];
                    else if (flag == 1) c = rb + (int)B.cols16[e];
                    else c = B.cols[e];
                    ac[q][j] = c < 0 ? 0 : (c < n ? c : n - 1);
                    av[q][j] = B.vals[e];
                }
            }
        }
    }
    double bi[R], xi[R], di[R], ri[R], zi[R], pi[R];
    double wr[R][YB > 0 ? YB : 1], awr[R][YB > 0 ? YB : 1];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        bi[q] = in[q] ? b[row[q]] : 0.0;
        xi[q] = in[q] ? x[row[q]] : 0.0;
        di[q] = in[q] ? B.dinv[row[q]] : 0.0;
        ri[q] = zi[q] = pi[q] = 0.0;
#pragma unroll
        for (int k = 0; k < YB; ++k) {
            wr[q][k] = in[q] && k < y ? W[(size_t)k * B.ld + row[q]] : 0.0;
            awr[q][k] = in[q] && k < y ? AW[(size_t)k * B.ld + row[q]] : 0.0;
        }
    }
    if (YB > 0)
        for (int e = threadIdx.x; e < y * y; e += kLdsBlock) sginv[(e / y) * YB + e % y] = B.Ginv[e];
    // (A v) of row q, v gathered from sp
    auto product = [&](int q) {
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < kLdsWidth; ++j)
            if (j < mw[q]) acc = fma(av[q][j], sp[ac[q][j]], acc);
        return acc;
    };
    auto share = [&](const double (&v)[R]) {
#pragma unroll
        for (int q = 0; q < R; ++q) sp[row[q]] = v[q];
    };

    // ---- Stage 1 (Alg. 2): rbar = b - A xbar, (b, b), (rbar, rbar), W^T rbar
    share(xi);
    __syncthreads();
    {
        double v[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] = 0.0;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            ri[q] = in[q] ? bi[q] - product(q) : 0.0;
            v[0] += bi[q] * bi[q];
            v[1] += ri[q] * ri[q];
#pragma unroll
            for (int k = 0; k < YB; ++k) v[2 + k] += wr[q][k] * ri[q];
        }
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
    // this lane's row of G^{-1} (lane k < y), for mu = G^{-1} c in the loop
    double ginv_row[YB > 0 ? YB : 1];
    {
        const int kl = lane < YB ? lane : 0;
#pragma unroll
        for (int j = 0; j < YB; ++j) ginv_row[j] = (lane < y && j < y) ? sginv[kl * YB + j] : 0.0;
    }
    if (state == kRunning) {
        // x = xbar + W what, r = rbar - (A W) what, z = M^{-1} r,
        // sums (r, z), (r, r), c = (A W)^T z; mu = G^{-1} c
        {
            double v[NV];
#pragma unroll
            for (int k = 0; k < NV; ++k) v[k] = 0.0;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                if (YB > 0) {
                    double wx = 0.0, awx = 0.0;
#pragma unroll
                    for (int k = 0; k < YB; ++k) {
                        const double wh = k < y ? smu[k] : 0.0;
                        wx += wr[q][k] * wh;
                        awx += awr[q][k] * wh;
                    }
                    xi[q] += wx;
                    ri[q] -= awx;
                }
                zi[q] = di[q] * ri[q];
                v[0] += ri[q] * zi[q];
                v[1] += ri[q] * ri[q];
#pragma unroll
                for (int k = 0; k < YB; ++k) v[2 + k] += awr[q][k] * zi[q];
            }
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
#pragma unroll
        for (int q = 0; q < R; ++q) {
            double s = zi[q];
#pragma unroll
            for (int k = 0; k < YB; ++k) s -= wr[q][k] * (k < y ? smu[k] : 0.0);
            pi[q] = s;
        }
        state = sh.state;
        status = sh.status;
        // ---- the loop of Alg. 1; every thread keeps the same state, so no
        // barrier is needed to share the decisions
        while (state == kRunning) {
            share(pi);
            __syncthreads();
            // q = A p, gamma = (A p, p)
            double qv[R];
            double g[1] = {0.0};
#pragma unroll
            for (int q = 0; q < R; ++q) {
                qv[q] = in[q] ? product(q) : 0.0;
                g[0] += qv[q] * pi[q];
            }
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
            {
                double v[NV];
#pragma unroll
                for (int k = 0; k < NV; ++k) v[k] = 0.0;
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    xi[q] = xi[q] + alpha * pi[q];
                    ri[q] = ri[q] - alpha * qv[q];
                    zi[q] = di[q] * ri[q];
                    v[0] += ri[q] * zi[q];
                    v[1] += ri[q] * ri[q];
#pragma unroll
                    for (int k = 0; k < YB; ++k) v[2 + k] += awr[q][k] * zi[q];
                }
                lds_wave_partials<NV>(v, red);
            }
            __syncthreads();
            ++iters;
            // every wave sums the wave partials itself: lane t < NV holds
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
#pragma unroll
            for (int j = 0; j < YB; ++j) muk += ginv_row[j] * lane_value(tot, 2 + j);
            // p = z + beta p - W mu, beta = (r', z') / (r, z)
            const double beta = rz / rho;
            rho = rz;
            beta_last = beta;
            double mu[YB > 0 ? YB : 1];
#pragma unroll
            for (int k = 0; k < YB; ++k) mu[k] = k < y ? lane_value(muk, k) : 0.0;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                double s = zi[q] + beta * pi[q];
#pragma unroll
                for (int k = 0; k < YB; ++k) s -= wr[q][k] * mu[k];
                pi[q] = s;
            }
        }
        rho_last = rho;
    }
    // ---- the true residual ||b - A x|| and the solution
    __syncthreads();
    share(xi);
    __syncthreads();
    double t[1] = {0.0};
#pragma unroll
    for (int q = 0; q < R; ++q) {
        if (in[q]) {
            const double rt = bi[q] - product(q);
            t[0] += rt * rt;
            x[row[q]] = xi[q];
        }
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

// Basis dimensions of the one-workgroup solve: up to kLdsYMax.
int lds_tier(int n, int y) { return n >= 1 && n <= kLdsThreads && y >= 0 && y <= kLdsYMax ? y : -1; }

hipError_t launch_lds_solve(const DevBufs& B, int yb, const double* b, double* x, const double* W,
                            const double* AW, hipStream_t s) {
    if (lds_tier(B.n, yb) != yb || B.nslices > kLdsWaves * kLdsRows) return hipErrorInvalidValue;
    const dim3 g(1), t(kLdsBlock);
    switch (yb) {
#define CASE(T) case T: hipLaunchKernelGGL((k_lds_solve<T>), g, t, 0, s, B, b, x, W, AW); break;
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace podcg
