// Streaming kernels of libpodcg: the vector updates of augmented PCG with their
// fused reductions, Stage 1, the tall-skinny Gram products and the POD basis
// formation.  All column blocks (W, A W, S) are column-major with leading
// dimension ld, so lane i of a wave touches row i of every column and each
// load instruction reads 512 contiguous bytes.
#include "podcg_device.h"

namespace podcg {

int basis_tier(int y) {
    if (y < 0) return -1;
    if (y <= kExactTierMax) return y;
    static const int wide[] = {20, 24, 28, 32};
    for (int t : wide)
        if (y <= t) return t;
    return -1;
}

// Loop kernel 2 of augmented PCG (Alg. 1): with alpha from kernel 1,
//   r <- r - alpha q,  z <- M^{-1} r  (Jacobi),
// and the sums (r, z), (r, r), c = (A W)^T z.  The last workgroup forms
//   beta = (r', z') / (r, z),  mu = G^{-1} c  (the solve with W^T A W of
// Alg. 1, with G^{-1} from the Cholesky factor of Stage 1),
// counts the iteration and tests ||r|| <= tol ||b||.
// Column of W or A W: read once per iteration, so loaded nontemporally when
// NTB (keeps the smaller vectors resident in the caches).
template <bool NTB, typename T>
__device__ __forceinline__ T basis_load(const T* p) {
    return NTB ? __builtin_nontemporal_load(p) : *p;
}

// T: storage and arithmetic type of the vectors and of A W (FP64, or FP32
// for the inner solve of mixed precision); all sums are accumulated in FP64.
template <typename T, int YB, bool NTB = false>
__global__ __launch_bounds__(kBlock) void k_update(DevBufs B, int y, T* __restrict__ r,
                                                   T* __restrict__ z, const T* __restrict__ q,
                                                   const T* __restrict__ AW) {
    constexpr int NV = 2 + YB;
    __shared__ double lds[kWavesPerBlock * NV + NV + 1];
    DevState* st = B.st;
    if (st->done != kRunning) return;
    const T alpha = (T)st->alpha;
    const T* __restrict__ dinv = mat_dinv<T>(B);
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = 0.0;
    const int n = B.n;
    const int stride = gridDim.x * kBlock;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const T ri = r[i] - alpha * q[i];
        const T zi = dinv[i] * ri;
        r[i] = ri;
        z[i] = zi;
        v[0] += (double)ri * (double)zi;
        v[1] += (double)ri * (double)ri;
#pragma unroll
        for (int k = 0; k < YB; ++k) {
            const T a = basis_load<NTB>(AW + (size_t)tier_col<YB>(k, y) * B.ld + i);
            if (tier_live<YB>(k, y)) v[2 + k] += (double)a * (double)zi;
        }
    }
    if (!grid_sum_last<NV>(v, B.part, B.counter, lds)) return;
    if (threadIdx.x == 0) {
        const double rz = lds[0], rr = lds[1];
        const int it = st->iter + 1;
        st->iter = it;
        st->rr = rr;
        if (!is_finite(rr) || !is_finite(rz)) {
            st->status = kStNonfinite;
            st->done = kFailed;
        } else {
            st->beta = rz / st->rho;
            st->rho = rz;
            if (rr <= st->tol2) {
                st->status = kStOk;
                st->done = kConvergedPending;
            } else if (it >= st->maxit) {
                st->status = kStNotConverged;
                st->done = kCapPending;
            }
        }
    }
    if (threadIdx.x < y) {
        double s = 0.0;
        for (int j = 0; j < y; ++j) s += B.Ginv[threadIdx.x * y + j] * lds[2 + j];
        st->mu[threadIdx.x] = s;
    }
}

// Loop kernel 2 in the implicit form of the direction, p = pt - W nu.  The
// SpMV has produced qt = A pt, and
//   A p = A pt - (A W) nu,  r <- r - alpha A p,  z <- M^{-1} r,
// with the sums (r, z), (r, r), c = (A W)^T z: each column of A W is loaded
// once and serves both A p and c.  The last workgroup forms beta and
// mu = G^{-1} c as in the explicit form and then advances
//   xi <- xi + alpha nu        (x += alpha p is alpha pt, minus W alpha nu),
//   nu <- mu + beta nu         (p' = z + beta p - W mu = pt' - W nu'),
//   a  <- c + beta a           (a = (A W)^T pt, by the same recurrence),
//   gcorr = nu^T a,
// so that the next SpMV turns (A pt, pt) into (A p, p) = (A pt, pt) - nu^T a
// (this uses (A W)^T p = 0, the property Alg. 1's projection maintains).
template <int YB>
__global__ __launch_bounds__(kBlock) void k_update_imp(DevBufs B, int y, double* __restrict__ r,
                                                       double* __restrict__ z,
                                                       const double* __restrict__ qt,
                                                       const double* __restrict__ AW) {
    constexpr int NV = 2 + YB;
    __shared__ double lds[kWavesPerBlock * NV + NV + 1];
    DevState* st = B.st;
    if (st->done != kRunning) return;
    const double alpha = st->alpha;
    double nu[YB > 0 ? YB : 1];
#pragma unroll
    for (int k = 0; k < YB; ++k) nu[k] = k < y ? st->nu[k] : 0.0;
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = 0.0;
    const int n = B.n;
    const int stride = gridDim.x * kBlock;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        double a[YB > 0 ? YB : 1];
        double qi = qt[i];
#pragma unroll
        for (int k = 0; k < YB; ++k) {
            a[k] = basis_load<true>(AW + (size_t)tier_col<YB>(k, y) * B.ld + i);
            if (tier_live<YB>(k, y)) qi -= a[k] * nu[k];
        }
        const double ri = r[i] - alpha * qi;
        const double zi = B.dinv[i] * ri;
        r[i] = ri;
        z[i] = zi;
        v[0] += ri * zi;
        v[1] += ri * ri;
#pragma unroll
        for (int k = 0; k < YB; ++k)
            if (tier_live<YB>(k, y)) v[2 + k] += a[k] * zi;
    }
    if (!grid_sum_last<NV>(v, B.part, B.counter, lds)) return;
    if (threadIdx.x == 0) {
        const double rz = lds[0], rr = lds[1];
        const int it = st->iter + 1;
        st->iter = it;
        st->rr = rr;
        double beta = 0.0, stepped = 1.0;
        if (!is_finite(rr) || !is_finite(rz)) {
            st->status = kStNonfinite;
            st->done = kFailed;
            stepped = 0.0;     // the direction kernel will not apply this step to x
        } else {
            beta = rz / st->rho;
            st->beta = beta;
            st->rho = rz;
            if (rr <= st->tol2) {
                st->status = kStOk;
                st->done = kConvergedPending;
            } else if (it >= st->maxit) {
                st->status = kStNotConverged;
                st->done = kCapPending;
            }
        }
        lds[NV] = beta;
        lds[NV + 1] = stepped;
    }
    __syncthreads();
    if (threadIdx.x < kWave) {
        const int k = threadIdx.x;
        double prod = 0.0;
        if (k < y) {
            double mu = 0.0;
            for (int j = 0; j < y; ++j) mu += B.Ginv[k * y + j] * lds[2 + j];
            st->mu[k] = mu;
            const double beta = lds[NV];
            const double nu_old = st->nu[k];
            if (lds[NV + 1] != 0.0) st->xi[k] += alpha * nu_old;
            const double nu_new = mu + beta * nu_old;
            const double a_new = lds[2 + k] + beta * st->acc[k];
            st->nu[k] = nu_new;
            st->acc[k] = a_new;
            prod = nu_new * a_new;
        }
        prod = wave_sum(prod);
        if (k == 0) st->gcorr = prod;
    }
}

// Loop kernel 3: x <- x + alpha p, then (while iterating) the new direction
//   p <- z + beta p - W mu,
// which keeps p A-orthogonal to range(W) (Alg. 1).  INIT forms the first
// direction p = z - W mu and leaves x alone.
// The solution x is always FP64: with FP32 vectors (mixed precision) the
// update x += alpha p is carried out in FP64, so the correction of a
// refinement step is accumulated without FP32 rounding.
// Directions recorded by REC (the Krylov basis V and Gamma, alpha of Alg. 1's
// outputs): p_k / sqrt(gamma_k) (unit A-norm) goes to column k of V while
// k < cap, with gamma_k and alpha_k.
struct DirRecord {
    double* V;
    size_t ld;
    int cap;
    double* gamma;
    double* alpha;
};

template <typename T, int YB, bool INIT, bool NTB = false, bool REC = false>
__global__ __launch_bounds__(kBlock) void k_dir(DevBufs B, int y, T* __restrict__ p,
                                                double* __restrict__ x, const T* __restrict__ z,
                                                const T* __restrict__ W, DirRecord rec) {
    const DevState* st = B.st;
    const int done = st->done;
    if (INIT) {
        if (done != kRunning) return;
    } else if (done != kRunning && done != kConvergedPending && done != kCapPending) {
        return;
    }
    const bool new_dir = INIT || done == kRunning;
    const double alpha = st->alpha;
    const T beta = (T)st->beta;
    T mu[YB > 0 ? YB : 1];
#pragma unroll
    for (int k = 0; k < YB; ++k) mu[k] = k < y ? (T)st->mu[k] : (T)0;
    const int n = B.n;
    const int stride = gridDim.x * kBlock;
    // index of the direction applied in this launch (the update kernel has
    // already counted its iteration)
    const int krec = REC && !INIT ? st->iter - 1 : -1;
    double* __restrict__ vrec = (REC && krec >= 0 && krec < rec.cap) ? rec.V + (size_t)krec * rec.ld : nullptr;
    const double vscale = REC ? 1.0 / sqrt(st->gamma) : 1.0;
    if (REC && vrec && blockIdx.x == 0 && threadIdx.x == 0) {
        rec.gamma[krec] = st->gamma;
        rec.alpha[krec] = alpha;
    }
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        T s;
        if (INIT) {
            s = z[i];
        } else {
            const T pi = p[i];
            x[i] += alpha * (double)pi;
            if (REC && vrec) vrec[i] = (double)pi * vscale;
            if (!new_dir) continue;
            s = z[i] + beta * pi;
        }
#pragma unroll
        for (int k = 0; k < YB; ++k) s -= basis_load<NTB>(W + (size_t)tier_col<YB>(k, y) * B.ld + i) * mu[k];
        p[i] = s;
    }
}

// Stage 1 (Alg. 2 and the first steps of Alg. 1).  With what = G^{-1} W^T rbar
// from the residual kernel and r = rbar:
//   x <- xbar + W what,  r <- rbar - (A W) what,  z = M^{-1} r,
// and the sums (r, z), (r, r), c = (A W)^T z; the last workgroup forms
// mu = G^{-1} c and tests the Stage-1 residual against the tolerance.
template <int YB>
__global__ __launch_bounds__(kBlock) void k_stage1_apply(DevBufs B, int y, double* __restrict__ x,
                                                         double* __restrict__ r,
                                                         double* __restrict__ z,
                                                         const double* __restrict__ W,
                                                         const double* __restrict__ AW) {
    constexpr int NV = 2 + YB;
    __shared__ double lds[kWavesPerBlock * NV + NV + 1];
    DevState* st = B.st;
    if (st->done != kRunning) return;
    double what[YB > 0 ? YB : 1];
#pragma unroll
    for (int k = 0; k < YB; ++k) what[k] = k < y ? st->what[k] : 0.0;
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = 0.0;
    const int n = B.n;
    const int stride = gridDim.x * kBlock;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        double ri = r[i];
        if (YB > 0) {
            double wx = 0.0, awx = 0.0;
#pragma unroll
            for (int k = 0; k < YB; ++k) {
                const int kc = tier_col<YB>(k, y);
                wx += W[(size_t)kc * B.ld + i] * what[k];
                awx += AW[(size_t)kc * B.ld + i] * what[k];
            }
            x[i] += wx;
            ri -= awx;
            r[i] = ri;
        }
        const double zi = B.dinv[i] * ri;
        z[i] = zi;
        v[0] += ri * zi;
        v[1] += ri * ri;
#pragma unroll
        for (int k = 0; k < YB; ++k) {
            const double a = AW[(size_t)tier_col<YB>(k, y) * B.ld + i];
            if (tier_live<YB>(k, y)) v[2 + k] += a * zi;
        }
    }
    if (!grid_sum_last<NV>(v, B.part, B.counter, lds)) return;
    if (threadIdx.x == 0) {
        const double rz = lds[0], rr = lds[1];
        st->rho = rz;
        st->rr = rr;
        st->rr0 = rr;
        if (!is_finite(rr) || !is_finite(rz)) {
            st->status = kStNonfinite;
            st->done = kFailed;
        } else if (rr <= st->tol2) {
            st->status = kStOk;
            st->done = kFinished;
        } else if (st->maxit <= 0) {
            st->status = kStNotConverged;
            st->done = kFinished;
        }
    }
    // implicit form: the first direction is p = z - W mu = pt - W nu with
    // pt = z, nu = mu, a = (A W)^T z and xi = 0
    const bool imp = st->implicit != 0;
    if (threadIdx.x < kWave) {
        const int k = threadIdx.x;
        double prod = 0.0;
        if (k < y) {
            double s = 0.0;
            for (int j = 0; j < y; ++j) s += B.Ginv[k * y + j] * lds[2 + j];
            st->mu[k] = s;
            if (imp) {
                st->nu[k] = s;
                st->acc[k] = lds[2 + k];
                st->xi[k] = 0.0;
                prod = s * lds[2 + k];
            }
        }
        if (imp) {
            prod = wave_sum(prod);
            if (k == 0) st->gcorr = prod;
        }
    }
}

// Implicit form, after the loop: x = xt - W xi.
template <int YB>
__global__ __launch_bounds__(kBlock) void k_implicit_finish(DevBufs B, int y, double* __restrict__ x,
                                                            const double* __restrict__ W) {
    const DevState* st = B.st;
    double xi[YB > 0 ? YB : 1];
#pragma unroll
    for (int k = 0; k < YB; ++k) xi[k] = k < y ? st->xi[k] : 0.0;
    const int n = B.n;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < YB; ++k) {
            const double w = basis_load<true>(W + (size_t)tier_col<YB>(k, y) * B.ld + i);
            if (tier_live<YB>(k, y)) s += w * xi[k];
        }
        x[i] -= s;
    }
}

// W(:, i) = sum_k S(:, k) T(k, i) for i < y, k < count (Eq. (podAlgebraicDefinition)
// with T = diag(w) V_y Sigma_y^{-1}).
template <int KB>
__global__ __launch_bounds__(kBlock) void k_pod_form(int n, size_t ld, const double* __restrict__ S,
                                                     int count, const double* __restrict__ T, int y,
                                                     double* __restrict__ W) {
    __shared__ double t[kYMax * kYMax];
    for (int e = threadIdx.x; e < count * y; e += kBlock) t[e] = T[e];
    __syncthreads();
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        double s[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const double v = S[(size_t)(k < count ? k : count - 1) * ld + i];
            s[k] = k < count ? v : 0.0;
        }
        for (int c = 0; c < y; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < KB; ++k)
                if (k < count) acc += s[k] * t[k * y + c];
            W[(size_t)c * ld + i] = acc;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_copy(const double* __restrict__ a, double* __restrict__ c,
                                                 size_t n) {
    for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
        c[i] = a[i];
}

__global__ __launch_bounds__(kBlock) void k_triad(const double* __restrict__ a,
                                                  const double* __restrict__ b,
                                                  double* __restrict__ c, size_t n, double s) {
    for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
        c[i] = a[i] + s * b[i];
}

__global__ void k_state_init(DevState* st, int maxit, double tol2, int y, int implicit) {
    if (threadIdx.x != 0) return;
    st->implicit = implicit;
    st->gcorr = 0.0;
    for (int k = 0; k < kYMax; ++k) st->nu[k] = st->acc[k] = st->xi[k] = 0.0;
    st->iter = 0;
    st->done = kRunning;
    st->status = kStNotConverged;
    st->y = y;
    st->maxit = maxit;
    st->rr = st->rr0 = st->bnorm2 = st->true_rr = 0.0;
    st->tol2 = tol2;
    st->rho = st->alpha = st->beta = st->gamma = 0.0;
    for (int k = 0; k < kYMax; ++k) st->mu[k] = st->what[k] = 0.0;
}

// Stage 1 of one refinement step of the mixed-precision solve.  In FP64:
// x64 += W what and r = r64 - (A W) what (what = G^{-1} W^T r64 from the
// residual kernel); then the inner system starts in FP32: r32 = r,
// z32 = M^{-1} r32, with the sums (r, z), (r, r) and (A W)^T z accumulated in
// FP64.  The inner iterations add their steps to x64 directly.  The last workgroup sets mu = G^{-1} (A W)^T z and the
// inner tolerance tol2 = inner_rtol2 (r, r).
template <int YB>
__global__ __launch_bounds__(kBlock) void k_stage1_mixed(DevBufs B, int y, double* __restrict__ x64,
                                                         const double* __restrict__ r64,
                                                         float* __restrict__ r32,
                                                         float* __restrict__ z32,
                                                         const double* __restrict__ W,
                                                         const double* __restrict__ AW,
                                                         const float* __restrict__ AW32,
                                                         double inner_rtol2) {
    constexpr int NV = 2 + YB;
    __shared__ double lds[kWavesPerBlock * NV + NV + 1];
    DevState* st = B.st;
    if (st->done != kRunning) return;
    double what[YB > 0 ? YB : 1];
#pragma unroll
    for (int k = 0; k < YB; ++k) what[k] = k < y ? st->what[k] : 0.0;
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = 0.0;
    const int n = B.n;
    const int stride = gridDim.x * kBlock;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        double ri = r64[i];
        if (YB > 0) {
            double wx = 0.0, awx = 0.0;
#pragma unroll
            for (int k = 0; k < YB; ++k) {
                const int kc = tier_col<YB>(k, y);
                wx += W[(size_t)kc * B.ld + i] * what[k];
                awx += AW[(size_t)kc * B.ld + i] * what[k];
            }
            x64[i] += wx;
            ri -= awx;
        }
        const float rf = (float)ri;
        const float zf = B.dinv32[i] * rf;
        r32[i] = rf;
        z32[i] = zf;
        v[0] += (double)rf * (double)zf;
        v[1] += (double)rf * (double)rf;
#pragma unroll
        for (int k = 0; k < YB; ++k) {
            const float a = AW32[(size_t)tier_col<YB>(k, y) * B.ld + i];
            if (tier_live<YB>(k, y)) v[2 + k] += (double)a * (double)zf;
        }
    }
    if (!grid_sum_last<NV>(v, B.part, B.counter, lds)) return;
    if (threadIdx.x == 0) {
        const double rz = lds[0], rr = lds[1];
        st->rho = rz;
        st->rr = rr;
        st->rr0 = rr;
        // the inner solve aims at inner_rtol relative to its own right-hand
        // side, but never below half of the outer target (st->tol2 holds
        // rtol^2 ||b||^2 from the residual kernel)
        st->tol2 = fmax(inner_rtol2 * rr, 0.25 * st->tol2);
        if (!is_finite(rr) || !is_finite(rz)) {
            st->status = kStNonfinite;
            st->done = kFailed;
        } else if (rr == 0.0 || st->maxit <= 0) {
            st->status = rr == 0.0 ? kStOk : kStNotConverged;
            st->done = kFinished;
        }
    }
    if (threadIdx.x < y) {
        double sum = 0.0;
        for (int j = 0; j < y; ++j) sum += B.Ginv[threadIdx.x * y + j] * lds[2 + j];
        st->mu[threadIdx.x] = sum;
    }
}

__global__ __launch_bounds__(kBlock) void k_to_float(const double* __restrict__ a, float* __restrict__ b,
                                                     size_t n) {
    for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
        b[i] = (float)a[i];
}

// ---------------------------------------------------------------- launchers

static int vec_grid(int64_t n, int cap = kVecBlocksMax) {
    if (cap <= 0) cap = kVecBlocksMax;
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    return (int)(g < cap ? g : cap);
}

hipError_t launch_update(const DevBufs& B, int yb, int y, double* r, double* z, const double* q,
                         const double* AW, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    dim3 g(vec_grid(B.n, B.update_grid)), t(kBlock);
    switch (yb) {
#define CASE(T) case T: PODCG_LAUNCH((k_update<double, T, true>), g, t, s, e0, e1, B, y, r, z, q, AW); break;
        PODCG_TIERS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_update_implicit(const DevBufs& B, int yb, int y, double* r, double* z, const double* qt,
                                  const double* AW, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (y < 1) return hipErrorInvalidValue;
    dim3 g(vec_grid(B.n, B.update_grid)), t(kBlock);
    switch (yb) {
#define CASE(T) case T: PODCG_LAUNCH((k_update_imp<T>), g, t, s, e0, e1, B, y, r, z, qt, AW); break;
        PODCG_POS_TIERS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_implicit_finish(const DevBufs& B, int yb, int y, double* x, const double* W, hipStream_t s) {
    if (y < 1) return hipErrorInvalidValue;
    dim3 g(vec_grid(B.n)), t(kBlock);
    switch (yb) {
#define CASE(T) case T: hipLaunchKernelGGL((k_implicit_finish<T>), g, t, 0, s, B, y, x, W); break;
        PODCG_POS_TIERS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dir(const DevBufs& B, int yb, int y, double* p, double* x, const double* z,
                      const double* W, bool init, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    dim3 g(vec_grid(B.n, B.dir_grid)), t(kBlock);
    const DirRecord none{};
    switch (yb) {
#define CASE(T)                                                                                    \
    case T:                                                                                        \
        if (init) PODCG_LAUNCH((k_dir<double, T, true, true>), g, t, s, e0, e1, B, y, p, x, z, W, none); \
        else PODCG_LAUNCH((k_dir<double, T, false, true>), g, t, s, e0, e1, B, y, p, x, z, W, none);     \
        break;
        PODCG_TIERS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dir_rec(const DevBufs& B, int yb, int y, double* p, double* x, const double* z,
                          const double* W, double* V, size_t ldv, int cap, double* gamma,
                          double* alpha, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    dim3 g(vec_grid(B.n, B.dir_grid)), t(kBlock);
    const DirRecord rec{V, ldv, cap, gamma, alpha};
    switch (yb) {
#define CASE(T) case T: PODCG_LAUNCH((k_dir<double, T, false, true, true>), g, t, s, e0, e1, B, y, p, x, z, W, rec); break;
        PODCG_TIERS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_stage1_apply(const DevBufs& B, int yb, int y, double* x, double* r, double* z,
                               const double* W, const double* AW, hipStream_t s) {
    dim3 g(vec_grid(B.n, B.update_grid)), t(kBlock);
    switch (yb) {
#define CASE(T) case T: hipLaunchKernelGGL((k_stage1_apply<T>), g, t, 0, s, B, y, x, r, z, W, AW); break;
        PODCG_TIERS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pod_form(int n, size_t ld, const double* S, int count, const double* T, int y,
                           double* W, hipStream_t s) {
    if (y < 1) return hipSuccess;
    dim3 g(vec_grid(n)), t(kBlock);
    switch (basis_tier(count)) {
#define CASE(K) case K: hipLaunchKernelGGL((k_pod_form<K>), g, t, 0, s, n, ld, S, count, T, y, W); break;
        PODCG_POS_TIERS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_copy(const double* src, double* dst, size_t n, hipStream_t s) {
    int64_t g = ((int64_t)n + kBlock - 1) / kBlock;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_copy, dim3((int)g), dim3(kBlock), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_triad(const double* a, const double* b, double* c, size_t n, double sc,
                        hipStream_t s) {
    int64_t g = ((int64_t)n + kBlock - 1) / kBlock;
    if (g > 16384) g = 16384;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_triad, dim3((int)g), dim3(kBlock), 0, s, a, b, c, n, sc);
    return hipGetLastError();
}

hipError_t launch_state_init(DevState* st, int maxit, double tol2, int y, hipStream_t s, bool implicit) {
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, st, maxit, tol2, y, implicit ? 1 : 0);
    return hipGetLastError();
}

}  // namespace podcg

namespace podcg {

hipError_t launch_update32(const DevBufs& B, int yb, int y, float* r, float* z, const float* q,
                           const float* AW, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    dim3 g(vec_grid(B.n, B.update_grid)), t(kBlock);
    switch (yb) {
#define CASE(T) case T: PODCG_LAUNCH((k_update<float, T, true>), g, t, s, e0, e1, B, y, r, z, q, AW); break;
        PODCG_TIERS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dir32(const DevBufs& B, int yb, int y, float* p, double* x, const float* z,
                        const float* W, bool init, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    dim3 g(vec_grid(B.n, B.dir_grid)), t(kBlock);
    const DirRecord none{};
    switch (yb) {
#define CASE(T)                                                                                    \
    case T:                                                                                        \
        if (init) PODCG_LAUNCH((k_dir<float, T, true, true>), g, t, s, e0, e1, B, y, p, x, z, W, none);  \
        else PODCG_LAUNCH((k_dir<float, T, false, true>), g, t, s, e0, e1, B, y, p, x, z, W, none);      \
        break;
        PODCG_TIERS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_stage1_mixed(const DevBufs& B, int yb, int y, double* x64, const double* r64,
                               float* r32, float* z32, const double* W, const double* AW,
                               const float* AW32, double inner_rtol, hipStream_t s) {
    dim3 g(vec_grid(B.n, B.update_grid)), t(kBlock);
    const double r2 = inner_rtol * inner_rtol;
    switch (yb) {
#define CASE(T) case T: hipLaunchKernelGGL((k_stage1_mixed<T>), g, t, 0, s, B, y, x64, r64, r32, z32, W, AW, AW32, r2); break;
        PODCG_TIERS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_to_float(const double* src, float* dst, size_t n, hipStream_t s) {
    int64_t g = ((int64_t)n + kBlock - 1) / kBlock;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_to_float, dim3((int)g), dim3(kBlock), 0, s, src, dst, n);
    return hipGetLastError();
}

}  // namespace podcg
