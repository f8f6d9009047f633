// Streaming kernels of libpodcg: the vector updates of augmented PCG with their
// fused reductions, Stage 1, the tall-skinny Gram products and the POD basis
// formation.  All column blocks (W, A W, S) are column-major with leading
// dimension ld, so lane i of a wave touches row i of every column and each
// load instruction reads 512 contiguous bytes; the implicit update also reads
// a copy of A W in 64-row tiles.
#include "podcg_launch.h"

namespace podcg {

int basis_tier(int y) {
    if (y < 0) return -1;
    if (y <= kExactTierMax) return y;
    static const int wide[] = {20, 24, 28, 32};
    for (int t : wide)
        if (y <= t) return t;
    return -1;
}

// Column of W or A W: read once per iteration, so loaded nontemporally when
// NTB (keeps the smaller vectors resident in the caches).  The tiled A W of
// the implicit update is loaded normally: measured at 128^3 and rank 6, the
// update takes 28.2 us that way against 29.0 us with nontemporal loads (the
// last-level cache then keeps part of it from one iteration to the next).
template <bool NTB, typename T>
__device__ __forceinline__ T basis_load(const T* p) {
    return NTB ? __builtin_nontemporal_load(p) : *p;
}

// alpha of iteration k, at the start of every update workgroup: the SpMV's
// per-workgroup partials of (A p, p) are summed here in a fixed order (the
// same in every workgroup), minus gcorr in the implicit form.  Workgroup 0
// records alpha and gamma in slot k & 1.  Returns false when gamma is not
// positive and finite; then workgroup 0 records the failure and stops the loop.
// The first kPartEarly partials of each thread are loaded by loop_partials at
// the very start of the kernel, ahead of the kernel's own operand prefetch:
// vector loads complete in order, so the wait for them here does not also wait
// for the prefetched operands (a wait on a partial loaded after the prefetch
// would).  The sum keeps the order t, t + kBlock, ... of each thread.
constexpr int kPartEarly = 4;   // covers SpMV grids up to 1024
__device__ __forceinline__ void loop_partials(const DevBufs& B, int nsp, double (&gp)[kPartEarly]) {
#pragma unroll
    for (int j = 0; j < kPartEarly; ++j) {
        const int t = threadIdx.x + j * kBlock;
        gp[j] = t < nsp ? B.gpart[t] : 0.0;   // the SpMV is the previous kernel: plain loads see its writes
    }
}
__device__ __forceinline__ bool loop_alpha(const DevBufs& B, int k, int nsp, const double (&gp)[kPartEarly],
                                           double gcorr, double* ldsg, double& alpha) {
    DevState* st = B.st;
    const int par = k & 1;
    const double rho = st->lrho[par];       // read next to the partials, before the barrier
    double g[1] = {0.0};
#pragma unroll
    for (int j = 0; j < kPartEarly; ++j)
        if ((int)threadIdx.x + j * kBlock < nsp) g[0] += gp[j];
    for (int t = threadIdx.x + kPartEarly * kBlock; t < nsp; t += kBlock) g[0] += B.gpart[t];
    block_sum<1>(g, ldsg);
    const double gamma = ldsg[0] - gcorr;
    const bool ok = gamma > 0.0 && is_finite(gamma);
    if (ok) alpha = rho / gamma;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->gamma = gamma;
        if (ok) {
            st->lgamma[par] = gamma;
            st->lalpha[par] = alpha;
            st->alpha = alpha;
        } else {
            st->status = is_finite(gamma) ? kStNotSpd : kStNonfinite;
            st->done = kFailed;
            st->stop = k;
        }
    }
    return ok;
}

// Loop kernel 2 of augmented PCG (Alg. 1), iteration k: with alpha from the
// SpMV's partials,
//   r <- r - alpha q,  z <- M^{-1} r  (Jacobi),
// and the sums (r, z), (r, r), c = (A W)^T z, reduced per group of
// workgroups; the direction kernel finishes the sums.  In FP64 only z is
// stored: with the Jacobi preconditioner r = M z, so the kernel reads z,
// recovers r = z / dinv and writes z alone (one vector of traffic less; r
// then carries one more rounding per iteration).  The FP32 inner solve of
// mixed precision keeps r and z.
// T: storage and arithmetic type of the vectors and of A W (FP64, or FP32
// for the inner solve of mixed precision); all sums are accumulated in FP64.
template <typename T, int YB, bool NTB = false>
__global__ __launch_bounds__(kBlock) void k_update(DevBufs B, int y, T* __restrict__ r,
                                                   T* __restrict__ z, const T* __restrict__ q,
                                                   const T* __restrict__ AW, int k, int nsp) {
    constexpr int NV = 2 + YB;
    __shared__ double lds[kWavesPerBlock * NV + NV + 1];
    __shared__ double ldsg[kWavesPerBlock + 2];
    if (k >= B.st->stop) return;
    double gp[kPartEarly];
    loop_partials(B, nsp, gp);
    const T* __restrict__ dinv = mat_dinv<T>(B);
    const int n = B.n;
    const int stride = gridDim.x * kBlock;
    // the operands of this thread's first kPrefetch elements are loaded
    // before alpha is formed, so the memory system is busy while every
    // workgroup sums the SpMV partials (fewer for wide bases, to bound the
    // registers)
    constexpr int kPrefetch = YB <= 7 ? 4 : (YB <= 10 ? 3 : (YB <= 14 ? 2 : 1));
    constexpr bool kZOnly = sizeof(T) == 8;
    const int i0 = blockIdx.x * kBlock + threadIdx.x;
    T rf[kPrefetch], qf[kPrefetch], df[kPrefetch], af[kPrefetch][YB > 0 ? YB : 1];
    // elements base, base + stride, ... (kPrefetch of them): all loads first
    auto load_block = [&](int base) {
#pragma unroll
        for (int u = 0; u < kPrefetch; ++u) {
            const int ic = base + u * stride < n ? base + u * stride : 0;
            rf[u] = kZOnly ? z[ic] : r[ic];
            qf[u] = q[ic];
            df[u] = dinv[ic];
#pragma unroll
            for (int j = 0; j < YB; ++j) af[u][j] = basis_load<NTB>(AW + (size_t)tier_col<YB>(j, y) * B.ld + ic);
        }
    };
    load_block(i0);
    double alpha_d;
    if (!loop_alpha(B, k, nsp, gp, 0.0, ldsg, alpha_d)) return;
    const T alpha = (T)alpha_d;
    double v[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = 0.0;
    auto step = [&](int i, T rold, T qi, T di, const T* a) {
        if (kZOnly) rold = rold / di;   // r = M z (Jacobi): only z is stored
        const T ri = rold - alpha * qi;
        const T zi = di * ri;
        if (!kZOnly) r[i] = ri;
        z[i] = zi;
        v[0] += (double)ri * (double)zi;
        v[1] += (double)ri * (double)ri;
#pragma unroll
        for (int j = 0; j < YB; ++j)
            if (tier_live<YB>(j, y)) v[2 + j] += (double)a[j] * (double)zi;
    };
    // the rest in blocks of kPrefetch elements, each block's loads issued
    // together (one round trip a block), in the same element order
    for (int base = i0; base < n; base += kPrefetch * stride) {
        if (base != i0) load_block(base);
#pragma unroll
        for (int u = 0; u < kPrefetch; ++u)
            if (base + u * stride < n) step(base + u * stride, rf[u], qf[u], df[u], af[u]);
    }
    group_sum_store<NV>(v, B.part, B.counter, lds);
}

// Loop kernel 2 in the implicit form of the direction, p = pt - W nu.  The
// SpMV has produced qt = A pt, and
//   A p = A pt - (A W) nu,  r <- r - alpha A p,  z <- M^{-1} r
// (only z is stored, r = z / dinv recovered, as in k_update),
// with the sums (r, z), (r, r), c = (A W)^T z: each column of A W is loaded
// once and serves both A p and c.  gamma = (A p, p) = (A pt, pt) - nu^T a with
// a = (A W)^T pt (this uses (A W)^T p = 0, the property Alg. 1's projection
// maintains).
// A W is read from its tiled copy AWt (64-row tiles, the y columns of a tile
// contiguous), so each wave streams one block instead of y separate columns.
template <int YB>
__global__ __launch_bounds__(kBlock) void k_update_imp(DevBufs B, int y, double* __restrict__ r,
                                                       double* __restrict__ z,
                                                       const double* __restrict__ qt,
                                                       const double* __restrict__ AWt, int k, int nsp) {
    constexpr int NV = 2 + YB;
    __shared__ double lds[kWavesPerBlock * NV + NV + 1];
    __shared__ double ldsg[kWavesPerBlock + 2];
    const DevState* st = B.st;
    if (k >= st->stop) return;
    double gp[kPartEarly];
    loop_partials(B, nsp, gp);
    const int par = k & 1;
    const int n = B.n;
    const int stride = gridDim.x * kBlock;
    // the operands of this thread's first kPrefetch elements are in flight
    // while alpha is formed (fewer for wide bases, to bound the registers)
    constexpr int kPrefetch = YB <= 7 ? 4 : (YB <= 10 ? 3 : (YB <= 14 ? 2 : 1));
    const int i0 = blockIdx.x * kBlock + threadIdx.x;
    double rf[kPrefetch], qf[kPrefetch], df[kPrefetch], af[kPrefetch][YB > 0 ? YB : 1];
    // elements base, base + stride, ... (kPrefetch of them): all loads first
    auto load_block = [&](int base) {
#pragma unroll
        for (int u = 0; u < kPrefetch; ++u) {
            const int i = base + u * stride;
            const int ic = i < n ? i : 0;
            rf[u] = z[ic];
            qf[u] = qt[ic];
            df[u] = B.dinv[ic];
            const double* t0 = AWt + (size_t)(ic / kSlice) * (kSlice * y) + (ic % kSlice);
#pragma unroll
            for (int j = 0; j < YB; ++j) af[u][j] = basis_load<false>(t0 + tier_col<YB>(j, y) * kSlice);
        }
    };
    load_block(i0);
    double nu[YB > 0 ? YB : 1];
#pragma unroll
    for (int j = 0; j < YB; ++j) nu[j] = j < y ? st->lnu[par][j] : 0.0;
    double alpha;
    if (!loop_alpha(B, k, nsp, gp, st->lgcorr[par], ldsg, alpha)) return;
    double v[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = 0.0;
    auto step = [&](int i, double rold, double qi, double di, const double* a) {
#pragma unroll
        for (int j = 0; j < YB; ++j)
            if (tier_live<YB>(j, y)) qi -= a[j] * nu[j];
        rold = rold / di;   // r = M z (Jacobi): only z is stored
        const double ri = rold - alpha * qi;
        const double zi = di * ri;
        z[i] = zi;
        v[0] += ri * zi;
        v[1] += ri * ri;
#pragma unroll
        for (int j = 0; j < YB; ++j)
            if (tier_live<YB>(j, y)) v[2 + j] += a[j] * zi;
    };
    // the rest in blocks of kPrefetch elements, each block's loads issued
    // together (one round trip a block), in the same element order
    for (int base = i0; base < n; base += kPrefetch * stride) {
        if (base != i0) load_block(base);
#pragma unroll
        for (int u = 0; u < kPrefetch; ++u)
            if (base + u * stride < n) step(base + u * stride, rf[u], qf[u], df[u], af[u]);
    }
    group_sum_store<NV>(v, B.part, B.counter, lds);
}

// Start of loop kernel 3 of iteration k, in every workgroup: the update's
// group partials summed in group order (lds[0] = (r', z'), lds[1] = (r', r'),
// lds[2 + j] = c_j); beta = (r', z') / (r, z), the convergence test
// ||r'|| <= tol ||b||, the iteration cap, and, when MU, mu = G^{-1} c into smu
// (Alg. 1's projection solve).  Workgroup 0 records the iteration (count,
// ||r'||^2, (r', z') in slot (k + 1) & 1, status and stop).  Returns false
// when the sums are not finite (no step is applied then).
// The group partials ga were loaded by the kernel before its operand
// prefetch (dir_partials), and when MU the caller has filled sginv with
// G^{-1} (from registers loaded at the same time); the state scalars are read
// here at entry.
struct DirStep {
    double alpha, beta;
    bool new_dir;
};
// The update's group partials (one per group of kGroup update workgroups,
// ng <= kBlock), loaded by each kernel before its own operand prefetch, for
// the same reason as loop_partials.
template <int NV>
__device__ __forceinline__ void dir_partials(const DevBufs& B, int nbu, double (&ga)[NV]) {
    const int ng = (nbu + kGroup - 1) / kGroup;
    const double* part2 = B.part + (size_t)NV * nbu;
#pragma unroll
    for (int k = 0; k < NV; ++k) ga[k] = (int)threadIdx.x < ng ? part2[(size_t)k * ng + threadIdx.x] : 0.0;
}
template <int NV, int YB, bool MU>
__device__ __forceinline__ bool dir_begin(const DevBufs& B, int y, int k, double (&ga)[NV], double* lds,
                                          double* smu, double* sginv, DirStep& d) {
    DevState* st = B.st;
    const int par = k & 1;
    const double alpha = st->lalpha[par], rho = st->lrho[par], tol2 = st->tol2;
    const int maxit = st->maxit;
    block_sum<NV>(ga, lds);   // the group sums in group order; ends with a barrier, after which sginv is complete
    const double rz = lds[0], rr = lds[1];
    const bool ok = is_finite(rr) && is_finite(rz);
    const bool conv = rr <= tol2, cap = k + 1 >= maxit;
    d.alpha = alpha;
    d.beta = ok ? rz / rho : 0.0;
    d.new_dir = ok && !conv && !cap;
    if (MU && threadIdx.x < y) {
        double s = 0.0;
        for (int j = 0; j < y; ++j) s += sginv[threadIdx.x * y + j] * lds[2 + j];
        smu[threadIdx.x] = s;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->iter = k + 1;
        st->rr = rr;
        if (!ok) {
            st->status = kStNonfinite;
            st->done = kFailed;
            st->stop = k;
        } else {
            st->beta = d.beta;
            st->rho = rz;
            st->lrho[par ^ 1] = rz;
            if (conv || cap) {
                st->status = conv ? kStOk : kStNotConverged;
                st->done = kFinished;
                st->stop = k + 1;
            }
        }
    }
    if (MU) __syncthreads();
    return ok;
}

// Loop kernel 3: x <- x + alpha p, then (while iterating) the new direction
//   p <- z + beta p - W mu,
// which keeps p A-orthogonal to range(W) (Alg. 1).  INIT forms the first
// direction p = z - W mu (mu from Stage 1) and leaves x alone.
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
                                                const T* __restrict__ W, DirRecord rec, int k, int nbu) {
    constexpr int NV = 2 + YB;
    __shared__ double lds[kWavesPerBlock * NV + NV + 1];
    __shared__ double smu[YB > 0 ? YB : 1];
    __shared__ double sginv[YB > 0 ? YB * YB : 1];
    const DevState* st = B.st;
    const int n = B.n;
    const int stride = gridDim.x * kBlock;
    DirStep d{0.0, 0.0, true};
    // the operands of this thread's first kPrefetch elements are loaded before
    // the reduction is finished, so the memory system is busy meanwhile; the
    // rest follow in blocks of kPrefetch elements, each block's loads issued
    // together (fewer for wide bases, to bound the registers)
    constexpr int kPrefetch = YB == 0 ? 4 : (YB <= 6 ? 2 : 1);
    const int i0 = blockIdx.x * kBlock + threadIdx.x;
    T pf[kPrefetch], zf[kPrefetch], wf[kPrefetch][YB > 0 ? YB : 1];
    double xf[kPrefetch];
    auto load_block = [&](int base, bool need_w) {
#pragma unroll
        for (int u = 0; u < kPrefetch; ++u) {
            const int ic = base + u * stride < n ? base + u * stride : 0;
            pf[u] = p[ic];
            zf[u] = z[ic];
            xf[u] = x[ic];
            if (need_w) {
#pragma unroll
                for (int j = 0; j < YB; ++j) wf[u][j] = basis_load<NTB>(W + (size_t)tier_col<YB>(j, y) * B.ld + ic);
            }
        }
    };
    if (INIT) {
        if (st->stop <= 0) return;
        if (threadIdx.x < y) smu[threadIdx.x] = st->mu[threadIdx.x];
        __syncthreads();
    } else {
        if (k >= st->stop) return;
        double ga[NV];
        dir_partials<NV>(B, nbu, ga);
        constexpr int kGi = YB > 0 ? (YB * YB + kBlock - 1) / kBlock : 1;
        double gi[kGi];
#pragma unroll
        for (int u = 0; u < kGi; ++u) {
            const int e = threadIdx.x + u * kBlock;
            gi[u] = YB > 0 && e < y * y ? B.Ginv[e] : 0.0;
        }
        load_block(i0, true);
        if (YB > 0) {
#pragma unroll
            for (int u = 0; u < kGi; ++u) {
                const int e = threadIdx.x + u * kBlock;
                if (e < y * y) sginv[e] = gi[u];
            }
        }
        if (!dir_begin<NV, YB, (YB > 0)>(B, y, k, ga, lds, smu, sginv, d)) return;
    }
    T mu[YB > 0 ? YB : 1];
#pragma unroll
    for (int j = 0; j < YB; ++j) mu[j] = j < y ? (T)smu[j] : (T)0;
    const T beta = (T)d.beta;
    const double alpha = d.alpha;
    double* __restrict__ vrec = (REC && !INIT && k < rec.cap) ? rec.V + (size_t)k * rec.ld : nullptr;
    const double gamma = REC && !INIT ? st->lgamma[k & 1] : 1.0;
    const double vscale = REC ? 1.0 / sqrt(gamma) : 1.0;
    if (REC && vrec && blockIdx.x == 0 && threadIdx.x == 0) {
        rec.gamma[k] = gamma;
        rec.alpha[k] = alpha;
    }
    auto step = [&](int i, T pi, T zi, double xi, const T* w) {
        T s;
        if (INIT) {
            s = zi;
        } else {
            x[i] = xi + alpha * (double)pi;
            if (REC && vrec) vrec[i] = (double)pi * vscale;
            if (!d.new_dir) return;
            s = zi + beta * pi;
        }
#pragma unroll
        for (int j = 0; j < YB; ++j) s -= w[j] * mu[j];
        p[i] = s;
    };
    if (INIT) {
        for (int i = i0; i < n; i += stride) {
            T w[YB > 0 ? YB : 1];
#pragma unroll
            for (int j = 0; j < YB; ++j) w[j] = basis_load<NTB>(W + (size_t)tier_col<YB>(j, y) * B.ld + i);
            step(i, (T)0, z[i], 0.0, w);
        }
        return;
    }
    for (int base = i0; base < n; base += kPrefetch * stride) {
        if (base != i0) load_block(base, d.new_dir);
#pragma unroll
        for (int u = 0; u < kPrefetch; ++u)
            if (base + u * stride < n) step(base + u * stride, pf[u], zf[u], xf[u], wf[u]);
    }
}

// Loop kernel 3 in the implicit form: x <- x + alpha pt and, while iterating,
// pt <- z + beta pt (no basis column is read).  Workgroup 0 advances the
// coefficients:
//   xi <- xi + alpha nu        (x += alpha p is alpha pt, minus W alpha nu),
//   nu <- mu + beta nu         (p' = z + beta p - W mu = pt' - W nu'),
//   a  <- c + beta a           (a = (A W)^T pt, by the same recurrence),
//   gcorr = nu^T a             (for the next update's gamma).
// YB is the basis tier of the update kernel (the layout of its partials).
template <int YB>
__global__ __launch_bounds__(kBlock) void k_dir_imp(DevBufs B, int y, double* __restrict__ p,
                                                    double* __restrict__ x, const double* __restrict__ z,
                                                    int k, int nbu) {
    constexpr int NV = 2 + YB;
    __shared__ double lds[kWavesPerBlock * NV + NV + 1];
    __shared__ double smu[YB > 0 ? YB : 1];
    __shared__ double sgi[YB > 0 ? YB * YB : 1];
    DevState* st = B.st;
    if (k >= st->stop) return;
    double ga[NV];
    dir_partials<NV>(B, nbu, ga);
    // workgroup 0's inputs of the coefficient recurrences (G^{-1}, nu, a, xi)
    // are requested up front as well, so its work after the streaming needs no
    // memory round trip
    const int par = k & 1;
    constexpr int kGi = YB > 0 ? (YB * YB + kBlock - 1) / kBlock : 1;
    double gi[kGi], nu_old = 0.0, acc_old = 0.0, xi_old = 0.0;
    if (YB > 0 && blockIdx.x == 0) {
#pragma unroll
        for (int u = 0; u < kGi; ++u) {
            const int e = threadIdx.x + u * kBlock;
            gi[u] = e < y * y ? B.Ginv[e] : 0.0;
        }
        if ((int)threadIdx.x < y) {
            nu_old = st->lnu[par][threadIdx.x];
            acc_old = st->lacc[par][threadIdx.x];
            xi_old = st->xi[threadIdx.x];
        }
    }
    const int n = B.n;
    const int stride = gridDim.x * kBlock;
    // the operands of this thread's first kPrefetch elements (all of them at
    // the default grid and 128^3) are in flight while the reduction is
    // finished, so the memory system stays busy during the prologue
    constexpr int kPrefetch = 8;
    const int i0 = blockIdx.x * kBlock + threadIdx.x;
    double pf[kPrefetch], zf[kPrefetch], xf[kPrefetch];
#pragma unroll
    for (int u = 0; u < kPrefetch; ++u) {
        const int i = i0 + u * stride;
        pf[u] = i < n ? p[i] : 0.0;
        zf[u] = i < n ? z[i] : 0.0;
        xf[u] = i < n ? x[i] : 0.0;
    }
    if (YB > 0 && blockIdx.x == 0) {   // visible to wave 0 after dir_begin's barriers
#pragma unroll
        for (int u = 0; u < kGi; ++u) {
            const int e = threadIdx.x + u * kBlock;
            if (e < y * y) sgi[e] = gi[u];
        }
    }
    DirStep d;
    if (!dir_begin<NV, YB, false>(B, y, k, ga, lds, smu, nullptr, d)) return;
#pragma unroll
    for (int u = 0; u < kPrefetch; ++u) {
        const int i = i0 + u * stride;
        if (i < n) {
            x[i] = xf[u] + d.alpha * pf[u];
            if (d.new_dir) p[i] = zf[u] + d.beta * pf[u];
        }
    }
    for (int i = i0 + kPrefetch * stride; i < n; i += stride) {
        const double pi = p[i];
        x[i] += d.alpha * pi;
        if (d.new_dir) p[i] = z[i] + d.beta * pi;
    }
    if (blockIdx.x == 0 && threadIdx.x < kWave) {
        // mu = G^{-1} c is needed here only (the direction pt carries no basis)
        const int j = threadIdx.x;
        double prod = 0.0;
        if (j < y) {
            double mu = 0.0;
            for (int i = 0; i < y; ++i) mu += sgi[j * y + i] * lds[2 + i];
            st->xi[j] = xi_old + d.alpha * nu_old;
            const double nu_new = mu + d.beta * nu_old;
            const double a_new = lds[2 + j] + d.beta * acc_old;
            st->lnu[par ^ 1][j] = nu_new;
            st->lacc[par ^ 1][j] = a_new;
            prod = nu_new * a_new;
        }
        prod = wave_sum(prod);
        if (j == 0) st->lgcorr[par ^ 1] = prod;
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
        st->lrho[0] = rz;
        st->rr = rr;
        st->rr0 = rr;
        if (!is_finite(rr) || !is_finite(rz)) {
            st->status = kStNonfinite;
            st->done = kFailed;
            st->stop = 0;
        } else if (rr <= st->tol2) {
            st->status = kStOk;
            st->done = kFinished;
            st->stop = 0;
        } else if (st->maxit <= 0) {
            st->status = kStNotConverged;
            st->done = kFinished;
            st->stop = 0;
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
                st->lnu[0][k] = s;
                st->lacc[0][k] = lds[2 + k];
                st->xi[k] = 0.0;
                prod = s * lds[2 + k];
            }
        }
        if (imp) {
            prod = wave_sum(prod);
            if (k == 0) st->lgcorr[0] = prod;
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
// with T = diag(w) V_y Sigma_y^{-1}).  y is the rank the eigen-solve wrote to
// *ydev, at most ymax.
template <int KB>
__global__ __launch_bounds__(kBlock) void k_pod_form(int n, size_t ld, const double* __restrict__ S,
                                                     int count, const double* __restrict__ T, int ymax,
                                                     const int* __restrict__ ydev, double* __restrict__ W) {
    __shared__ double t[kYMax * kYMax];
    const int yd = *ydev;
    const int y = yd < 0 ? 0 : (yd < ymax ? yd : ymax);
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

// Batched POD form: W = S T for every member with a POD (aux.count > 0), over
// the vector work list (row ranges of one member); the member's rank is read
// on the device, as in k_pod_form.
template <int KB>
__global__ __launch_bounds__(kBlock) void k_batch_pod_form(const BatchMember* __restrict__ mem,
                                                           const BatchAux* __restrict__ aux,
                                                           const BatchItem* __restrict__ items, int nitems) {
    __shared__ double t[kYMax * kYMax];
    const int G = gridDim.x;
    for (int base = 0; base < nitems; base += G) {
        const int m = min(G, nitems - base);
        if ((int)blockIdx.x >= m) break;
        const BatchItem it = items[base + xcd_block(blockIdx.x, m)];
        const BatchAux& A = aux[it.member];
        const int count = A.count;
        if (count < 1) continue;
        const size_t ld = mem[it.member].B.ld;
        const int ymax = count < A.rank_max ? count : A.rank_max;
        const int yd = *A.yout;
        const int y = yd < 0 ? 0 : (yd < ymax ? yd : ymax);
        __syncthreads();   // the previous item's reads of t are done
        for (int e = threadIdx.x; e < count * y; e += kBlock) t[e] = A.T[e];
        __syncthreads();
        for (int i = it.begin + (int)threadIdx.x; i < it.end; i += kBlock) {
            double sv[KB];
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                const double v = A.S[(size_t)(k < count ? k : count - 1) * ld + i];
                sv[k] = k < count ? v : 0.0;
            }
            for (int c = 0; c < y; ++c) {
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < KB; ++k)
                    if (k < count) acc += sv[k] * t[k * y + c];
                A.W[(size_t)c * ld + i] = acc;
            }
        }
    }
}

// Batched snapshot push: column aux.slot of every member's ring = aux.src,
// over the vector work list.
__global__ __launch_bounds__(kBlock) void k_batch_push(const BatchMember* __restrict__ mem,
                                                       const BatchAux* __restrict__ aux,
                                                       const BatchItem* __restrict__ items, int nitems) {
    const int G = gridDim.x;
    for (int base = 0; base < nitems; base += G) {
        const int m = min(G, nitems - base);
        if ((int)blockIdx.x >= m) break;
        const BatchItem it = items[base + xcd_block(blockIdx.x, m)];
        const BatchAux& A = aux[it.member];
        double* dst = A.S + (size_t)A.slot * mem[it.member].B.ld;
        for (int i = it.begin + (int)threadIdx.x; i < it.end; i += kBlock) dst[i] = A.src[i];
    }
}

// dst[(i / 64) 64 y + 64 j + i mod 64] = src[j ld + i] for i < ld, j < y.
__global__ __launch_bounds__(kBlock) void k_tile_columns(const double* __restrict__ src, size_t ld, int y,
                                                         double* __restrict__ dst) {
    const size_t total = ld * (size_t)y;
    const size_t tile = (size_t)kSlice * y;
    for (size_t e = blockIdx.x * (size_t)kBlock + threadIdx.x; e < total; e += (size_t)gridDim.x * kBlock) {
        const size_t t = e / tile, rem = e % tile;
        const size_t j = rem / kSlice, l = rem % kSlice;
        dst[e] = src[j * ld + t * kSlice + l];
    }
}

__global__ __launch_bounds__(kBlock) void k_copy(const double* __restrict__ a, double* __restrict__ c,
                                                 size_t n) {
    for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
        c[i] = a[i];
}

__device__ void state_init(DevState* st, int maxit, double tol2, int y, int implicit) {
    st->implicit = implicit;
    st->stop = maxit;
    for (int h = 0; h < 2; ++h) {
        st->lrho[h] = st->lalpha[h] = st->lgamma[h] = st->lgcorr[h] = 0.0;
        for (int k = 0; k < kYMax; ++k) st->lnu[h][k] = st->lacc[h][k] = 0.0;
    }
    for (int k = 0; k < kYMax; ++k) st->xi[k] = 0.0;
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

__global__ void k_state_init(DevState* st, int maxit, double tol2, int y, int implicit) {
    if (threadIdx.x == 0) state_init(st, maxit, tol2, y, implicit);
}

// Batched: thread m initialises member m.
__global__ void k_batch_state_init(const BatchMember* __restrict__ mem, const BatchSetup* __restrict__ su,
                                   int count) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < count) state_init(mem[m].B.st, su[m].maxit, su[m].tol2, mem[m].y, mem[m].implicit);
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
        st->lrho[0] = rz;
        st->rr = rr;
        st->rr0 = rr;
        // the inner solve aims at inner_rtol relative to its own right-hand
        // side, but never below half of the outer target (st->tol2 holds
        // rtol^2 ||b||^2 from the residual kernel)
        st->tol2 = fmax(inner_rtol2 * rr, 0.25 * st->tol2);
        if (!is_finite(rr) || !is_finite(rz)) {
            st->status = kStNonfinite;
            st->done = kFailed;
            st->stop = 0;
        } else if (rr == 0.0 || st->maxit <= 0) {
            st->status = rr == 0.0 ? kStOk : kStNotConverged;
            st->done = kFinished;
            st->stop = 0;
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

int update_blocks(const DevBufs& B) { return vec_grid(B.n, B.update_grid); }

hipError_t launch_update(const DevBufs& B, int yb, int y, double* r, double* z, const double* q,
                         const double* AW, int k, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    dim3 g(update_blocks(B)), t(kBlock);
    const int nsp = spmv_blocks(B);
    switch (yb) {
#define CASE(T) case T: PODCG_LAUNCH((k_update<double, T, true>), g, t, s, e0, e1, B, y, r, z, q, AW, k, nsp); break;
        PODCG_TIERS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_update_implicit(const DevBufs& B, int yb, int y, double* r, double* z, const double* qt,
                                  const double* AW, int k, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (y < 1) return hipErrorInvalidValue;
    dim3 g(update_blocks(B)), t(kBlock);
    const int nsp = spmv_blocks(B);
    switch (yb) {
#define CASE(T) case T: PODCG_LAUNCH((k_update_imp<T>), g, t, s, e0, e1, B, y, r, z, qt, AW, k, nsp); break;
        PODCG_POS_TIERS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dir_implicit(const DevBufs& B, int yb, int y, double* p, double* x, const double* z, int k,
                               hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (y < 1) return hipErrorInvalidValue;
    dim3 g(vec_grid(B.n, B.dir_grid)), t(kBlock);
    const int nbu = update_blocks(B);
    switch (yb) {
#define CASE(T) case T: PODCG_LAUNCH((k_dir_imp<T>), g, t, s, e0, e1, B, y, p, x, z, k, nbu); break;
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
                      const double* W, bool init, int k, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    dim3 g(vec_grid(B.n, B.dir_grid)), t(kBlock);
    const DirRecord none{};
    const int nbu = update_blocks(B);
    switch (yb) {
#define CASE(T)                                                                                    \
    case T:                                                                                        \
        if (init) PODCG_LAUNCH((k_dir<double, T, true, true>), g, t, s, e0, e1, B, y, p, x, z, W, none, k, nbu); \
        else PODCG_LAUNCH((k_dir<double, T, false, true>), g, t, s, e0, e1, B, y, p, x, z, W, none, k, nbu);     \
        break;
        PODCG_TIERS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dir_rec(const DevBufs& B, int yb, int y, double* p, double* x, const double* z,
                          const double* W, double* V, size_t ldv, int cap, double* gamma,
                          double* alpha, int k, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    dim3 g(vec_grid(B.n, B.dir_grid)), t(kBlock);
    const DirRecord rec{V, ldv, cap, gamma, alpha};
    const int nbu = update_blocks(B);
    switch (yb) {
#define CASE(T) case T: PODCG_LAUNCH((k_dir<double, T, false, true, true>), g, t, s, e0, e1, B, y, p, x, z, W, rec, k, nbu); break;
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

hipError_t launch_pod_form(int n, size_t ld, const double* S, int count, const double* T, int ymax,
                           const int* ydev, double* W, hipStream_t s) {
    if (ymax < 1) return hipSuccess;
    dim3 g(vec_grid(n)), t(kBlock);
    switch (basis_tier(count)) {
#define CASE(K) case K: hipLaunchKernelGGL((k_pod_form<K>), g, t, 0, s, n, ld, S, count, T, ymax, ydev, W); break;
        PODCG_POS_TIERS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch_pod_form(int kb, const BatchMember* mem, const BatchAux* aux, const BatchItem* items,
                                 int nitems, int grid, hipStream_t s) {
    if (nitems < 1) return hipSuccess;
    const dim3 g(grid < nitems ? grid : nitems), t(kBlock);
    switch (basis_tier(kb)) {
#define CASE(K) case K: hipLaunchKernelGGL((k_batch_pod_form<K>), g, t, 0, s, mem, aux, items, nitems); break;
        PODCG_POS_TIERS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch_push(const BatchMember* mem, const BatchAux* aux, const BatchItem* items, int nitems,
                             int grid, hipStream_t s) {
    if (nitems < 1) return hipSuccess;
    hipLaunchKernelGGL(k_batch_push, dim3(grid < nitems ? grid : nitems), dim3(kBlock), 0, s, mem, aux, items,
                       nitems);
    return hipGetLastError();
}

hipError_t launch_tile_columns(const double* src, size_t ld, int y, double* dst, hipStream_t s) {
    if (y < 1 || ld % kSlice != 0) return hipErrorInvalidValue;
    int64_t g = (int64_t)((ld * (size_t)y + kBlock - 1) / kBlock);
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_tile_columns, dim3((int)g), dim3(kBlock), 0, s, src, ld, y, dst);
    return hipGetLastError();
}

hipError_t launch_copy(const double* src, double* dst, size_t n, hipStream_t s) {
    int64_t g = ((int64_t)n + kBlock - 1) / kBlock;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_copy, dim3((int)g), dim3(kBlock), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_batch_state_init(const BatchMember* mem, const BatchSetup* su, int count, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_state_init, dim3((count + 63) / 64), dim3(64), 0, s, mem, su, count);
    return hipGetLastError();
}

hipError_t launch_state_init(DevState* st, int maxit, double tol2, int y, hipStream_t s, bool implicit) {
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, st, maxit, tol2, y, implicit ? 1 : 0);
    return hipGetLastError();
}

}  // namespace podcg

namespace podcg {

hipError_t launch_update32(const DevBufs& B, int yb, int y, float* r, float* z, const float* q,
                           const float* AW, int k, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    dim3 g(update_blocks(B)), t(kBlock);
    const int nsp = spmv_blocks(B);
    switch (yb) {
#define CASE(T) case T: PODCG_LAUNCH((k_update<float, T, true>), g, t, s, e0, e1, B, y, r, z, q, AW, k, nsp); break;
        PODCG_TIERS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dir32(const DevBufs& B, int yb, int y, float* p, double* x, const float* z,
                        const float* W, bool init, int k, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    dim3 g(vec_grid(B.n, B.dir_grid)), t(kBlock);
    const DirRecord none{};
    const int nbu = update_blocks(B);
    switch (yb) {
#define CASE(T)                                                                                    \
    case T:                                                                                        \
        if (init) PODCG_LAUNCH((k_dir<float, T, true, true>), g, t, s, e0, e1, B, y, p, x, z, W, none, k, nbu);  \
        else PODCG_LAUNCH((k_dir<float, T, false, true>), g, t, s, e0, e1, B, y, p, x, z, W, none, k, nbu);      \
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
