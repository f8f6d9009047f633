// Batched loop kernels: one launch per loop kernel advances augmented PCG
// (Alg. 1) of many independent sequences at once.
//
// The work of an iteration is cut into items, contiguous ranges of one
// member (SELL slices for the SpMV, rows for the vector kernels).  A fixed
// grid walks the compacted item list in rounds; within a round, workgroup b
// takes item xcd_block(b, m), so each XCD covers a contiguous range of items
// and the neighbouring rows of a member share one L2.  Every item reduces its
// partial sums and stores them in its member's slot; the last item of a
// member to arrive (arrival counter per member) sums the member's slots in a
// fixed order and forms that member's scalars, exactly as the last workgroup
// of the single-sequence kernels does.  Results are deterministic for a given
// item partition.  A member with a single item reduces inside its workgroup
// and never touches global memory for the sums.
//
// Members that have finished (or failed) drop out of the lists at the start of
// every block of iterations (k_batch_compact); within a block they exit on
// their state flag.
#include "podcg_launch.h"

namespace podcg {

int batch_tier(int y) {
    static const int tiers[] = {0, 1, 2, 4, 6, 8, 12, 16, 24, 32};
    for (int t : tiers)
        if (y <= t) return t;
    return -1;
}

#define PODCG_BATCH_TIERS(X) X(0) X(1) X(2) X(4) X(6) X(8) X(12) X(16) X(24) X(32)

namespace {

// Column index of a batched basis load: clamped into [0, y) so every load of
// the unrolled tier is unconditional and in bounds (y >= 1 is checked by the
// caller).
__device__ __forceinline__ int bcol(int k, int y) { return k < y ? k : y - 1; }

// Sum of NV values over the items of one member.  Returns true in the last
// item to arrive, with the member totals in lds[0..NV).
template <int NV>
__device__ __forceinline__ bool member_sum_last(double (&v)[NV], double* part, unsigned* counter,
                                                int nitems, int local, double* lds) {
    block_sum<NV>(v, lds);
    if (nitems == 1) return true;
    const int t = threadIdx.x;
    if (t < NV) store_shared(part + (size_t)t * nitems + local, lds[t]);
    if (!arrive_last(counter, nitems)) return false;
    double a[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) a[k] = 0.0;
    for (int i = t; i < nitems; i += kBlock) {
#pragma unroll
        for (int k = 0; k < NV; ++k) a[k] += load_shared(part + (size_t)k * nitems + i);
    }
    block_sum<NV>(a, lds);
    return true;
}

// Marks a member that leaves the running state inside a loop kernel.
__device__ __forceinline__ void leave_running(int* active) {
    __hip_atomic_fetch_add(active, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace

// q = A p, gamma = (A p, p), alpha = (r, z) / gamma per member.
__global__ __launch_bounds__(kBlock) void k_batch_spmv(const BatchMember* __restrict__ mem,
                                                       const BatchItem* __restrict__ items,
                                                       const int* __restrict__ counts,
                                                       int* __restrict__ active) {
    __shared__ double lds[kWavesPerBlock + 2];
    const int nitems = counts[0];
    const int G = gridDim.x;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    for (int base = 0; base < nitems; base += G) {
        const int m = min(G, nitems - base);
        if ((int)blockIdx.x >= m) break;
        const BatchItem it = items[base + xcd_block(blockIdx.x, m)];
        const BatchMember& M = mem[it.member];
        DevState* st = M.B.st;
        const int done = st->done;
        __syncthreads();   // every thread has read the flag before anyone may change it
        if (done != kRunning) {
            if ((done == kConvergedPending || done == kCapPending) && it.local == 0 && threadIdx.x == 0)
                st->done = kFinished;
            continue;
        }
        const double* __restrict__ p = M.p;
        double* __restrict__ q = M.q;
        double g[1] = {0.0};
        // two slices a wave, two rows a lane (spmv_slice_pair)
        for (int s = it.begin + 2 * wid; s < it.end; s += 2 * kWavesPerBlock)
            spmv_slice_pair(M.B, s, s + 1 < it.end, lane, p, q, g[0]);
        if (member_sum_last<1>(g, M.B.part, M.B.counter, M.spmv_items, it.local, lds) &&
            threadIdx.x == 0) {
            // implicit form: p = pt - W nu and (A p, p) = (A pt, pt) - nu^T a (slot 0 of the state)
            const double gamma = lds[0] - (M.implicit ? st->lgcorr[0] : 0.0);
            st->gamma = gamma;
            if (!(gamma > 0.0) || !is_finite(gamma)) {
                st->status = is_finite(gamma) ? kStNotSpd : kStNonfinite;
                st->done = kFailed;
                leave_running(active);
            } else {
                st->alpha = st->rho / gamma;
            }
        }
        __syncthreads();   // lds is reused by the next item
    }
}

// r -= alpha q, z = M^{-1} r, sums (r, z), (r, r), (A W)^T z; the last item of
// a member forms beta, mu = G^{-1} (A W)^T z and tests convergence.  Only z is
// stored: with Jacobi r = M z is recovered as z / dinv, as in k_update.  For a
// member in the implicit form the SpMV multiplied pt, so A p = q - (A W) nu is
// formed from the A W columns loaded for the sums, and the last item advances
// xi += alpha nu, nu = mu + beta nu, a = c + beta a and nu^T a (state slot 0).
template <int YB>
__global__ __launch_bounds__(kBlock) void k_batch_update(const BatchMember* __restrict__ mem,
                                                         const BatchItem* __restrict__ items,
                                                         const int* __restrict__ counts,
                                                         int* __restrict__ active) {
    constexpr int NV = 2 + YB;
    __shared__ double lds[kWavesPerBlock * NV + NV + 1];
    const int nitems = counts[1];
    const int G = gridDim.x;
    for (int base = 0; base < nitems; base += G) {
        const int m = min(G, nitems - base);
        if ((int)blockIdx.x >= m) break;
        const BatchItem it = items[base + xcd_block(blockIdx.x, m)];
        const BatchMember& M = mem[it.member];
        DevState* st = M.B.st;
        if (st->done != kRunning) continue;   // only this kernel's last item changes it
        const double alpha = st->alpha;
        const int y = M.y;
        double* __restrict__ z = M.z;
        const double* __restrict__ q = M.q;
        const double* __restrict__ dinv = M.B.dinv;
        const double* __restrict__ AW = M.AW;
        const size_t ld = M.B.ld;
        const bool imp = M.implicit != 0;
        double nu[YB > 0 ? YB : 1];
#pragma unroll
        for (int k = 0; k < YB; ++k) nu[k] = (imp && k < y) ? st->lnu[0][k] : 0.0;
        double v[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] = 0.0;
        for (int i = it.begin + (int)threadIdx.x; i < it.end; i += kBlock) {
            double a[YB > 0 ? YB : 1];
            double qi = q[i];
            if (YB > 0 && y > 0) {
#pragma unroll
                for (int k = 0; k < YB; ++k) {
                    a[k] = __builtin_nontemporal_load(AW + (size_t)bcol(k, y) * ld + i);
                    if (imp && k < y) qi -= a[k] * nu[k];
                }
            }
            // r = M z (Jacobi): only z is stored, r recovered
            const double di = dinv[i];
            const double ri = z[i] / di - alpha * qi;
            const double zi = di * ri;
            z[i] = zi;
            v[0] += ri * zi;
            v[1] += ri * ri;
            if (YB > 0 && y > 0) {
#pragma unroll
                for (int k = 0; k < YB; ++k)
                    if (k < y) v[2 + k] += a[k] * zi;
            }
        }
        if (member_sum_last<NV>(v, M.B.part, M.B.counter, M.vec_items, it.local, lds)) {
            if (threadIdx.x == 0) {
                const double rz = lds[0], rr = lds[1];
                const int iter = st->iter + 1;
                st->iter = iter;
                st->rr = rr;
                double beta = 0.0, stepped = 1.0;
                if (!is_finite(rr) || !is_finite(rz)) {
                    st->status = kStNonfinite;
                    st->done = kFailed;
                    leave_running(active);
                    stepped = 0.0;
                } else {
                    beta = rz / st->rho;
                    st->beta = beta;
                    st->rho = rz;
                    if (rr <= st->tol2) {
                        st->status = kStOk;
                        st->done = kConvergedPending;
                        leave_running(active);
                    } else if (iter >= st->maxit) {
                        st->status = kStNotConverged;
                        st->done = kCapPending;
                        leave_running(active);
                    }
                }
                lds[NV] = beta;
                lds[NV + 1] = stepped;
            }
            __syncthreads();
            if ((int)threadIdx.x < kWave) {
                const int k = threadIdx.x;
                double prod = 0.0;
                if (k < y) {
                    double s = 0.0;
                    for (int j = 0; j < y; ++j) s += M.B.Ginv[k * y + j] * lds[2 + j];
                    st->mu[k] = s;
                    if (imp) {
                        const double beta = lds[NV];
                        const double nu_old = st->lnu[0][k];
                        if (lds[NV + 1] != 0.0) st->xi[k] += alpha * nu_old;
                        const double nu_new = s + beta * nu_old;
                        const double a_new = lds[2 + k] + beta * st->lacc[0][k];
                        st->lnu[0][k] = nu_new;
                        st->lacc[0][k] = a_new;
                        prod = nu_new * a_new;
                    }
                }
                if (imp) {
                    prod = wave_sum(prod);
                    if (k == 0) st->lgcorr[0] = prod;
                }
            }
        }
        __syncthreads();   // lds is reused by the next item
    }
}

// x += alpha p; while iterating p = z + beta p - W mu (p = z + beta p for a
// member in the implicit form, whose basis term is carried by nu).
template <int YB>
__global__ __launch_bounds__(kBlock) void k_batch_dir(const BatchMember* __restrict__ mem,
                                                      const BatchItem* __restrict__ items,
                                                      const int* __restrict__ counts) {
    const int nitems = counts[1];
    const int G = gridDim.x;
    for (int base = 0; base < nitems; base += G) {
        const int m = min(G, nitems - base);
        if ((int)blockIdx.x >= m) break;
        const BatchItem it = items[base + xcd_block(blockIdx.x, m)];
        const BatchMember& M = mem[it.member];
        const DevState* st = M.B.st;
        const int done = st->done;
        if (done != kRunning && done != kConvergedPending && done != kCapPending) continue;
        const bool new_dir = done == kRunning;
        const double alpha = st->alpha, beta = st->beta;
        const int y = M.y;
        double mu[YB > 0 ? YB : 1];
#pragma unroll
        for (int k = 0; k < YB; ++k) mu[k] = k < y ? st->mu[k] : 0.0;
        double* __restrict__ p = M.p;
        double* __restrict__ x = M.x;
        const double* __restrict__ z = M.z;
        const double* __restrict__ W = M.W;
        const size_t ld = M.B.ld;
        for (int i = it.begin + (int)threadIdx.x; i < it.end; i += kBlock) {
            const double pi = p[i];
            x[i] += alpha * pi;
            if (!new_dir) continue;
            double s = z[i] + beta * pi;
            if (YB > 0 && y > 0 && !M.implicit) {
#pragma unroll
                for (int k = 0; k < YB; ++k)
                    s -= __builtin_nontemporal_load(W + (size_t)bcol(k, y) * ld + i) * mu[k];
            }
            p[i] = s;
        }
    }
}

// Rebuilds the SpMV and vector lists from the members still running (or with
// their last update x += alpha p pending) and counts the running members.
// One workgroup.
__global__ __launch_bounds__(kBlock) void k_batch_compact(const BatchMember* __restrict__ mem,
                                                          int count,
                                                          const BatchItem* __restrict__ spmv_full,
                                                          const BatchItem* __restrict__ vec_full,
                                                          BatchItem* __restrict__ spmv,
                                                          BatchItem* __restrict__ vec,
                                                          int* __restrict__ counts,
                                                          int* __restrict__ active) {
    __shared__ int keep[kBatchMaxMembers];
    __shared__ int run[kBatchMaxMembers];
    __shared__ int off_s[kBatchMaxMembers], off_v[kBatchMaxMembers];
    const int t = threadIdx.x;
    for (int m = t; m < count; m += kBlock) {
        const int d = mem[m].B.st->done;
        keep[m] = d == kRunning || d == kConvergedPending || d == kCapPending;
        run[m] = d == kRunning;
    }
    __syncthreads();
    if (t == 0) {
        int ns = 0, nv = 0, na = 0;
        for (int m = 0; m < count; ++m) {
            off_s[m] = ns;
            off_v[m] = nv;
            if (keep[m]) {
                ns += mem[m].spmv_items;
                nv += mem[m].vec_items;
            }
            na += run[m];
        }
        counts[0] = ns;
        counts[1] = nv;
        *active = na;
    }
    __syncthreads();
    for (int m = 0; m < count; ++m) {
        if (!keep[m]) continue;
        const BatchMember& M = mem[m];
        for (int i = t; i < M.spmv_items; i += kBlock) spmv[off_s[m] + i] = spmv_full[M.spmv_first + i];
        for (int i = t; i < M.vec_items; i += kBlock) vec[off_v[m] + i] = vec_full[M.vec_first + i];
    }
}

// Copies the polled block of every member's state into one array.
__global__ void k_batch_gather(const BatchMember* __restrict__ mem, int count, PollBlock* out) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= count) return;
    const DevState* st = mem[m].B.st;
    PollBlock P;
    P.iter = st->iter;
    P.done = st->done;
    P.status = st->status;
    P.y = st->y;
    P.maxit = st->maxit;
    P.pad0 = P.stop = P.pad2 = 0;
    P.rr = st->rr;
    P.rr0 = st->rr0;
    P.bnorm2 = st->bnorm2;
    P.true_rr = st->true_rr;
    out[m] = P;
}

// ------------------------------------------------------------------ launchers

hipError_t launch_batch_compact(const BatchMember* mem, int count, const BatchItem* spmv_full,
                                const BatchItem* vec_full, BatchItem* spmv, BatchItem* vec,
                                int* counts, int* active, hipStream_t s) {
    if (count < 1 || count > kBatchMaxMembers) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_batch_compact, dim3(1), dim3(kBlock), 0, s, mem, count, spmv_full, vec_full,
                       spmv, vec, counts, active);
    return hipGetLastError();
}

hipError_t launch_batch_spmv(const BatchMember* mem, const BatchItem* items, const int* counts,
                             int* active, int grid, hipStream_t s) {
    if (grid < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_batch_spmv, dim3(grid), dim3(kBlock), 0, s, mem, items, counts, active);
    return hipGetLastError();
}

hipError_t launch_batch_update(int yb, const BatchMember* mem, const BatchItem* items,
                               const int* counts, int* active, int grid, hipStream_t s) {
    if (grid < 1) return hipErrorInvalidValue;
    switch (yb) {
#define CASE(T) case T: hipLaunchKernelGGL((k_batch_update<T>), dim3(grid), dim3(kBlock), 0, s, mem, items, counts, active); break;
        PODCG_BATCH_TIERS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch_dir(int yb, const BatchMember* mem, const BatchItem* items, const int* counts,
                            int grid, hipStream_t s) {
    if (grid < 1) return hipErrorInvalidValue;
    switch (yb) {
#define CASE(T) case T: hipLaunchKernelGGL((k_batch_dir<T>), dim3(grid), dim3(kBlock), 0, s, mem, items, counts); break;
        PODCG_BATCH_TIERS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ batched Stage 1
// The single-sequence Stage 1 (k_resid, k_stage1_apply and the first
// direction) for all members in three launches over the work lists; each
// member's sums are reduced by its last item, as in the loop kernels.

// rbar = b - A xbar with (b, b), (rbar, rbar), W^T rbar per member; the last
// item sets ||b||^2, the absolute tolerance and what = G^{-1} W^T rbar (Alg. 2).
template <int YB>
__global__ __launch_bounds__(kBlock) void k_batch_resid(const BatchMember* __restrict__ mem,
                                                        const BatchSetup* __restrict__ su,
                                                        const BatchItem* __restrict__ items, int nitems) {
    constexpr int NV = 2 + YB;
    __shared__ double lds[kWavesPerBlock * NV + NV + 1];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int G = gridDim.x;
    for (int base = 0; base < nitems; base += G) {
        const int m = min(G, nitems - base);
        if ((int)blockIdx.x >= m) break;
        const BatchItem it = items[base + xcd_block(blockIdx.x, m)];
        const BatchMember& M = mem[it.member];
        DevState* st = M.B.st;
        if (st->done != kRunning) continue;
        const double* __restrict__ b = su[it.member].b;
        const double* __restrict__ W = M.W;
        const size_t ld = M.B.ld;
        const int y = M.y;
        double v[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] = 0.0;
        for (int s = it.begin + wid; s < it.end; s += kWavesPerBlock) {
            const double ax = sell_row<double>(M.B, M.B.vals, s, lane, M.x);
            const int row = s * kSlice + lane;
            if (row < M.B.n) {
                const double bi = b[row];
                const double ri = bi - ax;
                M.r[row] = ri;
                v[0] += bi * bi;
                v[1] += ri * ri;
                if (YB > 0 && y > 0) {
#pragma unroll
                    for (int k = 0; k < YB; ++k) {
                        const double wk = W[(size_t)bcol(k, y) * ld + row];
                        if (k < y) v[2 + k] += wk * ri;
                    }
                }
            }
        }
        if (member_sum_last<NV>(v, M.B.part, M.B.counter, M.spmv_items, it.local, lds)) {
            if (threadIdx.x == 0) {
                const double bb = lds[0];
                st->bnorm2 = bb;
                st->true_rr = lds[1];
                st->tol2 = st->tol2 * bb;
                if (!is_finite(bb) || !is_finite(lds[1])) {
                    st->status = kStNonfinite;
                    st->done = kFailed;
                    st->stop = 0;
                }
            }
            if ((int)threadIdx.x < y) {
                double sum = 0.0;
                for (int j = 0; j < y; ++j) sum += M.B.Ginv[threadIdx.x * y + j] * lds[2 + j];
                st->what[threadIdx.x] = sum;
            }
        }
        __syncthreads();   // lds is reused by the next item
    }
}

// x <- xbar + W what, r <- rbar - (A W) what, z = M^{-1} r, with (r, z),
// (r, r), c = (A W)^T z per member; the last item sets mu = G^{-1} c, tests
// the Stage-1 residual, and for the implicit form starts nu = mu, a = c,
// xi = 0.  A member in the implicit form gets its first direction pt = z here.
template <int YB>
__global__ __launch_bounds__(kBlock) void k_batch_stage1(const BatchMember* __restrict__ mem,
                                                         const BatchItem* __restrict__ items, int nitems) {
    constexpr int NV = 2 + YB;
    __shared__ double lds[kWavesPerBlock * NV + NV + 1];
    const int G = gridDim.x;
    for (int base = 0; base < nitems; base += G) {
        const int m = min(G, nitems - base);
        if ((int)blockIdx.x >= m) break;
        const BatchItem it = items[base + xcd_block(blockIdx.x, m)];
        const BatchMember& M = mem[it.member];
        DevState* st = M.B.st;
        if (st->done != kRunning) continue;
        const int y = M.y;
        const bool imp = M.implicit != 0;
        const size_t ld = M.B.ld;
        double what[YB > 0 ? YB : 1];
#pragma unroll
        for (int k = 0; k < YB; ++k) what[k] = k < y ? st->what[k] : 0.0;
        double v[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] = 0.0;
        for (int i = it.begin + (int)threadIdx.x; i < it.end; i += kBlock) {
            double ri = M.r[i];
            if (YB > 0 && y > 0) {
                double wx = 0.0, awx = 0.0;
#pragma unroll
                for (int k = 0; k < YB; ++k) {
                    const int kc = bcol(k, y);
                    wx += M.W[(size_t)kc * ld + i] * what[k];
                    awx += M.AW[(size_t)kc * ld + i] * what[k];
                }
                M.x[i] += wx;
                ri -= awx;
                M.r[i] = ri;
            }
            const double zi = M.B.dinv[i] * ri;
            M.z[i] = zi;
            if (imp) M.p[i] = zi;
            v[0] += ri * zi;
            v[1] += ri * ri;
            if (YB > 0 && y > 0) {
#pragma unroll
                for (int k = 0; k < YB; ++k) {
                    const double a = M.AW[(size_t)bcol(k, y) * ld + i];
                    if (k < y) v[2 + k] += a * zi;
                }
            }
        }
        if (member_sum_last<NV>(v, M.B.part, M.B.counter, M.vec_items, it.local, lds)) {
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
            if ((int)threadIdx.x < kWave) {
                const int k = threadIdx.x;
                double prod = 0.0;
                if (k < y) {
                    double sum = 0.0;
                    for (int j = 0; j < y; ++j) sum += M.B.Ginv[k * y + j] * lds[2 + j];
                    st->mu[k] = sum;
                    if (imp) {
                        st->lnu[0][k] = sum;
                        st->lacc[0][k] = lds[2 + k];
                        st->xi[k] = 0.0;
                        prod = sum * lds[2 + k];
                    }
                }
                if (imp) {
                    prod = wave_sum(prod);
                    if (k == 0) st->lgcorr[0] = prod;
                }
            }
        }
        __syncthreads();   // lds is reused by the next item
    }
}

// First direction of the members in the explicit form: p = z - W mu.
template <int YB>
__global__ __launch_bounds__(kBlock) void k_batch_dir_init(const BatchMember* __restrict__ mem,
                                                           const BatchItem* __restrict__ items, int nitems) {
    const int G = gridDim.x;
    for (int base = 0; base < nitems; base += G) {
        const int m = min(G, nitems - base);
        if ((int)blockIdx.x >= m) break;
        const BatchItem it = items[base + xcd_block(blockIdx.x, m)];
        const BatchMember& M = mem[it.member];
        const DevState* st = M.B.st;
        if (M.implicit || st->stop <= 0 || st->done != kRunning) continue;
        const int y = M.y;
        const size_t ld = M.B.ld;
        double mu[YB > 0 ? YB : 1];
#pragma unroll
        for (int k = 0; k < YB; ++k) mu[k] = k < y ? st->mu[k] : 0.0;
        for (int i = it.begin + (int)threadIdx.x; i < it.end; i += kBlock) {
            double sum = M.z[i];
            if (YB > 0 && y > 0) {
#pragma unroll
                for (int k = 0; k < YB; ++k) sum -= M.W[(size_t)bcol(k, y) * ld + i] * mu[k];
            }
            M.p[i] = sum;
        }
    }
}

// The tiled copy of A W (element (i, j) at (i / 64) 64 y + 64 j + i mod 64)
// that the single-sequence implicit update reads, for the members whose basis
// products were just formed; the member's last item also covers the padding
// rows up to the leading dimension.
template <int YB>
__global__ __launch_bounds__(kBlock) void k_batch_tile_aw(const BatchMember* __restrict__ mem,
                                                          const BatchSetup* __restrict__ su,
                                                          const BatchItem* __restrict__ items, int nitems) {
    const int G = gridDim.x;
    for (int base = 0; base < nitems; base += G) {
        const int m = min(G, nitems - base);
        if ((int)blockIdx.x >= m) break;
        const BatchItem it = items[base + xcd_block(blockIdx.x, m)];
        const BatchSetup& S = su[it.member];
        const BatchMember& M = mem[it.member];
        const int y = M.y;
        if (!S.setup || !S.AWt || y < 1) continue;
        const size_t ld = M.B.ld;
        const int end = it.end == M.B.n ? (int)ld : it.end;
        for (int i = it.begin + (int)threadIdx.x; i < end; i += kBlock) {
            const size_t tb = (size_t)(i / kSlice) * kSlice * y + (i % kSlice);
#pragma unroll
            for (int k = 0; k < YB; ++k)
                if (k < y) S.AWt[tb + (size_t)k * kSlice] = M.AW[(size_t)k * ld + i];
        }
    }
}

hipError_t launch_batch_resid(int yb, const BatchMember* mem, const BatchSetup* su, const BatchItem* items,
                              int nitems, int grid, hipStream_t s) {
    if (nitems < 1) return hipSuccess;
    const dim3 g(grid < nitems ? grid : nitems), t(kBlock);
    switch (yb) {
#define CASE(T) case T: hipLaunchKernelGGL((k_batch_resid<T>), g, t, 0, s, mem, su, items, nitems); break;
        PODCG_BATCH_TIERS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch_stage1(int yb, const BatchMember* mem, const BatchItem* items, int nitems, int grid,
                               hipStream_t s) {
    if (nitems < 1) return hipSuccess;
    const dim3 g(grid < nitems ? grid : nitems), t(kBlock);
    switch (yb) {
#define CASE(T) case T: hipLaunchKernelGGL((k_batch_stage1<T>), g, t, 0, s, mem, items, nitems); break;
        PODCG_BATCH_TIERS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch_dir_init(int yb, const BatchMember* mem, const BatchItem* items, int nitems, int grid,
                                 hipStream_t s) {
    if (nitems < 1) return hipSuccess;
    const dim3 g(grid < nitems ? grid : nitems), t(kBlock);
    switch (yb) {
#define CASE(T) case T: hipLaunchKernelGGL((k_batch_dir_init<T>), g, t, 0, s, mem, items, nitems); break;
        PODCG_BATCH_TIERS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch_tile_aw(int yb, const BatchMember* mem, const BatchSetup* su, const BatchItem* items,
                                int nitems, int grid, hipStream_t s) {
    if (nitems < 1 || yb < 1) return hipSuccess;
    const dim3 g(grid < nitems ? grid : nitems), t(kBlock);
    switch (yb) {
#define CASE(T) case T: hipLaunchKernelGGL((k_batch_tile_aw<T>), g, t, 0, s, mem, su, items, nitems); break;
        PODCG_BATCH_TIERS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch_gather(const BatchMember* mem, int count, PollBlock* out, hipStream_t s) {
    if (count < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_batch_gather, dim3((count + kBlock - 1) / kBlock), dim3(kBlock), 0, s, mem,
                       count, out);
    return hipGetLastError();
}

}  // namespace podcg
