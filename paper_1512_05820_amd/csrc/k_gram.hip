// The fused SpMM + Gram kernel of libpodcg: A X for k columns (optionally
// stored) and the k x k product X^T (A X) on the FP64 matrix cores, the
// products of Alg. 2 (W^T A W) and of Alg. pod_evd (S^T A S).
#include "podcg_launch.h"

namespace podcg {

// Fused AX = A X (optionally stored) and G = X^T (A X) for k <= KS columns,
// the products of Alg. 2 (W^T A W) and of Alg. pod_evd (S^T A S).  Each wave
// computes A X for one slice of 64 rows (lane = row), stages that block in
// LDS, and accumulates the 64-row contraction X^T (A X) on the FP64 matrix
// cores with v_mfma_f64_16x16x4f64: per instruction lane l supplies
// X[row 4 s + l / 16][col l % 16] (loaded directly) and
// (A X)[row 4 s + l / 16][col l % 16] (from LDS), and register r of lane l
// accumulates G[4 r + l / 16][l % 16].  Columns are padded to KB = 16 or 32
// (padding columns of A X are zero).
typedef double d4_t __attribute__((ext_vector_type(4)));
constexpr int kMfmaGroup = 4;   // MFMA steps (4 rows each) per X operand load group

template <int KS>
struct GramShape {
    static constexpr int KB = KS <= 16 ? 16 : 32;
    static constexpr int KT = KB / 16;
    static constexpr int LDSW = KS + 1;                        // padded row stride of a tile
    static constexpr int TILE = kSlice * LDSW;                 // doubles per wave tile
    static constexpr int RED = KT * KT * 4 * kWave;            // doubles per wave accumulator
    static constexpr int SH = kWavesPerBlock * (TILE > RED ? TILE : RED);
};

// Slice s (wave-uniform; s >= nslices adds nothing) of A X and X^T (A X):
// stores the slice's rows of A X when `store` is set and adds the slice's
// contraction to the accumulators d.  tw is this wave's LDS tile; only the
// calling wave touches it, so the only ordering needed is within the wave.
template <int KS>
__device__ __forceinline__ void gram_slice(const DevBufs& B, int k, const double* __restrict__ X,
                                           double* __restrict__ AX, int store, int s,
                                           d4_t (&d)[GramShape<KS>::KT][GramShape<KS>::KT], double* tw) {
    constexpr int KT = GramShape<KS>::KT;
    constexpr int LDSW = GramShape<KS>::LDSW;
    const int lane = threadIdx.x & (kWave - 1);
    const int r4 = lane >> 4, cc = lane & 15;
    const bool sv = s < B.nslices;
    double acc[KS];
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) acc[kk] = 0.0;
    const int row = s * kSlice + lane;
    // X operand of MFMA step st for column tile a: X[row 4 st + r4][col
    // 16 a + cc] of this slice (rows past n read row n - 1 and count as
    // zero; columns past k repeat column k - 1 and feed unused G rows).
    // Group 0 is loaded here, under the SpMM below.
    double xg[kMfmaGroup][KT];
    auto load_xgroup = [&](int g) {
#pragma unroll
        for (int u = 0; u < kMfmaGroup; ++u)
#pragma unroll
            for (int a = 0; a < KT; ++a) {
                const int grow = s * kSlice + 4 * (g * kMfmaGroup + u) + r4;
                const int colx = 16 * a + cc;
                const int colc = colx < k ? colx : k - 1;
                const double v = X[(size_t)colc * B.ld + (grow < B.n ? grow : B.n - 1)];
                xg[u][a] = grow < B.n ? v : 0.0;
            }
    };
    load_xgroup(0);
    if (sv) {
        const int64_t base = B.sptr[s];
        const int w = (int)((B.sptr[s + 1] - base) / kSlice);
        const int* c = B.cols + base + lane;
        const double* vv = B.vals + base + lane;
        // entry j + 1's value and column are loaded while entry j's k
        // gathers are in flight; a slice with an offset table computes the
        // column from its (scalar) offsets, with no index load at all
        const bool tabled = B.sflag[s] == 2;
        const int* __restrict__ tab = B.soff + (size_t)s * kTabMax;
        auto column = [&](int j) {
            if (tabled) {
                const int col = row + tab[j];
                return col < 0 ? 0 : (col < B.n ? col : B.n - 1);
            }
            return c[j * kSlice];
        };
        double a_next = vv[0];
        int col_next = column(0);
        for (int j = 0; j < w; ++j) {
            const double a = a_next;
            const int col = col_next;
            if (j + 1 < w) {
                a_next = vv[(j + 1) * kSlice];
                col_next = column(j + 1);
            }
            double xv[KS];
#pragma unroll
            for (int kk = 0; kk < KS; ++kk) xv[kk] = X[(size_t)(kk < k ? kk : k - 1) * B.ld + col];
#pragma unroll
            for (int kk = 0; kk < KS; ++kk) acc[kk] += a * xv[kk];
        }
        if (store && row < B.n) {
#pragma unroll
            for (int kk = 0; kk < KS; ++kk)
                if (kk < k) AX[(size_t)kk * B.ld + row] = acc[kk];
        }
    }
    const bool live = sv && row < B.n;
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) tw[lane * LDSW + kk] = (kk < k && live) ? acc[kk] : 0.0;
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    // the X operands of group g + 1 are in flight while group g's MFMAs run
    double xc[kMfmaGroup][KT];
#pragma unroll
    for (int u = 0; u < kMfmaGroup; ++u)
#pragma unroll
        for (int a = 0; a < KT; ++a) xc[u][a] = xg[u][a];
#pragma unroll
    for (int g = 0; g < kSlice / 4 / kMfmaGroup; ++g) {
        if (g + 1 < kSlice / 4 / kMfmaGroup) load_xgroup(g + 1);
#pragma unroll
        for (int u = 0; u < kMfmaGroup; ++u) {
            const int rr = 4 * (g * kMfmaGroup + u) + r4;
            double bb[KT];
#pragma unroll
            for (int b = 0; b < KT; ++b) {
                const int colx = 16 * b + cc;
                bb[b] = colx < KS ? tw[rr * LDSW + (colx < KS ? colx : 0)] : 0.0;
            }
#pragma unroll
            for (int a = 0; a < KT; ++a)
#pragma unroll
                for (int b = 0; b < KT; ++b)
                    d[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xc[u][a], bb[b], d[a][b], 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < kMfmaGroup; ++u)
#pragma unroll
            for (int a = 0; a < KT; ++a) xc[u][a] = xg[u][a];
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// The workgroup's k x k partial Gram: the four waves' accumulators summed in
// wave order through LDS (shm, which the wave tiles also use); output o = i k
// + j is owned by one thread, which calls emit(o, value).
template <int KS, class Emit>
__device__ __forceinline__ void gram_block_outputs(int k, d4_t (&d)[GramShape<KS>::KT][GramShape<KS>::KT],
                                                   double* shm, Emit&& emit) {
    constexpr int KT = GramShape<KS>::KT;
    constexpr int RED = GramShape<KS>::RED;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    __syncthreads();
    double* red = shm;
#pragma unroll
    for (int a = 0; a < KT; ++a)
#pragma unroll
        for (int b = 0; b < KT; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) red[wid * RED + ((a * KT + b) * 4 + r) * kWave + lane] = d[a][b][r];
    __syncthreads();
    for (int o = threadIdx.x; o < k * k; o += kBlock) {
        const int i = o / k, j = o % k;
        const int a = i / 16, b = j / 16, ii = i % 16, jj = j % 16;
        const int r = ii / 4, ln = (ii % 4) * 16 + jj;
        const int idx = ((a * KT + b) * 4 + r) * kWave + ln;
        double v = red[idx];
#pragma unroll
        for (int wv = 1; wv < kWavesPerBlock; ++wv) v += red[wv * RED + idx];
        emit(o, v);
    }
}

// Single system: the grid walks the slices; per-workgroup partial Grams are
// summed in a fixed two-level order.
template <int KS>
__global__ __launch_bounds__(kBlock) void k_spmm_gram(DevBufs B, int k, const double* __restrict__ X,
                                                      double* __restrict__ AX, int store,
                                                      double* __restrict__ G, double* part,
                                                      unsigned* counter) {
    constexpr int KT = GramShape<KS>::KT;
    constexpr int SH = GramShape<KS>::SH;
    __shared__ double shm[SH];
    const int wid = threadIdx.x / kWave;
    const int nb = gridDim.x;
    const int ngroups = (B.nslices + kWavesPerBlock - 1) / kWavesPerBlock;
    d4_t d[KT][KT];
#pragma unroll
    for (int a = 0; a < KT; ++a)
#pragma unroll
        for (int b = 0; b < KT; ++b) d[a][b] = d4_t{0.0, 0.0, 0.0, 0.0};
    double* tw = shm + wid * (SH / kWavesPerBlock);            // this wave's private tile
    // the trip count is uniform over the workgroup
    for (int L = xcd_block(blockIdx.x, nb); L < ngroups; L += nb) {
        const int s = __builtin_amdgcn_readfirstlane(L * kWavesPerBlock + wid);
        gram_slice<KS>(B, k, X, AX, store, s, d, tw);
    }
    const int nout = k * k;
    const int ng = (nb + kGroup - 1) / kGroup;
    const int g = blockIdx.x / kGroup;
    const int gsize = min(kGroup, nb - g * kGroup);
    gram_block_outputs<KS>(k, d, shm, [&](int o, double v) { store_shared(part + (size_t)o * nb + blockIdx.x, v); });
    if (!arrive_last(counter + 1 + g, gsize)) return;
    double* part2 = part + (size_t)nout * nb;
    for (int o = threadIdx.x; o < nout; o += kBlock) {
        double t[kGroup];
#pragma unroll
        for (int q = 0; q < kGroup; ++q) t[q] = q < gsize ? load_shared(part + (size_t)o * nb + g * kGroup + q) : 0.0;
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < kGroup; ++q) sum += t[q];
        store_shared(part2 + (size_t)o * ng + g, sum);
    }
    if (!arrive_last(counter, ng)) return;
    for (int o = threadIdx.x; o < nout; o += kBlock) {
        double sum = 0.0;
        for (int q0 = 0; q0 < ng; q0 += kGroup) {
            double t[kGroup];
#pragma unroll
            for (int q = 0; q < kGroup; ++q) t[q] = q0 + q < ng ? load_shared(part2 + (size_t)o * ng + q0 + q) : 0.0;
#pragma unroll
            for (int q = 0; q < kGroup; ++q) sum += t[q];
        }
        G[o] = sum;
    }
}

// Batched basis setup: A W and G = W^T A W of every member with `setup` set,
// over the SpMV work list (items are slice ranges of one member).  Each item
// leaves its partial Gram in the member's partial slots; the member's last
// item to arrive sums them in item order into the member's G.  A member table
// with AW null forms the Gram only (the POD Gram S^T A S, with W = S).
template <int KS>
__global__ __launch_bounds__(kBlock) void k_batch_spmm_gram(const BatchMember* __restrict__ mem,
                                                            const BatchSetup* __restrict__ su,
                                                            const BatchItem* __restrict__ items, int nitems) {
    constexpr int KT = GramShape<KS>::KT;
    constexpr int SH = GramShape<KS>::SH;
    __shared__ double shm[SH];
    const int wid = threadIdx.x / kWave;
    double* tw = shm + wid * (SH / kWavesPerBlock);
    const int G = gridDim.x;
    for (int base = 0; base < nitems; base += G) {
        const int m = min(G, nitems - base);
        if ((int)blockIdx.x >= m) break;
        const BatchItem it = items[base + xcd_block(blockIdx.x, m)];
        const BatchSetup& S = su[it.member];
        if (!S.setup) continue;
        const BatchMember& M = mem[it.member];
        const int k = S.ynom;
        d4_t d[KT][KT];
#pragma unroll
        for (int a = 0; a < KT; ++a)
#pragma unroll
            for (int b = 0; b < KT; ++b) d[a][b] = d4_t{0.0, 0.0, 0.0, 0.0};
        // waves take the item's slices in turn (a wave past the end adds nothing)
        const int nsl = it.end - it.begin;
        for (int q = 0; q < nsl; q += kWavesPerBlock) {
            const int s = __builtin_amdgcn_readfirstlane(q + wid < nsl ? it.begin + q + wid : M.B.nslices);
            gram_slice<KS>(M.B, k, M.W, const_cast<double*>(M.AW), M.AW != nullptr, s, d, tw);
        }
        const int nit = M.spmv_items;
        double* part = M.B.part;
        if (nit == 1) {
            gram_block_outputs<KS>(k, d, shm, [&](int o, double v) { S.G[o] = v; });
        } else {
            gram_block_outputs<KS>(k, d, shm, [&](int o, double v) { store_shared(part + (size_t)o * nit + it.local, v); });
            if (arrive_last(M.B.counter, nit)) {
                for (int o = threadIdx.x; o < k * k; o += kBlock) {
                    double sum = 0.0;
                    for (int i = 0; i < nit; ++i) sum += load_shared(part + (size_t)o * nit + i);
                    S.G[o] = sum;
                }
            }
        }
        __syncthreads();   // shm is reused by the next item
    }
}

// AX = A X for k <= KS columns, with no Gram (the truncation of the
// three-stage method forms its M x M Gram separately).  One wave per slice of
// 64 rows, lane = row; entry j + 1's value and column are requested while
// entry j's k gathers are in flight.
template <int KS>
__global__ __launch_bounds__(kBlock) void k_spmm(DevBufs B, int k, const double* __restrict__ X,
                                                 double* __restrict__ AX) {
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int nb = gridDim.x;
    const int ngroups = (B.nslices + kWavesPerBlock - 1) / kWavesPerBlock;
    for (int L = xcd_block(blockIdx.x, nb); L < ngroups; L += nb) {
        const int s = __builtin_amdgcn_readfirstlane(L * kWavesPerBlock + wid);
        if (s >= B.nslices) continue;
        const int row = s * kSlice + lane;
        double acc[KS];
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) acc[kk] = 0.0;
        const int64_t base = B.sptr[s];
        const int w = (int)((B.sptr[s + 1] - base) / kSlice);
        const int* c = B.cols + base + lane;
        const double* vv = B.vals + base + lane;
        const bool tabled = B.sflag[s] == 2;
        const int* __restrict__ tab = B.soff + (size_t)s * kTabMax;
        auto column = [&](int j) {
            if (tabled) {
                const int col = row + tab[j];
                return col < 0 ? 0 : (col < B.n ? col : B.n - 1);
            }
            return c[j * kSlice];
        };
        double a_next = w > 0 ? vv[0] : 0.0;
        int col_next = w > 0 ? column(0) : 0;
        for (int j = 0; j < w; ++j) {
            const double a = a_next;
            const int col = col_next;
            if (j + 1 < w) {
                a_next = vv[(j + 1) * kSlice];
                col_next = column(j + 1);
            }
            double xv[KS];
#pragma unroll
            for (int kk = 0; kk < KS; ++kk) xv[kk] = X[(size_t)(kk < k ? kk : k - 1) * B.ld + col];
#pragma unroll
            for (int kk = 0; kk < KS; ++kk) acc[kk] += a * xv[kk];
        }
        if (row < B.n) {
#pragma unroll
            for (int kk = 0; kk < KS; ++kk)
                if (kk < k) AX[(size_t)kk * B.ld + row] = acc[kk];
        }
    }
}

hipError_t launch_spmm(const DevBufs& B, int k, const double* X, double* AX, hipStream_t s) {
    if (k < 1 || k > kYMax) return hipErrorInvalidValue;
    const int groups = (B.nslices + kWavesPerBlock - 1) / kWavesPerBlock;
    const dim3 g(groups < 2048 ? groups : 2048), t(kBlock);
    switch (basis_tier(k)) {
#define CASE(T) case T: hipLaunchKernelGGL((k_spmm<T>), g, t, 0, s, B, k, X, AX); break;
        PODCG_POS_TIERS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch_spmm_gram(int ks, const BatchMember* mem, const BatchSetup* su, const BatchItem* items,
                                  int nitems, int grid, hipStream_t s) {
    if (ks < 1 || ks > kYMax || nitems < 1) return hipErrorInvalidValue;
    const dim3 g(grid < nitems ? grid : nitems), t(kBlock);
    switch (basis_tier(ks)) {
#define CASE(T) case T: hipLaunchKernelGGL((k_batch_spmm_gram<T>), g, t, 0, s, mem, su, items, nitems); break;
        PODCG_POS_TIERS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_spmm_gram(const DevBufs& B, int k, const double* X, double* AX, bool store, double* G,
                            hipStream_t s) {
    if (k < 1 || k > kYMax) return hipErrorInvalidValue;
    const int groups = (B.nslices + kWavesPerBlock - 1) / kWavesPerBlock;
    // grid cap measured on MI355X at 128^3: 1024 workgroups for up to 16
    // columns (6-7 columns: 150-166 us against 223-235 us at 512), 512 above
    // (20 columns: 350 us against 386 us at 1024); never more than the partial
    // sums buffer holds (k^2 slots per workgroup plus the group level)
    int cap = k <= 16 ? 2 * kGramBlocksMax : kGramBlocksMax;
    const int capk = kPartials / (k * k + (k * k + kGroup - 1) / kGroup + 1);
    if (cap > capk) cap = capk;
    dim3 g(groups < cap ? groups : cap), t(kBlock);
    switch (basis_tier(k)) {
#define CASE(T) case T: hipLaunchKernelGGL((k_spmm_gram<T>), g, t, 0, s, B, k, X, AX, store ? 1 : 0, G, B.part, B.counter); break;
        PODCG_POS_TIERS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
}  // namespace podcg
