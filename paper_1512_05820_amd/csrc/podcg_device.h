// Internal declarations of libpodcg: device-side state, reduction helpers and
// the row kernels shared by the translation units (the launchers are in
// podcg_launch.h).  Not a public header.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace podcg {

constexpr int kWave = 64;                 // CDNA wavefront
constexpr int kBlock = 256;               // threads per workgroup (4 waves)
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kSlice = 64;                // SELL slice height = one row per lane
constexpr int kYMax = 32;                 // largest basis / snapshot count
constexpr int kTabMax = 8;                // widest slice stored with a per-slice offset table
constexpr int kMetaWords = 16;            // words of a slice's metadata record (64 bytes)
constexpr int kNVMax = kYMax + 3;         // reduced values carried by one kernel
constexpr int kVecBlocksMax = 2048;       // partial-sum capacity of the streaming kernels
constexpr int kSpmvBlocksMax = 2048;      // partial-sum capacity of the SELL kernels
// Default launch grids of the loop kernels, measured on MI355X at 128^3.
// Each workgroup of the update and direction kernels first finishes the
// previous kernel's reduction, so fewer, longer-lived workgroups amortise that
// prologue.  Options override them.
constexpr int kSpmvGrid = 1024;
constexpr int kUpdateGrid = 512;
constexpr int kUpdateGridImplicit = 1024;   // the implicit form's update, which prefetches deeper
constexpr int kDirGrid = 1024;
constexpr int kCounters = 1 + kSpmvBlocksMax;        // arrival counters (level 2 + groups)
constexpr int kGramBlocksMax = 512;       // grid cap of the fused SpMM + Gram kernel
// doubles in the partials buffer: the larger of the loop kernels' need and the
// Gram kernel's (one slot per output entry per workgroup)
constexpr int kPartials = (2 * kNVMax * kSpmvBlocksMax > 2 * kYMax * kYMax * kGramBlocksMax)
                              ? 2 * kNVMax * kSpmvBlocksMax
                              : 2 * kYMax * kYMax * kGramBlocksMax;

// `done` values of the iteration state machine (see the loop kernels).
constexpr int kRunning = 0;
constexpr int kFinished = 1;
constexpr int kConvergedPending = 2;      // x += alpha p still to apply in this iteration
constexpr int kCapPending = 3;            // iteration cap reached, same pending update
constexpr int kFailed = -1;

// Scalar state of one solve, resident in device memory.  The first block is
// what the host polls.
struct DevState {
    int iter, done, status, y;
    int maxit, implicit, stop, pad2;   // implicit: the direction is kept as p = pt - W nu;
                                       // stop: loop kernels of iteration k run while k < stop
    double rr, rr0, bnorm2, true_rr;
    double tol2, rho, alpha, beta, gamma;
    double pad3[3];
    double mu[kYMax];      // projection coefficients G^{-1} (A W)^T z
    double what[kYMax];    // Stage-1 coefficients G^{-1} W^T rbar
    double xi[kYMax];      // implicit form: x = xt - W xi
    // Scalars of the loop, in two slots by iteration parity: iteration k reads
    // slot k & 1 and its direction kernel writes slot (k + 1) & 1, so no kernel
    // overwrites a value that another workgroup of the same kernel still reads.
    double lrho[2];        // (r, z) entering iteration k
    double lalpha[2];      // alpha_k (written by the update kernel)
    double lgamma[2];      // (A p_k, p_k)
    double lgcorr[2];      // implicit form: nu^T a, subtracted from (A pt, pt) to give (A p, p)
    double lnu[2][kYMax];  // implicit form: p = pt - W nu
    double lacc[2][kYMax]; // implicit form: a = (A W)^T pt, carried by its recurrence
};

struct PollBlock {         // host mirror of the first 48 bytes of DevState
    int iter, done, status, y;
    int maxit, pad0, stop, pad2;
    double rr, rr0, bnorm2, true_rr;
};

// Codes written by kernels into DevState::status (same values as the ABI).
constexpr int kStOk = 0, kStNotConverged = 1, kStNotSpd = -4, kStNonfinite = -5;

__device__ __forceinline__ bool is_finite(double v) { return v == v && fabs(v) <= 1.0e308; }

// Butterfly sum over the 64 lanes of a wave; every lane gets the total, and
// the order of additions is fixed.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Workgroup-wide reduction of NV values (fixed order).  `lds` needs
// kWavesPerBlock * NV doubles.  The result is left in lds[0..NV) for all threads.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[wid * NV + k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = lds[threadIdx.x];
#pragma unroll
        for (int w = 1; w < kWavesPerBlock; ++w) s += lds[w * NV + threadIdx.x];
        lds[kWavesPerBlock * NV + threadIdx.x] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) lds[threadIdx.x] = lds[kWavesPerBlock * NV + threadIdx.x];
    __syncthreads();
}

// Stores and loads that are coherent across the XCDs (relaxed atomics at agent
// scope: written through to, and read from, the level shared by all L2s).
// They let one workgroup read the partials of all others without an
// agent-scope fence, which on gfx950 writes back the whole L2 of the XCD.
__device__ __forceinline__ void store_shared(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_shared(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Wait until this wave's outstanding memory operations (the coherent stores
// above) have completed; also a compiler barrier.
__device__ __forceinline__ void wait_stores() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Arrival counter: returns true in the last of `expected` workgroups to
// arrive; that workgroup also returns the counter to zero.
__device__ __forceinline__ bool arrive_last(unsigned* counter, int expected) {
    __shared__ int is_last;
    wait_stores();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned prev =
            __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        is_last = (prev == (unsigned)(expected - 1));
        if (is_last) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    return is_last != 0;
}

constexpr int kGroup = 16;   // workgroups per first-level reduction group

// Deterministic two-level grid reduction of NV values.
//   level 1: each workgroup stores its NV sums in part[k * nb + block]; the
//            last workgroup of each group of kGroup consecutive workgroups
//            sums the group's entries (in block order) into
//            part[NV * nb + k * ng + group];
//   level 2: the last group to finish sums the ng group entries.
// Returns true in that final workgroup, with the totals in lds[0..NV).
// Requires nb <= kGroup * kBlock.  counter[0] is the level-2 counter,
// counter[1 + g] the counter of group g.  Each level issues all its loads
// before it sums, so the tail costs two memory round trips.
template <int NV>
__device__ __forceinline__ bool grid_sum_last(double (&v)[NV], double* part, unsigned* counter,
                                              double* lds) {
    block_sum<NV>(v, lds);
    const int nb = gridDim.x;
    const int ng = (nb + kGroup - 1) / kGroup;
    const int g = blockIdx.x / kGroup;
    if (threadIdx.x < NV) store_shared(part + (size_t)threadIdx.x * nb + blockIdx.x, lds[threadIdx.x]);
    const int gsize = min(kGroup, nb - g * kGroup);
    if (!arrive_last(counter + 1 + g, gsize)) return false;
    double a[NV];
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < NV; ++k)
        a[k] = t < gsize ? load_shared(part + (size_t)k * nb + g * kGroup + t) : 0.0;
    block_sum<NV>(a, lds);
    double* part2 = part + (size_t)NV * nb;
    if (t < NV) store_shared(part2 + (size_t)t * ng + g, lds[t]);
    if (!arrive_last(counter, ng)) return false;
#pragma unroll
    for (int k = 0; k < NV; ++k) a[k] = t < ng ? load_shared(part2 + (size_t)k * ng + t) : 0.0;
    block_sum<NV>(a, lds);
    return true;
}

// The loop kernels split the grid reduction between producer and consumer,
// so that no kernel ends with a serial tail in one workgroup.
// Producer side (level 1): the workgroup's NV sums go to part[k * nb + block];
// the last workgroup of each group of kGroup consecutive workgroups sums the
// group's entries (in block order) into part[NV * nb + k * ng + group].
template <int NV>
__device__ __forceinline__ void group_sum_store(double (&v)[NV], double* part, unsigned* counter, double* lds) {
    block_sum<NV>(v, lds);
    const int nb = gridDim.x;
    const int ng = (nb + kGroup - 1) / kGroup;
    const int g = blockIdx.x / kGroup;
    if (threadIdx.x < NV) store_shared(part + (size_t)threadIdx.x * nb + blockIdx.x, lds[threadIdx.x]);
    const int gsize = min(kGroup, nb - g * kGroup);
    if (!arrive_last(counter + 1 + g, gsize)) return;
    double a[NV];
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < NV; ++k)
        a[k] = t < gsize ? load_shared(part + (size_t)k * nb + g * kGroup + t) : 0.0;
    block_sum<NV>(a, lds);
    if (t < NV) store_shared(part + (size_t)NV * nb + (size_t)t * ng + g, lds[t]);
}
// Consumer side (level 2), run by every workgroup of the next kernel: the ng
// group sums of each value, added in group order (the same order in every
// workgroup, so every workgroup obtains bitwise the same totals), left in
// lds[0..NV).  nb is the producer's grid; requires ng <= kBlock.  The
// producer is an earlier kernel of the same stream, whose writes plain loads
// see, so these loads may hit in L2 (only the first workgroup on each XCD
// fetches the partials from memory).
template <int NV>
__device__ __forceinline__ void group_sum_load(const double* part, int nb, double* lds) {
    const int ng = (nb + kGroup - 1) / kGroup;
    const double* part2 = part + (size_t)NV * nb;
    double a[NV];
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < NV; ++k) a[k] = t < ng ? part2[(size_t)k * ng + t] : 0.0;
    block_sum<NV>(a, lds);
}

// Workgroup index remapped so that each XCD (workgroups are dealt to the 8
// XCDs round-robin) walks a contiguous range of the problem.  A bijection on
// [0, nb).
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7;
    const int t = b >> 3;
    return x * q + (x < r ? x : r) + t;
}

// Row (64 s + lane) of A x for the slice s handled by this wave.  Offset-table
// slices (widths 1..8, stencil matrices) branch on their width to a path of
// exactly that many value and gather loads, then the sums in order j = 0, 1,
// ...; the other storages loop in chunks of 8 (all column indices and values
// of a chunk first, padding slots re-reading the last valid slot and skipped
// with a select, then the gathers, then the sums).  s is wave-uniform, so the
// slice bounds and the format flag are scalar loads.  Three storages of the
// columns, chosen per slice at ingest:
//   flag 2: every row of the slice draws its columns from one list of w <= 8
//           offsets (a stencil), stored once per slice (offset j of the list
//           is slot j of every row; a row without that neighbour holds a zero
//           value there); the offsets are scalar loads and no per-entry index
//           is read;
//   flag 1: per-entry 16-bit offsets col - row (2 bytes per entry);
//   flag 0: per-entry int32 columns.
// Gather indices of padding are kept inside [0, n); rows past n read zeros.
template <typename T, typename C>
__device__ __forceinline__ double sell_row_cols(const C* __restrict__ c, const T* __restrict__ v, int w,
                                                int rb, const T* __restrict__ x) {
    double acc = 0.0;   // FP32 operands multiply exactly in FP64; the row sum is FP64
    for (int j0 = 0; j0 < w; j0 += 8) {
        int ci[8];
        T vi[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int j = min(j0 + u, w - 1);
            ci[u] = rb + (int)__builtin_nontemporal_load(c + j * kSlice);
            vi[u] = __builtin_nontemporal_load(v + j * kSlice);
        }
        T xi[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) xi[u] = x[ci[u]];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = (j0 + u < w) ? fma((double)vi[u], (double)xi[u], acc) : acc;
    }
    return acc;
}


// ------------------------------------------------------------------ launchers
// Device buffers of one context, passed to the launchers.
struct DevBufs {
    int n;
    int nslices;
    size_t ld;                 // leading dimension of column blocks (W, AW, S, AS)
    const int64_t* sptr;       // slice offsets, nslices + 1
    const int* cols;           // SELL column indices
    const int16_t* cols16;     // column offsets col - row of the 16-bit slices
    const uint8_t* sflag;      // per slice: 2 = offset table, 1 = read cols16, 0 = read cols
    const int* soff;           // per slice: kTabMax offsets (the slices with flag 2)
    const int* smeta;          // per slice: kMetaWords words {base lo, base hi, w, flag, tab[8], 0...}
    const double* vals;        // SELL values
    const double* dinv;        // 1 / diag(A)
    DevState* st;
    double* part;
    unsigned* counter;
    double* gpart;             // per-workgroup (A p, p) partials of the loop SpMV
    const double* Ginv;        // y x y row-major
    const float* vals32;       // FP32 copy of the SELL values (mixed precision)
    const float* dinv32;       // FP32 copy of dinv
    int spmv_grid, update_grid, dir_grid;   // launch grids of the loop kernels
};

constexpr int kLoopGridMax = 4096;

// Launch through hipExtLaunchKernel when timing events are given.
#define PODCG_LAUNCH(K, G, T, S, E0, E1, ...)                                                        \
    do {                                                                                            \
        if ((E0) || (E1)) hipExtLaunchKernelGGL(K, G, T, 0, S, E0, E1, 0, __VA_ARGS__);              \
        else hipLaunchKernelGGL(K, G, T, 0, S, __VA_ARGS__);                                        \
    } while (0)        // largest loop grid (partial and counter capacity)


// The per-slice metadata a wave needs before its first vector load (slice
// offset, width, column storage, offset table).  The loop SpMV reads it as one
// 64-byte record per slice with an ordinary vector load (lane l holds word
// l % 16) and extracts the fields with readlane: vector loads complete in
// order, so the next slice's record can be requested one slice ahead without
// any wait on it until it is used.
struct SliceMeta {
    int64_t base;
    int w, flag;
    int tab[kTabMax];
};
__device__ __forceinline__ int slice_meta_load(const DevBufs& B, int s) {
    return B.smeta[(size_t)s * kMetaWords + (threadIdx.x & (kMetaWords - 1))];
}
__device__ __forceinline__ SliceMeta slice_meta_unpack(int v) {
    SliceMeta m;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane(v, 0);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane(v, 1);
    m.base = (int64_t)(((uint64_t)hi << 32) | lo);
    m.w = __builtin_amdgcn_readlane(v, 2);
    m.flag = __builtin_amdgcn_readlane(v, 3);
    m.tab[0] = __builtin_amdgcn_readlane(v, 4);
    m.tab[1] = __builtin_amdgcn_readlane(v, 5);
    m.tab[2] = __builtin_amdgcn_readlane(v, 6);
    m.tab[3] = __builtin_amdgcn_readlane(v, 7);
    m.tab[4] = __builtin_amdgcn_readlane(v, 8);
    m.tab[5] = __builtin_amdgcn_readlane(v, 9);
    m.tab[6] = __builtin_amdgcn_readlane(v, 10);
    m.tab[7] = __builtin_amdgcn_readlane(v, 11);
    return m;
}
// Offset-table widths with a path of their own, the stencil widths first.
#define PODCG_TAB_WIDTHS(X) X(7) X(5) X(6) X(4) X(3) X(8) X(2) X(1)

// The row of an offset-table slice of width WN: exactly WN value and WN
// gather loads, each offset read straight from its (scalar) table entry
// tab(u); the row sum and, when the table holds the zero offset, x at the
// row itself as gathered (has = false otherwise).
template <typename T>
struct RowDiag {
    double acc;
    T xd;
    bool has;
};
template <typename T, int WN, typename Tab>
__device__ __forceinline__ RowDiag<T> sell_row_tab_diag(const DevBufs& B, Tab tab, const T* __restrict__ v,
                                                        int row, const T* __restrict__ x) {
    int ci[WN];
    T vi[WN];
#pragma unroll
    for (int u = 0; u < WN; ++u) {
        const int c = row + tab(u);
        ci[u] = c < 0 ? 0 : (c < B.n ? c : B.n - 1);
        vi[u] = __builtin_nontemporal_load(v + u * kSlice);
    }
    T xi[WN];
#pragma unroll
    for (int u = 0; u < WN; ++u) xi[u] = x[ci[u]];
    RowDiag<T> o{0.0, (T)0, false};
#pragma unroll
    for (int u = 0; u < WN; ++u) o.acc = fma((double)vi[u], (double)xi[u], o.acc);
#pragma unroll
    for (int u = 0; u < WN; ++u) {
        const bool z = tab(u) == 0;
        o.xd = z ? xi[u] : o.xd;
        o.has = o.has || z;
    }
    return o;
}

template <typename T, int WN, typename Tab>
__device__ __forceinline__ double sell_row_tab(const DevBufs& B, Tab tab, const T* __restrict__ v, int row,
                                              const T* __restrict__ x) {
    return sell_row_tab_diag<T, WN>(B, tab, v, row, x).acc;
}

template <typename T>
__device__ __forceinline__ double sell_row(const DevBufs& B, const T* __restrict__ vals, int s, int lane,
                                          const T* __restrict__ x) {
    s = __builtin_amdgcn_readfirstlane(s);
    const int64_t base = B.sptr[s];
    const int w = (int)((B.sptr[s + 1] - base) / kSlice);
    const T* v = vals + base + lane;
    const int flag = B.sflag[s];
    if (flag == 2) {
        const int row = s * kSlice + lane;
        const int* __restrict__ tab = B.soff + (size_t)s * kTabMax;
        const auto tabf = [&](int u) { return tab[u]; };
        switch (w) {
#define PODCG_TAB_CASE(WN) case WN: return sell_row_tab<T, WN>(B, tabf, v, row, x);
            PODCG_TAB_WIDTHS(PODCG_TAB_CASE)
#undef PODCG_TAB_CASE
            default: break;
        }
        int ci[kTabMax];
        T vi[kTabMax];
#pragma unroll
        for (int u = 0; u < kTabMax; ++u) {
            const int j = min(u, w - 1);
            const int c = row + tab[j];
            ci[u] = c < 0 ? 0 : (c < B.n ? c : B.n - 1);
            vi[u] = __builtin_nontemporal_load(v + j * kSlice);
        }
        T xi[kTabMax];
#pragma unroll
        for (int u = 0; u < kTabMax; ++u) xi[u] = x[ci[u]];
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < kTabMax; ++u) acc = u < w ? fma((double)vi[u], (double)xi[u], acc) : acc;
        return acc;
    }
    if (flag == 1) {
        const int row = s * kSlice + lane;
        return sell_row_cols<T, int16_t>(B.cols16 + base + lane, v, w, row < B.n ? row : 0, x);
    }
    return sell_row_cols<T, int>(B.cols + base + lane, v, w, 0, x);
}

// sell_row with the metadata already loaded.  Offset-table slices branch on
// their (wave-uniform) width to a path of exactly that width.
template <typename T>
__device__ __forceinline__ double sell_row_meta(const DevBufs& B, const SliceMeta& m, const T* __restrict__ vals,
                                               int s, int lane, const T* __restrict__ x) {
    const int w = m.w;
    const T* v = vals + m.base + lane;
    const int row = s * kSlice + lane;
    if (m.flag == 2) {
        const auto tab = [&](int u) { return m.tab[u]; };
        switch (w) {
#define PODCG_TAB_CASE(WN) case WN: return sell_row_tab<T, WN>(B, tab, v, row, x);
            PODCG_TAB_WIDTHS(PODCG_TAB_CASE)
#undef PODCG_TAB_CASE
            default: break;
        }
        int ci[kTabMax];
        T vi[kTabMax];
#pragma unroll
        for (int u = 0; u < kTabMax; ++u) {
            const int j = min(u, w - 1);
            int off = m.tab[0];
#pragma unroll
            for (int t = 1; t < kTabMax; ++t) off = j == t ? m.tab[t] : off;
            const int c = row + off;
            ci[u] = c < 0 ? 0 : (c < B.n ? c : B.n - 1);
            vi[u] = __builtin_nontemporal_load(v + j * kSlice);
        }
        T xi[kTabMax];
#pragma unroll
        for (int u = 0; u < kTabMax; ++u) xi[u] = x[ci[u]];
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < kTabMax; ++u) acc = u < w ? fma((double)vi[u], (double)xi[u], acc) : acc;
        return acc;
    }
    if (m.flag == 1) return sell_row_cols<T, int16_t>(B.cols16 + m.base + lane, v, w, row < B.n ? row : 0, x);
    return sell_row_cols<T, int>(B.cols + m.base + lane, v, w, 0, x);
}

// q = A p on two consecutive slices s0, s0 + 1 by one wave, two rows per
// lane: lane l holds rows r = 64 s0 + 2 l and r + 1 (lanes 0..31 in slice
// s0, 32..63 in slice s0 + 1) and loads their values, the even-offset entries
// of p and the products as 16-byte pairs; the +-1 offsets of the table come
// from the neighbouring lanes' own pairs (lane moves), so a 7-point row needs
// 5 instead of 7 gathers.  Row sums run over the table in order, as in
// sell_row_tab.  p and q must be 16-byte aligned.
typedef double dbl2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ dbl2 ld2(const double* __restrict__ a) {
    return *reinterpret_cast<const dbl2*>(a);
}
// entries c, c + 1 of p, each clamped into [0, n) (padding slots multiply a
// clamped entry by a zero value); one 16-byte load when c is even and in range
__device__ __forceinline__ dbl2 gather2(const double* __restrict__ p, int c, int n) {
    if (c >= 0 && c + 1 < n) {
        if ((c & 1) == 0) return ld2(p + c);
        return dbl2{p[c], p[c + 1]};
    }
    const int c0 = c < 0 ? 0 : (c < n ? c : n - 1);
    const int c1 = c + 1 < 0 ? 0 : (c + 1 < n ? c + 1 : n - 1);
    return dbl2{p[c0], p[c1]};
}
template <int WN>
__device__ __forceinline__ void pair_rows(const DevBufs& B, const SliceMeta& m0, const SliceMeta& m1, int s0,
                                          int lane, const double* __restrict__ p, double* __restrict__ q,
                                          double& g) {
    const int r = s0 * kSlice + 2 * lane;
    const int64_t base = lane < 32 ? m0.base : m1.base;
    const double* v = B.vals + base + 2 * (lane & 31);
    dbl2 vv[WN];
#pragma unroll
    for (int u = 0; u < WN; ++u) vv[u] = __builtin_nontemporal_load(reinterpret_cast<const dbl2*>(v + u * kSlice));
    const dbl2 own = gather2(p, r, B.n);
    // neighbours' pairs for the +-1 offsets; the wave's ends load theirs
    const double left = __shfl_up(own.y, 1, kWave);
    const double right = __shfl_down(own.x, 1, kWave);
    const int rl = s0 * kSlice - 1, rr = s0 * kSlice + 2 * kSlice;
    const double pl = lane == 0 ? p[rl < 0 ? 0 : (rl < B.n ? rl : B.n - 1)] : left;
    const double pr = lane == kWave - 1 ? p[rr < B.n ? rr : B.n - 1] : right;
    dbl2 xi[WN];
#pragma unroll
    for (int u = 0; u < WN; ++u) {
        const int off = m0.tab[u];
        if (off == 0) xi[u] = own;
        else if (off == -1) xi[u] = dbl2{pl, own.x};
        else if (off == 1) xi[u] = dbl2{own.y, pr};
        else xi[u] = gather2(p, r + off, B.n);
    }
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int u = 0; u < WN; ++u) {
        a0 = fma(vv[u].x, xi[u].x, a0);
        a1 = fma(vv[u].y, xi[u].y, a1);
    }
    if (r + 1 < B.n) {
        *reinterpret_cast<dbl2*>(q + r) = dbl2{a0, a1};
        g += a0 * own.x;
        g += a1 * own.y;
    } else if (r < B.n) {
        q[r] = a0;
        g += a0 * own.x;
    }
}

// Slices s0 and (when has1) s0 + 1 of q = A p, with the (q, p) partial added
// to g: the two-rows-per-lane path of pair_rows when both are offset-table
// slices with one table, else one slice at a time with lane = row.
__device__ __forceinline__ void spmv_slice_pair(const DevBufs& B, int s0, bool has1, int lane,
                                                const double* __restrict__ p, double* __restrict__ q, double& g) {
    const int s1 = has1 ? s0 + 1 : s0;
    const int mw = B.smeta[(size_t)(lane < kMetaWords ? s0 : s1) * kMetaWords + (lane & (kMetaWords - 1))];
    SliceMeta m0, m1;
    m0.base = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane(mw, 1) << 32) |
                        (uint32_t)__builtin_amdgcn_readlane(mw, 0));
    m0.w = __builtin_amdgcn_readlane(mw, 2);
    m0.flag = __builtin_amdgcn_readlane(mw, 3);
    m1.base = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane(mw, 17) << 32) |
                        (uint32_t)__builtin_amdgcn_readlane(mw, 16));
    m1.w = __builtin_amdgcn_readlane(mw, 18);
    m1.flag = __builtin_amdgcn_readlane(mw, 19);
#pragma unroll
    for (int u = 0; u < kTabMax; ++u) {
        m0.tab[u] = __builtin_amdgcn_readlane(mw, 4 + u);
        m1.tab[u] = __builtin_amdgcn_readlane(mw, 20 + u);
    }
    bool uni = has1 && m0.flag == 2 && m1.flag == 2 && m0.w == m1.w && m0.w >= 1 && m0.w <= kTabMax;
#pragma unroll
    for (int u = 0; u < kTabMax; ++u) uni = uni && (u >= m0.w || m0.tab[u] == m1.tab[u]);
    if (uni) {
        switch (m0.w) {
#define PODCG_PAIR_CASE(WN) case WN: pair_rows<WN>(B, m0, m1, s0, lane, p, q, g); break;
            PODCG_TAB_WIDTHS(PODCG_PAIR_CASE)
#undef PODCG_PAIR_CASE
            default: break;
        }
        return;
    }
    for (int h = 0; h < (has1 ? 2 : 1); ++h) {
        const int s = s0 + h;
        const SliceMeta m = h == 0 ? m0 : m1;
        const int row = s * kSlice + lane;
        RowDiag<double> o{0.0, 0.0, false};
        if (m.flag == 2 && m.w >= 1 && m.w <= kTabMax) {
            const auto tab = [&](int u) { return m.tab[u]; };
            const double* v = B.vals + m.base + lane;
            switch (m.w) {
#define PODCG_TAB_CASE(WN) case WN: o = sell_row_tab_diag<double, WN>(B, tab, v, row, p); break;
                PODCG_TAB_WIDTHS(PODCG_TAB_CASE)
#undef PODCG_TAB_CASE
                default: break;
            }
        } else {
            o.acc = sell_row_meta<double>(B, m, B.vals, s, lane, p);
        }
        if (row < B.n) {
            q[row] = o.acc;
            g += o.acc * (o.has ? o.xd : p[row]);
        }
    }
}

// Matrix values and Jacobi inverse in the storage type T of a kernel.
template <typename T> __device__ __forceinline__ const T* mat_vals(const DevBufs& B);
template <> __device__ __forceinline__ const double* mat_vals<double>(const DevBufs& B) { return B.vals; }
template <> __device__ __forceinline__ const float* mat_vals<float>(const DevBufs& B) { return B.vals32; }
template <typename T> __device__ __forceinline__ const T* mat_dinv(const DevBufs& B);
template <> __device__ __forceinline__ const double* mat_dinv<double>(const DevBufs& B) { return B.dinv; }
template <> __device__ __forceinline__ const float* mat_dinv<float>(const DevBufs& B) { return B.dinv32; }

// Register tiers compiled for the basis dimension.  Up to 16 the kernels are
// instantiated for the exact dimension (every column load is unconditional
// and issued together); above 16 a tier serves all y <= tier, with clamped
// column indices so loads stay unconditional and in bounds.
#define PODCG_WIDE_TIERS(X) X(20) X(24) X(28) X(32)
#define PODCG_POS_TIERS(X)                                                                         \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)        \
        PODCG_WIDE_TIERS(X)
#define PODCG_TIERS(X) X(0) PODCG_POS_TIERS(X)
constexpr int kExactTierMax = 16;

// Column index used for a load in tier YB with runtime dimension y: the
// column itself for exact tiers, clamped into [0, y) otherwise.
template <int YB>
__device__ __forceinline__ int tier_col(int k, int y) {
    return YB <= kExactTierMax ? k : (k < y ? k : y - 1);
}
template <int YB>
__device__ __forceinline__ bool tier_live(int k, int y) {
    return YB <= kExactTierMax ? true : k < y;
}

// ------------------------------------------------------------------ batches
// One member (an independent sequence) of a batched solve, as the batched loop
// kernels see it.  Rebuilt by the host before every batched solve.
struct BatchMember {
    DevBufs B;                 // the member context's matrix, state and scratch
    double* r;
    double* z;
    double* p;
    double* q;
    double* x;
    const double* W;
    const double* AW;
    int y;                     // basis columns used in this solve (0 = plain PCG)
    int spmv_items;            // work items of this member in the SpMV list
    int vec_items;             // work items of this member in the vector list
    int spmv_first;            // offset of its items in the full SpMV list
    int vec_first;             // offset of its items in the full vector list
    int implicit;              // 1: the direction is kept as p = pt - W nu (state slot 0 holds nu, a)
    int pad[2];
};

// A contiguous range of one member: SELL slices [begin, end) in the SpMV
// list, rows [begin, end) in the vector list.  `local` numbers the items of
// the member (its partial-sum slot).
struct BatchItem {
    int member, begin, end, local;
};

constexpr int kBatchMaxMembers = 1024;

// ------------------------------------------------------------ three stages
constexpr int kTsCap = 512;      // largest accumulated basis (columns of Y / Z)
constexpr int kTsChunks = 256;   // row chunks of the tall transposed products

// Device state of the three-stage method: the reduced vectors of Stage 2,
// the recorded Stage-3 scalars and the POD weights of the accumulated vectors.
struct TsDev {
    double xh[kTsCap], rh[kTsCap], ph[kTsCap], gh[kTsCap];
    double wtgy[kYMax * kTsCap];   // (A W)^T Y, w x m row-major
    double alp2[kYMax], gam2[kYMax];
    double rz2, rn0, rn, tau;
    int k2, done2, k2max, pad;
    double gam3[kTsCap], alp3[kTsCap];
    double eta_prev[kTsCap], eta_acc[kTsCap];
    // iterative Stage 3 (phi = 1): the stage-2 increment sum alpha p (reduced),
    // the current projection solve (right-hand side, solution; its residual
    // and direction reuse rh / ph and Ghat p reuses gh), and the kept
    // augmenting directions: naug of them (P and Ghat P in the separate
    // augmentation block, (Ghat p, p) here), naug0 at the start of the
    // current solve, knew kept by it so far
    double xinc[kTsCap], cin[kTsCap], muin[kTsCap];
    double gam_aug[kTsCap];
    double rzin, rn0in, tauin, cnin;   // cnin = ||c||
    int kin, donein, kinmax, naug;
    int naug0, knew, pad6, pad7;
};
// Augmentation block of the iterative Stage 3: direction l at P + l kTsCap,
// Ghat times it at P + (kTsCap + l) kTsCap.
constexpr size_t kTsAugDoubles = (size_t)2 * kTsCap * kTsCap;
// Directions formed from a residual below this fraction of their solve's
// right-hand side (Stage 2: its initial residual) are not kept (iterative
// Stage 3).
constexpr double kTsKeepFloor = 1e-6;

// One-workgroup solve of small systems (k_lds.hip): threads per workgroup,
// widest slice and largest basis it holds in registers.
constexpr int kLdsThreads = 1024;
constexpr int kLdsWidth = 8;
constexpr int kLdsYMax = 5;

}  // namespace podcg
