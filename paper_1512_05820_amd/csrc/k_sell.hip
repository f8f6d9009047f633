// Sparse kernels of libpodcg: CSR ingest into SELL-64 and the products with A.
//
// Layout (SELL-C-sigma with C = 64, sigma = 1, i.e. no row sorting): rows are
// cut into slices of 64 consecutive rows, one row per lane of a wavefront.
// Slice s stores its entries column-major: entry j of row 64 s + lane sits at
// sptr[s] + 64 j + lane, for j < width(s) = the longest row of the slice.
// Shorter rows are padded with value 0 and column = the row itself, so every
// gather stays inside the vector.  One load instruction of a wave then reads
// 64 consecutive values (512 B) and 64 consecutive column indices (256 B).
#include "podcg_launch.h"

namespace podcg {

// ---------------------------------------------------------------- ingest

// flag |= 1: rowptr not a valid offset array; |= 2: column out of range.
__global__ __launch_bounds__(kBlock) void k_validate_csr(int n, int64_t nnz,
                                                         const int32_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ colind,
                                                         int* flag) {
    int bad = 0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const int64_t s = rowptr[i], e = rowptr[i + 1];
        if (i == 0 && s != 0) bad |= 1;
        if (i == n - 1 && e != nnz) bad |= 1;
        if (s < 0 || e < s || e > nnz) { bad |= 1; continue; }
        for (int64_t k = s; k < e; ++k) {
            const int c = colind[k];
            if (c < 0 || c >= n) bad |= 2;
        }
    }
    if (bad) atomicOr(flag, bad);
}

// sptr[s + 1] = 64 * (longest row of slice s); one wave per slice.
__global__ __launch_bounds__(kBlock) void k_slice_widths(int n, int nslices,
                                                         const int32_t* __restrict__ rowptr,
                                                         int64_t* __restrict__ sptr) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = (blockIdx.x * kBlock + threadIdx.x) / kWave;
    const int nwaves = gridDim.x * kWavesPerBlock;
    for (int s = wave; s < nslices; s += nwaves) {
        const int row = s * kSlice + lane;
        int len = row < n ? rowptr[row + 1] - rowptr[row] : 0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) len = max(len, __shfl_xor(len, off, kWave));
        if (lane == 0) sptr[s + 1] = (int64_t)len * kSlice;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) sptr[0] = 0;
}

// In-place inclusive scan of sptr[1..nslices] by one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_scan_slices(int nslices, int64_t* sptr) {
    __shared__ int64_t sums[1024];
    const int t = threadIdx.x;
    const int chunk = (nslices + 1023) / 1024;
    const int beg = 1 + t * chunk;
    const int end = min(beg + chunk, nslices + 1);
    int64_t acc = 0;
    for (int i = beg; i < end; ++i) acc += sptr[i];
    sums[t] = acc;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int64_t v = t >= off ? sums[t - off] : 0;
        __syncthreads();
        sums[t] += v;
        __syncthreads();
    }
    int64_t run = t > 0 ? sums[t - 1] : 0;
    for (int i = beg; i < end; ++i) {
        run += sptr[i];
        sptr[i] = run;
    }
}

// Column indices and the CSR position of every SELL slot (-1 for padding).
__global__ __launch_bounds__(kBlock) void k_fill_pattern(int n, int nslices,
                                                         const int32_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ colind,
                                                         const int64_t* __restrict__ sptr,
                                                         int* __restrict__ cols, int* __restrict__ map) {
    const int total = nslices * kSlice;
    for (int row = blockIdx.x * kBlock + threadIdx.x; row < total; row += gridDim.x * kBlock) {
        const int s = row / kSlice, lane = row % kSlice;
        const int64_t base = sptr[s];
        const int w = (int)((sptr[s + 1] - base) / kSlice);
        const int beg = row < n ? rowptr[row] : 0;
        const int len = row < n ? rowptr[row + 1] - beg : 0;
        const int pad_col = row < n ? row : 0;
        for (int j = 0; j < w; ++j) {
            const int64_t slot = base + (int64_t)j * kSlice + lane;
            if (j < len) {
                cols[slot] = colind[beg + j];
                map[slot] = beg + j;
            } else {
                cols[slot] = pad_col;
                map[slot] = -1;
            }
        }
    }
}

// One wave per slice: 16-bit column offsets when they all fit (rows < n);
// padding rows (>= n) store 0 and gather entry 0.
__device__ __forceinline__ int wave_min_int(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int o = __shfl_xor(v, off, kWave);
        v = o < v ? o : v;
    }
    return v;
}

// One wave per slice.  The union of the rows' column offsets is built by
// repeatedly taking the smallest offset not yet consumed by any lane (rows are
// checked to be strictly increasing); the slice takes the table form when the
// union has exactly w entries (w = the slice width <= kTabMax), so its storage
// does not grow.  Slot j of each row then holds the entry with offset tab[j],
// or a zero-valued padding slot (map -1, column = the row) when the row has no
// such neighbour.
__global__ __launch_bounds__(kBlock) void k_fill_table(int n, int nslices, const int32_t* __restrict__ rowptr,
                                                       const int64_t* __restrict__ sptr, int* __restrict__ cols,
                                                       int* __restrict__ map, int* __restrict__ soff,
                                                       uint8_t* __restrict__ sflag) {
    constexpr int kNone = 0x7fffffff;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    for (int s = blockIdx.x * kWavesPerBlock + wid; s < nslices; s += gridDim.x * kWavesPerBlock) {
        const int64_t base = sptr[s];
        const int w = (int)((sptr[s + 1] - base) / kSlice);
        bool table = false;
        int tab[kTabMax];
        if (w >= 1 && w <= kTabMax) {
            const int row = s * kSlice + lane;
            const int beg = row < n ? rowptr[row] : 0;
            const int len = row < n ? rowptr[row + 1] - beg : 0;
            int off[kTabMax];
            bool sorted = true;
#pragma unroll
            for (int j = 0; j < kTabMax; ++j) {
                off[j] = (j < len) ? cols[base + (int64_t)j * kSlice + lane] - row : kNone;
                if (j > 0 && j < len && off[j] <= off[j - 1]) sorted = false;
            }
            int cnt = 0, ptr = 0;
            for (int round = 0; round <= kTabMax; ++round) {
                int mine = kNone;
#pragma unroll
                for (int j = 0; j < kTabMax; ++j)
                    if (j == ptr) mine = off[j];
                const int m = wave_min_int(mine);
                if (m == kNone) break;
                if (cnt < kTabMax) {
#pragma unroll
                    for (int j = 0; j < kTabMax; ++j)
                        if (j == cnt) tab[j] = m;
                }
                ++cnt;
                if (mine == m) ++ptr;
            }
            table = __all(sorted) && cnt == w;
            if (table) {
                int e = 0;
#pragma unroll
                for (int j = 0; j < kTabMax; ++j) {
                    if (j >= w) break;
                    const int64_t slot = base + (int64_t)j * kSlice + lane;
                    int cur = kNone;
#pragma unroll
                    for (int u = 0; u < kTabMax; ++u)
                        if (u == e) cur = off[u];
                    if (e < len && cur == tab[j]) {
                        cols[slot] = row + tab[j];
                        map[slot] = beg + e;
                        ++e;
                    } else {
                        cols[slot] = row < n ? row : 0;
                        map[slot] = -1;
                    }
                }
                if (lane == 0)
#pragma unroll
                    for (int j = 0; j < kTabMax; ++j) soff[(size_t)s * kTabMax + j] = j < w ? tab[j] : 0;
            }
        }
        if (lane == 0) {
            sflag[s] = table ? 2 : 0;
            if (!table)   // defined contents for slices without a table (read, not used, by the SpMV)
#pragma unroll
                for (int j = 0; j < kTabMax; ++j) soff[(size_t)s * kTabMax + j] = 0;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_fill_offsets16(int n, int nslices, const int64_t* __restrict__ sptr,
                                                           const int* __restrict__ cols,
                                                           int16_t* __restrict__ cols16,
                                                           uint8_t* __restrict__ sflag) {
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    for (int s = blockIdx.x * kWavesPerBlock + wid; s < nslices; s += gridDim.x * kWavesPerBlock) {
        if (sflag[s] == 2) continue;   // offset-table slice
        const int64_t base = sptr[s];
        const int w = (int)((sptr[s + 1] - base) / kSlice);
        const int row = s * kSlice + lane;
        bool fits = true;
        for (int j = 0; j < w; ++j) {
            const int d = cols[base + (int64_t)j * kSlice + lane] - row;
            if (row < n && (d > 32767 || d < -32767)) fits = false;
        }
        const bool all = __all(fits);
        if (all)
            for (int j = 0; j < w; ++j) {
                const int64_t slot = base + (int64_t)j * kSlice + lane;
                cols16[slot] = row < n ? (int16_t)(cols[slot] - row) : (int16_t)0;
            }
        if (lane == 0) sflag[s] = all ? 1 : 0;
    }
}

// SELL values of one stored row (row < nslices * 64) from the CSR values, and
// dinv[row] = 1 / (sum of its diagonal entries).  Returns the flags: 4 a
// diagonal entry missing or not positive, 8 a non-finite value.
__device__ __forceinline__ int fill_values_row(int row, int n, const int64_t* __restrict__ sptr,
                                               const int* __restrict__ cols, const int* __restrict__ map,
                                               const uint8_t* __restrict__ sflag, const int* __restrict__ soff,
                                               const double* __restrict__ csr_vals, double* __restrict__ vals,
                                               double* __restrict__ dinv) {
    int bad = 0;
    {
        const int s = row / kSlice, lane = row % kSlice;   // s is wave-uniform
        const int64_t base = sptr[s];
        const int w = (int)((sptr[s + 1] - base) / kSlice);
        double d = 0.0;
        if (w <= kTabMax) {
            // all slot indices, then all value gathers, then the stores; an
            // offset-table slice takes its diagonal from the zero offset (a
            // table lists distinct offsets), the others compare columns
            int m[kTabMax];
#pragma unroll
            for (int u = 0; u < kTabMax; ++u) m[u] = u < w ? map[base + (int64_t)u * kSlice + lane] : -1;
            double v[kTabMax];
#pragma unroll
            for (int u = 0; u < kTabMax; ++u) v[u] = m[u] >= 0 ? csr_vals[m[u]] : 0.0;
            const bool tabled = sflag[s] == 2;
            int c[kTabMax];
#pragma unroll
            for (int u = 0; u < kTabMax; ++u)
                c[u] = u < w ? (tabled ? row + soff[(size_t)s * kTabMax + u] : cols[base + (int64_t)u * kSlice + lane]) : -1;
#pragma unroll
            for (int u = 0; u < kTabMax; ++u) {
                if (u < w) {
                    vals[base + (int64_t)u * kSlice + lane] = v[u];
                    if (!is_finite(v[u])) bad |= 8;
                    if (m[u] >= 0 && c[u] == row) d += v[u];
                }
            }
        } else {
            for (int jj = 0; jj < w; ++jj) {
                const int64_t slot = base + (int64_t)jj * kSlice + lane;
                const int mm = map[slot];
                const double vv = mm >= 0 ? csr_vals[mm] : 0.0;
                vals[slot] = vv;
                if (!is_finite(vv)) bad |= 8;
                if (mm >= 0 && cols[slot] == row) d += vv;
            }
        }
        if (row < n) {
            if (!(d > 0.0)) bad |= 4;
            dinv[row] = d > 0.0 ? 1.0 / d : 0.0;
        } else {
            dinv[row] = 0.0;
        }
    }
    return bad;
}

// SELL values from CSR values, and dinv = 1 / (sum of the diagonal entries).
// flag |= 4: a diagonal entry missing or not positive; |= 8: non-finite value.
__global__ __launch_bounds__(kBlock) void k_fill_values(int n, int nslices,
                                                        const int64_t* __restrict__ sptr,
                                                        const int* __restrict__ cols,
                                                        const int* __restrict__ map,
                                                        const uint8_t* __restrict__ sflag,
                                                        const int* __restrict__ soff,
                                                        const double* __restrict__ csr_vals,
                                                        double* __restrict__ vals,
                                                        double* __restrict__ dinv, int* flag) {
    const int total = nslices * kSlice;
    int bad = 0;
    for (int row = blockIdx.x * kBlock + threadIdx.x; row < total; row += gridDim.x * kBlock)
        bad |= fill_values_row(row, n, sptr, cols, map, sflag, soff, csr_vals, vals, dinv);
    if (bad) atomicOr(flag, bad);
}

// Batched value ingest: every member's SELL values and dinv from its CSR
// values (aux.src), over the SpMV work list (slice ranges of one member).
__global__ __launch_bounds__(kBlock) void k_batch_fill_values(const BatchMember* __restrict__ mem,
                                                              const BatchAux* __restrict__ aux,
                                                              const BatchItem* __restrict__ items, int nitems) {
    const int G = gridDim.x;
    for (int base = 0; base < nitems; base += G) {
        const int m = min(G, nitems - base);
        if ((int)blockIdx.x >= m) break;
        const BatchItem it = items[base + xcd_block(blockIdx.x, m)];
        const BatchMember& M = mem[it.member];
        const BatchAux& A = aux[it.member];
        int bad = 0;
        for (int row = it.begin * kSlice + (int)threadIdx.x; row < it.end * kSlice; row += kBlock)
            bad |= fill_values_row(row, M.B.n, M.B.sptr, M.B.cols, A.map, M.B.sflag, M.B.soff, A.src, A.vals,
                                   A.dinv);
        if (bad) atomicOr(A.flag, bad);
    }
}

// out[e] = scale * u[row(e)] * v[col(e)] for every stored CSR entry e, in CSR
// order (the slot -> CSR map of the ingest).  With u = lambda, v = x and
// scale = -1 this is the derivative of lambda^T (b - A x) with respect to the
// matrix values.
__global__ __launch_bounds__(kBlock) void k_pattern_outer(int n, int nslices,
                                                          const int64_t* __restrict__ sptr,
                                                          const int* __restrict__ cols,
                                                          const int* __restrict__ map,
                                                          const double* __restrict__ u,
                                                          const double* __restrict__ v, double scale,
                                                          double* __restrict__ out) {
    const int total = nslices * kSlice;
    for (int row = blockIdx.x * kBlock + threadIdx.x; row < total; row += gridDim.x * kBlock) {
        if (row >= n) continue;
        const int s = row / kSlice, lane = row % kSlice;
        const int64_t base = sptr[s];
        const int w = (int)((sptr[s + 1] - base) / kSlice);
        const double ur = scale * u[row];
        for (int j = 0; j < w; ++j) {
            const int64_t slot = base + (int64_t)j * kSlice + lane;
            const int m = map[slot];
            if (m >= 0) out[m] = ur * v[cols[slot]];
        }
    }
}

// ---------------------------------------------------------------- products

// Loop kernel 1 of augmented PCG (Alg. 1), iteration k: q = A p and the
// workgroup's share of gamma = (A p, p), stored in gpart[block].  The update
// kernel that follows sums the partials itself (every workgroup, in the same
// order) and forms alpha = (r, z) / gamma, so this kernel ends without a
// serial reduction tail.  T is the storage type of the matrix and vectors
// (FP64, or FP32 for the inner solve of mixed precision); row sums and gamma
// are accumulated in FP64 and q is rounded to T once.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_spmv_gamma(DevBufs B, const T* __restrict__ p,
                                                       T* __restrict__ q, int k) {
    __shared__ double lds[kWavesPerBlock * 1 + 1 + 1];
    if (k >= B.st->stop) return;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int nb = gridDim.x;
    const int ngroups = (B.nslices + kWavesPerBlock - 1) / kWavesPerBlock;
    double g[1] = {0.0};
    // the next slice's metadata is fetched while this slice is processed; the
    // wait for it sits at the end of the iteration, when it has long arrived
    int L = xcd_block(blockIdx.x, nb);
    const int last = B.nslices - 1;
    int cur = slice_meta_load(B, min(L * kWavesPerBlock + wid, last));
    for (; L < ngroups; L += nb) {
        const int s = L * kWavesPerBlock + wid;
        const int nxt = slice_meta_load(B, min((L + nb) * kWavesPerBlock + wid, last));
        if (s < B.nslices) {
            const SliceMeta m = slice_meta_unpack(cur);
            const int row = s * kSlice + lane;
            // offset-table rows return p[row] as gathered at the zero offset,
            // so the (q, p) partial needs no second load of it
            RowDiag<T> o{0.0, (T)0, false};
            if (m.flag == 2 && m.w >= 1 && m.w <= kTabMax) {
                const auto tab = [&](int u) { return m.tab[u]; };
                const T* v = mat_vals<T>(B) + m.base + lane;
                switch (m.w) {
#define PODCG_TAB_CASE(WN) case WN: o = sell_row_tab_diag<T, WN>(B, tab, v, row, p); break;
                    PODCG_TAB_WIDTHS(PODCG_TAB_CASE)
#undef PODCG_TAB_CASE
                    default: break;
                }
            } else {
                o.acc = sell_row_meta<T>(B, m, mat_vals<T>(B), s, lane, p);
            }
            if (row < B.n) {
                const T qv = (T)o.acc;
                q[row] = qv;
                g[0] += (double)qv * (double)(o.has ? o.xd : p[row]);
            }
        }
        cur = nxt;
    }
    block_sum<1>(g, lds);
    if (threadIdx.x == 0) store_shared(B.gpart + blockIdx.x, lds[0]);
}

// Loop kernel 1 in FP64 with two rows per lane and two slices per wave (the
// same products and partials as k_spmv_gamma<double>, row sums in the same
// order; spmv_slice_pair): one pair of slices a wave at a time.
__global__ __launch_bounds__(kBlock) void k_spmv_gamma2(DevBufs B, const double* __restrict__ p,
                                                        double* __restrict__ q, int k) {
    __shared__ double lds[kWavesPerBlock * 1 + 1 + 1];
    if (k >= B.st->stop) return;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int nb = gridDim.x;
    const int npairs = (B.nslices + 1) / 2;
    const int ngroups = (npairs + kWavesPerBlock - 1) / kWavesPerBlock;
    double g[1] = {0.0};
    for (int L = xcd_block(blockIdx.x, nb); L < ngroups; L += nb) {
        const int P = L * kWavesPerBlock + wid;
        if (P < npairs) spmv_slice_pair(B, 2 * P, 2 * P + 1 < B.nslices, lane, p, q, g[0]);
    }
    block_sum<1>(g, lds);
    if (threadIdx.x == 0) store_shared(B.gpart + blockIdx.x, lds[0]);
}

__global__ __launch_bounds__(kBlock) void k_matvec(DevBufs B, const double* __restrict__ x,
                                                   double* __restrict__ y) {
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int nb = gridDim.x;
    const int ngroups = (B.nslices + kWavesPerBlock - 1) / kWavesPerBlock;
    for (int L = xcd_block(blockIdx.x, nb); L < ngroups; L += nb) {
        const int s = L * kWavesPerBlock + wid;
        if (s < B.nslices) {
            const double acc = sell_row<double>(B, B.vals, s, lane, x);
            const int row = s * kSlice + lane;
            if (row < B.n) y[row] = acc;
        }
    }
}

// r = b - A x with reductions.  STAGE1: partials (b, b), (r, r), W^T r; the
// last workgroup sets ||b||^2, the absolute tolerance and the Stage-1
// coefficients what = G^{-1} W^T r (Alg. 2).  Otherwise only (r, r) is kept
// (the true residual at exit).  STORE writes r.
template <int YB, bool STORE, bool STAGE1>
__global__ __launch_bounds__(kBlock) void k_resid(DevBufs B, int y, const double* __restrict__ b,
                                                  const double* __restrict__ x, double* __restrict__ r,
                                                  const double* __restrict__ W) {
    constexpr int NV = 2 + YB;
    __shared__ double lds[kWavesPerBlock * NV + NV + 1];
    DevState* st = B.st;
    if (STAGE1 && st->done != kRunning) return;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int nb = gridDim.x;
    const int ngroups = (B.nslices + kWavesPerBlock - 1) / kWavesPerBlock;
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = 0.0;
    for (int L = xcd_block(blockIdx.x, nb); L < ngroups; L += nb) {
        const int s = L * kWavesPerBlock + wid;
        if (s < B.nslices) {
            const double ax = sell_row<double>(B, B.vals, s, lane, x);
            const int row = s * kSlice + lane;
            if (row < B.n) {
                const double bi = b[row];
                const double ri = bi - ax;
                if (STORE) r[row] = ri;
                v[0] += bi * bi;
                v[1] += ri * ri;
#pragma unroll
                for (int k = 0; k < YB; ++k) {
                    const double wk = W[(size_t)tier_col<YB>(k, y) * B.ld + row];
                    if (tier_live<YB>(k, y)) v[2 + k] += wk * ri;
                }
            }
        }
    }
    if (!grid_sum_last<NV>(v, B.part, B.counter, lds)) return;
    if (STAGE1) {
        if (threadIdx.x == 0) {
            const double bb = lds[0];
            st->bnorm2 = bb;
            st->true_rr = lds[1];
            st->tol2 = st->tol2 * bb;
            if (!is_finite(bb) || !is_finite(lds[1])) {
                st->status = kStNonfinite;
                st->done = kFailed;
                st->stop = 0;       // no loop kernel runs
            }
        }
        if (threadIdx.x < y) {
            double s = 0.0;
            for (int j = 0; j < y; ++j) s += B.Ginv[threadIdx.x * y + j] * lds[2 + j];
            st->what[threadIdx.x] = s;
        }
    } else if (threadIdx.x == 0) {
        st->true_rr = lds[1];
    }
}

// ---------------------------------------------------------------- launchers

static int grid_for_slices(int nslices, int cap = kSpmvGrid) {
    const int groups = (nslices + kWavesPerBlock - 1) / kWavesPerBlock;
    if (cap <= 0) cap = kSpmvGrid;
    return groups < cap ? groups : cap;
}

int spmv_blocks(const DevBufs& B) { return grid_for_slices(B.nslices, B.spmv_grid); }

static int grid_for(int64_t items, int cap) {
    int64_t g = (items + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    return (int)(g < cap ? g : cap);
}

hipError_t launch_validate_csr(int n, int64_t nnz, const int32_t* rowptr, const int32_t* colind,
                               int* flag, hipStream_t s) {
    hipLaunchKernelGGL(k_validate_csr, dim3(grid_for(n, 4096)), dim3(kBlock), 0, s, n, nnz, rowptr,
                       colind, flag);
    return hipGetLastError();
}

hipError_t launch_slice_widths(int n, int nslices, const int32_t* rowptr, int64_t* sptr, hipStream_t s) {
    hipLaunchKernelGGL(k_slice_widths, dim3(grid_for_slices(nslices)), dim3(kBlock), 0, s, n, nslices,
                       rowptr, sptr);
    return hipGetLastError();
}

hipError_t launch_scan_slices(int nslices, int64_t* sptr, hipStream_t s) {
    hipLaunchKernelGGL(k_scan_slices, dim3(1), dim3(1024), 0, s, nslices, sptr);
    return hipGetLastError();
}

hipError_t launch_fill_pattern(int n, int nslices, const int32_t* rowptr, const int32_t* colind,
                               const int64_t* sptr, int* cols, int* map, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_pattern, dim3(grid_for((int64_t)nslices * kSlice, 8192)), dim3(kBlock),
                       0, s, n, nslices, rowptr, colind, sptr, cols, map);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_fill_meta(int nslices, const int64_t* __restrict__ sptr,
                                                      const uint8_t* __restrict__ sflag,
                                                      const int* __restrict__ soff, int* __restrict__ smeta) {
    const int64_t total = (int64_t)nslices * kMetaWords;
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < total; e += (int64_t)gridDim.x * kBlock) {
        const int s = (int)(e / kMetaWords), f = (int)(e % kMetaWords);
        const int64_t base = sptr[s];
        int v = 0;
        if (f == 0) v = (int)(uint32_t)((uint64_t)base & 0xffffffffu);
        else if (f == 1) v = (int)(uint32_t)((uint64_t)base >> 32);
        else if (f == 2) v = (int)((sptr[s + 1] - base) / kSlice);
        else if (f == 3) v = sflag[s];
        else if (f < 4 + kTabMax) v = soff[(size_t)s * kTabMax + (f - 4)];
        smeta[e] = v;
    }
}

hipError_t launch_fill_meta(int nslices, const int64_t* sptr, const uint8_t* sflag, const int* soff, int* smeta,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_fill_meta, dim3(grid_for((int64_t)nslices * kMetaWords, 8192)), dim3(kBlock), 0, s,
                       nslices, sptr, sflag, soff, smeta);
    return hipGetLastError();
}

hipError_t launch_fill_table(int n, int nslices, const int32_t* rowptr, const int64_t* sptr, int* cols,
                             int* map, int* soff, uint8_t* sflag, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_table, dim3(grid_for((int64_t)nslices * kSlice, 8192)), dim3(kBlock), 0, s, n,
                       nslices, rowptr, sptr, cols, map, soff, sflag);
    return hipGetLastError();
}

hipError_t launch_fill_offsets16(int n, int nslices, const int64_t* sptr, const int* cols, int16_t* cols16,
                                 uint8_t* sflag, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_offsets16, dim3(grid_for((int64_t)nslices * kSlice, 8192)), dim3(kBlock), 0, s, n,
                       nslices, sptr, cols, cols16, sflag);
    return hipGetLastError();
}

hipError_t launch_fill_values(int n, int nslices, const int64_t* sptr, const int* cols,
                              const int* map, const uint8_t* sflag, const int* soff, const double* csr_vals,
                              double* vals, double* dinv, int* flag, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_values, dim3(grid_for((int64_t)nslices * kSlice, 8192)), dim3(kBlock),
                       0, s, n, nslices, sptr, cols, map, sflag, soff, csr_vals, vals, dinv, flag);
    return hipGetLastError();
}

hipError_t launch_batch_fill_values(const BatchMember* mem, const BatchAux* aux, const BatchItem* items,
                                    int nitems, int grid, hipStream_t s) {
    if (nitems < 1) return hipSuccess;
    hipLaunchKernelGGL(k_batch_fill_values, dim3(grid < nitems ? grid : nitems), dim3(kBlock), 0, s, mem, aux,
                       items, nitems);
    return hipGetLastError();
}

hipError_t launch_pattern_outer(int n, int nslices, const int64_t* sptr, const int* cols, const int* map,
                                const double* u, const double* v, double scale, double* out,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_pattern_outer, dim3(grid_for((int64_t)nslices * kSlice, 8192)), dim3(kBlock), 0,
                       s, n, nslices, sptr, cols, map, u, v, scale, out);
    return hipGetLastError();
}

hipError_t launch_spmv_gamma(const DevBufs& B, const double* p, double* q, int k, bool pairs, hipStream_t s,
                             hipEvent_t e0, hipEvent_t e1) {
    // the pair kernel's 16-byte accesses need 16-byte aligned vectors; its
    // fallback for slices without a table has no metadata prefetch
    if (pairs && (((uintptr_t)p | (uintptr_t)q) & 15) == 0)
        PODCG_LAUNCH(k_spmv_gamma2, dim3(spmv_blocks(B)), dim3(kBlock), s, e0, e1, B, p, q, k);
    else
        PODCG_LAUNCH((k_spmv_gamma<double>), dim3(spmv_blocks(B)), dim3(kBlock), s, e0, e1, B, p, q, k);
    return hipGetLastError();
}

hipError_t launch_spmv_gamma32(const DevBufs& B, const float* p, float* q, int k, hipStream_t s, hipEvent_t e0,
                               hipEvent_t e1) {
    PODCG_LAUNCH((k_spmv_gamma<float>), dim3(spmv_blocks(B)), dim3(kBlock), s, e0, e1, B, p, q, k);
    return hipGetLastError();
}

hipError_t launch_matvec(const DevBufs& B, const double* x, double* y, hipStream_t s) {
    hipLaunchKernelGGL(k_matvec, dim3(grid_for_slices(B.nslices)), dim3(kBlock), 0, s, B, x, y);
    return hipGetLastError();
}

hipError_t launch_resid(const DevBufs& B, int yb, int y, const double* b, const double* x, double* r,
                        const double* W, bool store, bool stage1, hipStream_t s) {
    dim3 g(grid_for_slices(B.nslices)), t(kBlock);
    if (!stage1) {   // true residual ||b - A x||^2 only
        if (store || yb != 0) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_resid<0, false, false>), g, t, 0, s, B, 0, b, x, r, W);
        return hipGetLastError();
    }
    if (!store) return hipErrorInvalidValue;
    switch (yb) {
#define CASE(T) case T: hipLaunchKernelGGL((k_resid<T, true, true>), g, t, 0, s, B, y, b, x, r, W); break;
        PODCG_TIERS(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace podcg
