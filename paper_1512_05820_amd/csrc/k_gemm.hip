// Tall-skinny dense products of the three-stage truncation (Alg. pod_evd
// applied to the accumulated basis, Alg. 3) on the FP64 matrix cores:
//   Gram   Zbar = Z^T (A Z)       M x M, inner dimension n (millions of rows);
//   basis  Y   = Z T               n x y, T = diag(eta) V_y Sigma_y^{-1} (M x y).
// Both run on v_mfma_f64_16x16x4f64 with the lane layout used throughout the
// library: lane l supplies A[i = l % 16][k = l / 16] and B[k = l / 16][j = l % 16],
// and register r of lane l accumulates D[4 r + l / 16][l % 16].
//
// A workgroup of four wavefronts owns a 64-row output tile (2 x 2 wavefronts of
// 32 x 32, each 2 x 2 MFMA blocks; the basis product uses 2 x 4 blocks per
// wavefront for 128 output columns).  Operand panels of 32 inner rows are
// staged through LDS with coalesced loads (one column's rows are contiguous
// in the column-major blocks), the next panel's loads in flight while the
// current one feeds the matrix cores.
#include "podcg_launch.h"

namespace podcg {

typedef double dv4_t __attribute__((ext_vector_type(4)));

constexpr int kGemmTile = 64;                 // output rows (and Gram columns) per workgroup
constexpr int kGemmPanel = 32;                // inner rows per LDS panel
constexpr int kGemmLd = kGemmTile + 1;        // padded LDS row stride
constexpr int kGemmLoads = kGemmPanel * kGemmTile / kBlock;   // doubles per thread per operand panel (8)

// Partial Gram of row chunk c: P_c[i][j] = sum over rows r of chunk c of
// X[r][ti 64 + i] Y[r][tj 64 + j], written at P + c pstride + (ti 64 + i) ldp
// + tj 64 + j for the rows < M and columns < N of the tile.  SYM (X^T A X with
// Y = A X): only tiles ti <= tj are computed (the sum mirrors the rest).
// Grid: (tiles, chunks); tile t enumerates (ti, tj) row-major over the
// computed tiles.
template <bool SYM>
__global__ __launch_bounds__(kBlock) void k_gemm_tn_part(int n, size_t ld, const double* __restrict__ X, int M,
                                                         const double* __restrict__ Y, int N, int rows_per_chunk,
                                                         double* __restrict__ P, size_t pstride, int ldp) {
    __shared__ double xs[kGemmPanel * kGemmLd], ys[kGemmPanel * kGemmLd];
    const int tilesN = (N + kGemmTile - 1) / kGemmTile;
    int ti, tj;
    {
        int t = blockIdx.x;
        if (SYM) {                                // upper-triangle tile t -> (ti, tj), ti <= tj
            ti = 0;
            while (t >= tilesN - ti) {
                t -= tilesN - ti;
                ++ti;
            }
            tj = ti + t;
        } else {
            ti = t / tilesN;
            tj = t % tilesN;
        }
    }
    const int c = blockIdx.y;
    const int r0 = c * rows_per_chunk;
    const int r1 = min(n, r0 + rows_per_chunk);
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    const int wi = wid >> 1, wj = wid & 1;
    const int cx0 = ti * kGemmTile, cy0 = tj * kGemmTile;
    dv4_t d[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) d[a][b] = dv4_t{0.0, 0.0, 0.0, 0.0};
    // this thread's share of a panel: element e = tid + kBlock u is column
    // e / 32 of the tile, inner row e % 32 (a wave reads two columns' 32 rows)
    double xr[kGemmLoads], yr[kGemmLoads];
    auto load = [&](int k0) {
#pragma unroll
        for (int u = 0; u < kGemmLoads; ++u) {
            const int e = tid + kBlock * u;
            const int col = e / kGemmPanel, row = k0 + e % kGemmPanel;
            const bool rin = row < r1;
            const int cx = cx0 + col, cy = cy0 + col;
            xr[u] = (rin && cx < M) ? X[(size_t)cx * ld + row] : 0.0;
            yr[u] = (rin && cy < N) ? Y[(size_t)cy * ld + row] : 0.0;
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int u = 0; u < kGemmLoads; ++u) {
            const int e = tid + kBlock * u;
            const int col = e / kGemmPanel, row = e % kGemmPanel;
            xs[row * kGemmLd + col] = xr[u];
            ys[row * kGemmLd + col] = yr[u];
        }
    };
    const int r4 = lane >> 4, cc = lane & 15;
    if (r0 < r1) load(r0);
    for (int k0 = r0; k0 < r1; k0 += kGemmPanel) {
        __syncthreads();                          // the previous panel has been consumed
        stash();
        __syncthreads();
        if (k0 + kGemmPanel < r1) load(k0 + kGemmPanel);   // next panel in flight
#pragma unroll
        for (int kk = 0; kk < kGemmPanel / 4; ++kk) {
            const int kr = 4 * kk + r4;
            double a[2], b[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                a[q] = xs[kr * kGemmLd + 32 * wi + 16 * q + cc];
                b[q] = ys[kr * kGemmLd + 32 * wj + 16 * q + cc];
            }
#pragma unroll
            for (int qa = 0; qa < 2; ++qa)
#pragma unroll
                for (int qb = 0; qb < 2; ++qb)
                    d[qa][qb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[qa], b[qb], d[qa][qb], 0, 0, 0);
        }
    }
    double* Pc = P + (size_t)c * pstride;
#pragma unroll
    for (int qa = 0; qa < 2; ++qa)
#pragma unroll
        for (int qb = 0; qb < 2; ++qb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gi = cx0 + 32 * wi + 16 * qa + 4 * r + r4;
                const int gj = cy0 + 32 * wj + 16 * qb + cc;
                if (gi < M && gj < N) Pc[(size_t)gi * ldp + gj] = d[qa][qb][r];
            }
}

// G[i][j] = sum over the chunks, in chunk order, of P_c[i][j]; with SYM the
// entries of tiles below the diagonal come from the mirrored entry.
__global__ __launch_bounds__(kBlock) void k_gram_sum(const double* __restrict__ P, int nparts, size_t pstride,
                                                     int M, int N, int ldp, int sym, double* __restrict__ G,
                                                     int ldg) {
    for (int e = blockIdx.x * kBlock + threadIdx.x; e < M * N; e += gridDim.x * kBlock) {
        int i = e / N, j = e % N;
        if (sym && i / kGemmTile > j / kGemmTile) {
            const int t = i;
            i = j;
            j = t;
        }
        double s = 0.0;
        for (int c = 0; c < nparts; ++c) s += P[(size_t)c * pstride + (size_t)i * ldp + j];
        G[(size_t)(e / N) * ldg + e % N] = s;
    }
}

// Out[r][c] = sum_k X[r][k] T[k][c] for r < n, c < Ny: X n x M and Out n x Ny
// column-major (leading dimension ld), T column-major M x Ny (leading
// dimension ldt).  A workgroup computes 64 rows by 128 columns; each
// wavefront 32 rows by 64 columns (2 x 4 MFMA blocks).  The output tile is
// staged through LDS so that each column's 64 rows are stored contiguously.
constexpr int kNnCols = 128;
constexpr int kNnLdT = kNnCols + 1;
__global__ __launch_bounds__(kBlock) void k_gemm_nn(int n, size_t ld, const double* __restrict__ X, int M,
                                                    const double* __restrict__ T, int ldt, int Ny,
                                                    double* __restrict__ Out) {
    // xs: 32 inner rows (k) x 64 output rows; ts: 32 x 128 columns; the output
    // tile (128 columns x 64 rows) reuses the same space after the inner loop
    constexpr int XS = kGemmPanel * kGemmLd, TS = kGemmPanel * kNnLdT;
    constexpr int OS = kNnCols * kGemmLd;
    __shared__ double sh[(XS + TS) > OS ? (XS + TS) : OS];
    double* xs = sh;
    double* ts = sh + XS;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    const int wi = wid >> 1, wj = wid & 1;
    const int r0 = blockIdx.x * kGemmTile;
    const int c0 = blockIdx.y * kNnCols;
    dv4_t d[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) d[a][b] = dv4_t{0.0, 0.0, 0.0, 0.0};
    // X panel: element e = tid + kBlock u is inner row e / 64, output row e % 64
    // (a wave reads 64 contiguous rows of one column of X); T panel: element
    // e is column e / 32, inner row e % 32 (one column's 32 rows contiguous)
    constexpr int XL = kGemmPanel * kGemmTile / kBlock;   // 8
    constexpr int TL = kGemmPanel * kNnCols / kBlock;     // 16
    double xr[XL], tr[TL];
    auto load = [&](int k0) {
#pragma unroll
        for (int u = 0; u < XL; ++u) {
            const int e = tid + kBlock * u;
            const int k = k0 + e / kGemmTile, r = r0 + e % kGemmTile;
            xr[u] = (k < M && r < n) ? X[(size_t)k * ld + r] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < TL; ++u) {
            const int e = tid + kBlock * u;
            const int col = c0 + e / kGemmPanel, k = k0 + e % kGemmPanel;
            tr[u] = (k < M && col < Ny) ? T[(size_t)col * ldt + k] : 0.0;
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int u = 0; u < XL; ++u) {
            const int e = tid + kBlock * u;
            xs[(e / kGemmTile) * kGemmLd + e % kGemmTile] = xr[u];
        }
#pragma unroll
        for (int u = 0; u < TL; ++u) {
            const int e = tid + kBlock * u;
            ts[(e % kGemmPanel) * kNnLdT + e / kGemmPanel] = tr[u];
        }
    };
    const int r4 = lane >> 4, cc = lane & 15;
    load(0);
    for (int k0 = 0; k0 < M; k0 += kGemmPanel) {
        __syncthreads();
        stash();
        __syncthreads();
        if (k0 + kGemmPanel < M) load(k0 + kGemmPanel);
#pragma unroll
        for (int kk = 0; kk < kGemmPanel / 4; ++kk) {
            const int kr = 4 * kk + r4;
            double a[2], b[4];
#pragma unroll
            for (int q = 0; q < 2; ++q) a[q] = xs[kr * kGemmLd + 32 * wi + 16 * q + cc];
#pragma unroll
            for (int q = 0; q < 4; ++q) b[q] = ts[kr * kNnLdT + 64 * wj + 16 * q + cc];
#pragma unroll
            for (int qa = 0; qa < 2; ++qa)
#pragma unroll
                for (int qb = 0; qb < 4; ++qb)
                    d[qa][qb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[qa], b[qb], d[qa][qb], 0, 0, 0);
        }
    }
    __syncthreads();                              // every wave is done with xs / ts
    double* os = sh;                              // os[col * kGemmLd + row]
#pragma unroll
    for (int qa = 0; qa < 2; ++qa)
#pragma unroll
        for (int qb = 0; qb < 4; ++qb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 32 * wi + 16 * qa + 4 * r + r4;
                const int j = 64 * wj + 16 * qb + cc;
                os[j * kGemmLd + i] = d[qa][qb][r];
            }
    __syncthreads();
    for (int e = tid; e < kNnCols * kGemmTile; e += kBlock) {
        const int j = e / kGemmTile, i = e % kGemmTile;
        if (c0 + j < Ny && r0 + i < n) Out[(size_t)(c0 + j) * ld + r0 + i] = os[j * kGemmLd + i];
    }
}

// ---------------------------------------------------------------- launchers

int gemm_tn_tiles(int M, int N, bool sym) {
    const int tm = (M + kGemmTile - 1) / kGemmTile, tn = (N + kGemmTile - 1) / kGemmTile;
    return sym ? tn * (tn + 1) / 2 : tm * tn;
}

hipError_t launch_gemm_tn_parts(int n, size_t ld, const double* X, int M, const double* Y, int N, int chunks,
                                bool sym, double* P, size_t pstride, int ldp, hipStream_t s) {
    if (n < 1 || M < 1 || N < 1 || chunks < 1 || ldp < N || (sym && M != N) || pstride < (size_t)M * ldp)
        return hipErrorInvalidValue;
    int rows = (n + chunks - 1) / chunks;
    rows = (rows + kGemmPanel - 1) / kGemmPanel * kGemmPanel;
    chunks = (n + rows - 1) / rows;
    const dim3 g(gemm_tn_tiles(M, N, sym), chunks);
    if (sym)
        hipLaunchKernelGGL((k_gemm_tn_part<true>), g, dim3(kBlock), 0, s, n, ld, X, M, Y, N, rows, P, pstride, ldp);
    else
        hipLaunchKernelGGL((k_gemm_tn_part<false>), g, dim3(kBlock), 0, s, n, ld, X, M, Y, N, rows, P, pstride, ldp);
    return hipGetLastError();
}

int gemm_tn_chunks(int n, int chunks) {
    int rows = (n + chunks - 1) / chunks;
    rows = (rows + kGemmPanel - 1) / kGemmPanel * kGemmPanel;
    return (n + rows - 1) / rows;
}

hipError_t launch_gram_sum(const double* P, int nparts, size_t pstride, int M, int N, int ldp, bool sym,
                           double* G, int ldg, hipStream_t s) {
    if (M < 1 || N < 1 || nparts < 1) return hipErrorInvalidValue;
    int g = (M * N + kBlock - 1) / kBlock;
    if (g > 2048) g = 2048;
    hipLaunchKernelGGL(k_gram_sum, dim3(g), dim3(kBlock), 0, s, P, nparts, pstride, M, N, ldp, sym ? 1 : 0, G, ldg);
    return hipGetLastError();
}

hipError_t launch_gemm_nn(int n, size_t ld, const double* X, int M, const double* T, int ldt, int Ny,
                          double* Out, hipStream_t s) {
    if (n < 1 || M < 1 || Ny < 1 || ldt < M) return hipErrorInvalidValue;
    const dim3 g((n + kGemmTile - 1) / kGemmTile, (Ny + kNnCols - 1) / kNnCols);
    hipLaunchKernelGGL(k_gemm_nn, g, dim3(kBlock), 0, s, n, ld, X, M, T, ldt, Ny, Out);
    return hipGetLastError();
}

}  // namespace podcg
