// Kernels of the three-stage method (Alg. 3): products with the tall
// accumulated basis Y (n x m, m <= kTsCap, column-major with leading dimension
// ld), the reduced iteration of Stage 2 (Section 4.2), the factor of the
// Stage-3 basis, the bookkeeping of the accumulated vectors and weights
// (Section 3.3.2) and the eigen-decomposition of the weighted snapshot Gram of
// a truncation (Alg. pod_evd).
#include "podcg_launch.h"

namespace podcg {

// ------------------------------------------------------------ tall products

// out = sign * Y c (accumulate: out += sign * Y c); c has m entries.
__global__ __launch_bounds__(kBlock) void k_gemv_n(int n, size_t ld, const double* __restrict__ Y, int m,
                                                   const double* __restrict__ c, double* __restrict__ out,
                                                   double sign, int accumulate) {
    __shared__ double cs[kTsCap];
    for (int k = threadIdx.x; k < m; k += kBlock) cs[k] = c[k];
    __syncthreads();
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        double acc = 0.0;
#pragma unroll 8
        for (int k = 0; k < m; ++k) acc += Y[(size_t)k * ld + i] * cs[k];
        out[i] = accumulate ? out[i] + sign * acc : sign * acc;
    }
}

// part[g * m + k] = sum over the rows of chunk g of Y(i, k) v(i): each wave
// takes 16 columns at a time (one load of v per row for all 16), lanes over
// the rows; the last group re-reads the last column instead of branching.  The
// grid is row chunks (x) by groups of 64 columns (y).  Measured at 128^3 with
// 100 columns: 305 us (5.5 TB/s) against 515 us with 8 columns a wave (and
// 350 us with 4, 516 us with 8 and deeper unrolling).
constexpr int kGemvCols = 16;
__global__ __launch_bounds__(kBlock) void k_gemv_t_part(int n, size_t ld, const double* __restrict__ Y,
                                                        int m, const double* __restrict__ v,
                                                        double* __restrict__ part, int rows) {
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int r0 = blockIdx.x * rows;
    const int r1 = min(n, r0 + rows);
    for (int k0 = (blockIdx.y * kWavesPerBlock + wid) * kGemvCols; k0 < m;
         k0 += gridDim.y * kWavesPerBlock * kGemvCols) {
        double acc[kGemvCols];
        const double* __restrict__ yk[kGemvCols];
#pragma unroll
        for (int u = 0; u < kGemvCols; ++u) {
            acc[u] = 0.0;
            yk[u] = Y + (size_t)min(k0 + u, m - 1) * ld;
        }
#pragma unroll 2
        for (int i = r0 + lane; i < r1; i += kWave) {
            const double vi = v[i];
#pragma unroll
            for (int u = 0; u < kGemvCols; ++u) acc[u] += yk[u][i] * vi;
        }
#pragma unroll
        for (int u = 0; u < kGemvCols; ++u) {
            const double t = wave_sum(acc[u]);
            if (lane == 0 && k0 + u < m) part[(size_t)blockIdx.x * m + k0 + u] = t;
        }
    }
}

// out[k] = sum_g part[g * m + k]: one wave per k, lane l adding the chunks
// l, l + 64, ... in order, then the wave's butterfly (a fixed order).
__global__ __launch_bounds__(kBlock) void k_gemv_t_reduce(const double* __restrict__ part, int chunks, int m,
                                                          double* __restrict__ out) {
    const int lane = threadIdx.x & (kWave - 1);
    const int k = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (k >= m) return;   // wave-uniform
    double s = 0.0;
    for (int g = lane; g < chunks; g += kWave) s += part[(size_t)g * m + k];
    s = wave_sum(s);
    if (lane == 0) out[k] = s;
}

// ------------------------------------------------------------------ Stage 2
// Augmented CG (Alg. 1 with M = I) on Ghat = Y^T A Y in reduced coordinates,
// augmented by What (W = Y What: the columns sel of Y).  The solves with
// What^T Ghat What = W^T A W reuse G_W^{-1} from Stage 1; What^T Ghat z is
// (A W)^T Y z = wtgy z with wtgy = (A W)^T Y computed once per system.

// Sum of a value over the workgroup, fixed order; every thread gets it.
__device__ __forceinline__ double ts_block_sum(double v, double* lds) {
    double a[1] = {v};
    block_sum<1>(a, lds);
    const double r = lds[0];
    __syncthreads();
    return r;
}

// mu = G_W^{-1} (wtgy z) into mu_s (LDS, w entries); then p = z + beta p - What mu.
__device__ __forceinline__ void ts_project(TsDev* T, int m, const int* sel, int w, const double* GinvW,
                                           double beta, bool first, double* c_s, double* mu_s) {
    const int t = threadIdx.x;
    if (t < w) {
        double s = 0.0;
        for (int k = 0; k < m; ++k) s += T->wtgy[(size_t)t * m + k] * T->rh[k];
        c_s[t] = s;
    }
    __syncthreads();
    if (t < w) {
        double s = 0.0;
        for (int j = 0; j < w; ++j) s += GinvW[t * w + j] * c_s[j];
        mu_s[t] = s;
    }
    __syncthreads();
    for (int k = t; k < m; k += kBlock) T->ph[k] = first ? T->rh[k] : T->rh[k] + beta * T->ph[k];
    __syncthreads();
    if (t < w) T->ph[sel[t]] -= mu_s[t];
    __syncthreads();
}

// Start of Stage 2: rh = Y^T (b - A xbar - A W what) is already in T->rh.
// xh = What what, p = z - What mu, rz = (r, z), the tolerance
// max(tau_rel ||b||, floor ||rh||) and the iteration cap.
// The stage-2 increment xinc and the augmentation count of the iterative
// Stage 3 start at zero.
__global__ __launch_bounds__(kBlock) void k_ts_s2_init(TsDev* T, const DevState* st, int m,
                                                       const int* __restrict__ sel, int w,
                                                       const double* __restrict__ GinvW, double tau_rel,
                                                       double floor_rel, int k2max) {
    __shared__ double lds[kWavesPerBlock + 2];
    __shared__ double c_s[kYMax], mu_s[kYMax];
    const int t = threadIdx.x;
    for (int k = t; k < m; k += kBlock) {
        T->xh[k] = 0.0;
        T->xinc[k] = 0.0;
    }
    if (t == 0) {
        T->naug = 0;
        T->knew = 0;
    }
    __syncthreads();
    if (t < w) T->xh[sel[t]] = st->what[t];
    double a = 0.0;
    for (int k = t; k < m; k += kBlock) a += T->rh[k] * T->rh[k];
    const double rz = ts_block_sum(a, lds);
    ts_project(T, m, sel, w, GinvW, 0.0, true, c_s, mu_s);
    if (t == 0) {
        const double rn0 = sqrt(rz);
        T->rz2 = rz;
        T->rn0 = rn0;
        T->rn = rn0;
        T->tau = fmax(tau_rel * sqrt(st->bnorm2), floor_rel * rn0);
        T->k2 = 0;
        T->k2max = k2max;
        T->done2 = (rn0 <= T->tau || k2max <= 0) ? 1 : 0;
    }
}

// One Stage-2 iteration once gh = Ghat p is in T->gh.  With aug (the
// iterative Stage 3), the direction joins the augmentation when it was formed
// from a residual of at least kTsKeepFloor of the initial one, and the
// increment sum alpha p is kept in xinc; the per-step scalars of the
// [W, X] basis are recorded for the first kYMax steps.
__global__ __launch_bounds__(kBlock) void k_ts_s2_step(TsDev* T, int m, const int* __restrict__ sel, int w,
                                                       const double* __restrict__ GinvW, double* __restrict__ aug) {
    __shared__ double lds[kWavesPerBlock + 2];
    __shared__ double c_s[kYMax], mu_s[kYMax];
    __shared__ int stop;
    const int t = threadIdx.x;
    if (T->done2) return;
    double a = 0.0;
    for (int k = t; k < m; k += kBlock) a += T->ph[k] * T->gh[k];
    const double g = ts_block_sum(a, lds);
    if (t == 0) stop = !(g > 0.0);
    __syncthreads();
    if (stop) {
        if (t == 0) T->done2 = 1;
        return;
    }
    const double alpha = T->rz2 / g;
    const int naug = T->naug;
    const bool keep = aug && T->rn >= kTsKeepFloor * T->rn0 && naug < m;
    if (keep)
        for (int k = t; k < m; k += kBlock) {
            aug[(size_t)naug * kTsCap + k] = T->ph[k];
            aug[(size_t)(kTsCap + naug) * kTsCap + k] = T->gh[k];
        }
    double b2 = 0.0;
    for (int k = t; k < m; k += kBlock) {
        T->xh[k] += alpha * T->ph[k];
        T->xinc[k] += alpha * T->ph[k];
        const double r = T->rh[k] - alpha * T->gh[k];
        T->rh[k] = r;
        b2 += r * r;
    }
    const double rz_new = ts_block_sum(b2, lds);
    const double beta = rz_new / T->rz2;
    const int k2 = T->k2;
    __syncthreads();   // every thread has read rz2, rn, naug and k2
    if (t == 0) {
        if (keep) {
            T->gam_aug[naug] = g;
            T->naug = naug + 1;
        }
        if (k2 < kYMax) {
            T->gam2[k2] = g;
            T->alp2[k2] = alpha;
        }
        T->rz2 = rz_new;
        T->k2 = k2 + 1;
        T->rn = sqrt(rz_new);
        T->done2 = (sqrt(rz_new) <= T->tau || k2 + 1 >= T->k2max) ? 1 : 0;
    }
    ts_project(T, m, sel, w, GinvW, beta, false, c_s, mu_s);
}

// ------------------------------------------- iterative Stage 3 (phi = 1)
// Projection solves Ghat mu = c (Section 4.3.1): augmented CG on Ghat (M = I)
// against the reduced stage-1 columns What and the kept directions P_l
// (l < naug0), mutually Ghat-orthogonal, so the solves with B^T Ghat B use
// blockdiag(G_W^{-1}, diag(1 / gam_aug)); Ghat What = ((A W)^T Y)^T = wtgy^T and
// Ghat P_l are kept, so no product with Ghat is needed to use them.  One
// workgroup of kTsThreads threads; vectors of m <= kTsCap entries.
constexpr int kTsThreads = 1024;
constexpr int kTsWaves = kTsThreads / kWave;

__device__ __forceinline__ double ts_sum(double v, double* red) {
    v = wave_sum(v);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    double s = red[0];
    for (int w = 1; w < kTsWaves; ++w) s += red[w];
    __syncthreads();
    return s;
}

// ph = rh + beta ph - What nu_w - sum_{l < na} P_l nu_l with
// nu = blockdiag(G_W^{-1}, 1 / gam_aug) B^T Ghat rh (the projection of steps
// aug2 / aug3 of Alg. 1 on Ghat).
__device__ void ts_in_direction(TsDev* T, const double* __restrict__ aug, int m, const int* __restrict__ sel,
                                int w, const double* __restrict__ GinvW, int na, double beta, bool first,
                                double* cw, double* nuw, double* nd) {
    const int t = threadIdx.x;
    const double* __restrict__ G = aug + (size_t)kTsCap * kTsCap;
    if (t < w) {
        double s = 0.0;
        for (int k = 0; k < m; ++k) s += T->wtgy[(size_t)t * m + k] * T->rh[k];
        cw[t] = s;
    }
    for (int l = t; l < na; l += kTsThreads) {
        double s = 0.0;
        for (int k = 0; k < m; ++k) s += G[(size_t)l * kTsCap + k] * T->rh[k];
        nd[l] = s / T->gam_aug[l];
    }
    __syncthreads();
    if (t < w) {
        double s = 0.0;
        for (int j = 0; j < w; ++j) s += GinvW[t * w + j] * cw[j];
        nuw[t] = s;
    }
    __syncthreads();
    for (int k = t; k < m; k += kTsThreads) {
        double v = first ? T->rh[k] : T->rh[k] + beta * T->ph[k];
        for (int l = 0; l < na; ++l) v -= aug[(size_t)l * kTsCap + k] * nd[l];
        for (int i = 0; i < w; ++i) v -= sel[i] == k ? nuw[i] : 0.0;
        T->ph[k] = v;
    }
    __syncthreads();
}

// gh = Ghat ph for Stage 2 when Ghat = Y^T A Y has been formed (one
// workgroup; Ghat row-major m x m).
__global__ __launch_bounds__(kTsThreads) void k_ts_ghat_mv(TsDev* T, const double* __restrict__ Ghat, int m) {
    for (int k = threadIdx.x; k < m; k += kTsThreads) {
        const double* __restrict__ g = Ghat + (size_t)k * m;
        double s = 0.0;
        for (int l = 0; l < m; ++l) s += g[l] * T->ph[l];
        T->gh[k] = s;
    }
}

// A whole projection solve Ghat mu = c (c in T->cin) in one launch, with the
// reduced matrix Ghat = Y^T A Y formed beforehand (row-major m x m).  Start:
// the Galerkin solution over the kept directions (mu = B nu, nu =
// blockdiag(G_W^{-1}, 1 / gam_aug) B^T c, B^T c = (c[sel], P_l^T c)), its
// residual rh = c - Ghat B nu, the tolerance rel ||c|| and the first
// direction.  Steps: gh = Ghat ph, mu += alpha ph, rh -= alpha gh; a
// direction joins the augmentation (after the kept ones) when it was formed
// from a residual of at least kTsKeepFloor of ||c|| (the residual is computed
// with cancellation against c), then the next direction, projected against
// the directions kept before this solve.  The start and the projections
// assume the kept directions Ghat-orthogonal; kept from many solves they can
// lose that in rounding, and a solve can then stall.  A solve that ends
// above its tolerance after kinmax steps is therefore done once more with
// none kept (the stage-1 columns only), and the directions of that second
// solve replace the kept set.  The solve's scalars stay in registers (the
// same in every thread); acc[0] accumulates the steps and acc[1] the solves.
__global__ __launch_bounds__(kTsThreads) void k_ts_in_solve(TsDev* T, double* __restrict__ aug, int m,
                                                            const int* __restrict__ sel, int w,
                                                            const double* __restrict__ GinvW,
                                                            const double* __restrict__ Ghat, double rel,
                                                            int kinmax, int* __restrict__ acc) {
    __shared__ double red[kTsWaves];
    __shared__ double cw[kYMax], nuw[kYMax], nd[kTsCap];
    const int t = threadIdx.x;
    const double* __restrict__ G = aug + (size_t)kTsCap * kTsCap;
    int na = T->naug;
    int kin = 0, knew = 0, kall = 0;
    double rz = 0.0, rn0 = 0.0, cn = 0.0, tau = 0.0;
    bool conv = false;
    for (int attempt = 0; attempt < 2; ++attempt) {
        if (t < w) cw[t] = T->cin[sel[t]];
        for (int l = t; l < na; l += kTsThreads) {
            double s = 0.0;
            for (int k = 0; k < m; ++k) s += aug[(size_t)l * kTsCap + k] * T->cin[k];
            nd[l] = s / T->gam_aug[l];
        }
        __syncthreads();
        if (t < w) {
            double s = 0.0;
            for (int j = 0; j < w; ++j) s += GinvW[t * w + j] * cw[j];
            nuw[t] = s;
        }
        __syncthreads();
        double rr = 0.0, cc = 0.0;
        for (int k = t; k < m; k += kTsThreads) {
            const double c = T->cin[k];
            double mu = 0.0, r = c;
            for (int i = 0; i < w; ++i) {
                mu += sel[i] == k ? nuw[i] : 0.0;
                r -= T->wtgy[(size_t)i * m + k] * nuw[i];
            }
            for (int l = 0; l < na; ++l) {
                mu += aug[(size_t)l * kTsCap + k] * nd[l];
                r -= G[(size_t)l * kTsCap + k] * nd[l];
            }
            T->muin[k] = mu;
            T->rh[k] = r;
            rr += r * r;
            cc += c * c;
        }
        rz = ts_sum(rr, red);
        cn = sqrt(ts_sum(cc, red));
        rn0 = sqrt(rz);
        tau = rel * cn;
        conv = rn0 <= tau;
        bool done = conv || kinmax <= 0;
        kin = 0;
        knew = 0;
        if (!done) ts_in_direction(T, aug, m, sel, w, GinvW, na, 0.0, true, cw, nuw, nd);
        while (!done) {
            // gh = Ghat ph
            for (int k = t; k < m; k += kTsThreads) {
                const double* __restrict__ g = Ghat + (size_t)k * m;
                double s = 0.0;
                for (int l = 0; l < m; ++l) s += g[l] * T->ph[l];
                T->gh[k] = s;
            }
            __syncthreads();
            double a = 0.0;
            for (int k = t; k < m; k += kTsThreads) a += T->ph[k] * T->gh[k];
            const double g = ts_sum(a, red);
            if (!(g > 0.0)) break;
            const double alpha = rz / g;
            const int slot = na + knew;
            const bool keep = sqrt(rz) >= kTsKeepFloor * cn && slot < m;
            double b2 = 0.0;
            for (int k = t; k < m; k += kTsThreads) {
                const double p = T->ph[k], gk = T->gh[k];
                if (keep) {
                    aug[(size_t)slot * kTsCap + k] = p;
                    aug[(size_t)(kTsCap + slot) * kTsCap + k] = gk;
                }
                T->muin[k] += alpha * p;
                const double r = T->rh[k] - alpha * gk;
                T->rh[k] = r;
                b2 += r * r;
            }
            const double rz_new = ts_sum(b2, red);
            if (keep && t == 0) T->gam_aug[slot] = g;
            ++kin;
            if (keep) ++knew;
            conv = sqrt(rz_new) <= tau;
            done = conv || kin >= kinmax;
            if (!done) ts_in_direction(T, aug, m, sel, w, GinvW, na, rz_new / rz, false, cw, nuw, nd);
            rz = rz_new;
        }
        kall += kin;
        if (conv || na == 0) break;
        na = 0;   // stalled with kept directions: once more with none
        __syncthreads();
    }
    if (t == 0) {
        T->rzin = rz;
        T->rn0in = rn0;
        T->tauin = tau;
        T->cnin = cn;
        T->kin = kall;
        T->kinmax = kinmax;
        T->naug0 = na;
        T->knew = knew;
        T->donein = 1;
        T->naug = na + knew;
        acc[0] += kall;
        acc[1] += 1;
    }
}

// ------------------------------------------------------------------ Stage 3
// Inverse of the reused factor blockdiag(R, sqrt(Gammahat)) of [W, X]^T A [W, X]
// (Section 4.3): blockdiag(G_W^{-1}, Gammahat^{-1}), row-major (w + k2)^2.
__global__ void k_ts_ginv_blockdiag(const double* __restrict__ GinvW, int w, const TsDev* T, int k2,
                                    double* __restrict__ GinvB) {
    const int y = w + k2;
    for (int e = threadIdx.x; e < y * y; e += blockDim.x) {
        const int i = e / y, j = e % y;
        double v = 0.0;
        if (i < w && j < w) v = GinvW[i * w + j];
        else if (i == j) v = 1.0 / T->gam2[i - w];
        GinvB[e] = v;
    }
}

// ------------------------------------------------------- accumulated vectors

// eta_prev = [xh (m); alpha_k sqrt(gamma_k) (kr)] (coefficients of x - xbar in
// Z = [Y, V Gamma^{-1/2}]); eta_acc = eta_prev + eta_acc / 2 (RBF weights with
// 2^{1-i}, Section 3.3.2).
__global__ __launch_bounds__(kBlock) void k_ts_eta(TsDev* T, int m, int kr) {
    for (int e = blockIdx.x * kBlock + threadIdx.x; e < m + kr; e += gridDim.x * kBlock) {
        const double prev = e < m ? T->xh[e] : T->alp3[e - m] * sqrt(T->gam3[e - m]);
        T->eta_prev[e] = prev;
        T->eta_acc[e] = prev + 0.5 * T->eta_acc[e];
    }
}

// B(:, c) = Y(:, sel[c]).
__global__ __launch_bounds__(kBlock) void k_ts_gather(const double* __restrict__ Y, size_t ld, int n,
                                                      const int* __restrict__ sel, double* __restrict__ B) {
    const int c = blockIdx.y;
    const double* __restrict__ src = Y + (size_t)sel[c] * ld;
    double* __restrict__ dst = B + (size_t)c * ld;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) dst[i] = src[i];
}

// ------------------------------------------------------------- truncation

// G <- diag(eta) sym(G) diag(eta), M x M.
__global__ __launch_bounds__(kBlock) void k_ts_weight_sym(double* __restrict__ G, int M,
                                                          const double* __restrict__ eta) {
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= M * M) return;
    const int i = e / M, j = e % M;
    if (j < i) return;
    const double s = 0.5 * (G[i * M + j] + G[j * M + i]) * eta[i] * eta[j];
    G[i * M + j] = s;
    G[j * M + i] = s;
}

constexpr int kJacobiThreads = 1024;

// Cyclic Jacobi eigen-decomposition of the symmetric M x M matrix A
// (row-major), spread over the whole GPU: each sweep runs Mp - 1 rounds
// (Mp = M rounded up to even) of Mp / 2 disjoint rotations in round-robin
// pairing.  Disjoint rotations commute, so J^T A J splits into independent
// 2 x 2 blocks (rows of pair a, columns of pair b): one launch per round
// reads A from one buffer and writes the rotated blocks to the other (every
// entry is written once), and the (p, q) entries of the rotated pairs are set
// to zero.  Every workgroup first forms the round's rotations from the input
// buffer.

__device__ __forceinline__ void jac_pair(int i, int r, int Mp, int& p, int& q) {
    int a, b;
    if (i == 0) {
        a = Mp - 1;
        b = r;
    } else {
        a = (r + i) % (Mp - 1);
        b = (r - i + Mp - 1) % (Mp - 1);
    }
    p = a < b ? a : b;
    q = a < b ? b : a;
}

__global__ __launch_bounds__(kBlock) void k_jac_round(const double* __restrict__ A, double* __restrict__ An,
                                                      double* __restrict__ V, int M, int r) {
    __shared__ double cs[kTsCap / 2], sn[kTsCap / 2];
    __shared__ int pp[kTsCap / 2], qq[kTsCap / 2];
    const int Mp = M + (M & 1);
    const int np = Mp / 2;
    for (int i = threadIdx.x; i < np; i += kBlock) {
        int p, q;
        jac_pair(i, r, Mp, p, q);
        double c = 1.0, s = 0.0;
        if (q < M) {
            const double apq = A[p * M + q];
            if (apq != 0.0) {
                const double tau = (A[q * M + q] - A[p * M + p]) / (2.0 * apq);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                c = 1.0 / sqrt(1.0 + t * t);
                s = t * c;
            }
        }
        cs[i] = c;
        sn[i] = s;
        pp[i] = p;
        qq[i] = q < M ? q : -1;
    }
    __syncthreads();
    const int nblk = np * np;
    const int total = nblk + M * np;
    for (int e = blockIdx.x * kBlock + threadIdx.x; e < total; e += gridDim.x * kBlock) {
        if (e < nblk) {                                   // block (a, b) of A
            const int a = e / np, b = e % np;
            const int pa = pp[a], qa = qq[a], pb = pp[b], qb = qq[b];
            const double ca = cs[a], sa = sn[a], cb = cs[b], sb = sn[b];
            const double x11 = A[pa * M + pb];
            const double x12 = qb >= 0 ? A[pa * M + qb] : 0.0;
            const double x21 = qa >= 0 ? A[qa * M + pb] : 0.0;
            const double x22 = (qa >= 0 && qb >= 0) ? A[qa * M + qb] : 0.0;
            const double y11 = ca * x11 - sa * x21, y21 = sa * x11 + ca * x21;
            const double y12 = ca * x12 - sa * x22, y22 = sa * x12 + ca * x22;
            double z11 = cb * y11 - sb * y12, z12 = sb * y11 + cb * y12;
            double z21 = cb * y21 - sb * y22;
            const double z22 = sb * y21 + cb * y22;
            if (a == b && sa != 0.0) {
                z12 = 0.0;
                z21 = 0.0;
            }
            An[pa * M + pb] = z11;
            if (qb >= 0) An[pa * M + qb] = z12;
            if (qa >= 0) An[qa * M + pb] = z21;
            if (qa >= 0 && qb >= 0) An[qa * M + qb] = z22;
        } else {                                          // columns p_b, q_b of V
            const int f = e - nblk;
            const int k = f / np, b = f % np;
            const int pb = pp[b], qb = qq[b];
            const double sb = sn[b];
            if (qb < 0 || sb == 0.0) continue;
            const double cb = cs[b];
            const double vkp = V[k * M + pb], vkq = V[k * M + qb];
            V[k * M + pb] = cb * vkp - sb * vkq;
            V[k * M + qb] = sb * vkp + cb * vkq;
        }
    }
}

// V = I.
__global__ __launch_bounds__(kBlock) void k_jac_init(double* __restrict__ V, int M) {
    for (int e = blockIdx.x * kBlock + threadIdx.x; e < M * M; e += gridDim.x * kBlock)
        V[e] = (e / M == e % M) ? 1.0 : 0.0;
}

// off = sum of squared off-diagonal entries, fro = all; flag = off <= 1e-30 fro
// (off-diagonal norm <= 1e-15 of the Frobenius norm).  One workgroup.
__global__ __launch_bounds__(kJacobiThreads) void k_jac_offnorm(const double* __restrict__ A, int M,
                                                                int* __restrict__ flag) {
    __shared__ double red[2 * (kJacobiThreads / kWave)];
    const int t = threadIdx.x;
    double off = 0.0, fro = 0.0;
    for (int e = t; e < M * M; e += kJacobiThreads) {
        const double v = A[e] * A[e];
        fro += v;
        if (e / M != e % M) off += v;
    }
    off = wave_sum(off);
    fro = wave_sum(fro);
    if ((t & (kWave - 1)) == 0) {
        red[2 * (t / kWave)] = off;
        red[2 * (t / kWave) + 1] = fro;
    }
    __syncthreads();
    if (t == 0) {
        double o = 0.0, f = 0.0;
        for (int w = 0; w < kJacobiThreads / kWave; ++w) {
            o += red[2 * w];
            f += red[2 * w + 1];
        }
        *flag = (o <= 1e-30 * f) ? 1 : 0;
    }
}

// Eigenvalues (diagonal of A) sorted descending (ties by index) into lam; the
// eigenvectors (columns of V) in the same order into A (A[k * M + c] =
// component k of eigenvector c) with the largest-magnitude component of each
// positive.  One workgroup.
__global__ __launch_bounds__(kJacobiThreads) void k_jac_finish(double* __restrict__ A, int M,
                                                               double* __restrict__ V,
                                                               double* __restrict__ lam) {
    __shared__ int rk[kTsCap];
    __shared__ double d[kTsCap];
    const int t = threadIdx.x, nt = kJacobiThreads;
    for (int i = t; i < M; i += nt) d[i] = A[i * M + i];
    __syncthreads();
    for (int i = t; i < M; i += nt) {
        const double li = d[i];
        int rank = 0;
        for (int j = 0; j < M; ++j) rank += (d[j] > li) || (d[j] == li && j < i);
        rk[i] = rank;
        lam[rank] = li;
    }
    __syncthreads();
    for (int e = t; e < M * M; e += nt) {
        const int k = e / M, i = e % M;
        A[k * M + rk[i]] = V[k * M + i];
    }
    __syncthreads();
    for (int c = t; c < M; c += nt) {
        int kmax = 0;
        double vmax = -1.0;
        for (int k = 0; k < M; ++k) {
            const double v = fabs(A[k * M + c]);
            if (v > vmax) {
                vmax = v;
                kmax = k;
            }
        }
        if (A[kmax * M + c] < 0.0)
            for (int k = 0; k < M; ++k) A[k * M + c] = -A[k * M + c];
    }
}

// T(k, c) = eta_k V(k, c) / sqrt(lam_c), column-major M x y (a GEMM operand).
__global__ __launch_bounds__(kBlock) void k_ts_pod_coeffs(const double* __restrict__ Vs, int M,
                                                          const double* __restrict__ lam,
                                                          const double* __restrict__ eta, int y,
                                                          double* __restrict__ T) {
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= M * y) return;
    const int k = e % M, c = e / M;
    T[e] = eta[k] * Vs[k * M + c] / sqrt(lam[c]);
}

// ---------------------------------------------------------------- launchers

namespace {
int rows_grid(int n) {
    int g = (n + kBlock - 1) / kBlock;
    return g < 1024 ? (g < 1 ? 1 : g) : 1024;
}
}  // namespace

hipError_t launch_gemv_n(int n, size_t ld, const double* Y, int m, const double* c, double* out,
                         double sign, bool accumulate, hipStream_t s) {
    if (m < 0 || m > kTsCap) return hipErrorInvalidValue;
    if (m == 0 && accumulate) return hipSuccess;
    hipLaunchKernelGGL(k_gemv_n, dim3(rows_grid(n)), dim3(kBlock), 0, s, n, ld, Y, m, c, out, sign,
                       accumulate ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_gemv_t(int n, size_t ld, const double* Y, int m, const double* v, double* part,
                         double* out, hipStream_t s) {
    if (m < 1 || m > kTsCap) return hipErrorInvalidValue;
    int chunks = (n + 2047) / 2048;
    if (chunks > kTsChunks) chunks = kTsChunks;
    if (chunks < 1) chunks = 1;
    int rows = (n + chunks - 1) / chunks;
    rows = (rows + kWave - 1) / kWave * kWave;
    const int colgroups = (m + kWavesPerBlock * kGemvCols - 1) / (kWavesPerBlock * kGemvCols);
    hipLaunchKernelGGL(k_gemv_t_part, dim3(chunks, colgroups), dim3(kBlock), 0, s, n, ld, Y, m, v, part, rows);
    hipLaunchKernelGGL(k_gemv_t_reduce, dim3((m + kWavesPerBlock - 1) / kWavesPerBlock), dim3(kBlock), 0, s, part,
                       chunks, m, out);
    return hipGetLastError();
}

hipError_t launch_ts_s2_init(TsDev* T, const DevState* st, int m, const int* sel, int w,
                             const double* GinvW, double tau_rel, double floor_rel, int k2max,
                             hipStream_t s) {
    if (m < 1 || m > kTsCap || w < 0 || w > kYMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_ts_s2_init, dim3(1), dim3(kBlock), 0, s, T, st, m, sel, w, GinvW, tau_rel,
                       floor_rel, k2max);
    return hipGetLastError();
}

hipError_t launch_ts_s2_step(TsDev* T, int m, const int* sel, int w, const double* GinvW, double* aug,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_ts_s2_step, dim3(1), dim3(kBlock), 0, s, T, m, sel, w, GinvW, aug);
    return hipGetLastError();
}

hipError_t launch_ts_ghat_mv(TsDev* T, const double* Ghat, int m, hipStream_t s) {
    if (m < 1 || m > kTsCap) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_ts_ghat_mv, dim3(1), dim3(kTsThreads), 0, s, T, Ghat, m);
    return hipGetLastError();
}

hipError_t launch_ts_in_solve(TsDev* T, double* aug, int m, const int* sel, int w, const double* GinvW,
                              const double* Ghat, double rel, int kinmax, int* acc, hipStream_t s) {
    if (m < 1 || m > kTsCap || w < 0 || w > kYMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_ts_in_solve, dim3(1), dim3(kTsThreads), 0, s, T, aug, m, sel, w, GinvW, Ghat, rel, kinmax,
                       acc);
    return hipGetLastError();
}

hipError_t launch_ts_ginv_blockdiag(const double* GinvW, int w, const TsDev* T, int k2, double* GinvB,
                                    hipStream_t s) {
    if (w + k2 > kYMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_ts_ginv_blockdiag, dim3(1), dim3(kBlock), 0, s, GinvW, w, T, k2, GinvB);
    return hipGetLastError();
}

hipError_t launch_ts_eta(TsDev* T, int m, int kr, hipStream_t s) {
    if (m + kr > kTsCap) return hipErrorInvalidValue;
    if (m + kr == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ts_eta, dim3((m + kr + kBlock - 1) / kBlock), dim3(kBlock), 0, s, T, m, kr);
    return hipGetLastError();
}

hipError_t launch_ts_gather(const double* Y, size_t ld, int n, const int* sel, int w, double* B,
                            hipStream_t s) {
    if (w < 1) return hipSuccess;
    hipLaunchKernelGGL(k_ts_gather, dim3(rows_grid(n) < 64 ? rows_grid(n) : 64, w), dim3(kBlock), 0, s, Y,
                       ld, n, sel, B);
    return hipGetLastError();
}

hipError_t launch_ts_weight_sym(double* G, int M, const double* eta, hipStream_t s) {
    if (M < 1) return hipSuccess;
    hipLaunchKernelGGL(k_ts_weight_sym, dim3((M * M + kBlock - 1) / kBlock), dim3(kBlock), 0, s, G, M, eta);
    return hipGetLastError();
}

hipError_t launch_ts_jacobi_init(double* V, int M, hipStream_t s) {
    if (M < 1 || M > kTsCap) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_jac_init, dim3(rows_grid(M * M)), dim3(kBlock), 0, s, V, M);
    return hipGetLastError();
}

// One sweep; the matrix alternates between *A and *A2 (the pointers are
// swapped so that *A holds the current matrix on return); ends with the
// convergence flag of the result.
hipError_t launch_ts_jacobi_sweep(double** A, double** A2, double* V, int M, int* flag, hipStream_t s) {
    if (M < 1 || M > kTsCap) return hipErrorInvalidValue;
    const int Mp = M + (M & 1);
    const int np = Mp / 2;
    const int g = rows_grid(np * np + M * np);
    for (int r = 0; r < Mp - 1; ++r) {
        hipLaunchKernelGGL(k_jac_round, dim3(g), dim3(kBlock), 0, s, (const double*)*A, *A2, V, M, r);
        double* t = *A;
        *A = *A2;
        *A2 = t;
    }
    hipLaunchKernelGGL(k_jac_offnorm, dim3(1), dim3(kJacobiThreads), 0, s, (const double*)*A, M, flag);
    return hipGetLastError();
}

hipError_t launch_ts_jacobi_offnorm(const double* A, int M, int* flag, hipStream_t s) {
    hipLaunchKernelGGL(k_jac_offnorm, dim3(1), dim3(kJacobiThreads), 0, s, A, M, flag);
    return hipGetLastError();
}

hipError_t launch_ts_jacobi_finish(double* A, int M, double* V, double* lam, hipStream_t s) {
    if (M < 1 || M > kTsCap) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_jac_finish, dim3(1), dim3(kJacobiThreads), 0, s, A, M, V, lam);
    return hipGetLastError();
}

hipError_t launch_ts_pod_coeffs(const double* Vs, int M, const double* lam, const double* eta, int y,
                                double* T, hipStream_t s) {
    if (y < 1) return hipSuccess;
    hipLaunchKernelGGL(k_ts_pod_coeffs, dim3((M * y + kBlock - 1) / kBlock), dim3(kBlock), 0, s, Vs, M, lam,
                       eta, y, T);
    return hipGetLastError();
}

}  // namespace podcg
