// Small dense kernels of libpodcg, each run by one workgroup of kBlock threads:
// the factorisation of the reduced matrix W^T A W (Alg. 2) and the POD
// coefficients from the eigen-decomposition of the snapshot Gram matrix
// (Alg. pod_evd).  Matrices are at most 32 x 32 and live in LDS.
#include "podcg_launch.h"

namespace podcg {

constexpr int kLd = kYMax + 1;   // padded LDS row stride

// Pair t of round `step` of the round-robin (tournament) ordering of me
// players: position 0 is fixed, positions 1..me-1 rotate.  p < q; q = -1 for
// the bye (a player index >= m, when m is odd).
__device__ __forceinline__ void tournament_pair(int t, int step, int me, int m, int& p, int& q) {
    int p0 = 0, p1 = me - 2 - t + step;
    if (t > 0) {
        p0 = t - 1 + step;
        if (p0 >= me - 1) p0 -= me - 1;
        ++p0;
    }
    if (p1 >= me - 1) p1 -= me - 1;
    ++p1;
    p = p0 < p1 ? p0 : p1;
    q = p0 < p1 ? p1 : p0;
    if (q >= m) q = -1;
}

// Rotation (c, s) that annihilates a_pq: the symmetric Schur decomposition
// of the 2 x 2 block {p, q} (Golub & Van Loan), t = tan(theta) the root of
// t^2 + 2 tau t - 1 = 0 of smaller magnitude, tau = (a_qq - a_pp) / (2 a_pq).
// Written without divisions: with x = a_qq - a_pp, y = 2 a_pq (both scaled
// by the same power of two so that the larger has magnitude in [1/2, 1)),
// r = sqrt(x^2 + y^2), u = |x| + r and v = sign(x) y, t = v / u, so
// c = u / sqrt(u^2 + v^2) and s = v / sqrt(u^2 + v^2).  The identity for the
// bye or a zero a_pq.
__device__ __forceinline__ void schur2(const double* a, int p, int q, double& c, double& sn) {
    const int qq = q < 0 ? p : q;
    const double apq = a[p * kLd + qq], app = a[p * kLd + p], aqq = a[qq * kLd + qq];
    const double x0 = aqq - app, y0 = 2.0 * apq;
    const int e = __builtin_amdgcn_frexp_exp(fmax(fabs(x0), fabs(y0)));
    const double x = __builtin_amdgcn_ldexp(x0, -e), y = __builtin_amdgcn_ldexp(y0, -e);
    const double r = sqrt(x * x + y * y);
    const double u = fabs(x) + r, v = x >= 0.0 ? y : -y;
    const double h = rsqrt(u * u + v * v);
    const bool rot = q >= 0 && apq != 0.0;
    c = rot ? u * h : 1.0;
    sn = rot ? v * h : 0.0;
}

// Jacobi eigen-decomposition of the symmetric m x m matrix a (LDS, stride
// kLd) by one workgroup of kBlock threads; b is LDS scratch of the same
// shape; V (LDS, may be null) receives the eigenvectors as columns.  The
// rotations of one sweep are grouped by the round-robin ordering: each step
// holds m/2 disjoint pairs, so the step's whole similarity transform splits
// into independent 2 x 2 blocks, one per thread, and the eigenvector update
// into independent column pairs.  Every thread forms the rotations it applies
// from the step's input matrix itself, and writes its block into the other
// buffer, so a step costs one barrier.  Sweeps stop when the off-diagonal
// Frobenius norm drops below 1e-15 of the full norm.  On exit lam[0..m) holds
// the eigenvalues in decreasing order, V is permuted to match, and each
// eigenvector is signed so that its entry of largest magnitude (first such
// index) is positive.
__device__ void block_jacobi(double* a, double* b, double* V, double* lam, int m) {
    __shared__ double red[kWavesPerBlock + 1];
    const int tid = threadIdx.x;
    if (V)
        for (int e = tid; e < m * m; e += kBlock) V[(e / m) * kLd + e % m] = (e / m == e % m) ? 1.0 : 0.0;
    double f[1] = {0.0};
    for (int e = tid; e < m * m; e += kBlock) {
        const double v = a[(e / m) * kLd + e % m];
        f[0] += v * v;
    }
    block_sum<1>(f, red);
    const double fro = red[0];
    const int me = m + (m & 1);          // players, with a bye when m is odd
    const int npair = me / 2;
    // this thread's 2 x 2 block of pairs (t, u) (npair^2 <= kBlock)
    const bool has_blk = tid < npair * npair;
    const int bt = tid / npair, bu = tid % npair;
    __syncthreads();
    for (int sweep = 0; sweep < 100 && m > 1; ++sweep) {
        double o[1] = {0.0};
        for (int e = tid; e < m * m; e += kBlock) {
            const int i = e / m, j = e % m;
            if (i != j) o[0] += a[i * kLd + j] * a[i * kLd + j];
        }
        block_sum<1>(o, red);
        const double off = red[0];
        __syncthreads();
        if (off <= 1.0e-30 * fro) break;
        for (int step = 0; step < me - 1; ++step) {
            // b <- J^T a J with J the direct sum of the pairs' rotations: the
            // 2 x 2 block of rows {p_t, q_t} and columns {p_u, q_u} becomes
            // J_t^T a_tu J_u (rows first, then columns); V <- V J in place,
            // rows t and t + npair of the column pair u (each entry one owner)
            if (has_blk) {
                int pt, qt, pu, qu;
                tournament_pair(bt, step, me, m, pt, qt);
                tournament_pair(bu, step, me, m, pu, qu);
                double ct, st, cu, su;
                schur2(a, pt, qt, ct, st);
                schur2(a, pu, qu, cu, su);
                const double b0 = a[pt * kLd + pu];
                const double b1 = qu >= 0 ? a[pt * kLd + qu] : 0.0;
                const double b2 = qt >= 0 ? a[qt * kLd + pu] : 0.0;
                const double b3 = (qt >= 0 && qu >= 0) ? a[qt * kLd + qu] : 0.0;
                const double rp0 = ct * b0 - st * b2;
                const double rp1 = ct * b1 - st * b3;
                const double rq0 = st * b0 + ct * b2;
                const double rq1 = st * b1 + ct * b3;
                const bool zero = bt == bu && st != 0.0;   // the pair's own a_pq
                b[pt * kLd + pu] = cu * rp0 - su * rp1;
                if (qu >= 0) b[pt * kLd + qu] = zero ? 0.0 : su * rp0 + cu * rp1;
                if (qt >= 0) {
                    b[qt * kLd + pu] = zero ? 0.0 : cu * rq0 - su * rq1;
                    if (qu >= 0) b[qt * kLd + qu] = su * rq0 + cu * rq1;
                }
                if (V)
                    for (int kq = bt; kq < m; kq += npair) {
                        const double xp = V[kq * kLd + pu];
                        const double xq = qu >= 0 ? V[kq * kLd + qu] : 0.0;
                        V[kq * kLd + pu] = cu * xp - su * xq;
                        if (qu >= 0) V[kq * kLd + qu] = su * xp + cu * xq;
                    }
            }
            __syncthreads();
            double* t = a;
            a = b;
            b = t;
        }
    }
    if (tid < m) lam[tid] = a[tid * kLd + tid];
    __syncthreads();
    // selection sort, decreasing; threads swap the rows of V in parallel
    for (int i = 0; i < m; ++i) {
        int best = i;
        for (int j = i + 1; j < m; ++j)
            if (lam[j] > lam[best]) best = j;
        __syncthreads();
        if (best != i) {
            if (V && tid < m) {
                const double t = V[tid * kLd + i];
                V[tid * kLd + i] = V[tid * kLd + best];
                V[tid * kLd + best] = t;
            }
            if (tid == 0) {
                const double t = lam[i];
                lam[i] = lam[best];
                lam[best] = t;
            }
        }
        __syncthreads();
    }
    if (V && tid < m) {
        int big = 0;
        for (int k = 1; k < m; ++k)
            if (fabs(V[k * kLd + tid]) > fabs(V[big * kLd + tid])) big = k;
        if (V[big * kLd + tid] < 0.0)
            for (int k = 0; k < m; ++k) V[k * kLd + tid] = -V[k * kLd + tid];
    }
    __syncthreads();
}

// Reduced matrix of Stage 1: symmetrise G (m x m, row-major, in place),
// factor G = R^T R (R upper, row-major m x m) stopping at the first pivot
// <= 1e-14 max_i G_ii, and form Ginv = R^{-1} R^{-T} on the kept leading
// block (row-major, stride = kept rank).  st->y receives the kept rank and
// lam the eigenvalues of the kept block (for its condition number).
// The body, for one workgroup; `report` (if not null) receives the kept rank
// and the largest and smallest kept eigenvalue.
__device__ void reduced_factor(double* G, int m, double* R, double* Ginv, double* lam, DevState* st,
                               double* report) {
    __shared__ double g[kYMax * kLd], rr[kYMax * kLd], ri[kYMax * kLd], v[kYMax * kLd], vb[kYMax * kLd];
    __shared__ double lm[kYMax];
    __shared__ int kept_s;
    const int tid = threadIdx.x;
    for (int e = tid; e < m * m; e += kBlock) {
        const int i = e / m, j = e % m;
        g[i * kLd + j] = 0.5 * (G[i * m + j] + G[j * m + i]);
    }
    __syncthreads();
    for (int e = tid; e < m * m; e += kBlock) G[e] = g[(e / m) * kLd + e % m];
    for (int e = tid; e < kYMax * kLd; e += kBlock) { rr[e] = 0.0; ri[e] = 0.0; }
    __syncthreads();
    if (tid == 0) {
        double dmax = 0.0;
        for (int i = 0; i < m; ++i) dmax = fmax(dmax, g[i * kLd + i]);
        int kept = m;
        for (int j = 0; j < m; ++j) {
            double d = g[j * kLd + j];
            for (int k = 0; k < j; ++k) d -= rr[k * kLd + j] * rr[k * kLd + j];
            if (!(d > 1.0e-14 * dmax) || !is_finite(d)) { kept = j; break; }
            const double rjj = sqrt(d);
            rr[j * kLd + j] = rjj;
            for (int i = j + 1; i < m; ++i) {
                double s = g[j * kLd + i];
                for (int k = 0; k < j; ++k) s -= rr[k * kLd + j] * rr[k * kLd + i];
                rr[j * kLd + i] = s / rjj;
            }
        }
        kept_s = kept;
    }
    __syncthreads();
    const int y = kept_s;
    // column j of R^{-1} (upper) by back substitution, one thread per column
    if (tid < y) {
        const int j = tid;
        for (int i = j; i >= 0; --i) {
            double s = (i == j) ? 1.0 : 0.0;
            for (int k = i + 1; k <= j; ++k) s -= rr[i * kLd + k] * ri[k * kLd + j];
            ri[i * kLd + j] = s / rr[i * kLd + i];
        }
    }
    __syncthreads();
    for (int e = tid; e < y * y; e += kBlock) {
        const int i = e / y, j = e % y;
        double s = 0.0;
        for (int k = (i > j ? i : j); k < y; ++k) s += ri[i * kLd + k] * ri[j * kLd + k];
        Ginv[e] = s;
    }
    for (int e = tid; e < m * m; e += kBlock) R[e] = rr[(e / m) * kLd + e % m];
    // eigenvalues of the kept block (condition number of W^T A W)
    __syncthreads();
    for (int e = tid; e < y * y; e += kBlock) v[(e / y) * kLd + e % y] = g[(e / y) * kLd + e % y];
    __syncthreads();
    if (y > 0) block_jacobi(v, vb, nullptr, lm, y);   // eigenvalues only
    if (tid < y) lam[tid] = lm[tid];
    if (tid == 0) {
        st->y = y;
        if (report) {
            report[0] = (double)y;
            report[1] = y > 0 ? lm[0] : 0.0;
            report[2] = y > 0 ? lm[y - 1] : 0.0;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_reduced_factor(double* G, int m, double* R, double* Ginv,
                                                          double* lam, DevState* st) {
    reduced_factor(G, m, R, Ginv, lam, st, nullptr);
}

struct Weights {
    double w[kYMax];
};

// POD coefficients (Alg. pod_evd): Gbar = diag(w) Gs diag(w), symmetrised;
// Gbar = V diag(lam) V^T; y = #{lam_i > rank_rtol lam_1}, capped by rank_max
// and the energy criterion; T = diag(w) V_y diag(lam_y)^{-1/2} (count x y,
// row-major).  Writes lam[0..count), *y_out and, if not null, *y_copy.  The
// body, for one workgroup.
__device__ void pod_coeffs(const double* Gs, int count, const double* w, int rank_max, double rank_rtol,
                           double energy, double* T, double* lam_out, int* y_out, int* y_copy) {
    __shared__ double a[kYMax * kLd], b[kYMax * kLd], V[kYMax * kLd];
    __shared__ double lam[kYMax];
    __shared__ int y_s;
    const int tid = threadIdx.x;
    const int m = count;
    for (int e = tid; e < m * m; e += kBlock) {
        const int i = e / m, j = e % m;
        const double gij = w[i] * Gs[i * m + j] * w[j];
        const double gji = w[j] * Gs[j * m + i] * w[i];
        a[i * kLd + j] = 0.5 * (gij + gji);
    }
    __syncthreads();
    block_jacobi(a, b, V, lam, m);
    if (tid == 0) {
        int y = 0;
        if (lam[0] > 0.0)
            for (int i = 0; i < m; ++i)
                if (lam[i] > rank_rtol * lam[0]) y = i + 1;
        if (y > rank_max) y = rank_max;
        if (energy > 0.0 && energy < 1.0 && y > 0) {
            double tot = 0.0, acc = 0.0;
            for (int i = 0; i < m; ++i) tot += lam[i];
            int ye = y;
            for (int i = 0; i < y; ++i) {
                acc += lam[i];
                if (acc >= energy * tot) { ye = i + 1; break; }
            }
            y = ye;
        }
        y_s = y;
        *y_out = y;
        if (y_copy) *y_copy = y;
    }
    __syncthreads();
    const int y = y_s;
    for (int e = tid; e < m * y; e += kBlock) {
        const int k = e / y, i = e % y;
        T[e] = w[k] * V[k * kLd + i] / sqrt(lam[i]);
    }
    if (tid < m) lam_out[tid] = lam[tid];
}

__global__ __launch_bounds__(kBlock) void k_pod_coeffs(const double* Gs, int count, Weights wt,
                                                      int rank_max, double rank_rtol, double energy,
                                                      double* T, double* lam_out, int* y_out) {
    pod_coeffs(Gs, count, wt.w, rank_max, rank_rtol, energy, T, lam_out, y_out, nullptr);
}

// Batched: workgroup b solves the POD eigen-problem of member list[b].
__global__ __launch_bounds__(kBlock) void k_batch_pod_coeffs(const BatchAux* __restrict__ aux,
                                                            const int* __restrict__ list) {
    const BatchAux& A = aux[list[blockIdx.x]];
    pod_coeffs(A.Gs, A.count, A.w, A.rank_max, A.rank_rtol, A.energy, A.T, A.lam, A.yout, A.rank);
}

hipError_t launch_batch_pod_coeffs(const BatchAux* aux, const int* list, int nlist, hipStream_t s) {
    if (nlist < 1) return hipSuccess;
    hipLaunchKernelGGL(k_batch_pod_coeffs, dim3(nlist), dim3(kBlock), 0, s, aux, list);
    return hipGetLastError();
}

// Batched: workgroup b factors member list[b] (its G of ynom columns).
__global__ __launch_bounds__(kBlock) void k_batch_reduced_factor(const BatchMember* __restrict__ mem,
                                                                const BatchSetup* __restrict__ su,
                                                                const int* __restrict__ list) {
    const int m = list[blockIdx.x];
    const BatchSetup& S = su[m];
    reduced_factor(S.G, S.ynom, S.R, S.Ginv, S.lamG, mem[m].B.st, S.report);
}

hipError_t launch_batch_reduced_factor(const BatchMember* mem, const BatchSetup* su, const int* list, int nlist,
                                       hipStream_t s) {
    if (nlist < 1) return hipSuccess;
    hipLaunchKernelGGL(k_batch_reduced_factor, dim3(nlist), dim3(kBlock), 0, s, mem, su, list);
    return hipGetLastError();
}

hipError_t launch_reduced_factor(double* G, int m, double* R, double* Ginv, double* lam,
                                 DevState* st, hipStream_t s) {
    if (m < 1 || m > kYMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_reduced_factor, dim3(1), dim3(kBlock), 0, s, G, m, R, Ginv, lam, st);
    return hipGetLastError();
}

hipError_t launch_pod_coeffs(const double* Gs, int count, const double* w, int rank_max,
                             double rank_rtol, double energy, double* T, double* lam, int* y_out,
                             hipStream_t s) {
    if (count < 1 || count > kYMax) return hipErrorInvalidValue;
    Weights wt;
    for (int i = 0; i < kYMax; ++i) wt.w[i] = i < count ? w[i] : 0.0;
    hipLaunchKernelGGL(k_pod_coeffs, dim3(1), dim3(kBlock), 0, s, Gs, count, wt, rank_max, rank_rtol,
                       energy, T, lam, y_out);
    return hipGetLastError();
}

}  // namespace podcg
