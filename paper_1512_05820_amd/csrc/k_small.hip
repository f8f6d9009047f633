// Small dense kernels of libpodcg, each run by one workgroup of one wavefront:
// the factorisation of the reduced matrix W^T A W (Alg. 2) and the POD
// coefficients from the eigen-decomposition of the snapshot Gram matrix
// (Alg. pod_evd).  Matrices are at most 32 x 32 and live in LDS.
#include "podcg_device.h"

namespace podcg {

constexpr int kLd = kYMax + 1;   // padded LDS row stride

// Jacobi eigen-decomposition of the symmetric m x m matrix a (LDS, stride
// kLd) by one wavefront; V (LDS) receives the eigenvectors as columns.  Each
// rotation is the symmetric Schur decomposition of a 2 x 2 block (Golub & Van
// Loan).  The rotations of one sweep are grouped by the round-robin
// (tournament) ordering: each step holds m/2 disjoint pairs, so all their row
// rotations, then all their column rotations, run in parallel across the
// lanes.  Sweeps stop when the off-diagonal Frobenius norm drops below 1e-15
// of the full norm.  On exit lam[0..m) holds the eigenvalues in decreasing
// order, V is permuted to match, and each eigenvector is signed so that its
// entry of largest magnitude (first such index) is positive.
__device__ void wave_jacobi(double* a, double* V, double* lam, int m) {
    __shared__ double cs[2 * (kYMax / 2 + 1)];
    __shared__ int pq[2 * (kYMax / 2 + 1)];
    const int lane = threadIdx.x;
    for (int e = lane; e < m * m; e += kWave) V[(e / m) * kLd + e % m] = (e / m == e % m) ? 1.0 : 0.0;
    double f = 0.0;
    for (int e = lane; e < m * m; e += kWave) {
        const double v = a[(e / m) * kLd + e % m];
        f += v * v;
    }
    const double fro = wave_sum(f);
    const int me = m + (m & 1);          // players, with a bye when m is odd
    const int npair = me / 2;
    __syncthreads();
    for (int sweep = 0; sweep < 100 && m > 1; ++sweep) {
        double o = 0.0;
        {
            const int j = lane & 31;
            if (j < m)
                for (int i = lane >> 5; i < m; i += 2)
                    if (i != j) o += a[i * kLd + j] * a[i * kLd + j];
        }
        const double off = wave_sum(o);
        if (off <= 1.0e-30 * fro) break;
        for (int step = 0; step < me - 1; ++step) {
            // pairs of this round: position 0 is fixed, the others rotate
            if (lane < npair) {
                const int i0 = lane, i1 = me - 1 - lane;
                const int p0 = i0 == 0 ? 0 : 1 + (i0 - 1 + step) % (me - 1);
                const int p1 = 1 + (i1 - 1 + step) % (me - 1);
                int p = p0 < p1 ? p0 : p1, q = p0 < p1 ? p1 : p0;
                double c = 1.0, sn = 0.0;
                if (q < m) {
                    const double apq = a[p * kLd + q];
                    if (apq != 0.0) {
                        const double tau = (a[q * kLd + q] - a[p * kLd + p]) / (2.0 * apq);
                        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        sn = t * c;
                    }
                } else {
                    p = q = -1;                  // bye
                }
                pq[2 * lane] = p;
                pq[2 * lane + 1] = q;
                cs[2 * lane] = c;
                cs[2 * lane + 1] = sn;
            }
            __syncthreads();
            // rows p, q of every pair:  A <- J^T A.  Lane l updates entry
            // k = l % 32 of pairs t = l / 32, l / 32 + 2, ... (m <= 32, so no
            // index needs a division)
            const int kq = lane & 31, t0 = lane >> 5;
            if (kq < m)
                for (int t = t0; t < npair; t += 2) {
                    const int p = pq[2 * t], q = pq[2 * t + 1];
                    if (p < 0) continue;
                    const double c = cs[2 * t], sn = cs[2 * t + 1];
                    const double apk = a[p * kLd + kq], aqk = a[q * kLd + kq];
                    a[p * kLd + kq] = c * apk - sn * aqk;
                    a[q * kLd + kq] = sn * apk + c * aqk;
                }
            __syncthreads();
            // columns p, q of every pair:  A <- A J,  V <- V J
            if (kq < m)
                for (int t = t0; t < npair; t += 2) {
                    const int p = pq[2 * t], q = pq[2 * t + 1];
                    if (p < 0) continue;
                    const double c = cs[2 * t], sn = cs[2 * t + 1];
                    const double akp = a[kq * kLd + p], akq = a[kq * kLd + q];
                    a[kq * kLd + p] = c * akp - sn * akq;
                    a[kq * kLd + q] = sn * akp + c * akq;
                    const double vkp = V[kq * kLd + p], vkq = V[kq * kLd + q];
                    V[kq * kLd + p] = c * vkp - sn * vkq;
                    V[kq * kLd + q] = sn * vkp + c * vkq;
                }
            __syncthreads();
            if (lane < npair) {
                const int p = pq[2 * lane], q = pq[2 * lane + 1];
                if (p >= 0 && cs[2 * lane + 1] != 0.0) {
                    a[p * kLd + q] = 0.0;
                    a[q * kLd + p] = 0.0;
                }
            }
            __syncthreads();
        }
    }
    if (lane < m) lam[lane] = a[lane * kLd + lane];
    __syncthreads();
    // selection sort, decreasing; lanes swap the rows of V in parallel
    for (int i = 0; i < m; ++i) {
        int best = i;
        for (int j = i + 1; j < m; ++j)
            if (lam[j] > lam[best]) best = j;
        __syncthreads();
        if (best != i) {
            if (lane < m) {
                const double t = V[lane * kLd + i];
                V[lane * kLd + i] = V[lane * kLd + best];
                V[lane * kLd + best] = t;
            }
            if (lane == 0) {
                const double t = lam[i];
                lam[i] = lam[best];
                lam[best] = t;
            }
        }
        __syncthreads();
    }
    if (lane < m) {
        int big = 0;
        for (int k = 1; k < m; ++k)
            if (fabs(V[k * kLd + lane]) > fabs(V[big * kLd + lane])) big = k;
        if (V[big * kLd + lane] < 0.0)
            for (int k = 0; k < m; ++k) V[k * kLd + lane] = -V[k * kLd + lane];
    }
    __syncthreads();
}

// Reduced matrix of Stage 1: symmetrise G (m x m, row-major, in place),
// factor G = R^T R (R upper, row-major m x m) stopping at the first pivot
// <= 1e-14 max_i G_ii, and form Ginv = R^{-1} R^{-T} on the kept leading
// block (row-major, stride = kept rank).  st->y receives the kept rank and
// lam the eigenvalues of the kept block (for its condition number).
__global__ __launch_bounds__(kWave) void k_reduced_factor(double* G, int m, double* R, double* Ginv,
                                                          double* lam, DevState* st) {
    __shared__ double g[kYMax * kLd], rr[kYMax * kLd], ri[kYMax * kLd], v[kYMax * kLd];
    __shared__ double lm[kYMax];
    __shared__ int kept_s;
    const int lane = threadIdx.x;
    for (int e = lane; e < m * m; e += kWave) {
        const int i = e / m, j = e % m;
        g[i * kLd + j] = 0.5 * (G[i * m + j] + G[j * m + i]);
    }
    __syncthreads();
    for (int e = lane; e < m * m; e += kWave) G[e] = g[(e / m) * kLd + e % m];
    for (int e = lane; e < kYMax * kLd; e += kWave) { rr[e] = 0.0; ri[e] = 0.0; }
    __syncthreads();
    if (lane == 0) {
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
    // column j of R^{-1} (upper) by back substitution, one lane per column
    if (lane < y) {
        const int j = lane;
        for (int i = j; i >= 0; --i) {
            double s = (i == j) ? 1.0 : 0.0;
            for (int k = i + 1; k <= j; ++k) s -= rr[i * kLd + k] * ri[k * kLd + j];
            ri[i * kLd + j] = s / rr[i * kLd + i];
        }
    }
    __syncthreads();
    for (int e = lane; e < y * y; e += kWave) {
        const int i = e / y, j = e % y;
        double s = 0.0;
        for (int k = (i > j ? i : j); k < y; ++k) s += ri[i * kLd + k] * ri[j * kLd + k];
        Ginv[e] = s;
    }
    for (int e = lane; e < m * m; e += kWave) R[e] = rr[(e / m) * kLd + e % m];
    // eigenvalues of the kept block (condition number of W^T A W)
    __syncthreads();
    for (int e = lane; e < y * y; e += kWave) v[(e / y) * kLd + e % y] = g[(e / y) * kLd + e % y];
    __syncthreads();
    if (y > 0) wave_jacobi(v, ri, lm, y);
    if (lane < y) lam[lane] = lm[lane];
    if (lane == 0) st->y = y;
}

struct Weights {
    double w[kYMax];
};

// POD coefficients (Alg. pod_evd): Gbar = diag(w) Gs diag(w), symmetrised;
// Gbar = V diag(lam) V^T; y = #{lam_i > rank_rtol lam_1}, capped by rank_max
// and the energy criterion; T = diag(w) V_y diag(lam_y)^{-1/2} (count x y,
// row-major).  Writes lam[0..count) and *y_out.
__global__ __launch_bounds__(kWave) void k_pod_coeffs(const double* Gs, int count, Weights wt,
                                                      int rank_max, double rank_rtol, double energy,
                                                      double* T, double* lam_out, int* y_out) {
    __shared__ double a[kYMax * kLd], V[kYMax * kLd];
    __shared__ double lam[kYMax];
    __shared__ int y_s;
    const int lane = threadIdx.x;
    const int m = count;
    for (int e = lane; e < m * m; e += kWave) {
        const int i = e / m, j = e % m;
        const double gij = wt.w[i] * Gs[i * m + j] * wt.w[j];
        const double gji = wt.w[j] * Gs[j * m + i] * wt.w[i];
        a[i * kLd + j] = 0.5 * (gij + gji);
    }
    __syncthreads();
    wave_jacobi(a, V, lam, m);
    if (lane == 0) {
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
    }
    __syncthreads();
    const int y = y_s;
    for (int e = lane; e < m * y; e += kWave) {
        const int k = e / y, i = e % y;
        T[e] = wt.w[k] * V[k * kLd + i] / sqrt(lam[i]);
    }
    if (lane < m) lam_out[lane] = lam[lane];
}

hipError_t launch_reduced_factor(double* G, int m, double* R, double* Ginv, double* lam,
                                 DevState* st, hipStream_t s) {
    if (m < 1 || m > kYMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_reduced_factor, dim3(1), dim3(kWave), 0, s, G, m, R, Ginv, lam, st);
    return hipGetLastError();
}

hipError_t launch_pod_coeffs(const double* Gs, int count, const double* w, int rank_max,
                             double rank_rtol, double energy, double* T, double* lam, int* y_out,
                             hipStream_t s) {
    if (count < 1 || count > kYMax) return hipErrorInvalidValue;
    Weights wt;
    for (int i = 0; i < kYMax; ++i) wt.w[i] = i < count ? w[i] : 0.0;
    hipLaunchKernelGGL(k_pod_coeffs, dim3(1), dim3(kWave), 0, s, Gs, count, wt, rank_max, rank_rtol,
                       energy, T, lam, y_out);
    return hipGetLastError();
}

}  // namespace podcg
