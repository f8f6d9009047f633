/*
 * podcg_oracle.c -- plain CPU FP64 reference for the POD-augmented
 * conjugate-gradient method of Carlberg, Forstall and Tuminaro,
 * "Krylov-subspace recycling via the POD-augmented conjugate-gradient method".
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * helper with the GPU library, and it never calls it.
 *
 * Everything is written out directly from the paper, in double precision,
 * with no blocking or fusion: a CSR matrix-vector product, dot products and
 * axpys, a dense Cholesky factorisation and a cyclic Jacobi symmetric
 * eigensolver.  OpenMP only splits independent row loops and sums.
 *
 * What each function follows:
 *   orc_matvec        y = A x for CSR A (the matrices of the sequence, Eq. (sequence)).
 *   orc_cholesky      G = R^T R, R upper triangular (Alg. 2, second step).
 *   orc_sym_eig       G = V diag(lam) V^T by cyclic Jacobi rotations
 *                     (Alg. pod_evd, second step; any symmetric EVD serves).
 *   orc_plain_pcg     Jacobi-preconditioned CG, the minimiser of Eq. (KrylovSolve).
 *   orc_aug_pcg       Stage 1 (Alg. 2) followed by Alg. 1 (augmented PCG) with
 *                     augmenting basis W; this is Stage 3 of Section 4 with an
 *                     empty Stage 2 (the Cholesky factor of Stage 1 is reused
 *                     in the projection solves, Section 4.3).
 *   orc_pod_evd       Alg. pod_evd (Appendix A): POD basis of weighted snapshots
 *                     in the metric of a given SPD matrix, Eqs. (podOpt)-(podOrth).
 *
 * Readings where the paper leaves a choice (stated once more in the design notes):
 *   - the stopping test ||b - A x||_2 <= eps_j (Eq. (sequenceInexact)) is taken
 *     with eps_j = tol * ||b_j||_2 and is evaluated on the recursive residual,
 *     also before the first iteration (so zero iterations are possible);
 *   - Alg. 1 works on the increment: it is called with right-hand side
 *     b - A xbar and returns x = xbar + increment;
 *   - the iteration count k is the number of search directions used, which
 *     equals the number of preconditioner applications inside the loop;
 *   - the projection right-hand side W^T A z is formed as (A W)^T z with the
 *     product A W kept from Stage 1, as the paper does in Stage 3 (A symmetric);
 *   - the reduced Gram matrix is symmetrised, (G + G^T) / 2, before it is
 *     factored or diagonalised;
 *   - a Cholesky pivot <= 1e-14 * max diag(G) truncates the basis to the
 *     columns before it (POD columns are ordered by energy, Remark podvecorder).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_ERR_ARG (-1)
#define ORC_ERR_NOT_SPD (-4)
#define ORC_ERR_NONFINITE (-5)

typedef struct {
    int32_t iters;          /* search directions used (preconditioner applications in the loop) */
    int32_t matvecs;        /* products with A, setup included */
    int32_t status;         /* ORC_* code */
    int32_t rank;           /* augmenting-basis dimension actually used */
    double stage1_relres;   /* ||r|| / ||b|| after Stage 1 (before the loop) */
    double relres;          /* recursive ||r|| / ||b|| at exit */
    double true_relres;     /* ||b - A x|| / ||b|| at exit */
    double bnorm;           /* ||b|| */
    double cond_G;          /* condition number of W^T A W (1 if no basis) */
} orc_stats;

/* ---------------------------------------------------------------- basics */

void orc_matvec(int64_t n, const int32_t* rowptr, const int32_t* colind,
                const double* val, const double* x, double* y)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) s += val[e] * x[colind[e]];
        y[i] = s;
    }
}

/* Inner product a^T b.  The sum runs over fixed blocks of 4096 indices (at
 * most 256 blocks, so blocks grow with n), each summed in index order, and the
 * block sums are added in block order: the result does not depend on the
 * number of threads or on their timing (a reduction clause would leave the
 * combining order open). */
static double dot(int64_t n, const double* a, const double* b)
{
    enum { kBlocks = 256, kMinBlock = 4096 };
    double part[kBlocks];
    int64_t nb = (n + kMinBlock - 1) / kMinBlock;
    if (nb < 1) nb = 1;
    if (nb > kBlocks) nb = kBlocks;
    #pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < nb; ++t) {
        const int64_t lo = n * t / nb, hi = n * (t + 1) / nb;
        double s = 0.0;
        for (int64_t i = lo; i < hi; ++i) s += a[i] * b[i];
        part[t] = s;
    }
    double s = 0.0;
    for (int64_t t = 0; t < nb; ++t) s += part[t];
    return s;
}

static int finite(double v) { return v == v && fabs(v) <= 1.0e308; }

/* Jacobi preconditioner M = diag(A): dinv = 1 / a_ii.  Returns 0, or
 * ORC_ERR_NOT_SPD if a diagonal entry is missing or not positive. */
static int jacobi_inverse(int64_t n, const int32_t* rowptr, const int32_t* colind,
                          const double* val, double* dinv)
{
    int bad = 0;
    #pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
            if (colind[e] == i) d += val[e];
        if (!(d > 0.0)) { bad = 1; dinv[i] = 0.0; }
        else dinv[i] = 1.0 / d;
    }
    return bad ? ORC_ERR_NOT_SPD : ORC_OK;
}

/* ------------------------------------------------------ dense small algebra */

/* G = R^T R for a symmetric m x m matrix G (row-major), R upper triangular
 * (row-major, lower part zeroed).  Stops at the first pivot that is not
 * larger than 1e-14 * max_i G_ii and returns the number of accepted
 * columns (m on success). */
int orc_cholesky(int32_t m, const double* G, double* R)
{
    double dmax = 0.0;
    for (int32_t i = 0; i < m; ++i) if (G[i * m + i] > dmax) dmax = G[i * m + i];
    memset(R, 0, sizeof(double) * (size_t)m * (size_t)m);
    for (int32_t j = 0; j < m; ++j) {
        double d = G[j * m + j];
        for (int32_t k = 0; k < j; ++k) d -= R[k * m + j] * R[k * m + j];
        if (!(d > 1.0e-14 * dmax) || !finite(d)) return j;
        double rjj = sqrt(d);
        R[j * m + j] = rjj;
        for (int32_t i = j + 1; i < m; ++i) {
            double s = G[j * m + i];
            for (int32_t k = 0; k < j; ++k) s -= R[k * m + j] * R[k * m + i];
            R[j * m + i] = s / rjj;
        }
    }
    return m;
}

/* Solve R^T R u = c with R the leading y x y block of an m x m upper
 * triangular row-major matrix. */
static void chol_solve(int32_t m, int32_t y, const double* R, const double* c, double* u)
{
    for (int32_t i = 0; i < y; ++i) {            /* R^T v = c */
        double s = c[i];
        for (int32_t k = 0; k < i; ++k) s -= R[k * m + i] * u[k];
        u[i] = s / R[i * m + i];
    }
    for (int32_t i = y - 1; i >= 0; --i) {       /* R u = v */
        double s = u[i];
        for (int32_t k = i + 1; k < y; ++k) s -= R[i * m + k] * u[k];
        u[i] = s / R[i * m + i];
    }
}

/* Symmetric eigen-decomposition G = V diag(lam) V^T by cyclic Jacobi
 * rotations (Golub & Van Loan, symmetric Schur decomposition of 2x2 blocks).
 * G row-major m x m; V row-major with eigenvectors as columns.  Eigenvalues
 * are returned in decreasing order; each eigenvector is signed so that its
 * entry of largest magnitude (first such index) is positive.  Returns the
 * number of sweeps used. */
int orc_sym_eig(int32_t m, const double* G, double* V, double* lam)
{
    double* a = (double*)malloc(sizeof(double) * (size_t)m * (size_t)m);
    memcpy(a, G, sizeof(double) * (size_t)m * (size_t)m);
    for (int32_t i = 0; i < m; ++i)
        for (int32_t j = 0; j < m; ++j) V[i * m + j] = (i == j) ? 1.0 : 0.0;
    double fro = 0.0;
    for (int32_t i = 0; i < m * m; ++i) fro += a[i] * a[i];
    int sweeps = 0;
    for (; sweeps < 100; ++sweeps) {
        double off = 0.0;
        for (int32_t p = 0; p < m; ++p)
            for (int32_t q = 0; q < m; ++q)
                if (p != q) off += a[p * m + q] * a[p * m + q];
        if (off <= 1.0e-30 * fro) break;
        for (int32_t p = 0; p < m - 1; ++p) {
            for (int32_t q = p + 1; q < m; ++q) {
                double apq = a[p * m + q];
                if (apq == 0.0) continue;
                double tau = (a[q * m + q] - a[p * m + p]) / (2.0 * apq);
                double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t);
                double s = t * c;
                /* A <- J^T A J with J the rotation in the (p, q) plane */
                for (int32_t k = 0; k < m; ++k) {
                    double akp = a[k * m + p], akq = a[k * m + q];
                    a[k * m + p] = c * akp - s * akq;
                    a[k * m + q] = s * akp + c * akq;
                }
                for (int32_t k = 0; k < m; ++k) {
                    double apk = a[p * m + k], aqk = a[q * m + k];
                    a[p * m + k] = c * apk - s * aqk;
                    a[q * m + k] = s * apk + c * aqk;
                }
                a[p * m + q] = 0.0;
                a[q * m + p] = 0.0;
                for (int32_t k = 0; k < m; ++k) {
                    double vkp = V[k * m + p], vkq = V[k * m + q];
                    V[k * m + p] = c * vkp - s * vkq;
                    V[k * m + q] = s * vkp + c * vkq;
                }
            }
        }
    }
    for (int32_t i = 0; i < m; ++i) lam[i] = a[i * m + i];
    free(a);
    /* selection sort, decreasing */
    for (int32_t i = 0; i < m; ++i) {
        int32_t best = i;
        for (int32_t j = i + 1; j < m; ++j) if (lam[j] > lam[best]) best = j;
        if (best != i) {
            double t = lam[i]; lam[i] = lam[best]; lam[best] = t;
            for (int32_t k = 0; k < m; ++k) {
                double v = V[k * m + i]; V[k * m + i] = V[k * m + best]; V[k * m + best] = v;
            }
        }
    }
    for (int32_t i = 0; i < m; ++i) {
        int32_t big = 0;
        for (int32_t k = 1; k < m; ++k) if (fabs(V[k * m + i]) > fabs(V[big * m + i])) big = k;
        if (V[big * m + i] < 0.0)
            for (int32_t k = 0; k < m; ++k) V[k * m + i] = -V[k * m + i];
    }
    return sweeps;
}

/* ------------------------------------------------------- Krylov solvers */

/* Reduced quantities of Alg. 2 for the basis W (n x y, column-major, ld n):
 * AW = A W, G = W^T (A W) symmetrised, G = R^T R.  Returns the number of
 * columns kept after the pivot test. */
int orc_reduced_setup(int64_t n, const int32_t* rowptr, const int32_t* colind,
                      const double* val, const double* W, int32_t y,
                      double* AW, double* G, double* R)
{
    for (int32_t k = 0; k < y; ++k) orc_matvec(n, rowptr, colind, val, W + k * n, AW + k * n);
    for (int32_t i = 0; i < y; ++i)
        for (int32_t j = 0; j < y; ++j) G[i * y + j] = dot(n, W + i * n, AW + j * n);
    for (int32_t i = 0; i < y; ++i)
        for (int32_t j = i + 1; j < y; ++j) {
            double s = 0.5 * (G[i * y + j] + G[j * y + i]);
            G[i * y + j] = s; G[j * y + i] = s;
        }
    return orc_cholesky(y, G, R);
}

/*
 * Augmented PCG for A x = b from the initial guess xbar (in x on entry),
 * with augmenting basis W (n x y column-major; y = 0 gives plain PCG).
 *
 *   Stage 1 (Alg. 2):   rbar = b - A xbar;  G what = W^T rbar  (G = W^T A W = R^T R)
 *   Alg. 1, with Y = W, x0hat = what, on the increment system A d = rbar:
 *       d0 = W what;  r0 = rbar - A d0;  z0 = M^{-1} r0;
 *       G mu0 = (A W)^T z0;  p0 = z0 - W mu0;
 *       loop: gamma = (A p, p); alpha = (r, z) / gamma; d += alpha p;
 *             r -= alpha A p; z = M^{-1} r; beta = (r', z') / (r, z);
 *             G mu = (A W)^T z; p = z + beta p - W mu;  stop when ||r|| <= tol ||b||.
 *   x = xbar + d.
 *
 * Optional recording for tests: dirs (n x maxit, column k = p^k), iterates
 * (n x (maxit + 1), column k = xbar + d^k) and coef (2 maxit: alpha_k, beta_k
 * of every iteration, the coefficients of the Lanczos tridiagonal matrix that
 * CG implicitly builds).  Any of them may be NULL.
 */
int orc_aug_pcg(int64_t n, const int32_t* rowptr, const int32_t* colind, const double* val,
                const double* b, double* x, const double* W, int32_t y,
                double tol, int32_t maxit, orc_stats* st, double* dirs, double* iterates,
                double* coef)
{
    memset(st, 0, sizeof(*st));
    st->cond_G = 1.0;
    if (n <= 0 || y < 0 || maxit < 0 || !(tol >= 0.0)) { st->status = ORC_ERR_ARG; return st->status; }
    size_t nb = sizeof(double) * (size_t)n;
    double* dinv = (double*)malloc(nb);
    double* r = (double*)malloc(nb);
    double* z = (double*)malloc(nb);
    double* p = (double*)malloc(nb);
    double* q = (double*)malloc(nb);
    double* d = (double*)calloc((size_t)n, sizeof(double));
    double* AW = y ? (double*)malloc(nb * (size_t)y) : NULL;
    double* G = y ? (double*)malloc(sizeof(double) * (size_t)y * (size_t)y) : NULL;
    double* R = y ? (double*)malloc(sizeof(double) * (size_t)y * (size_t)y) : NULL;
    double cbuf[64], mu[64];
    int32_t yk = 0;
    int status = ORC_OK;

    if (y > 64) { status = ORC_ERR_ARG; goto done; }
    if (jacobi_inverse(n, rowptr, colind, val, dinv) != ORC_OK) { status = ORC_ERR_NOT_SPD; goto done; }

    double bnorm = sqrt(dot(n, b, b));
    st->bnorm = bnorm;
    if (!finite(bnorm)) { status = ORC_ERR_NONFINITE; goto done; }
    double eps = tol * bnorm;

    /* reduced setup: A W, W^T A W, Cholesky */
    if (y > 0) {
        yk = orc_reduced_setup(n, rowptr, colind, val, W, y, AW, G, R);
        st->matvecs += y;
        if (yk > 0) {
            double* Gk = (double*)malloc(sizeof(double) * (size_t)yk * (size_t)yk);
            double* Vk = (double*)malloc(sizeof(double) * (size_t)yk * (size_t)yk);
            double lk[64];
            for (int32_t i = 0; i < yk; ++i)
                for (int32_t j = 0; j < yk; ++j) Gk[i * yk + j] = G[i * y + j];
            orc_sym_eig(yk, Gk, Vk, lk);
            st->cond_G = lk[yk - 1] > 0.0 ? lk[0] / lk[yk - 1] : INFINITY;
            free(Gk); free(Vk);
        }
    }
    st->rank = yk;

    /* Stage 1: rbar = b - A xbar */
    orc_matvec(n, rowptr, colind, val, x, q);
    st->matvecs += 1;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
    if (yk > 0) {
        double what[64];
        for (int32_t k = 0; k < yk; ++k) cbuf[k] = dot(n, W + k * n, r);
        chol_solve(y, yk, R, cbuf, what);
        /* Alg. 1 first two steps: d0 = W what; r0 = rbar - A d0 */
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double s = 0.0;
            for (int32_t k = 0; k < yk; ++k) s += W[k * n + i] * what[k];
            d[i] = s;
        }
        orc_matvec(n, rowptr, colind, val, d, q);
        st->matvecs += 1;
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) r[i] -= q[i];
    }
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
    if (yk > 0) {
        for (int32_t k = 0; k < yk; ++k) cbuf[k] = dot(n, AW + k * n, z);
        chol_solve(y, yk, R, cbuf, mu);
    }
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = z[i];
        for (int32_t k = 0; k < yk; ++k) s -= W[k * n + i] * mu[k];
        p[i] = s;
    }
    double rho = dot(n, r, z);
    double rr = dot(n, r, r);
    st->stage1_relres = bnorm > 0.0 ? sqrt(rr) / bnorm : sqrt(rr);
    if (!finite(rr)) { status = ORC_ERR_NONFINITE; goto done; }
    if (iterates) {
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) iterates[i] = x[i] + d[i];
    }

    int32_t k = 0;
    status = ORC_NOT_CONVERGED;
    if (sqrt(rr) <= eps) status = ORC_OK;
    while (status != ORC_OK && k < maxit) {
        if (dirs) memcpy(dirs + (size_t)k * (size_t)n, p, nb);
        orc_matvec(n, rowptr, colind, val, p, q);
        st->matvecs += 1;
        double gamma = dot(n, p, q);
        if (!(gamma > 0.0)) { status = finite(gamma) ? ORC_ERR_NOT_SPD : ORC_ERR_NONFINITE; break; }
        double alpha = rho / gamma;
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            d[i] += alpha * p[i];
            r[i] -= alpha * q[i];
            z[i] = dinv[i] * r[i];
        }
        double rho_new = dot(n, r, z);
        rr = dot(n, r, r);
        double beta = rho_new / rho;
        if (coef) { coef[2 * k] = alpha; coef[2 * k + 1] = beta; }
        if (yk > 0) {
            for (int32_t j = 0; j < yk; ++j) cbuf[j] = dot(n, AW + j * n, z);
            chol_solve(y, yk, R, cbuf, mu);
        }
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double s = z[i] + beta * p[i];
            for (int32_t j = 0; j < yk; ++j) s -= W[j * n + i] * mu[j];
            p[i] = s;
        }
        rho = rho_new;
        k += 1;
        if (iterates) {
            double* xk = iterates + (size_t)k * (size_t)n;
            #pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < n; ++i) xk[i] = x[i] + d[i];
        }
        if (!finite(rr)) { status = ORC_ERR_NONFINITE; break; }
        if (sqrt(rr) <= eps) status = ORC_OK;
    }
    st->iters = k;
    st->relres = bnorm > 0.0 ? sqrt(rr) / bnorm : sqrt(rr);

    /* x = xbar + d, then the true residual */
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) x[i] += d[i];
    orc_matvec(n, rowptr, colind, val, x, q);
    st->matvecs += 1;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) q[i] = b[i] - q[i];
    double tr = sqrt(dot(n, q, q));
    st->true_relres = bnorm > 0.0 ? tr / bnorm : tr;

done:
    st->status = status;
    free(dinv); free(r); free(z); free(p); free(q); free(d);
    free(AW); free(G); free(R);
    return status;
}

/* Plain Jacobi PCG (Eq. (KrylovSolve)): the augmented solver with no basis. */
int orc_plain_pcg(int64_t n, const int32_t* rowptr, const int32_t* colind, const double* val,
                  const double* b, double* x, double tol, int32_t maxit, orc_stats* st,
                  double* dirs, double* iterates)
{
    return orc_aug_pcg(n, rowptr, colind, val, b, x, NULL, 0, tol, maxit, st, dirs, iterates, NULL);
}

/*
 * Alg. pod_evd with metric Theta = A:
 *   AS = A S;  Gbar = diag(w) S^T A S diag(w)  (symmetrised);
 *   Gbar = V Sigma^2 V^T (eigenvalues lam = sigma^2, decreasing);
 *   dimension: y = #{i : lam_i > rank_rtol * lam_1}, capped by rank_max and,
 *   when 0 < energy < 1, by the smallest i whose cumulative energy
 *   sum_{k<=i} lam_k / sum_l lam_l reaches energy;
 *   basis: W = S diag(w) [v_1 / sigma_1, ..., v_y / sigma_y]   (Eq. (podAlgebraicDefinition)).
 * S is n x s column-major; W (n x rank_max, column-major) receives the y
 * columns; lam (s) receives all eigenvalues.  Returns y.
 */
int orc_pod_evd(int64_t n, const int32_t* rowptr, const int32_t* colind, const double* val,
                const double* S, int32_t s, const double* w, int32_t rank_max,
                double rank_rtol, double energy, double* W, double* lam)
{
    if (s <= 0 || s > 64 || rank_max < 0) return 0;
    size_t nb = sizeof(double) * (size_t)n;
    double* AS = (double*)malloc(nb * (size_t)s);
    double* Gb = (double*)malloc(sizeof(double) * (size_t)s * (size_t)s);
    double* V = (double*)malloc(sizeof(double) * (size_t)s * (size_t)s);
    for (int32_t k = 0; k < s; ++k) orc_matvec(n, rowptr, colind, val, S + (size_t)k * n, AS + (size_t)k * n);
    for (int32_t i = 0; i < s; ++i)
        for (int32_t j = 0; j < s; ++j)
            Gb[i * s + j] = w[i] * dot(n, S + (size_t)i * n, AS + (size_t)j * n) * w[j];
    for (int32_t i = 0; i < s; ++i)
        for (int32_t j = i + 1; j < s; ++j) {
            double t = 0.5 * (Gb[i * s + j] + Gb[j * s + i]);
            Gb[i * s + j] = t; Gb[j * s + i] = t;
        }
    orc_sym_eig(s, Gb, V, lam);
    int32_t y = 0;
    if (lam[0] > 0.0)
        for (int32_t i = 0; i < s; ++i) if (lam[i] > rank_rtol * lam[0]) y = i + 1;
    if (y > rank_max) y = rank_max;
    if (energy > 0.0 && energy < 1.0 && y > 0) {
        double tot = 0.0, acc = 0.0;
        for (int32_t i = 0; i < s; ++i) tot += lam[i];
        int32_t ye = y;
        for (int32_t i = 0; i < y; ++i) {
            acc += lam[i];
            if (acc >= energy * tot) { ye = i + 1; break; }
        }
        y = ye;
    }
    for (int32_t i = 0; i < y; ++i) {
        double inv_sigma = 1.0 / sqrt(lam[i]);
        double coef[64];
        for (int32_t k = 0; k < s; ++k) coef[k] = w[k] * V[k * s + i] * inv_sigma;
        double* Wi = W + (size_t)i * n;
        #pragma omp parallel for schedule(static)
        for (int64_t r = 0; r < n; ++r) {
            double acc = 0.0;
            for (int32_t k = 0; k < s; ++k) acc += S[(size_t)k * n + r] * coef[k];
            Wi[r] = acc;
        }
    }
    free(AS); free(Gb); free(V);
    return y;
}
