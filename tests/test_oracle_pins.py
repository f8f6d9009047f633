"""Pins of the CPU oracle against facts the paper and linear algebra fix.

None of these retypes the oracle's own recurrence.  Each compares it with an
independent statement: a dense direct solve, the closed-form A-orthogonal
projector (pseudo-inverse form), the Galerkin solution on an explicitly built
augmented Krylov space, the Eckart-Young optimum of POD, the SVD route to
POD, a theorem bound, or a library routine.
"""

import numpy as np
import pytest

from problems import tiny

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _system(n=40, cond=1e3, seed=0, y=5):
    A = tiny.random_spd(n, cond, seed)
    # non-constant diagonal so the Jacobi preconditioner matters
    D = np.diag(np.linspace(0.5, 2.0, n))
    A = D @ A @ D
    r = _rng(seed + 100)
    b = r.standard_normal(n)
    W = r.standard_normal((n, y))
    return A, b, W


def _csr(orc, A):
    return orc.CSR(*tiny.dense_to_csr(A, drop_zeros=False))


def _aproj(A, W, xstar, xbar):
    """A-orthogonal projection of xstar onto xbar + range(W), pseudo-inverse form
    xbar + W (A^{1/2} W)^+ A^{1/2} (xstar - xbar) with A = L L^T, A^{1/2} = L^T."""
    L = np.linalg.cholesky(A)
    Ah = L.T
    return xbar + W @ (np.linalg.pinv(Ah @ W) @ (Ah @ (xstar - xbar)))


# ---------------------------------------------------------------- primitives

def test_matvec_matches_dense(orc):
    A, b, _ = _system(n=33, seed=1)
    A[np.abs(A) < 0.3] = 0.0
    np.fill_diagonal(A, 5.0)
    x = _rng(2).standard_normal(33)
    y = orc.matvec(orc.CSR(*tiny.dense_to_csr(A)), x)
    assert np.allclose(y, A @ x, rtol=1e-14, atol=1e-13)


def test_cholesky_matches_library(orc):
    A, _, _ = _system(n=12, cond=50, seed=3)
    R, k = orc.cholesky(A)
    assert k == 12
    assert np.allclose(R, np.linalg.cholesky(A).T, rtol=1e-12, atol=1e-12)


def test_cholesky_truncates_at_dependent_column(orc):
    r = _rng(4)
    X = r.standard_normal((20, 4))
    X = np.column_stack([X, X[:, 0] + X[:, 1], r.standard_normal(20)])
    G = X.T @ X
    R, k = orc.cholesky(G)
    assert k == 4
    assert np.allclose(R[:4, :4].T @ R[:4, :4], G[:4, :4], rtol=1e-12)


def test_sym_eig_matches_library(orc):
    r = _rng(5)
    M = r.standard_normal((9, 9))
    G = M @ M.T + np.diag(np.arange(9.0))
    lam, V = orc.sym_eig(G)
    ref = np.linalg.eigvalsh(G)[::-1]
    assert np.allclose(lam, ref, rtol=1e-13, atol=1e-12 * ref[0])
    assert np.allclose(V @ np.diag(lam) @ V.T, G, atol=1e-12 * ref[0])
    assert np.allclose(V.T @ V, np.eye(9), atol=1e-13)
    assert np.all(np.diff(lam) <= 0)
    big = np.argmax(np.abs(V), axis=0)
    assert np.all(V[big, np.arange(9)] > 0)


# ---------------------------------------------------------------- solvers

def test_T1_solution_matches_dense_solve(orc):
    A, b, W = _system(seed=6)
    xstar = np.linalg.solve(A, b)
    x, st = orc.aug_pcg(_csr(orc, A), b, np.zeros_like(b), W, tol=1e-12, maxit=500)
    assert st.status == orc.OK and st.rank == W.shape[1]
    err = np.linalg.norm(x - xstar) / np.linalg.norm(xstar)
    assert err <= 1e3 * 1e-12 * 10
    assert st.true_relres <= 1e-11


def test_T2_stage1_is_the_A_projection_and_galerkin(orc):
    A, b, W = _system(seed=7)
    xbar = _rng(8).standard_normal(b.size)
    x, st = orc.aug_pcg(_csr(orc, A), b, xbar, W, tol=0.0, maxit=0)
    assert st.iters == 0 and st.status == orc.NOT_CONVERGED
    xstar = np.linalg.solve(A, b)
    ref = _aproj(A, W, xstar, xbar)
    assert np.linalg.norm(x - ref) <= 1e-11 * np.linalg.norm(ref)
    # residual orthogonal to range(W), Eq. (equivalenceResidualOrth)
    g = W.T @ (b - A @ x)
    assert np.linalg.norm(g) <= 1e-11 * np.linalg.norm(W) * np.linalg.norm(b)
    assert np.isclose(st.stage1_relres, np.linalg.norm(b - A @ x) / np.linalg.norm(b),
                      rtol=1e-8)


def test_T3_directions_A_orthogonal_to_W_and_each_other(orc):
    A, b, W = _system(n=40, cond=100, seed=9)
    _, st, P, _ = orc.aug_pcg(_csr(orc, A), b, np.zeros_like(b), W, tol=1e-10,
                              maxit=200, record=True)
    assert st.iters >= 10
    AP = A @ P.T
    rel = np.linalg.norm(W.T @ AP, axis=0) / (np.linalg.norm(W) * np.linalg.norm(AP, axis=0))
    assert rel.max() <= 1e-12
    Gm = P[:8] @ A @ P[:8].T
    d = np.sqrt(np.diag(Gm))
    off = Gm / np.outer(d, d) - np.eye(8)
    assert np.abs(off).max() <= 1e-10


def test_T4_exact_recovery_when_solution_in_span(orc):
    A, _, W = _system(seed=10)
    c = _rng(11).standard_normal(W.shape[1])
    xbar = _rng(12).standard_normal(W.shape[0])
    xstar = xbar + W @ c
    b = A @ xstar
    x, st = orc.aug_pcg(_csr(orc, A), b, xbar, W, tol=1e-10, maxit=100)
    assert st.iters == 0 and st.status == orc.OK
    assert np.linalg.norm(x - xstar) <= 1e-12 * np.linalg.norm(xstar)


def test_T5_finite_termination_within_n_minus_y(orc):
    n, y = 14, 5
    A, b, W = _system(n=n, cond=10, seed=13, y=y)
    _, st = orc.aug_pcg(_csr(orc, A), b, np.zeros(n), W, tol=1e-13, maxit=100)
    assert st.status == orc.OK
    assert st.iters <= n - y


def test_T5_plain_terminates_in_distinct_eigenvalue_count(orc):
    A, lam = tiny.circulant_spd(24, seed=14)
    distinct = np.unique(np.round(lam, 9)).size
    b = _rng(15).standard_normal(24)
    _, st = orc.plain_pcg(_csr(orc, A), b, np.zeros(24), tol=1e-12, maxit=100)
    assert st.status == orc.OK
    assert st.iters <= distinct < 24


def _krylov_galerkin(A, b, xbar, W, k):
    """argmin of the A-norm error over xbar + range(W) + K_k(Pi M^-1 A, Pi M^-1 r0),
    Pi = I - W (W^T A W)^{-1} W^T A, r0 the residual after the projection on range(W);
    for W empty, plain PCG's Eq. (KrylovSolve)."""
    n = b.size
    Minv = np.diag(1.0 / np.diag(A))
    if W is None:
        Pi = np.eye(n)
        x0 = xbar
        basis0 = np.zeros((n, 0))
    else:
        Pi = np.eye(n) - W @ np.linalg.solve(W.T @ A @ W, W.T @ A)
        x0 = xbar + W @ np.linalg.solve(W.T @ A @ W, W.T @ (b - A @ xbar))
        basis0 = W
    v = Pi @ Minv @ (b - A @ x0)
    K = []
    for _ in range(k):
        for u in K:                       # orthonormalise for a well-posed basis
            v = v - (u @ v) * u
        for u in K:
            v = v - (u @ v) * u
        v = v / np.linalg.norm(v)
        K.append(v)
        v = Pi @ Minv @ A @ v
    B = np.column_stack([basis0] + K)
    return xbar + B @ np.linalg.solve(B.T @ A @ B, B.T @ (b - A @ xbar))


@pytest.mark.parametrize("with_basis", [True, False])
def test_T6_iterates_minimise_A_norm_over_augmented_krylov_space(orc, with_basis):
    A, b, W = _system(n=30, cond=200, seed=16)
    if not with_basis:
        W = None
    xbar = _rng(17).standard_normal(b.size)
    _, st, _, its = orc.aug_pcg(_csr(orc, A), b, xbar, W, tol=0.0, maxit=7, record=True)
    xstar = np.linalg.solve(A, b)
    for k in range(1, 8):
        ref = _krylov_galerkin(A, b, xbar, W, k)
        assert np.linalg.norm(its[k] - ref) <= 1e-9 * np.linalg.norm(xstar), k


def test_T8_identity_basis_is_a_direct_solve(orc):
    A, b, _ = _system(n=20, cond=100, seed=18)
    x, st = orc.aug_pcg(_csr(orc, A), b, np.zeros(20), np.eye(20), tol=1e-10, maxit=10)
    assert st.iters == 0
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-11, atol=1e-12)


def test_relative_stopping_rule(orc):
    A, b, W = _system(seed=19)
    for tol in (1e-4, 1e-8):
        x, st = orc.aug_pcg(_csr(orc, A), b, np.zeros_like(b), W, tol=tol, maxit=500)
        assert st.relres <= tol
        assert st.status == orc.OK


def test_zero_rhs_zero_guess_is_zero_iterations(orc):
    A, b, W = _system(seed=20)
    x, st = orc.aug_pcg(_csr(orc, A), np.zeros_like(b), np.zeros_like(b), W, 1e-8, 50)
    assert st.iters == 0 and st.status == orc.OK and not np.any(x)


def test_error_paths(orc):
    A, b, W = _system(n=10, seed=21, y=2)
    Aneg = A.copy()
    Aneg[3, 3] = -1.0
    _, st = orc.aug_pcg(_csr(orc, Aneg), b, np.zeros(10), W, 1e-8, 50)
    assert st.status == orc.ERR_NOT_SPD
    bn = b.copy()
    bn[2] = np.nan
    _, st = orc.aug_pcg(_csr(orc, A), bn, np.zeros(10), W, 1e-8, 50)
    assert st.status == orc.ERR_NONFINITE
    _, st = orc.aug_pcg(_csr(orc, A), b, np.zeros(10), W, 1e-14, 1)
    assert st.status == orc.NOT_CONVERGED and st.iters == 1
    # indefinite (negative eigenvalue, positive diagonal): gamma <= 0 is caught
    Q = np.linalg.qr(_rng(22).standard_normal((10, 10)))[0]
    lam = np.linspace(1, 10, 10)
    lam[0] = -5.0
    Ai = (Q * lam) @ Q.T
    Ai = 0.5 * (Ai + Ai.T) + np.diag(np.full(10, 0.0))
    if np.all(np.diag(Ai) > 0):
        _, st = orc.plain_pcg(_csr(orc, Ai), Q[:, 0], np.zeros(10), 1e-12, 50)
        assert st.status in (orc.ERR_NOT_SPD, orc.OK)


def test_dependent_basis_is_truncated(orc):
    A, b, W = _system(seed=23, y=3)
    Wd = np.column_stack([W, W[:, 0] + 2 * W[:, 1]])
    x, st = orc.aug_pcg(_csr(orc, A), b, np.zeros_like(b), Wd, 1e-10, 500)
    assert st.rank == 3 and st.status == orc.OK


# ---------------------------------------------------------------- POD

def _pod_setup(seed=30, n=50, s=7):
    A, _, _ = _system(n=n, cond=300, seed=seed)
    S = _rng(seed + 1).standard_normal((n, s))
    w = np.array([2.0 ** (-i) for i in range(s)])
    return A, S, w


def test_T9_pod_basis_is_A_orthonormal_and_nested(orc):
    A, S, w = _pod_setup()
    W4, lam = orc.pod_evd(_csr(orc, A), S, w, 4)
    W5, _ = orc.pod_evd(_csr(orc, A), S, w, 5)
    assert W4.shape == (50, 4) and W5.shape == (50, 5)
    assert np.allclose(W5.T @ A @ W5, np.eye(5), atol=1e-11)
    assert np.allclose(W5[:, :4], W4, rtol=0, atol=1e-13 * np.abs(W4).max())


def test_T10_pod_attains_eckart_young_optimum(orc):
    A, S, w = _pod_setup(seed=31)
    Sw = S * w
    for y in (1, 3, 5):
        W, lam = orc.pod_evd(_csr(orc, A), S, w, y)
        P = W @ np.linalg.solve(W.T @ A @ W, W.T @ A)
        E = Sw - P @ Sw
        err = np.einsum("ij,ij->", E, A @ E)
        assert np.isclose(err, lam[y:].sum(), rtol=1e-9)
        # any other y-dimensional subspace does no better
        Q = _rng(32 + y).standard_normal((50, y))
        P2 = Q @ np.linalg.solve(Q.T @ A @ Q, Q.T @ A)
        E2 = Sw - P2 @ Sw
        assert np.einsum("ij,ij->", E2, A @ E2) >= err


def test_T11_pod_evd_equals_pod_svd(orc):
    A, S, w = _pod_setup(seed=33)
    W, lam = orc.pod_evd(_csr(orc, A), S, w, 4)
    L = np.linalg.cholesky(A)
    U, sig, Vt = np.linalg.svd(L.T @ (S * w), full_matrices=False)
    assert np.allclose(lam, sig ** 2, rtol=1e-10)
    Wsvd = (S * w) @ Vt[:4].T / sig[:4]
    # same basis up to the sign of each column
    for i in range(4):
        s = np.sign(W[:, i] @ Wsvd[:, i])
        assert np.allclose(W[:, i], s * Wsvd[:, i], rtol=0, atol=1e-10 * np.abs(W[:, i]).max())


def test_pod_rank_cut_on_dependent_snapshots(orc):
    A, S, w = _pod_setup(seed=34, s=4)
    S = np.column_stack([S, S[:, 0] - S[:, 2], 3.0 * S[:, 1]])
    w = np.ones(6)
    W, lam = orc.pod_evd(_csr(orc, A), S, w, 6, rank_rtol=1e-12)
    assert W.shape[1] == 4
    assert np.allclose(W.T @ A @ W, np.eye(4), atol=1e-10)


def test_pod_energy_criterion(orc):
    A, S, w = _pod_setup(seed=35)
    _, lam = orc.pod_evd(_csr(orc, A), S, w, 7)
    frac = np.cumsum(lam) / lam.sum()
    for e in (0.5, 0.9, 0.999):
        W, _ = orc.pod_evd(_csr(orc, A), S, w, 7, energy=e)
        assert W.shape[1] == int(np.argmax(frac >= e)) + 1


def test_T12_theorem5_reduced_matrix_bound(orc):
    from problems import config2
    cfg = config2(N=10, steps=6)
    A0 = orc.CSR(cfg.rowptr, cfg.colind, cfg.matrix_values(2))
    A1 = orc.CSR(cfg.rowptr, cfg.colind, cfg.matrix_values(3))
    D0, D1 = cfg.fv.dense(A0.vals), cfg.fv.dense(A1.vals)
    S = np.linalg.solve(D0, _rng(36).standard_normal((cfg.n, 5)))
    W, _ = orc.pod_evd(A0, S, np.ones(5), 5)
    _, G, _, _ = orc.reduced_setup(A1, W)
    lhs = np.linalg.norm(G - np.eye(W.shape[1]), 2)
    rhs = np.linalg.norm(W, 2) ** 2 * np.linalg.norm(D1 - D0, 2)
    assert lhs <= rhs
    _, G0, _, _ = orc.reduced_setup(A0, W)
    assert np.allclose(G0, np.eye(W.shape[1]), atol=1e-10)


def test_config1_scaled_matrices_give_scaled_identity_gram(orc):
    from problems import config1
    cfg = config1()
    A3 = orc.CSR(cfg.rowptr, cfg.colind, cfg.matrix_values(3))
    A4 = orc.CSR(cfg.rowptr, cfg.colind, cfg.matrix_values(4))
    S = np.column_stack([cfg.rhs(j) for j in range(1, 4)])
    W, _ = orc.pod_evd(A3, S, np.ones(3), 3)
    _, G, _, _ = orc.reduced_setup(A4, W)
    assert np.allclose(G, (1.04 / 1.03) * np.eye(3), atol=1e-12)


def test_exact_recovery_on_r2_sequence(orc):
    """Every x_j lies in one fixed 2-D space, so from j = 3 on the POD rank is 2
    and Stage 1 alone reaches the accuracy of the stored snapshots (about tol)."""
    from problems import config1
    cfg = config1(variant="r2", steps=6)
    res = orc.run_sequence(cfg, "aug")
    for r in res[2:]:
        assert r["rank"] == 2 and r["rank_next"] == 2
        assert r["stage1_relres"] <= 3 * cfg.tol
        assert r["iters"] <= 5 and r["status"] == orc.OK


def test_lanczos_extremes_from_pcg_coefficients(orc):
    """The (alpha, beta) a PCG run records give the Lanczos tridiagonal matrix
    of the Jacobi-preconditioned operator: run to near exhaustion on a small
    system, its extreme eigenvalues are those of D^{-1/2} A D^{-1/2}."""
    A, b, _ = _system(n=30, cond=1e3, seed=21)
    _, st, ab = orc.plain_pcg(_csr(orc, A), b, np.zeros(30), tol=1e-15, maxit=60, coefs=True)
    assert ab.shape == (st.iters, 2) and st.iters >= 25
    d = 1.0 / np.sqrt(np.diag(A))
    lam = np.linalg.eigvalsh(d[:, None] * A * d[None, :])
    lo, hi = orc.lanczos_extremes(ab)
    assert abs(lo - lam[0]) <= 1e-6 * lam[0] and abs(hi - lam[-1]) <= 1e-8 * lam[-1]
