"""Small seeded SPD matrices in CSR form, for pins and edge cases."""

from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def dense_to_csr(A: np.ndarray, drop_zeros: bool = True):
    """(rowptr int32, colind int32, vals float64) of a dense matrix."""
    A = np.asarray(A, dtype=np.float64)
    mask = (A != 0.0) if drop_zeros else np.ones_like(A, dtype=bool)
    np.fill_diagonal(mask, True)
    rowptr = np.zeros(A.shape[0] + 1, dtype=np.int32)
    np.cumsum(mask.sum(axis=1), out=rowptr[1:])
    rows, cols = np.nonzero(mask)
    return rowptr, cols.astype(np.int32), A[rows, cols].copy()


def random_spd(n: int, cond: float, seed: int) -> np.ndarray:
    """Dense Q diag(lam) Q^T with eigenvalues log-spaced in [1, cond]."""
    r = _rng(seed)
    Q, _ = np.linalg.qr(r.standard_normal((n, n)))
    lam = np.logspace(0.0, np.log10(cond), n)
    A = (Q * lam) @ Q.T
    return 0.5 * (A + A.T)


def laplacian_1d(n: int, shift: float = 0.0) -> np.ndarray:
    A = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    return A + shift * np.eye(n)


def laplacian_2d(N: int, shift: float = 0.0) -> np.ndarray:
    T = laplacian_1d(N)
    I = np.eye(N)
    return np.kron(I, T) + np.kron(T, I) + shift * np.eye(N * N)


def circulant_spd(n: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Symmetric positive definite circulant matrix and its eigenvalues.

    First row c with c_k = c_{n-k}.  The eigenvalues are the real DFT of c,
    lam_m = sum_k c_k cos(2 pi k m / n), and lam_m = lam_{n-m}, so there are
    at most n // 2 + 1 distinct values.  The diagonal is constant, so a
    Jacobi preconditioner is a multiple of the identity.
    """
    r = _rng(seed)
    half = r.uniform(-1.0, 1.0, size=n // 2 + 1)
    c = np.zeros(n)
    c[: n // 2 + 1] = half
    for k in range(1, (n + 1) // 2):
        c[n - k] = c[k]
    lam = np.array([np.sum(c * np.cos(2 * np.pi * np.arange(n) * m / n)) for m in range(n)])
    c[0] += 1.0 - lam.min()                 # make the smallest eigenvalue 1
    lam += 1.0 - lam.min()
    A = np.array([[c[(j - i) % n] for j in range(n)] for i in range(n)])
    return A, lam

