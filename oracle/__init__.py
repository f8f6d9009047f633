"""CPU FP64 oracle for the POD-augmented CG method -- test infrastructure only.

The arithmetic lives in ``podcg_oracle.c`` (plain C, built with gcc); this
module only marshals NumPy arrays into it and runs sequences.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import
it.  It shares no code with the GPU library and never calls it.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "podcg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, NOT_CONVERGED, ERR_ARG, ERR_NOT_SPD, ERR_NONFINITE = 0, 1, -1, -4, -5


def build(verbose: bool = False, src: str = _SRC, out: str = _LIB) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` (gcc, OpenMP)."""
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
           "-std=c11", "-Wall", "-Wno-unknown-pragmas", "-o", out + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


class _Stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("matvecs", C.c_int32), ("status", C.c_int32),
                ("rank", C.c_int32), ("stage1_relres", C.c_double), ("relres", C.c_double),
                ("true_relres", C.c_double), ("bnorm", C.c_double), ("cond_G", C.c_double)]


@dataclass
class Stats:
    iters: int
    matvecs: int
    status: int
    rank: int
    stage1_relres: float
    relres: float
    true_relres: float
    bnorm: float
    cond_G: float


_lib = None
_lib_path = _LIB


def use_library(path: str | None):
    """Load the oracle from another build of podcg_oracle.c (None: the default).

    Used by the mutation tests, which compile altered copies of the source to
    show that the pins catch them."""
    global _lib, _lib_path
    _lib, _lib_path = None, (path or _LIB)


def lib():
    global _lib
    if _lib is None:
        if _lib_path == _LIB and not os.path.exists(_LIB):
            build()
        L = C.CDLL(_lib_path)
        P = C.c_void_p
        L.orc_matvec.argtypes = [C.c_int64, P, P, P, P, P]
        L.orc_matvec.restype = None
        L.orc_cholesky.argtypes = [C.c_int32, P, P]
        L.orc_cholesky.restype = C.c_int
        L.orc_sym_eig.argtypes = [C.c_int32, P, P, P]
        L.orc_sym_eig.restype = C.c_int
        L.orc_reduced_setup.argtypes = [C.c_int64, P, P, P, P, C.c_int32, P, P, P]
        L.orc_reduced_setup.restype = C.c_int
        L.orc_aug_pcg.argtypes = [C.c_int64, P, P, P, P, P, P, C.c_int32, C.c_double,
                                  C.c_int32, C.POINTER(_Stats), P, P, P]
        L.orc_aug_pcg.restype = C.c_int
        L.orc_plain_pcg.argtypes = [C.c_int64, P, P, P, P, P, C.c_double, C.c_int32,
                                    C.POINTER(_Stats), P, P]
        L.orc_plain_pcg.restype = C.c_int
        L.orc_pod_evd.argtypes = [C.c_int64, P, P, P, P, C.c_int32, P, C.c_int32,
                                  C.c_double, C.c_double, P, P]
        L.orc_pod_evd.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class CSR:
    """A CSR matrix held as NumPy arrays (int32 indices, float64 values)."""

    def __init__(self, rowptr, colind, vals):
        self.rowptr, self.colind, self.vals = _i32(rowptr), _i32(colind), _f64(vals)
        self.n = self.rowptr.size - 1

    def args(self):
        return (self.n, _p(self.rowptr), _p(self.colind), _p(self.vals))


def matvec(A: CSR, x: np.ndarray) -> np.ndarray:
    x = _f64(x)
    y = np.empty(A.n)
    lib().orc_matvec(*A.args(), _p(x), _p(y))
    return y


def cholesky(G: np.ndarray):
    """(R upper, accepted columns) with G = R^T R on the accepted block."""
    G = _f64(G)
    m = G.shape[0]
    R = np.zeros((m, m))
    k = lib().orc_cholesky(m, _p(G), _p(R))
    return R, k


def sym_eig(G: np.ndarray):
    """(lam decreasing, V columns) of a symmetric matrix by cyclic Jacobi."""
    G = _f64(G)
    m = G.shape[0]
    V = np.zeros((m, m))
    lam = np.zeros(m)
    lib().orc_sym_eig(m, _p(G), _p(V), _p(lam))
    return lam, V


def reduced_setup(A: CSR, W: np.ndarray):
    """(AW, G, R, kept) for a basis W given as (n, y) array."""
    Wc = _f64(np.asarray(W).T)               # column-major n x y
    y = Wc.shape[0]
    AW = np.zeros_like(Wc)
    G = np.zeros((y, y))
    R = np.zeros((y, y))
    kept = lib().orc_reduced_setup(*A.args(), _p(Wc), y, _p(AW), _p(G), _p(R))
    return AW.T.copy(), G, R, kept


def aug_pcg(A: CSR, b, xbar, W=None, tol=1e-8, maxit=10000, record=False, coefs=False):
    """Stage 1 + augmented PCG.  W is (n, y) or None.

    Returns (x, Stats) or, with record=True, (x, Stats, dirs, iterates) where
    dirs is (k, n) and iterates is (k + 1, n).  With coefs=True a last element
    is appended: the (k, 2) array of the iterations' (alpha, beta)."""
    n = A.n
    b = _f64(b)
    x = _f64(np.array(xbar, dtype=np.float64, copy=True))
    if W is None or np.asarray(W).size == 0:
        Wc, y = None, 0
    else:
        Wc = _f64(np.asarray(W).T)
        y = Wc.shape[0]
    st = _Stats()
    dirs = np.zeros((maxit, n)) if record else None
    its = np.zeros((maxit + 1, n)) if record else None
    ab = np.zeros((max(int(maxit), 1), 2)) if coefs else None
    lib().orc_aug_pcg(*A.args(), _p(b), _p(x), _p(Wc), y, float(tol), int(maxit),
                      C.byref(st), _p(dirs), _p(its), _p(ab))
    s = Stats(**{f: getattr(st, f) for f, _ in _Stats._fields_})
    out = (x, s, dirs[: s.iters], its[: s.iters + 1]) if record else (x, s)
    if coefs:
        out = out + (ab[: s.iters].copy(),)
    return out


def plain_pcg(A: CSR, b, xbar, tol=1e-8, maxit=10000, record=False, coefs=False):
    return aug_pcg(A, b, xbar, None, tol, maxit, record, coefs)


def lanczos_extremes(ab: np.ndarray):
    """Extreme eigenvalues of the preconditioned operator M^{-1} A estimated
    from the (alpha_k, beta_k) of a PCG run: they are the extreme eigenvalues
    of the Lanczos tridiagonal matrix T with T_kk = 1/alpha_k +
    beta_{k-1}/alpha_{k-1} and T_k,k+1 = sqrt(beta_k)/alpha_k (the standard
    CG-Lanczos relation; the estimates lie inside the true spectrum)."""
    a, b = ab[:, 0], ab[:, 1]
    k = a.size
    d = 1.0 / a
    d[1:] += b[:-1] / a[:-1]
    e = np.sqrt(b[:-1]) / a[:-1]
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    lam = np.linalg.eigvalsh(T) if k else np.zeros(1)
    return float(lam[0]), float(lam[-1])


def pod_evd(A: CSR, S: np.ndarray, weights, rank_max: int, rank_rtol: float = 1e-12,
            energy: float = 1.0):
    """POD basis of snapshots S ((n, s) array) in the A metric.

    Returns (W (n, y), lam (s,))."""
    Sc = _f64(np.asarray(S).T)
    s = Sc.shape[0]
    w = _f64(weights)
    W = np.zeros((max(rank_max, 1), A.n))
    lam = np.zeros(s)
    y = lib().orc_pod_evd(*A.args(), _p(Sc), s, _p(w), int(rank_max), float(rank_rtol),
                          float(energy), _p(W), _p(lam))
    return W[:y].T.copy(), lam


def idw_weights(count: int) -> np.ndarray:
    """Inverse-distance weights 1 / 2^(i - 1), i = 1 the most recent snapshot."""
    return np.array([2.0 ** (-(i - 1)) for i in range(1, count + 1)])


from .sequence import run_sequence  # noqa: E402

__all__ = ["build", "lib", "use_library", "CSR", "matvec", "cholesky", "sym_eig", "reduced_setup",
           "aug_pcg", "plain_pcg", "lanczos_extremes", "pod_evd", "idw_weights", "run_sequence", "Stats"]
