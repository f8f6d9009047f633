"""A 2-D diffusion sequence whose inputs are bitwise reproducible anywhere.

The other generators evaluate random Fourier fields with matrix products and
cos/exp, whose last bits depend on the BLAS build, its thread count and the
CPU's vector unit.  This one uses only integer hashing and the correctly
rounded operations + - * / in a fixed order, so every machine produces the
same bits.  It exists for tests that compare stored results exactly and for
small sequences that must exercise the snapshot ring (omega smaller than the
number of systems) with a matrix that changes from system to system.

* Coefficient on the extended (N+2)^2 node grid: k_j[a, c] = 1 + 0.75 u(a, c + j),
  u a dyadic hash in [0, 1) -- a rough field that shifts one node per system.
* Load: b_j = f_1 + c_j f_2 + s_j f_3 with f_i dyadic hash fields in [-1, 1),
  smoothed by two passes of a 5-point average, and (c_j, s_j) the rational
  rotation ((1 - t^2), 2 t) / (1 + t^2), t = j / 8.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .fv import FVDiffusion


def _hash_unit(a: np.ndarray, c: np.ndarray, salt: int) -> np.ndarray:
    """Dyadic values in [0, 1) from integer coordinates (exact in float64)."""
    h = (a.astype(np.uint64) * np.uint64(73856093)) ^ (c.astype(np.uint64) * np.uint64(19349663)) \
        ^ np.uint64(salt * 83492791 + 1)
    h = (h * np.uint64(2654435761)) & np.uint64(0xFFFFFFFF)
    h ^= h >> np.uint64(15)
    h = (h * np.uint64(2246822519)) & np.uint64(0xFFFFFFFF)
    h ^= h >> np.uint64(13)
    return (h >> np.uint64(8)).astype(np.float64) / float(1 << 24)


def _smooth(f: np.ndarray) -> np.ndarray:
    """One pass of (4 f + neighbours) / 8 on an N x N grid (zero outside)."""
    g = np.pad(f, 1)
    return (4.0 * f + g[:-2, 1:-1] + g[2:, 1:-1] + g[1:-1, :-2] + g[1:-1, 2:]) / 8.0


@dataclass
class ExactDiffusion2D:
    N: int = 16
    steps: int = 8
    omega: int = 3
    rank: int = 2
    tol: float = 1e-10
    amp: float = 0.75
    name: str = field(default="exact_diffusion2d")

    def __post_init__(self):
        self.fv = FVDiffusion(self.N, 2)
        self.n, self.nnz = self.fv.n, self.fv.nnz
        self.rowptr, self.colind = self.fv.rowptr, self.fv.colind
        M = self.N + 2
        a, c = np.meshgrid(np.arange(M), np.arange(M + self.steps + 1), indexing="ij")
        self._u = _hash_unit(a, c, 1)                       # (M, M + steps + 1)
        ia, ic = np.meshgrid(np.arange(self.N), np.arange(self.N), indexing="ij")
        self._f = []
        for salt in (2, 3, 4):
            f = 2.0 * _hash_unit(ia, ic, salt) - 1.0
            self._f.append(_smooth(_smooth(f)).ravel())

    def matrix_values(self, j: int) -> np.ndarray:
        M = self.N + 2
        k = 1.0 + self.amp * self._u[:, j:j + M]
        return self.fv.values(k)

    def rhs(self, j: int, x_prev: np.ndarray | None = None) -> np.ndarray:
        t = j / 8.0
        den = 1.0 + t * t
        cj, sj = (1.0 - t * t) / den, (2.0 * t) / den
        return self._f[0] + cj * self._f[1] + sj * self._f[2]

    def describe(self) -> dict:
        return {"workload": self.name, "N": self.N, "n": self.n, "nnz": self.nnz,
                "steps": self.steps, "omega": self.omega, "rank": self.rank, "tol": self.tol}


def exact2d(**kw) -> ExactDiffusion2D:
    return ExactDiffusion2D(**kw)
