"""Gaussian random fields by random Fourier features.

A stationary Gaussian field with squared-exponential covariance
exp(-|x - x'|^2 / (2 l^2)) is approximated (Rahimi & Recht, 2007) by

    g(x) = sqrt(2 / M) * sum_m cos(w_m . x + phi_m),
    w_m ~ N(0, l^-2 I),  phi_m ~ U[0, 2 pi).

The field has unit variance and can be evaluated at any point, so drifting or
rotated copies of one field are exact (no interpolation).
"""

from __future__ import annotations

import numpy as np


class FourierField:
    """A seeded random-Fourier-feature field on R^d."""

    def __init__(self, dim: int, corr_len: float, seed: int, n_features: int = 512):
        rng = np.random.Generator(np.random.PCG64(seed))
        self.dim = int(dim)
        self.corr_len = float(corr_len)
        self.n_features = int(n_features)
        self.omega = rng.normal(0.0, 1.0 / corr_len, size=(n_features, dim))
        self.phase = rng.uniform(0.0, 2.0 * np.pi, size=n_features)
        self.scale = np.sqrt(2.0 / n_features)

    def rotated(self, theta: float, center) -> "FourierField":
        """The field x -> g(c + R(theta) (x - c)), itself a Fourier-feature field:
        w_m . (c + R (x - c)) = (R^T w_m) . x + w_m . c - (R^T w_m) . c (2-D only)."""
        if self.dim != 2:
            raise ValueError("rotation is defined for 2-D fields")
        c = np.asarray(center, dtype=np.float64)
        rot = np.array([[np.cos(theta), -np.sin(theta)], [np.sin(theta), np.cos(theta)]])
        out = object.__new__(FourierField)
        out.dim, out.corr_len, out.n_features = self.dim, self.corr_len, self.n_features
        out.omega = self.omega @ rot                      # rows (R^T w_m)^T
        out.phase = self.phase + self.omega @ c - out.omega @ c
        out.scale = self.scale
        return out

    def at_points(self, pts: np.ndarray, chunk: int = 65536) -> np.ndarray:
        """Evaluate at an (m, dim) array of points."""
        pts = np.asarray(pts, dtype=np.float64).reshape(-1, self.dim)
        out = np.empty(pts.shape[0], dtype=np.float64)
        for s in range(0, pts.shape[0], chunk):
            arg = pts[s:s + chunk] @ self.omega.T + self.phase
            out[s:s + chunk] = self.scale * np.cos(arg).sum(axis=1)
        return out

    def on_grid(self, *axes: np.ndarray) -> np.ndarray:
        """Evaluate on the tensor grid of 1-D coordinate arrays ``axes``.

        ``axes[0]`` is the fastest-varying coordinate; the result has shape
        ``(len(axes[-1]), ..., len(axes[0]))`` (C order, x fastest).  The sum
        over features is done as complex products of 1-D factors,
        cos(a + b + c + phi) = Re(e^{i phi} e^{ia} e^{ib} e^{ic}).
        """
        if len(axes) != self.dim:
            raise ValueError("need one coordinate array per dimension")
        fac = [np.exp(1j * np.outer(self.omega[:, d], np.asarray(a, np.float64)))
               for d, a in enumerate(axes)]                      # (M, len_d)
        amp = np.exp(1j * self.phase)                            # (M,)
        if self.dim == 1:
            val = (amp[:, None] * fac[0]).sum(axis=0)
            return self.scale * val.real
        if self.dim == 2:
            # out[j, i] = Re sum_m amp_m Y[m, j] X[m, i]
            val = (fac[1] * amp[:, None]).T @ fac[0]
            return self.scale * val.real
        if self.dim == 3:
            nz, ny, nx = len(axes[2]), len(axes[1]), len(axes[0])
            out = np.empty((nz, ny, nx), dtype=np.float64)
            for k in range(nz):
                coef = amp * fac[2][:, k]
                out[k] = ((fac[1] * coef[:, None]).T @ fac[0]).real
            return self.scale * out
        raise ValueError("dim must be 1, 2 or 3")
