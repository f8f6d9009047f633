"""The synthetic sequences A_j x_j = b_j used by the tests and the benchmark.

Every constant lives here, so a run can record exactly what it solved.

* Config 1 -- 2-D 5-point variable-coefficient diffusion, N = 32 (n = 1024).
  k_j(x) = exp(0.5 g(x)) (1 + 0.01 j) with g a unit-variance field of
  correlation length 0.2 (seed 1).  Because the factor (1 + 0.01 j) is
  uniform, A_j = (1 + 0.01 j) A_0 exactly.  b_j(x) = f(c + R(theta_j)(x - c)),
  f a second field (seed 2), c the centre of the square, theta_j = 0.05 j rad:
  the load pattern rotates slowly about the centre.  Ten systems,
  snapshot memory 5, POD rank 4, relative tolerance 1e-8.
  Variant "r2": b_j = cos(theta_j) f_1 + sin(theta_j) f_2, so every x_j lies
  in a fixed two-dimensional space (exact-recovery case).

* Config 2 -- 3-D 7-point diffusion, N = 128 (n = 2,097,152), one implicit
  time step per system: A_j = K(k_j) + (1/dt) I, dt = 1e-3.
  k_j(x) = exp(g(x - j h e_1)): a lognormal field (sigma = 1, correlation
  length 0.1) that drifts one cell along x per step.
  b_j = x_{j-1} / dt + s with s = 1 and x_0 = 0.  Fifty systems, snapshot
  memory 20, POD rank 10, relative tolerance 1e-10.
  Smaller N gives the same problem family at test sizes.

* Config 3 -- 3-D Q1 hexahedral linear elasticity on 64^3 nodes x 3 dof
  (n = 786,432, nnz = 61,731,000), Young's modulus exp(0.5 g) per element
  (correlation length 0.2, seed 5), nu = 0.3, face x = 0 clamped.  Body
  force (0, 0, -1)(1 + 0.05 sin j), j = 1..30; snapshot memory 10, POD rank 6,
  relative tolerance 1e-8, solved in FP32 inside FP64 refinement.  As stated,
  A is constant and the b_j are collinear, so from j = 2 on Stage 1 alone is
  exact.  Variant "moving": the load is additionally weighted by a Gaussian
  bump (width 0.15, amplitude 1) whose centre moves along x with j, which
  makes the solutions genuinely change.

* Config 4 -- a batch of 64 independent config-1-type sequences with uneven
  sizes: side N_i drawn uniformly from {64, ..., 512} (seed 3), member i
  with coefficient field seed 1000 + 2 i and load field seed 1001 + 2 i;
  A_j = (1 + 0.01 j) A_0 per member, b_j the load field rotated by 0.05 j rad
  about the centre; 20 systems, snapshot memory 10, POD rank 6, relative
  tolerance 1e-8, FP64.  The rotated load is evaluated on the grid as a
  Fourier field with rotated frequencies (same function as config 1's
  pointwise evaluation, computed by matrix products).

* Config 5 -- differentiation: the config-2 family at N = 96 (n = 884,736),
  200 systems, snapshot memory 20, POD rank 10, relative tolerance 1e-10.
  Outputs q_j = C x_j with C = 256 distinct seeded rows of the identity
  (seed 6).  Parameters: the log-coefficient field theta on the extended
  grid (kappa_j is the window of exp(theta) shifted by j cells) and the
  source s (b_j = x_{j-1} / dt + s).  Adjoint gradients are checkpointed every
  20 systems.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .elasticity import Q1Elasticity
from .fv import FVDiffusion
from .grf import FourierField


@dataclass
class Config1Diffusion2D:
    N: int = 32
    steps: int = 10
    omega: int = 5
    rank: int = 4
    tol: float = 1e-8
    corr_len: float = 0.2
    sigma: float = 0.5
    growth: float = 0.01
    dtheta: float = 0.05
    seed_kappa: int = 1
    seed_rhs: int = 2
    seed_rhs2: int = 3
    variant: str = "rotate"          # "rotate" or "r2"
    name: str = field(default="config1_diffusion2d")

    def __post_init__(self):
        self.fv = FVDiffusion(self.N, 2)
        self.n, self.nnz = self.fv.n, self.fv.nnz
        self.rowptr, self.colind = self.fv.rowptr, self.fv.colind
        ax = self.fv.node_axis()
        g = FourierField(2, self.corr_len, self.seed_kappa).on_grid(ax, ax)
        self._vals0 = self.fv.values(np.exp(self.sigma * g))
        self._pts = self.fv.interior_points()
        self._f1 = FourierField(2, self.corr_len, self.seed_rhs)
        self._f2 = FourierField(2, self.corr_len, self.seed_rhs2)

    def matrix_values(self, j: int) -> np.ndarray:
        return self._vals0 * (1.0 + self.growth * j)

    def rhs(self, j: int, x_prev: np.ndarray | None = None) -> np.ndarray:
        th = self.dtheta * j
        if self.variant == "r2":
            return np.cos(th) * self._f1.at_points(self._pts) + \
                np.sin(th) * self._f2.at_points(self._pts)
        c = np.array([0.5, 0.5])
        rot = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
        q = c + (self._pts - c) @ rot.T
        return self._f1.at_points(q)

    def describe(self) -> dict:
        return {"workload": self.name, "N": self.N, "n": self.n, "nnz": self.nnz,
                "steps": self.steps, "omega": self.omega, "rank": self.rank,
                "tol": self.tol, "variant": self.variant}


class Config4Member:
    """One sequence of the config-4 batch (config-1 type, side N)."""

    def __init__(self, N: int, seed_kappa: int, seed_rhs: int, steps: int, omega: int, rank: int,
                 tol: float, corr_len: float = 0.2, sigma: float = 0.5, growth: float = 0.01,
                 dtheta: float = 0.05):
        self.N, self.steps, self.omega, self.rank, self.tol = N, steps, omega, rank, tol
        self.growth, self.dtheta = growth, dtheta
        self.seed_kappa, self.seed_rhs = seed_kappa, seed_rhs
        self.fv = FVDiffusion(N, 2)
        self.n, self.nnz = self.fv.n, self.fv.nnz
        self.rowptr, self.colind = self.fv.rowptr, self.fv.colind
        ax = self.fv.node_axis()
        g = FourierField(2, corr_len, seed_kappa).on_grid(ax, ax)
        self._vals0 = self.fv.values(np.exp(sigma * g))
        self._f = FourierField(2, corr_len, seed_rhs)
        self._ax = (np.arange(N, dtype=np.float64) + 1.0) * self.fv.h

    def matrix_values(self, j: int) -> np.ndarray:
        return self._vals0 * (1.0 + self.growth * j)

    def rhs(self, j: int, x_prev: np.ndarray | None = None) -> np.ndarray:
        f = self._f.rotated(self.dtheta * j, (0.5, 0.5))
        return f.on_grid(self._ax, self._ax).ravel()


@dataclass
class Config4Batch:
    members_count: int = 64
    n_min: int = 64
    n_max: int = 512
    steps: int = 20
    omega: int = 10
    rank: int = 6
    tol: float = 1e-8
    seed_sizes: int = 3
    name: str = field(default="config4_batched")

    def __post_init__(self):
        rng = np.random.Generator(np.random.PCG64(self.seed_sizes))
        self.sides = rng.integers(self.n_min, self.n_max + 1, size=self.members_count)
        self.members = [Config4Member(int(N), 1000 + 2 * i, 1001 + 2 * i, self.steps, self.omega,
                                      self.rank, self.tol)
                        for i, N in enumerate(self.sides)]
        self.n_total = int(sum(m.n for m in self.members))
        self.nnz_total = int(sum(m.nnz for m in self.members))

    def describe(self) -> dict:
        return {"workload": self.name, "sequences": self.members_count,
                "side_range": [self.n_min, self.n_max], "n_total": self.n_total,
                "nnz_total": self.nnz_total, "steps": self.steps, "omega": self.omega,
                "rank": self.rank, "tol": self.tol}


@dataclass
class Config2Diffusion3D:
    N: int = 128
    steps: int = 50
    omega: int = 20
    rank: int = 10
    tol: float = 1e-10
    dt: float = 1e-3
    corr_len: float = 0.1
    sigma: float = 1.0
    source: float = 1.0
    seed_kappa: int = 4
    name: str = field(default="config2_diffusion3d")

    def __post_init__(self):
        self.fv = FVDiffusion(self.N, 3)
        self.n, self.nnz = self.fv.n, self.fv.nnz
        self.rowptr, self.colind = self.fv.rowptr, self.fv.colind
        h, J = self.fv.h, self.steps
        ax = self.fv.node_axis()
        ax_x = (np.arange(-J, self.N + 2, dtype=np.float64)) * h   # room for the drift
        self._g = FourierField(3, self.corr_len, self.seed_kappa).on_grid(ax_x, ax, ax)

    def matrix_values(self, j: int) -> np.ndarray:
        J, N = self.steps, self.N
        if not 0 <= j <= J:
            raise ValueError("step out of range")
        g = self._g[:, :, J - j: J - j + N + 2]          # g(x - j h e_1)
        return self.fv.values(np.exp(self.sigma * g), shift=1.0 / self.dt)

    def rhs(self, j: int, x_prev: np.ndarray | None) -> np.ndarray:
        b = np.full(self.n, self.source)
        if x_prev is not None:
            b += x_prev / self.dt
        return b

    def describe(self) -> dict:
        return {"workload": self.name, "N": self.N, "n": self.n, "nnz": self.nnz,
                "steps": self.steps, "omega": self.omega, "rank": self.rank,
                "tol": self.tol, "dt": self.dt, "corr_len": self.corr_len,
                "sigma": self.sigma}


@dataclass
class Config3Elasticity:
    N: int = 64
    steps: int = 30
    omega: int = 10
    rank: int = 6
    tol: float = 1e-8
    nu: float = 0.3
    sigma: float = 0.5
    corr_len: float = 0.2
    seed: int = 5
    variant: str = "scale"            # "scale" or "moving"
    name: str = field(default="config3_elasticity")

    def __post_init__(self):
        self.el = Q1Elasticity(self.N, self.nu, self.sigma, self.corr_len, self.seed)
        self.n, self.nnz = self.el.n, self.el.nnz
        self.rowptr, self.colind = self.el.rowptr, self.el.colind
        self._vals = self.el.vals

    def matrix_values(self, j: int) -> np.ndarray:
        return self._vals

    def rhs(self, j: int, x_prev: np.ndarray | None = None) -> np.ndarray:
        f = self.el.rhs(scale=1.0 + 0.05 * np.sin(j))
        if self.variant == "moving":
            N = self.N
            x = np.arange(N) / (N - 1.0)
            c = 0.2 + 0.6 * (j % self.steps) / max(self.steps - 1, 1)
            bump = 1.0 + np.exp(-(x - c) ** 2 / (2 * 0.15 ** 2))
            w = np.broadcast_to(bump[None, None, :], (N, N, N)).reshape(-1)
            f = f * np.repeat(w, 3)
        return f

    def describe(self) -> dict:
        return {"workload": self.name, "N": self.N, "n": self.n, "nnz": self.nnz,
                "steps": self.steps, "omega": self.omega, "rank": self.rank,
                "tol": self.tol, "variant": self.variant}


def config1(**kw) -> Config1Diffusion2D:
    return Config1Diffusion2D(**kw)


def config2(**kw) -> Config2Diffusion3D:
    return Config2Diffusion3D(**kw)


def config3(**kw) -> Config3Elasticity:
    return Config3Elasticity(**kw)


@dataclass
class Config5Adjoint:
    N: int = 96
    steps: int = 200
    omega: int = 20
    rank: int = 10
    tol: float = 1e-10
    dt: float = 1e-3
    corr_len: float = 0.1
    sigma: float = 1.0
    source: float = 1.0
    seed_kappa: int = 4
    seed_outputs: int = 6
    n_outputs: int = 256
    checkpoint_every: int = 20
    name: str = field(default="config5_adjoint")

    def __post_init__(self):
        self.fv = FVDiffusion(self.N, 3)
        self.n, self.nnz = self.fv.n, self.fv.nnz
        self.rowptr, self.colind = self.fv.rowptr, self.fv.colind
        h, J, N = self.fv.h, self.steps, self.N
        ax = self.fv.node_axis()
        ax_x = (np.arange(-J, N + 2, dtype=np.float64)) * h
        g = FourierField(3, self.corr_len, self.seed_kappa).on_grid(ax_x, ax, ax)
        self.theta = self.sigma * g                    # log kappa on the extended grid
        r = np.random.Generator(np.random.PCG64(self.seed_outputs))
        self.outputs = np.sort(r.choice(self.n, size=min(self.n_outputs, self.n), replace=False))

    def window(self, j: int):
        """Slice of theta giving log kappa_j on the (N+2)^3 node grid."""
        J, N = self.steps, self.N
        return (slice(None), slice(None), slice(J - j, J - j + N + 2))

    def matrix_values(self, j: int, theta: np.ndarray | None = None) -> np.ndarray:
        th = self.theta if theta is None else theta
        return self.fv.values(np.exp(th[self.window(j)]), shift=1.0 / self.dt)

    def rhs(self, j: int, x_prev: np.ndarray | None, s: np.ndarray | None = None) -> np.ndarray:
        b = np.full(self.n, self.source) if s is None else np.array(s, dtype=np.float64)
        if x_prev is not None:
            b = b + x_prev / self.dt
        return b

    def describe(self) -> dict:
        return {"workload": self.name, "N": self.N, "n": self.n, "nnz": self.nnz,
                "steps": self.steps, "omega": self.omega, "rank": self.rank, "tol": self.tol,
                "outputs": int(self.outputs.size), "checkpoint_every": self.checkpoint_every}


def config4(**kw) -> Config4Batch:
    return Config4Batch(**kw)


def config5(**kw) -> Config5Adjoint:
    return Config5Adjoint(**kw)
