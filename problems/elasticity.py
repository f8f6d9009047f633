"""Trilinear (Q1) hexahedral linear elasticity on a uniform grid of the unit cube.

Nodes sit at (i, j, k) h, i, j, k = 0..N-1, h = 1 / (N - 1); each node carries
three displacement unknowns (dof = 3 node + component, nodes numbered x
fastest).  Every element is a cube of side h; its stiffness is E_e times the
stiffness of a unit-modulus element, integrated with 2 x 2 x 2 Gauss points
for an isotropic material with Poisson ratio nu.  Young's modulus is
piecewise constant per element: E_e = exp(sigma g(centre_e)) with g a seeded
unit-variance random field.

The face x = 0 is clamped: its rows and columns become those of the identity
(the stored pattern keeps the zeros, so every interior row has 81 entries).
The load is a body force (0, 0, -1) scaled per system, lumped to the nodes.
"""

from __future__ import annotations

import numpy as np

from .grf import FourierField


def unit_element_stiffness(nu: float, h: float) -> np.ndarray:
    """24 x 24 stiffness of a cube of side h with E = 1 (dofs: 3 per corner,
    corner a = ax + 2 ay + 4 az)."""
    lam = nu / ((1 + nu) * (1 - 2 * nu))
    mu = 1.0 / (2 * (1 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[[0, 1, 2], [0, 1, 2]] += 2 * mu
    D[[3, 4, 5], [3, 4, 5]] = mu
    g = 1.0 / np.sqrt(3.0)
    K = np.zeros((24, 24))
    corners = [(a & 1, (a >> 1) & 1, (a >> 2) & 1) for a in range(8)]
    for xi in (-g, g):
        for eta in (-g, g):
            for zeta in (-g, g):
                dN = np.zeros((8, 3))          # derivatives w.r.t. physical x, y, z
                for a, (ax, ay, az) in enumerate(corners):
                    sx, sy, sz = 2 * ax - 1, 2 * ay - 1, 2 * az - 1
                    dN[a, 0] = sx * (1 + sy * eta) * (1 + sz * zeta) / 8 * (2 / h)
                    dN[a, 1] = sy * (1 + sx * xi) * (1 + sz * zeta) / 8 * (2 / h)
                    dN[a, 2] = sz * (1 + sx * xi) * (1 + sy * eta) / 8 * (2 / h)
                B = np.zeros((6, 24))
                for a in range(8):
                    dx, dy, dz = dN[a]
                    c = 3 * a
                    B[0, c], B[1, c + 1], B[2, c + 2] = dx, dy, dz
                    B[3, c], B[3, c + 1] = dy, dx
                    B[4, c + 1], B[4, c + 2] = dz, dy
                    B[5, c], B[5, c + 2] = dz, dx
                K += B.T @ D @ B * (h / 2) ** 3
    return 0.5 * (K + K.T)


class Q1Elasticity:
    """Pattern, values and loads of the clamped Q1 elasticity operator."""

    def __init__(self, N: int, nu: float = 0.3, sigma: float = 0.5, corr_len: float = 0.2,
                 seed: int = 5):
        self.N = int(N)
        self.h = 1.0 / (self.N - 1)
        self.nu = nu
        self.nnodes = self.N ** 3
        self.n = 3 * self.nnodes
        Ne = self.N - 1
        ctr = (np.arange(Ne) + 0.5) * self.h
        g = FourierField(3, corr_len, seed).on_grid(ctr, ctr, ctr)      # (z, y, x)
        self.E = np.exp(sigma * g)
        self.Kref = unit_element_stiffness(nu, self.h)
        self._offsets = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
        self._build()

    def _build(self):
        N, Ne = self.N, self.N - 1
        blocks = np.zeros((N, N, N, 27, 3, 3))                # (z, y, x, offset, c1, c2)
        corners = [(a & 1, (a >> 1) & 1, (a >> 2) & 1) for a in range(8)]
        oidx = {o: t for t, o in enumerate(self._offsets)}
        for a, (ax, ay, az) in enumerate(corners):
            for b, (bx, by, bz) in enumerate(corners):
                t = oidx[(bx - ax, by - ay, bz - az)]
                kab = self.Kref[3 * a:3 * a + 3, 3 * b:3 * b + 3]
                blocks[az:az + Ne, ay:ay + Ne, ax:ax + Ne, t] += self.E[..., None, None] * kab
        # clamp x = 0: identity rows and columns
        clamped = np.zeros((N, N, N), dtype=bool)
        clamped[:, :, 0] = True
        kz, ky, kx = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
        valid = np.zeros((N, N, N, 27), dtype=bool)
        nbr_clamped = np.zeros((N, N, N, 27), dtype=bool)
        for t, (dx, dy, dz) in enumerate(self._offsets):
            x2, y2, z2 = kx + dx, ky + dy, kz + dz
            ok = (x2 >= 0) & (x2 < N) & (y2 >= 0) & (y2 < N) & (z2 >= 0) & (z2 < N)
            valid[..., t] = ok
            nbr_clamped[..., t] = ok & (x2 == 0)
        kill = clamped[..., None] | nbr_clamped               # (z, y, x, offset)
        blocks[kill] = 0.0
        centre = self._offsets.index((0, 0, 0))
        cz = clamped
        blocks[cz, centre] = np.eye(3)
        self.clamped = np.repeat(clamped.reshape(-1), 3)
        # CSR: row (node, c1), entries over offsets (ascending node delta) then c2
        node = np.arange(self.nnodes).reshape(N, N, N)
        cols = np.empty((N, N, N, 27, 3), dtype=np.int64)
        for t, (dx, dy, dz) in enumerate(self._offsets):
            cols[..., t, :] = 3 * (node + dx + N * dy + N * N * dz)[..., None] + np.arange(3)
        per_node = valid.sum(axis=-1) * 3                      # entries per row of this node
        self.rowptr = np.zeros(self.n + 1, dtype=np.int64)
        np.cumsum(np.repeat(per_node.reshape(-1), 3), out=self.rowptr[1:])
        # gather (node, c1, offset, c2) in row order
        v = np.transpose(blocks, (0, 1, 2, 4, 3, 5))          # (z, y, x, c1, offset, c2)
        m = np.broadcast_to(valid[:, :, :, None, :, None], v.shape)
        cc = np.broadcast_to(cols[:, :, :, None, :, :], v.shape)
        self.vals = v[m]
        self.colind = cc[m].astype(np.int32)
        self.nnz = int(self.rowptr[-1])
        assert self.vals.size == self.nnz
        self.rowptr = self.rowptr.astype(np.int32)
        # lumped body-force weights: h^3 / 8 per adjacent element
        cnt = np.zeros((N, N, N))
        for (ax, ay, az) in corners:
            cnt[az:az + Ne, ay:ay + Ne, ax:ax + Ne] += 1.0
        self._load_z = -(cnt * self.h ** 3 / 8.0).reshape(-1)

    def rhs(self, scale: float = 1.0, direction=(0.0, 0.0, -1.0)) -> np.ndarray:
        f = np.zeros((self.nnodes, 3))
        w = -self._load_z                                     # positive nodal weights
        for c in range(3):
            f[:, c] = direction[c] * w * scale
        f = f.reshape(-1)
        f[self.clamped] = 0.0
        return f

    def dense(self) -> np.ndarray:
        A = np.zeros((self.n, self.n))
        for i in range(self.n):
            s, e = self.rowptr[i], self.rowptr[i + 1]
            A[i, self.colind[s:e]] += self.vals[s:e]
        return A
