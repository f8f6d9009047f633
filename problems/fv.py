"""Cell-centred finite-volume diffusion matrices on the unit square / cube.

Unknowns sit at the interior nodes x = (i + 1) h, i = 0..N-1, h = 1 / (N + 1),
of (0, 1)^d with homogeneous Dirichlet data on the boundary.  The flux
through the face between nodes a and b uses the harmonic mean
2 k_a k_b / (k_a + k_b) of the coefficient, scaled by 1 / h^2.  Faces that
touch the boundary use the coefficient at the boundary node.  An optional
diagonal shift c I (a 1/dt mass term) is added.

Rows are numbered x-fastest: row = i + N j (+ N^2 k).  Columns within a row
are ascending.  The result is symmetric and strictly diagonally dominant on
boundary rows, hence SPD.
"""

from __future__ import annotations

import numpy as np


class FVDiffusion:
    """Pattern and values of the 5-point (2-D) or 7-point (3-D) FV operator."""

    def __init__(self, N: int, dim: int):
        if dim not in (2, 3):
            raise ValueError("dim must be 2 or 3")
        self.N = int(N)
        self.dim = int(dim)
        self.n = self.N ** self.dim
        self.h = 1.0 / (self.N + 1)
        self._build_pattern()

    # axes ordered (z, y, x) in array space; offsets in row numbering
    def _offsets(self):
        N = self.N
        if self.dim == 2:
            return [(0, -1, -N), (1, -1, -1), (1, +1, +1), (0, +1, +N)]
        return [(0, -1, -N * N), (1, -1, -N), (2, -1, -1),
                (2, +1, +1), (1, +1, +N), (0, +1, +N * N)]

    def _build_pattern(self):
        N, d = self.N, self.dim
        shape = (N,) * d
        idx = np.arange(self.n, dtype=np.int64).reshape(shape)
        offs = self._offsets()
        half = len(offs) // 2
        slots = len(offs) + 1                          # neighbours + diagonal
        cols = np.empty(shape + (slots,), dtype=np.int64)
        valid = np.zeros(shape + (slots,), dtype=bool)
        order = list(range(half)) + [None] + list(range(half, len(offs)))
        for s, o in enumerate(order):
            if o is None:
                cols[..., s] = idx
                valid[..., s] = True
                continue
            axis, sgn, delta = offs[o]
            cols[..., s] = idx + delta
            pos = np.indices(shape)[axis]
            valid[..., s] = (pos + sgn >= 0) & (pos + sgn < N)
        self._valid = valid.reshape(self.n, slots)
        self._order = order
        cnt = self._valid.sum(axis=1)
        self.rowptr = np.zeros(self.n + 1, dtype=np.int32)
        np.cumsum(cnt, out=self.rowptr[1:])
        self.colind = cols.reshape(self.n, slots)[self._valid].astype(np.int32)
        self.nnz = int(self.rowptr[-1])

    def values(self, kappa_ext: np.ndarray, shift: float = 0.0) -> np.ndarray:
        """CSR values for a coefficient given on the extended (N+2)^d node grid.

        ``kappa_ext`` has shape (N+2,)*d in (z, y, x) order and includes the
        boundary nodes; entry [1:-1, ...] is the coefficient at the unknowns.
        """
        N, d = self.N, self.dim
        k = np.asarray(kappa_ext, dtype=np.float64)
        if k.shape != (N + 2,) * d:
            raise ValueError(f"kappa_ext must have shape {(N + 2,) * d}")
        inner = tuple(slice(1, N + 1) for _ in range(d))
        kc = k[inner]
        offs = self._offsets()
        inv_h2 = 1.0 / (self.h * self.h)
        face = []
        for axis, sgn, _ in offs:
            sl = [slice(1, N + 1)] * d
            sl[axis] = slice(1 + sgn, N + 1 + sgn)
            kn = k[tuple(sl)]
            face.append(2.0 * kc * kn / (kc + kn) * inv_h2)
        diag = np.zeros_like(kc)
        for f in face:
            diag += f
        diag += shift
        slots = len(offs) + 1
        vals = np.empty(kc.shape + (slots,), dtype=np.float64)
        for s, o in enumerate(self._order):
            vals[..., s] = diag if o is None else -face[o]
        return vals.reshape(self.n, slots)[self._valid]

    def node_axis(self) -> np.ndarray:
        """Coordinates of the extended node line 0, h, ..., 1 (N + 2 points)."""
        return np.arange(self.N + 2, dtype=np.float64) * self.h

    def interior_points(self) -> np.ndarray:
        """(n, d) coordinates of the unknowns, x fastest."""
        ax = (np.arange(self.N, dtype=np.float64) + 1.0) * self.h
        grids = np.meshgrid(*([ax] * self.dim), indexing="ij")   # (z.., y, x) order
        pts = np.stack([g.ravel() for g in reversed(grids)], axis=1)
        return pts

    def dense(self, vals: np.ndarray) -> np.ndarray:
        A = np.zeros((self.n, self.n))
        for i in range(self.n):
            s, e = self.rowptr[i], self.rowptr[i + 1]
            A[i, self.colind[s:e]] = vals[s:e]
        return A
