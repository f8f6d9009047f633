"""The finite-volume diffusion values of problems.fv written with torch ops,
so that the matrix values are differentiable in the coefficient field.

Same formulas and the same CSR order as FVDiffusion.values: harmonic-mean face
coefficients 2 k_a k_b / (k_a + k_b) / h^2, boundary faces using the
coefficient at the boundary node, plus a diagonal shift.
"""

from __future__ import annotations

import torch

from .fv import FVDiffusion


class FVDiffusionTorch:
    def __init__(self, fv: FVDiffusion, device="cuda"):
        self.fv = fv
        self.device = device
        self.valid = torch.from_numpy(fv._valid).to(device)

    def values(self, kappa_ext: torch.Tensor, shift: float = 0.0) -> torch.Tensor:
        fv = self.fv
        N, d = fv.N, fv.dim
        inner = tuple(slice(1, N + 1) for _ in range(d))
        kc = kappa_ext[inner]
        inv_h2 = 1.0 / (fv.h * fv.h)
        face = []
        for axis, sgn, _ in fv._offsets():
            sl = [slice(1, N + 1)] * d
            sl[axis] = slice(1 + sgn, N + 1 + sgn)
            kn = kappa_ext[tuple(sl)]
            face.append(2.0 * kc * kn / (kc + kn) * inv_h2)
        diag = face[0]
        for f in face[1:]:
            diag = diag + f
        diag = diag + shift
        cols = []
        for o in fv._order:
            cols.append(diag if o is None else -face[o])
        vals = torch.stack(cols, dim=-1).reshape(fv.n, len(fv._order))
        return vals[self.valid]
