"""Dense adjoint of an output functional of a diffusion sequence -- test infrastructure only.

For the sequence A_j(theta) x_j = b_j, b_j = s + x_{j-1} / dt (b_1 = s), with
A_j the finite-volume operator of the coefficient kappa_j = exp(window_j(theta))
plus (1/dt) I, and the functional J = sum_j w_j . (C x_j) (outputs q_j = C x_j,
Eq. (outputs) of Section 2), the gradient follows from the adjoint recursion

    lambda_j = A_j^{-1} (C^T w_j + lambda_{j+1} / dt)        (A_j symmetric)
    dJ/ds     = sum_j lambda_j
    dJ/dA_j   = -lambda_j x_j^T

and the derivative of each face coefficient t = 2 k_a k_b / (k_a + k_b) / h^2,
dt/dk_a = 2 k_b^2 / (k_a + k_b)^2 / h^2, written out by hand below.  Every
solve is a dense Cholesky solve (small grids only).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def _dense(cfg, vals):
    return cfg.fv.dense(vals)


def face_adjoint(fv, kappa_ext: np.ndarray, lam: np.ndarray, x: np.ndarray) -> np.ndarray:
    """dJ/dkappa_ext for the term -lambda^T A(kappa) x of one system."""
    N, d = fv.N, fv.dim
    inner = tuple(slice(1, N + 1) for _ in range(d))
    lam_e = np.zeros_like(kappa_ext)
    x_e = np.zeros_like(kappa_ext)
    lam_e[inner] = lam.reshape((N,) * d)
    x_e[inner] = x.reshape((N,) * d)
    kbar = np.zeros_like(kappa_ext)
    kc = kappa_ext[inner]
    inv_h2 = 1.0 / (fv.h * fv.h)
    for axis, sgn, _ in fv._offsets():
        sl = [slice(1, N + 1)] * d
        sl[axis] = slice(1 + sgn, N + 1 + sgn)
        sl = tuple(sl)
        kn = kappa_ext[sl]
        # node a's face toward b adds t to A[a, a] and -t to A[a, b] (b interior)
        g = -(lam_e[inner] * x_e[inner] - lam_e[inner] * x_e[sl])
        den = (kc + kn) ** 2
        kbar[inner] += g * 2.0 * kn * kn / den * inv_h2
        kbar[sl] += g * 2.0 * kc * kc / den * inv_h2
    return kbar


def sequence_gradient(cfg, theta: np.ndarray, s: np.ndarray, weights: np.ndarray, steps: int):
    """(J, dJ/dtheta, dJ/ds, xs) for J = sum_j weights[j-1] . x_j[cfg.outputs]."""
    facs, xs, kappas = [], [], []
    x_prev = None
    J = 0.0
    for j in range(1, steps + 1):
        kappa = np.exp(theta[cfg.window(j)])
        A = _dense(cfg, cfg.fv.values(kappa, shift=1.0 / cfg.dt))
        f = sla.cho_factor(A)
        b = s.copy() if x_prev is None else s + x_prev / cfg.dt
        x = sla.cho_solve(f, b)
        J += float(weights[j - 1] @ x[cfg.outputs])
        facs.append(f)
        xs.append(x)
        kappas.append(kappa)
        x_prev = x
    gtheta = np.zeros_like(theta)
    gs = np.zeros(cfg.n)
    carry = np.zeros(cfg.n)
    for j in range(steps, 0, -1):
        xbar = carry.copy()
        xbar[cfg.outputs] += weights[j - 1]
        lam = sla.cho_solve(facs[j - 1], xbar)
        gs += lam
        carry = lam / cfg.dt
        kbar = face_adjoint(cfg.fv, kappas[j - 1], lam, xs[j - 1])
        gtheta[cfg.window(j)] += kbar * kappas[j - 1]
    return J, gtheta, gs, xs
