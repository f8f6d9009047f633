"""Three-stage POD-augmented CG (Alg. 3, Section 4) -- TEST INFRASTRUCTURE ONLY.

Plain NumPy, FP64, small problems.  One call of `ts_solve` is one pass of the
loop of Alg. 3 for system j, with the non-iterative Stage 3 (phi = 0,
Section 4.3) or, with phi = 1, the iterative Stage 3 of Section 4.3.1:

  Stage 1 (Alg. 2)     direct Galerkin solve over the stage-1 basis W_j;
  Stage 2 (Sect. 4.2)  augmented CG (Alg. 1, M = I) on the reduced system
                       Y^T A Y xhat = Y^T (b - A xbar) from xhat0 = What what,
                       augmented by What (W_j = Y_j What, a column selection),
                       to the stage-2 tolerance; full-space directions
                       X = Y Xhat with X^T A X = Gammahat;
  Stage 3 (Sect. 4.3)  augmented PCG (Alg. 1, Jacobi M) on A from
                       x0 = Y xhat with the basis [W, X] and the reused
                       factor blockdiag(R, sqrt(Gammahat)), recording its
                       directions V and Gamma = diag(p^T A p);
  Stage 3, phi = 1      augmented PCG on A from the same x0 with all of Y as
                       the augmenting basis; each projection
                       Y^T A Y mu = Y^T A z is solved iteratively (augmented
                       CG on the reduced matrix, M = I) against the reduced
                       stage-1 columns, the stage-2 directions and the
                       directions of the earlier projection solves, with the
                       block-diagonal factor they share;
  then the accumulated vectors Z_j = [Y_j, V_j Gamma_j^{-1/2}] either become
  Y_{j+1} (W_{j+1} gains the new vectors the rho rule selects) or, when they
  exceed ybar, are truncated by POD (Eq. (podAlgebraicDefinition), metric
  A_j, weights eta^prev or eta^RBF of Section 3.3.2, energy criteria of
  Sections 3.3.4 and 4.5) and W_{j+1} is the leading POD vectors.

Readings where the paper is garbled or silent (stated again in the design
notes): the new Krylov vectors enter Y and W scaled by Gamma^{-1/2} (A_j-
orthonormal; the printed sqrt(Gamma) would not give the well-conditioned
reduced matrix of Theorem wellConditioned); rho = 0 selects no new vector,
rho = 1 all of them, 0 < rho < 1 those with gamma_k / sum gamma > rho;
eta^prev(j) is the coefficient vector of the computed x_j - xbar_j in Z_j;
eta^RBF = sum_i 2^{1-i} eta^prev(j+1-i) over the systems since the last
truncation; both stages stop on ||r|| before their first iteration too; the
stage-2 tolerance is stage2_factor * rtol * ||b||, but not below 1e-6 of the
initial reduced residual ||Y^T r|| (the loose end of the paper's range);
Stage 3 uses the reused block-diagonal factor or, as an option, the computed
and factored Gram of [W, X]; Stage 2 runs at most
min(stage2_maxit, basis_max - w) iterations and at most `cap - m` Stage-3
directions are recorded.  With phi = 1, Stage 2 runs to its tolerance with
only a rounding-level floor (1e-13 of its initial residual) and up to
min(stage2_maxit, m - w) steps: Alg. 1 over all of Y never corrects the part
of the error that lies in range(Y), so that part has to be solved to below
the overall tolerance first.  The iterative Stage 3 starts each projection solve
from the Galerkin solution over the augmenting directions it already has (the
direct block-diagonal solve): Alg. 1 started from zero, as printed, never
resolves the part of mu in their span, and the outer directions would then not
be A-orthogonal to them, which the paper states they are.  The projection
solves stop at inner_rtol times the norm of their right-hand side (the paper
gives no value) and after inner_maxit steps; by default that tolerance is
1e-2 of the solve's own relative tolerance (never below the rounding-level
floor): the error an inexact projection leaves in range(Y) is never corrected
by the later directions, which are A-orthogonal to Y.  Measured: with 1e-8
against an overall 1e-10 the iteration diverged after reaching 2e-9 (2-D,
24^2); on the 128^3 sequence it diverged with 1e-10 and 1e-8 and converged
with 1e-12.  Directions formed after a solve's residual (Stage 2
or a projection solve) has fallen below 1e-6 of its initial value still
advance that solve but do not join the augmentation (for a projection solve
the measure is the norm of its right-hand side, which its Galerkin start may
already have cancelled to a small residual): they are orthogonal to the
earlier ones only to about the rounding error divided by that reduction, and
the reused block-diagonal factor needs them orthogonal (a late stage-2
direction made the projection solves diverge, and at 128^3 kept directions
formed from small post-start residuals made the iteration diverge).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import CSR, matvec

BASIS_MAX = 32          # columns of the Stage-1 / Stage-3 augmenting bases
STAGE2_FLOOR = 1e-6     # stage-2 tolerance floor, relative to the initial reduced residual
ROUNDING_FLOOR = 1e-13  # phi = 1: floor of Stage 2 and of the projection solves, relative to
                        # their initial residual
INNER_MARGIN = 1e-2     # phi = 1: default projection-solve tolerance relative to the overall one
KEEP_FLOOR = 1e-6       # phi = 1: a direction joins the reduced augmentation only if it was
                        # formed from a residual at least this fraction of its solve's
                        # right-hand side (Stage 2: its initial residual)


@dataclass
class TSOptions:
    ybar: int = 60             # truncate when the accumulated vectors exceed ybar
    y_trunc: int = 20          # POD dimension after a truncation
    w_max: int = 5             # stage-1 basis dimension after a truncation
    energy_y: float = 1.0      # energy criterion of the truncated basis (1: off)
    energy_w: float = 1.0      # energy criterion of the stage-1 basis (1: off)
    rho: float = 0.0           # new-vector rule of Alg. 3
    w_cap: int = 16            # largest stage-1 basis outside truncations
    stage2_factor: float = 1e-4
    stage2_maxit: int = 24
    weights: str = "rbf"       # "rbf" (IDW 2^{1-i}) or "previous"
    stage3_gram: str = "blockdiag"   # factor of [W, X]^T A [W, X]: reused blockdiag(R, sqrt(Gammahat))
                                     # (Section 4.3) or "exact" (computed and factored)
    rank_rtol: float = 1e-12
    cap: int = 512             # columns of the accumulated-vector store
    phi: int = 0               # Stage 3 over [W, X] (0, Section 4.3) or over all of Y (1, Section 4.3.1)
    inner_rtol: float = 0.0    # phi = 1: tolerance of each projection solve, relative to its right-hand
                               # side; <= 0: INNER_MARGIN times the solve's own relative tolerance
    inner_maxit: int = 256     # phi = 1: step cap of each projection solve


@dataclass
class TSState:
    n: int
    Y: np.ndarray = None                   # (n, m) augmenting basis Y_j
    sel: list = field(default_factory=list)  # columns of Y forming W_j
    eta_acc: np.ndarray = None             # running eta^RBF since the last truncation
    jc: int = 0                            # latest truncation index
    j: int = 0                             # systems solved

    def __post_init__(self):
        if self.Y is None:
            self.Y = np.zeros((self.n, 0))
        if self.eta_acc is None:
            self.eta_acc = np.zeros(0)

    @property
    def m(self) -> int:
        return self.Y.shape[1]


def _mv(A: CSR, X: np.ndarray) -> np.ndarray:
    if X.ndim == 1:
        return matvec(A, X)
    return np.stack([matvec(A, X[:, k]) for k in range(X.shape[1])], axis=1)


def _chol_truncated(G: np.ndarray):
    """Upper Cholesky factor of the symmetrised G; a pivot <= 1e-14 max diag
    drops that column and the ones after it.  Returns (R (kept x kept), kept)."""
    G = 0.5 * (G + G.T)
    y = G.shape[0]
    if y == 0:
        return np.zeros((0, 0)), 0
    dmax = max(np.max(np.diag(G)), 0.0)
    R = np.zeros((y, y))
    for i in range(y):
        s = G[i, i] - R[:i, i] @ R[:i, i]
        if not s > 1e-14 * dmax:
            return R[:i, :i].copy(), i
        R[i, i] = np.sqrt(s)
        for k in range(i + 1, y):
            R[i, k] = (G[i, k] - R[:i, i] @ R[:i, k]) / R[i, i]
    return R, y


def _chol_solve(R: np.ndarray, v: np.ndarray) -> np.ndarray:
    """G^{-1} v with G = R^T R."""
    t = np.linalg.solve(R.T, v)
    return np.linalg.solve(R, t)


def pod_evd_dense(A: CSR, Z: np.ndarray, eta: np.ndarray, y_max: int, rank_rtol: float,
                  energy: float):
    """POD of the columns of Z with weights eta in the A metric (Alg. pod_evd):
    Gbar = diag(eta) Z^T A Z diag(eta) = V Sigma^2 V^T (decreasing), y by the
    rank cut, the cap and the energy criterion, basis Z diag(eta) V_y Sigma_y^{-1}.
    Returns (basis (n, y), eigenvalues)."""
    AZ = _mv(A, Z)
    Gb = (eta[:, None] * (Z.T @ AZ)) * eta[None, :]
    Gb = 0.5 * (Gb + Gb.T)
    lam, V = np.linalg.eigh(Gb)
    order = np.argsort(lam)[::-1]
    lam, V = lam[order], V[:, order]
    for i in range(V.shape[1]):              # largest-magnitude component positive
        k = np.argmax(np.abs(V[:, i]))
        if V[k, i] < 0:
            V[:, i] = -V[:, i]
    y = int(np.sum(lam > rank_rtol * lam[0])) if lam.size and lam[0] > 0 else 0
    y = min(y, y_max)
    y = _energy_count(lam, y, energy)
    T = (eta[:, None] * V[:, :y]) / np.sqrt(lam[:y])[None, :]
    return Z @ T, lam


def _energy_count(lam: np.ndarray, y: int, energy: float) -> int:
    if 0.0 < energy < 1.0 and y > 0:
        tot = float(np.sum(lam[lam > 0]))
        acc = 0.0
        for i in range(y):
            acc += lam[i]
            if acc >= energy * tot:
                return i + 1
    return y


@dataclass
class TSStats:
    j: int = 0
    w: int = 0              # stage-1 dimension used
    m: int = 0              # dim Y_j
    k2: int = 0             # stage-2 iterations
    k3: int = 0             # stage-3 iterations (preconditioner applications)
    matvecs: int = 0
    stage1_relres: float = 0.0
    stage2_relres: float = 0.0
    relres: float = 0.0
    true_relres: float = 0.0
    truncated: bool = False
    m_next: int = 0         # dim Y_{j+1}
    w_next: int = 0         # dim W_{j+1}
    cond_YAY: float = 1.0   # condition number of Y_j^T A_j Y_j (E6 diagnostic)
    status: int = 0
    k_in: int = 0           # phi = 1: steps of all projection solves


def stage2(A: CSR, Y: np.ndarray, sel: list, AW: np.ndarray, R: np.ndarray, what: np.ndarray,
           rbar: np.ndarray, tol: float, maxit: int, red: dict | None = None,
           floor_rel: float = None):
    """Augmented CG on Y^T A Y xhat = Y^T rbar, M = I, from xhat0 = What what,
    augmented by What (Section 4.2).  Returns (xhat, X, AX, gammahat, k, ||rhat||);
    `red`, if given, receives the reduced directions ("P", m x k), Ghat times
    them ("G") and their (Ghat p, p) ("gam"), of the steps whose direction was
    formed from a residual of at least KEEP_FLOOR of the initial one."""
    n, m = Y.shape
    w = len(sel)
    xh = np.zeros(m)
    if w:
        xh[sel] = what
    rh = Y.T @ (rbar - _mv(A, Y @ xh))                 # rhat0 = bhat - Ghat xhat0
    zh = rh.copy()

    def proj(zv):                                      # What G_W^{-1} What^T Ghat z
        if w == 0:
            return np.zeros(0)
        return _chol_solve(R, AW.T @ (Y @ zv))

    mu = proj(zh)
    ph = zh.copy()
    if w:
        ph[sel] -= mu
    rz = rh @ zh
    X, AX, gam = [], [], []
    k = 0
    rn0 = float(np.linalg.norm(rh))
    # never below 1e-6 of the initial reduced residual: directions formed from
    # a much smaller residual are A-orthogonal to the earlier ones only to a
    # relative accuracy that breaks the block-diagonal factor reused in Stage 3
    floor_rel = STAGE2_FLOOR if floor_rel is None else floor_rel
    tol = max(tol, floor_rel * float(np.linalg.norm(rh)))
    while np.linalg.norm(rh) > tol and k < maxit:
        rn_formed = float(np.linalg.norm(rh))      # the residual ph was formed from
        u = Y @ ph
        q = matvec(A, u)
        gh = Y.T @ q                                   # Ghat p
        g = ph @ gh
        if not g > 0:
            break
        alpha = rz / g
        xh += alpha * ph
        rh -= alpha * gh
        zh = rh.copy()
        rz_new = rh @ zh
        beta = rz_new / rz
        rz = rz_new
        X.append(u)
        AX.append(q)
        gam.append(g)
        if red is not None and rn_formed >= KEEP_FLOOR * rn0:
            red.setdefault("P", []).append(ph.copy())
            red.setdefault("G", []).append(gh)
            red.setdefault("gam", []).append(g)
        k += 1
        mu = proj(zh)
        ph = zh + beta * ph
        if w:
            ph[sel] -= mu
    X = np.stack(X, axis=1) if X else np.zeros((n, 0))
    AX = np.stack(AX, axis=1) if AX else np.zeros((n, 0))
    if red is not None:
        for key in ("P", "G"):
            red[key] = np.stack(red[key], axis=1) if red.get(key) else np.zeros((m, 0))
        red["gam"] = np.array(red.get("gam", []))
    return xh, X, AX, np.array(gam), k, float(np.linalg.norm(rh))


def stage3(A: CSR, b: np.ndarray, x0: np.ndarray, B: np.ndarray, AB: np.ndarray,
           Ginv: np.ndarray, dinv: np.ndarray, tol: float, maxit: int, rec_max: int):
    """Augmented PCG (Alg. 1) from x0 (no re-projection), basis B with A B and
    the inverse of the reused block-diagonal factor; records up to rec_max
    directions.  Returns (x, V, gamma, alpha, k, ||r||)."""
    y = B.shape[1]
    x = x0.copy()
    r = b - matvec(A, x)
    z = dinv * r
    mu = Ginv @ (AB.T @ z) if y else np.zeros(0)
    p = z - B @ mu if y else z.copy()
    rz = r @ z
    V, gam, alp = [], [], []
    k = 0
    while np.linalg.norm(r) > tol and k < maxit:
        q = matvec(A, p)
        g = p @ q
        if not g > 0:
            raise RuntimeError("stage 3: (A p, p) <= 0")
        alpha = rz / g
        x += alpha * p
        r -= alpha * q
        z = dinv * r
        rz_new = r @ z
        beta = rz_new / rz
        rz = rz_new
        if k < rec_max:
            V.append(p.copy())
            gam.append(g)
            alp.append(alpha)
        k += 1
        mu = Ginv @ (AB.T @ z) if y else np.zeros(0)
        p = z + beta * p - (B @ mu if y else 0.0)
    V = np.stack(V, axis=1) if V else np.zeros((len(b), 0))
    return x, V, np.array(gam), np.array(alp), k, float(np.linalg.norm(r))


class ReducedAugmentation:
    """The augmenting directions of the projection solves of the iterative
    Stage 3, in Y coordinates (Section 4.3.1): the stage-1 columns What
    (W = Y What, a column selection; W^T A W = R^T R), the stage-2 directions
    and the directions of the earlier projection solves.  They are mutually
    Ghat-orthogonal (Ghat = Y^T A Y), so (B^T Ghat B)^{-1} is
    blockdiag(G_W^{-1}, diag(1 / gamma)); Ghat What = Y^T (A W) and Ghat p of
    every other direction are kept, so no product with Ghat is needed to use
    them."""

    def __init__(self, Y: np.ndarray, sel: list, AW: np.ndarray, R: np.ndarray, P2: np.ndarray,
                 G2: np.ndarray, gam2: np.ndarray):
        self.m = Y.shape[1]
        self.sel = list(sel)
        self.R = R
        self.GW = Y.T @ AW if sel else np.zeros((self.m, 0))
        self.P = [P2[:, k] for k in range(P2.shape[1])]
        self.G = [G2[:, k] for k in range(G2.shape[1])]
        self.gam = [float(g) for g in gam2]

    def solve_coeffs(self, cw: np.ndarray, cd: np.ndarray):
        """blockdiag(G_W^{-1}, diag(1 / gamma)) applied to (cw, cd)."""
        nw = _chol_solve(self.R, cw) if self.sel else np.zeros(0)
        return nw, cd / np.array(self.gam) if self.gam else np.zeros(0)

    def combine(self, nw: np.ndarray, nd: np.ndarray) -> np.ndarray:
        """B nu in Y coordinates."""
        v = np.zeros(self.m)
        if self.sel:
            v[self.sel] += nw
        for p, c in zip(self.P, nd):
            v += c * p
        return v

    def combine_G(self, nw: np.ndarray, nd: np.ndarray) -> np.ndarray:
        """Ghat B nu."""
        v = self.GW @ nw if self.sel else np.zeros(self.m)
        for g, c in zip(self.G, nd):
            v = v + c * g
        return v

    def galerkin(self, c: np.ndarray):
        """Coefficients of the Galerkin solution of Ghat mu = c over range(B):
        (B^T Ghat B)^{-1} B^T c."""
        cw = c[self.sel] if self.sel else np.zeros(0)
        cd = np.array([p @ c for p in self.P])
        return self.solve_coeffs(cw, cd)

    def project(self, z: np.ndarray):
        """Coefficients of steps aug2 / aug3 of Alg. 1 on Ghat: (B^T Ghat B)^{-1} B^T Ghat z."""
        cw = self.GW.T @ z if self.sel else np.zeros(0)
        cd = np.array([g @ z for g in self.G])
        return self.solve_coeffs(cw, cd)


def projection_solve(c: np.ndarray, aug: ReducedAugmentation, ghat_mv, tol: float, maxit: int):
    """Ghat mu = c by augmented CG (Alg. 1, M = I) against the directions of
    `aug`, from the Galerkin solution over their span.  Its own directions
    join `aug` afterwards, those formed from a residual of at least KEEP_FLOOR
    of ||c|| (the residual is computed with cancellation against c, so later
    directions are orthogonal to the earlier ones only to about the rounding
    error of c divided by that reduction, and the block-diagonal factor needs
    them orthogonal).  Returns (mu, steps)."""
    nw, nd = aug.galerkin(c)
    mu = aug.combine(nw, nd)
    r = c - aug.combine_G(nw, nd)
    z = r.copy()
    nw, nd = aug.project(z)
    p = z - aug.combine(nw, nd)
    rz = r @ z
    newP, newG, newgam = [], [], []
    k = 0
    cn = float(np.linalg.norm(c))
    while np.linalg.norm(r) > tol and k < maxit:
        keep = float(np.linalg.norm(r)) >= KEEP_FLOOR * cn      # p was formed from this residual
        g = ghat_mv(p)
        gam = p @ g
        if not gam > 0:
            break
        alpha = rz / gam
        mu += alpha * p
        r -= alpha * g
        z = r.copy()
        rz_new = r @ z
        beta = rz_new / rz
        rz = rz_new
        if keep:
            newP.append(p.copy())
            newG.append(g)
            newgam.append(gam)
        k += 1
        nw, nd = aug.project(z)
        p = z + beta * p - aug.combine(nw, nd)
    room = max(0, aug.m - len(aug.P))     # at most m mutually Ghat-orthogonal directions
    aug.P += newP[:room]
    aug.G += newG[:room]
    aug.gam += newgam[:room]
    return mu, k


def stage3_iterative(A: CSR, b: np.ndarray, x0: np.ndarray, Y: np.ndarray, aug: ReducedAugmentation,
                     dinv: np.ndarray, tol: float, maxit: int, rec_max: int, inner_rel: float,
                     inner_maxit: int):
    """Augmented PCG (Alg. 1) from x0 with all of Y as the augmenting basis,
    each solve Y^T A Y mu = Y^T A z of steps aug2 / aug3 done by
    projection_solve (Section 4.3.1).  Records up to rec_max directions.
    Returns (x, V, gamma, alpha, k, ||r||, projection-solve steps, matvecs)."""
    x = x0.copy()
    r = b - matvec(A, x)
    z = dinv * r
    rz = r @ z
    V, gam, alp = [], [], []
    k = kin = 0
    mv = 1

    def ghat_mv(v):
        return Y.T @ matvec(A, Y @ v)

    def mu_of(zv):
        nonlocal kin, mv
        c = Y.T @ matvec(A, zv)
        rel = max(inner_rel, ROUNDING_FLOOR)
        mu, ks = projection_solve(c, aug, ghat_mv, rel * float(np.linalg.norm(c)), inner_maxit)
        kin += ks
        mv += 1 + ks
        return mu

    if np.linalg.norm(r) > tol and maxit > 0:
        p = z - Y @ mu_of(z)
    while np.linalg.norm(r) > tol and k < maxit:
        q = matvec(A, p)
        mv += 1
        g = p @ q
        if not g > 0:
            raise RuntimeError("stage 3: (A p, p) <= 0")
        alpha = rz / g
        x += alpha * p
        r -= alpha * q
        z = dinv * r
        rz_new = r @ z
        beta = rz_new / rz
        rz = rz_new
        if k < rec_max:
            V.append(p.copy())
            gam.append(g)
            alp.append(alpha)
        k += 1
        if np.linalg.norm(r) <= tol or k >= maxit:
            break
        p = z + beta * p - Y @ mu_of(z)
    V = np.stack(V, axis=1) if V else np.zeros((len(b), 0))
    return x, V, np.array(gam), np.array(alp), k, float(np.linalg.norm(r)), kin, mv


def ts_solve(A: CSR, b: np.ndarray, xbar: np.ndarray, st: TSState, rtol: float, maxit: int,
             opt: TSOptions, keep: dict | None = None):
    """One system of Alg. 3 (phi = 0).  Updates st to Y_{j+1}, W_{j+1}.
    Returns (x, TSStats); `keep`, if given, receives intermediate quantities."""
    n = len(b)
    st.j += 1
    S = TSStats(j=st.j, m=st.m)
    diag = np.zeros(n)
    for i in range(n):
        row = slice(A.rowptr[i], A.rowptr[i + 1])
        cols = A.colind[row]
        diag[i] = A.vals[row][cols == i].sum()
    dinv = 1.0 / diag
    bn = float(np.linalg.norm(b))
    tol = rtol * bn
    rbar = b - matvec(A, xbar)
    Y = st.Y
    m = st.m
    if m:
        G = Y.T @ _mv(A, Y)
        ev = np.linalg.eigvalsh(0.5 * (G + G.T))
        S.cond_YAY = float(ev[-1] / ev[0]) if ev[0] > 0 else np.inf
    # Stage 1 (Alg. 2) over W = Y[:, sel]
    sel = list(st.sel)
    if sel:
        W = Y[:, sel]
        AW = _mv(A, W)
        R, kept = _chol_truncated(W.T @ AW)
        sel = sel[:kept]
        W, AW = W[:, :kept], AW[:, :kept]
        what = _chol_solve(R, W.T @ rbar) if kept else np.zeros(0)
    else:
        W, AW, R, what = np.zeros((n, 0)), np.zeros((n, 0)), np.zeros((0, 0)), np.zeros(0)
    w = len(sel)
    S.w = w
    x1 = W @ what if w else np.zeros(n)
    S.stage1_relres = float(np.linalg.norm(rbar - (AW @ what if w else 0.0)) / bn) if bn else 0.0
    # Stage 2 over Y
    # phi = 0: [W, X] is Stage 3's augmenting basis, at most BASIS_MAX columns;
    # phi = 1: the stage-2 directions only join the reduced augmentation, and
    # Stage 2 runs to its tolerance with no floor (Alg. 1 over all of Y never
    # corrects the part of the error in range(Y) that Stage 2 leaves)
    it = opt.phi == 1
    k2_max = min(opt.stage2_maxit, m - w) if it else min(opt.stage2_maxit, BASIS_MAX - w)
    red = {}
    if m:
        xh, X, AX, gh, k2, rhn = stage2(A, Y, sel, AW, R, what, rbar,
                                         opt.stage2_factor * tol, k2_max, red,
                                         floor_rel=ROUNDING_FLOOR if it else STAGE2_FLOOR)
    else:
        xh, X, AX, gh, k2, rhn = np.zeros(0), np.zeros((n, 0)), np.zeros((n, 0)), np.zeros(0), 0, 0.0
    S.k2 = k2
    S.stage2_relres = rhn / bn if bn else 0.0
    x0 = Y @ xh if m else x1
    # Stage 3 with [W, X] and blockdiag(R, sqrt(Gammahat))
    B = np.concatenate([W, X], axis=1)
    AB = np.concatenate([AW, AX], axis=1)
    if opt.stage3_gram == "exact" and B.shape[1]:
        RB, kb = _chol_truncated(B.T @ AB)
        B, AB = B[:, :kb], AB[:, :kb]
        Ginv = _chol_solve(RB, np.eye(kb)) if kb else np.zeros((0, 0))
    else:
        y = B.shape[1]
        Ginv = np.zeros((y, y))
        if w:
            Ginv[:w, :w] = _chol_solve(R, np.eye(w))
        for k in range(k2):
            Ginv[w + k, w + k] = 1.0 / gh[k]
    rec_max = max(0, opt.cap - m)
    aug = None
    if opt.phi == 1 and m:
        aug = ReducedAugmentation(Y, sel, AW, R, red["P"], red["G"], red["gam"])
        inner_rel = opt.inner_rtol if opt.inner_rtol > 0 else INNER_MARGIN * rtol
        dx, V, gam, alp, k3, rn, kin, mv3 = stage3_iterative(A, rbar, x0, Y, aug, dinv, tol, maxit, rec_max,
                                                             inner_rel, opt.inner_maxit)
        S.k_in = kin
        S.matvecs = 1 + w + k2 + mv3 + 1
    else:
        dx, V, gam, alp, k3, rn = stage3(A, rbar, x0, B, AB, Ginv, dinv, tol, maxit, rec_max)
        S.matvecs = 1 + w + k2 + 1 + k3 + 1
    x = xbar + dx
    S.k3 = k3
    S.relres = rn / bn if bn else rn
    S.true_relres = float(np.linalg.norm(b - matvec(A, x)) / bn) if bn else 0.0
    S.status = 0 if rn <= tol else 1
    # accumulation: Z_j = [Y_j, V Gamma^{-1/2}], eta^prev = [xhat; alpha sqrt(gamma)]
    kr = V.shape[1]
    Znew = V / np.sqrt(gam)[None, :] if kr else np.zeros((n, 0))
    Z = np.concatenate([Y, Znew], axis=1)
    eta_prev = np.concatenate([xh if m else np.zeros(0), alp * np.sqrt(gam)])
    eta_acc = np.concatenate([st.eta_acc, np.zeros(kr)])
    eta_acc = eta_prev + 0.5 * eta_acc
    if keep is not None:
        keep.update(dict(W=W, X=X, AX=AX, gammahat=gh, V=V, gamma=gam, alpha=alp, xhat=xh,
                         what=what, Z=Z, eta_prev=eta_prev, eta_rbf=eta_acc.copy(), x0=x0,
                         Ginv=Ginv, sel=list(sel), red=red, aug=aug))
    if Z.shape[1] > opt.ybar:
        eta = eta_acc if opt.weights == "rbf" else eta_prev
        Ynew, lam = pod_evd_dense(A, Z, eta, opt.y_trunc, opt.rank_rtol, opt.energy_y)
        yk = Ynew.shape[1]
        wk = min(opt.w_max, yk)
        wk = _energy_count(lam, wk, opt.energy_w)
        st.Y = Ynew
        st.sel = list(range(wk))
        st.eta_acc = np.zeros(yk)
        st.jc = st.j
        S.truncated = True
        if keep is not None:
            keep["pod_lam"] = lam
    else:
        st.Y = Z
        new = list(range(m, m + kr))
        if opt.rho >= 1.0:
            pick = new
        elif opt.rho <= 0.0 or kr == 0:
            pick = []
        else:
            tot = float(np.sum(gam))
            pick = [m + k for k in range(kr) if gam[k] / tot > opt.rho]
        st.sel = (sel + pick)[:opt.w_cap]
        st.eta_acc = eta_acc
    S.m_next = st.m
    S.w_next = len(st.sel)
    return x, S


def run_three_stage(cfg, opt: TSOptions, steps: int | None = None, maxit: int = 100000,
                    keep_x: bool = False):
    """Sequence driver: ts_solve for j = 1..steps with xbar_j = 0."""
    steps = cfg.steps if steps is None else steps
    st = TSState(cfg.n)
    out = []
    x_prev = None
    for j in range(1, steps + 1):
        A = CSR(cfg.rowptr, cfg.colind, cfg.matrix_values(j))
        b = cfg.rhs(j, x_prev)
        x, S = ts_solve(A, b, np.zeros(cfg.n), st, cfg.tol, maxit, opt)
        rec = S.__dict__.copy()
        if keep_x:
            rec["x"] = x
            rec["b"] = b
        out.append(rec)
        x_prev = x
    return out
