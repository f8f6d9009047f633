"""Pins of the three-stage oracle (Alg. 3) against what the paper and the
mathematics fix, and mutants of it that the pins must catch.

* Stage 2 with a zero tolerance reaches the Galerkin solution over range(Y)
  (a dense solve of Y^T A Y), its directions are A-orthogonal to each other
  and to W (Section 4.2), and it terminates in at most m - w steps.
* Stage-3 directions are A-orthogonal to each other and to [W, X]
  (Section 4.3); the solution is reconstructed exactly from the accumulated
  vectors and the previous weights (Section 3.3.2).
* A truncated basis is A_j-orthonormal (Eq. (podOrth)) and equals the POD of
  the independent C oracle (Alg. pod_evd) when both apply.
* With rho = 1 and a constant matrix the second solve of the same system
  needs no Stage-3 iteration (the solution lies in the accumulated span).
* eta^RBF equals the explicit sum of Section 3.3.2 with weights 2^{1-i}.
* Theorem wellConditioned: ||Y_j^T A_j Y_j - I|| <= sum ||Y_k||^2 ||A_k - A_{k-1}||.
* Iterative Stage 3 (phi = 1, Section 4.3.1): with tight projection solves it
  is Alg. 1 with all of Y as the augmenting basis (the C oracle's dense
  Cholesky projection); its directions are A-orthogonal to all of Y; the
  augmenting directions of the projection solves stay mutually orthogonal in
  the reduced metric, so all projection solves together take at most
  m - w - k2 steps (exact arithmetic; two spare for rounding).
"""

import importlib.util
import os
import sys
import tempfile

import numpy as np
import pytest

import oracle
from oracle import three_stage as TS
from problems import Config4Member


def _A(cfg, j):
    return oracle.CSR(cfg.rowptr, cfg.colind, cfg.matrix_values(j))


def _dense(A):
    n = A.n
    D = np.zeros((n, n))
    for i in range(n):
        for e in range(A.rowptr[i], A.rowptr[i + 1]):
            D[i, A.colind[e]] += A.vals[e]
    return D


def pin_stage2_galerkin(ts):
    cfg = Config4Member(12, 1000, 1001, 3, 5, 4, 1e-10)
    A = _A(cfg, 1)
    r = np.random.Generator(np.random.PCG64(70))
    Y = r.standard_normal((cfg.n, 10))
    sel = [0, 1, 2]
    W = Y[:, sel]
    AW = np.stack([oracle.matvec(A, W[:, k]) for k in range(3)], axis=1)
    R, kept = ts._chol_truncated(W.T @ AW)
    assert kept == 3
    rbar = cfg.rhs(1)
    what = ts._chol_solve(R, W.T @ rbar)
    # finite termination: m - w = 7 steps reach the Galerkin solution over range(Y)
    xh, X, AX, gh, k, rhn = ts.stage2(A, Y, sel, AW, R, what, rbar, 0.0, 7)
    D = _dense(A)
    ref = np.linalg.solve(Y.T @ D @ Y, Y.T @ rbar)
    assert k == 7
    assert np.linalg.norm(xh - ref) <= 1e-9 * np.linalg.norm(ref)
    # X^T A X diagonal (= Gammahat), X^T A W = 0
    XAX = X.T @ AX
    off = XAX - np.diag(np.diag(XAX))
    assert np.abs(off).max() <= 1e-9 * np.abs(np.diag(XAX)).max()
    assert np.allclose(np.diag(XAX), gh, rtol=1e-10)
    assert np.abs(X.T @ AW).max() <= 1e-9 * np.linalg.norm(X) * np.linalg.norm(AW)


def pin_stage3_orthogonality_and_reconstruction(ts):
    cfg = Config4Member(14, 1002, 1003, 4, 5, 4, 1e-10)
    opt = ts.TSOptions(ybar=1000, rho=0.0, stage2_factor=1e-4, stage2_maxit=30)
    st = ts.TSState(cfg.n)
    for j in (1, 2):
        A = _A(cfg, j)
        b = cfg.rhs(j)
        keep = {}
        x, S = ts.ts_solve(A, b, np.zeros(cfg.n), st, cfg.tol, 10000, opt, keep)
        assert S.true_relres <= cfg.tol * 1.01
        # x - xbar = Z eta^prev
        assert np.linalg.norm(keep["Z"] @ keep["eta_prev"] - x) <= 1e-11 * np.linalg.norm(x)
        V = keep["V"]
        AV = np.stack([oracle.matvec(A, V[:, k]) for k in range(V.shape[1])], axis=1)
        G = V.T @ AV
        assert np.allclose(np.diag(G), keep["gamma"], rtol=1e-10)
        off = G - np.diag(np.diag(G))
        assert np.abs(off).max() <= 1e-6 * np.abs(np.diag(G)).max()
        B = np.concatenate([keep["W"], keep["X"]], axis=1)
        if B.shape[1]:
            c = np.abs(B.T @ AV) / (np.linalg.norm(B, axis=0)[:, None] * np.linalg.norm(V, axis=0)[None, :])
            assert c.max() <= 1e-6
    assert S.k2 > 0


def pin_truncation_orthonormal_and_c_pod(ts):
    cfg = Config4Member(10, 1004, 1005, 3, 5, 4, 1e-10)
    A = _A(cfg, 2)
    r = np.random.Generator(np.random.PCG64(71))
    Z = r.standard_normal((cfg.n, 12))
    eta = r.uniform(0.2, 1.0, 12)
    Yn, lam = ts.pod_evd_dense(A, Z, eta, 6, 1e-12, 1.0)
    D = _dense(A)
    assert np.abs(Yn.T @ D @ Yn - np.eye(6)).max() <= 1e-10
    Wc, lam_c = oracle.pod_evd(A, Z, eta, 6)
    assert np.allclose(lam, lam_c, rtol=1e-10, atol=1e-12 * lam[0])
    P1 = Yn @ Yn.T @ D
    P2 = Wc @ Wc.T @ D
    assert np.abs(P1 - P2).max() <= 1e-9 * np.abs(P2).max()
    # energy criterion: smallest y reaching the energy fraction
    Ye, _ = ts.pod_evd_dense(A, Z, eta, 12, 1e-12, 0.9)
    frac = np.cumsum(lam) / lam.sum()
    assert Ye.shape[1] == int(np.argmax(frac >= 0.9)) + 1


def pin_exact_recovery(ts):
    cfg = Config4Member(6, 1006, 1007, 2, 5, 4, 1e-10)
    A = _A(cfg, 1)
    b = cfg.rhs(1)
    for rho in (1.0, 0.0):
        opt = ts.TSOptions(ybar=1000, rho=rho, w_cap=32, stage2_factor=1e-6, stage2_maxit=32)
        st = ts.TSState(cfg.n)
        x1, S1 = ts.ts_solve(A, b, np.zeros(cfg.n), st, cfg.tol, 10000, opt)
        keep = {}
        x2, S2 = ts.ts_solve(A, b, np.zeros(cfg.n), st, cfg.tol, 10000, opt, keep)
        assert S1.k3 > 0 and S1.k3 <= 32
        assert S2.true_relres <= cfg.tol * 1.01
        if rho == 1.0:        # Stage 1 alone reproduces x_1
            assert S2.w == S1.k3 and S2.k3 == 0 and S2.k2 == 0
        else:                 # Stage 2 reproduces x_1 to its tolerance
            assert S2.w == 0 and S2.k2 > 0
            assert np.linalg.norm(keep["x0"] - x1) <= 1e-4 * np.linalg.norm(x1)
            assert S2.k3 < S1.k3 // 2


def pin_rbf_weights(ts):
    cfg = Config4Member(9, 1008, 1009, 4, 5, 4, 1e-8)
    opt = ts.TSOptions(ybar=1000, rho=0.0, stage2_maxit=8)
    st = ts.TSState(cfg.n)
    hist = []
    for j in range(1, 5):
        keep = {}
        ts.ts_solve(_A(cfg, j), cfg.rhs(j), np.zeros(cfg.n), st, cfg.tol, 10000, opt, keep)
        hist.append(keep["eta_prev"])
        L = len(keep["eta_rbf"])
        expl = np.zeros(L)
        for i in range(1, len(hist) + 1):
            e = hist[-i]
            expl[:len(e)] += 2.0 ** (1 - i) * e
        assert np.allclose(keep["eta_rbf"], expl, rtol=1e-14, atol=0)


def pin_well_conditioned_bound(ts):
    cfg = Config4Member(8, 1010, 1011, 4, 5, 4, 1e-6)
    opt = ts.TSOptions(ybar=1000, rho=1.0, w_cap=32, stage2_factor=1e-6)
    st = ts.TSState(cfg.n)
    bound = 0.0
    D_prev = None
    for j in range(1, 5):
        A = _A(cfg, j)
        D = _dense(A)
        if st.m:
            Y = st.Y
            bound += np.linalg.norm(Y, 2) ** 2 * np.linalg.norm(D - D_prev, 2)
            err = np.linalg.norm(Y.T @ D @ Y - np.eye(st.m), 2)
            assert err <= bound * (1 + 1e-8) + 1e-10, (j, err, bound)
        if st.m + 12 > 32:
            break
        ts.ts_solve(A, cfg.rhs(j), np.zeros(cfg.n), st, cfg.tol, 10000, opt)
        assert st.sel == list(range(st.m))            # W = Y throughout
        D_prev = D
    assert st.m > 0


def pin_stage3_exact_factor(ts):
    cfg = Config4Member(16, 1014, 1015, 3, 5, 4, 1e-10)
    opt = ts.TSOptions(ybar=1000, rho=0.0, stage2_maxit=20, stage3_gram="exact")
    st = ts.TSState(cfg.n)
    for j in (1, 2, 3):
        A = _A(cfg, j)
        keep = {}
        x, S = ts.ts_solve(A, cfg.rhs(j), np.zeros(cfg.n), st, cfg.tol, 10000, opt, keep)
        assert S.status == 0 and S.true_relres <= cfg.tol * 1.01
    B = np.concatenate([keep["W"], keep["X"]], axis=1)
    AB = np.stack([oracle.matvec(A, B[:, k]) for k in range(B.shape[1])], axis=1)
    kb = keep["Ginv"].shape[0]
    assert np.abs(keep["Ginv"] @ (B[:, :kb].T @ AB[:, :kb]) - np.eye(kb)).max() <= 1e-8
    V = keep["V"]
    AV = np.stack([oracle.matvec(A, V[:, k]) for k in range(V.shape[1])], axis=1)
    c = np.abs(B[:, :kb].T @ AV) / (np.linalg.norm(B[:, :kb], axis=0)[:, None] * np.linalg.norm(V, axis=0)[None, :])
    assert c.max() <= 1e-8


def _dinv(A):
    d = np.zeros(A.n)
    for i in range(A.n):
        for e in range(A.rowptr[i], A.rowptr[i + 1]):
            if A.colind[e] == i:
                d[i] += A.vals[e]
    return 1.0 / d


def pin_iterative_stage3_is_full_projection(ts):
    cfg = Config4Member(12, 1050, 1051, 2, 5, 4, 1e-10)
    A = _A(cfg, 1)
    D = _dense(A)
    r = np.random.Generator(np.random.PCG64(73))
    m = 12
    Y = r.standard_normal((cfg.n, m))
    sel = [0, 1, 2]
    W = Y[:, sel]
    AW = D @ W
    R, kept = ts._chol_truncated(W.T @ AW)
    rbar = cfg.rhs(1)
    what = ts._chol_solve(R, W.T @ rbar)
    red = {}
    _, X, AX, gh, k2, _ = ts.stage2(A, Y, sel, AW, R, what, rbar, 0.0, 3, red)
    assert k2 == 3 and red["P"].shape == (m, 3)
    aug = ts.ReducedAugmentation(Y, sel, AW, R, red["P"], red["G"], gh)
    # start from the Galerkin solution over range(Y), as the reference does
    x0 = Y @ np.linalg.solve(Y.T @ D @ Y, Y.T @ rbar)
    K = 12
    x, V, gam, alp, k3, rn, kin, mv = ts.stage3_iterative(A, rbar, x0, Y, aug, _dinv(A), 0.0, K, K, 1e-14, 200)
    xr, so = oracle.aug_pcg(A, rbar, x0, Y, tol=0.0, maxit=K)
    assert k3 == K == so.iters
    assert np.linalg.norm(x - xr) <= 1e-9 * np.linalg.norm(xr)
    assert 0 < kin <= m - len(sel) - k2 + 2
    assert mv == 1 + K + K + kin      # r0, one A p a step, one A z a projection (K of them), the solve steps


def pin_iterative_stage3_orthogonality(ts):
    cfg = Config4Member(14, 1052, 1053, 3, 5, 4, 1e-10)
    opt = ts.TSOptions(ybar=1000, rho=0.0, stage2_factor=1e-2, stage2_maxit=512, phi=1, inner_rtol=1e-11,
                       inner_maxit=32)
    st = ts.TSState(cfg.n)
    for j in (1, 2, 3):
        A = _A(cfg, j)
        keep = {}
        Y = st.Y.copy()
        x, S = ts.ts_solve(A, cfg.rhs(j), np.zeros(cfg.n), st, cfg.tol, 200, opt, keep)
        assert S.status == 0 and S.true_relres <= cfg.tol * 1.01
    D = _dense(A)
    m, w, k2 = Y.shape[1], S.w, S.k2
    assert m > 0 and S.k_in > 0
    V = keep["V"]
    c = np.abs(Y.T @ D @ V) / (np.linalg.norm(Y, axis=0)[:, None] * np.linalg.norm(D @ V, axis=0)[None, :])
    assert c.max() <= 1e-7, c.max()
    aug = keep["aug"]
    P = np.stack(aug.P, axis=1)
    Gh = Y.T @ D @ Y
    Q = P.T @ Gh @ P
    off = Q - np.diag(np.diag(Q))
    assert np.abs(off).max() <= 1e-7 * np.abs(np.diag(Q)).max()
    assert np.allclose(np.diag(Q), aug.gam, rtol=1e-9)
    if w:
        Wh = np.eye(m)[:, keep["sel"]]
        assert np.abs(P.T @ Gh @ Wh).max() <= 1e-7 * np.abs(Gh).max()
    assert S.k_in <= m - w - k2 + 2


PINS = [pin_iterative_stage3_is_full_projection, pin_iterative_stage3_orthogonality, pin_stage2_galerkin, pin_stage3_orthogonality_and_reconstruction, pin_stage3_exact_factor,
        pin_truncation_orthonormal_and_c_pod, pin_exact_recovery, pin_rbf_weights,
        pin_well_conditioned_bound]


@pytest.mark.parametrize("pin", PINS, ids=lambda f: f.__name__)
def test_three_stage_oracle_pins(pin):
    pin(TS)


def test_e6_reduced_matrix_is_scaled_identity_after_truncation():
    """Synthetic rerun of the paper's reduced-matrix diagnostic: with
    A_j = (1 + 0.01 j) A_0, a basis truncated with the metric A_{j-1} gives
    Y_j^T A_j Y_j = (1 + 0.01 j) / (1 + 0.01 (j - 1)) I, condition number 1."""
    cfg = Config4Member(16, 1030, 1031, 7, 5, 4, 1e-8)
    opt = TS.TSOptions(ybar=30, y_trunc=10, w_max=3, stage2_maxit=10)
    out = TS.run_three_stage(cfg, opt)
    after = [o for prev, o in zip(out, out[1:]) if prev["truncated"]]
    assert after
    for o in after:
        print(f"j={o['j']} m={o['m']} cond(Y^T A Y) = {o['cond_YAY']:.12f}")
        assert abs(o["cond_YAY"] - 1.0) <= 1e-9


def test_three_stage_sequence_with_truncations_meets_tolerance():
    cfg = Config4Member(20, 1012, 1013, 6, 5, 4, 1e-8)
    opt = TS.TSOptions(ybar=40, y_trunc=12, w_max=4, rho=1e-3, stage2_maxit=20)
    out = TS.run_three_stage(cfg, opt)
    ex = TS.run_three_stage(cfg, TS.TSOptions(ybar=40, y_trunc=12, w_max=4, rho=1e-3,
                                              stage2_maxit=20, stage3_gram="exact"))
    for a, e in zip(out, ex):
        assert e["status"] == 0 and abs(a["k3"] - e["k3"]) <= max(2, a["k3"] // 10)
    assert any(o["truncated"] for o in out)
    for o in out:
        assert o["status"] == 0 and o["true_relres"] <= cfg.tol * 1.01
        assert o["m_next"] <= max(opt.ybar, o["m"]) + o["k3"]
    later = [o["k3"] for o in out[2:]]
    assert max(later) < out[0]["k3"]


def test_iterative_stage3_sequence_meets_tolerance():
    """The iterative Stage 3 (phi = 1) over a sequence with truncations meets
    the tolerance in every system with at most the iterations of the
    non-iterative Stage 3, whose augmenting space it contains."""
    cfg = Config4Member(20, 1012, 1013, 6, 5, 4, 1e-8)
    base = dict(ybar=40, y_trunc=12, w_max=4, rho=1e-3)
    out0 = TS.run_three_stage(cfg, TS.TSOptions(**base, stage2_maxit=20))
    out1 = TS.run_three_stage(cfg, TS.TSOptions(**base, stage2_maxit=512, phi=1))
    for a, b in zip(out0, out1):
        print(f"j={a['j']}: phi=0 k3 {a['k3']} matvecs {a['matvecs']} | phi=1 k3 {b['k3']} "
              f"projection steps {b['k_in']} matvecs {b['matvecs']}")
        assert b["status"] == 0 and b["true_relres"] <= cfg.tol * 1.01
        assert b["k3"] <= a["k3"]
    assert sum(b["k_in"] for b in out1) > 0


# ------------------------------------------------------------------ mutants

SRC = TS.__file__

MUTANTS = {
    "new_vectors_scaled_by_sqrt_gamma": (
        "Znew = V / np.sqrt(gam)[None, :] if kr else np.zeros((n, 0))",
        "Znew = V * np.sqrt(gam)[None, :] if kr else np.zeros((n, 0))"),
    "stage2_without_projection": (
        "        ph = zh + beta * ph\n        if w:\n            ph[sel] -= mu",
        "        ph = zh + beta * ph\n        if False:\n            ph[sel] -= mu"),
    "rbf_factor_quarter": ("eta_acc = eta_prev + 0.5 * eta_acc", "eta_acc = eta_prev + 0.25 * eta_acc"),
    "stage3_residual_ignores_x0": ("    y = B.shape[1]\n    x = x0.copy()\n    r = b - matvec(A, x)",
                                   "    y = B.shape[1]\n    x = x0.copy()\n    r = b.copy()"),
    "stage2_rhs_without_stage1": ("rh = Y.T @ (rbar - _mv(A, Y @ xh))", "rh = Y.T @ rbar"),
    "stage3_exact_gram_without_A": ("RB, kb = _chol_truncated(B.T @ AB)", "RB, kb = _chol_truncated(B.T @ B)"),
    "projection_solve_from_zero": (
        "    nw, nd = aug.galerkin(c)\n    mu = aug.combine(nw, nd)\n    r = c - aug.combine_G(nw, nd)",
        "    mu = np.zeros_like(c)\n    r = c.copy()"),
    "projection_directions_not_kept": ("    aug.P += newP[:room]\n    aug.G += newG[:room]\n    aug.gam += newgam[:room]",
                                       "    pass"),
    "outer_direction_unprojected": ("        p = z + beta * p - Y @ mu_of(z)", "        p = z + beta * p"),
    "pod_missing_weight": ("T = (eta[:, None] * V[:, :y]) / np.sqrt(lam[:y])[None, :]",
                           "T = V[:, :y] / np.sqrt(lam[:y])[None, :]"),
}


def _load_mutant(name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    src = src.replace(old, new).replace("from . import CSR, matvec", "from oracle import CSR, matvec")
    d = tempfile.mkdtemp()
    path = os.path.join(d, f"ts_{name}.py")
    with open(path, "w") as f:
        f.write(src)
    spec = importlib.util.spec_from_file_location(f"ts_mutant_{name}", path)
    mod = importlib.util.module_from_spec(spec)
    sys.modules[spec.name] = mod
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_three_stage_mutant_is_caught(name):
    mod = _load_mutant(name)
    caught = []
    for pin in PINS:
        try:
            pin(mod)
        except Exception:
            caught.append(pin.__name__)
    assert caught, f"mutant {name} passed every pin"


def test_e8_pod_weights_synthetic():
    """Synthetic rerun of the paper's POD-weights experiment (Section 5.3): the
    vectors accumulated over systems 1..10 (no truncation) are truncated by POD
    in the metric A_10 with the ideal, previous and RBF weights, and system 11
    is solved over the first k POD vectors.  Reported: the A_11-norm error of
    the Stage-1 solution and the Stage-3 iterations to 1e-6.  Pinned: the
    error is non-increasing in k for every weighting (nested subspaces), and the
    ideal weights are at least as good as the computable ones at the largest k
    (within 5%)."""
    cfg = Config4Member(18, 1040, 1041, 11, 5, 4, 1e-6)
    opt = TS.TSOptions(ybar=10_000, cap=10_000, rho=0.0, stage2_maxit=8)
    st = TS.TSState(cfg.n)
    prev = []
    for j in range(1, 11):
        keep = {}
        TS.ts_solve(_A(cfg, j), cfg.rhs(j), np.zeros(cfg.n), st, cfg.tol, 10_000, opt, keep)
        prev.append(keep["eta_prev"])
    Z = st.Y
    A10, A11 = _A(cfg, 10), _A(cfg, 11)
    D11 = _dense(A11)
    b11 = cfg.rhs(11)
    x11 = np.linalg.solve(D11, b11)
    AZ11 = D11 @ Z
    # Eq. (weightsIdealAj) with xbar = 0.  The accumulated Krylov vectors of ten
    # similar solves are linearly dependent in floating point (Z^T A Z has
    # eigenvalues at rounding level), so the weights are the minimum-norm
    # solution: eigenvalues below 1e-12 of the largest are dropped
    G = Z.T @ AZ11
    lam, U = np.linalg.eigh(0.5 * (G + G.T))
    live = lam > 1e-12 * lam[-1]
    ideal = U[:, live] @ ((U[:, live].T @ (Z.T @ b11)) / lam[live])
    rbf = np.zeros(Z.shape[1])
    for i, e in enumerate(reversed(prev), start=1):
        rbf[:len(e)] += 2.0 ** (1 - i) * e
    weights = {"ideal": ideal, "previous": prev[-1], "rbf": rbf}
    ks = [1, 2, 4, 8, 16]
    rows = []
    for name, eta in weights.items():
        basis, _ = TS.pod_evd_dense(A10, Z, eta, max(ks), 1e-12, 1.0)
        errs, its = [], []
        for k in ks:
            W = basis[:, :k]
            c = np.linalg.solve(W.T @ D11 @ W, W.T @ b11)
            d = x11 - W @ c
            errs.append(float(np.sqrt(d @ D11 @ d) / np.sqrt(x11 @ D11 @ x11)))
            _, so = oracle.aug_pcg(A11, b11, np.zeros(cfg.n), W, cfg.tol, 10_000)
            its.append(so.iters)
        rows.append((name, errs, its))
        assert all(errs[i + 1] <= errs[i] * (1 + 1e-9) + 1e-14 for i in range(len(errs) - 1)), (name, errs)
    final = {name: errs[-1] for name, errs, _ in rows}
    assert final["ideal"] <= 1.05 * min(final["previous"], final["rbf"])
    print(f"\nE8 synthetic: Z_10 has {Z.shape[1]} vectors; k = {ks}")
    for name, errs, its in rows:
        print(f"{name:9s} A-norm error {' '.join(f'{e:.2e}' for e in errs)} | stage-3 iterations {its}")
