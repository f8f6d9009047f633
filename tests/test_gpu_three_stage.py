"""The three-stage method (Alg. 3) on the GPU against the three-stage oracle,
with the non-iterative Stage 3 (phi = 0) and the iterative one (phi = 1).

Lockstep: from identical states (Y, stage-1 columns, weights), matrix and
right-hand side, with tolerance 0 and the same Stage-3 iteration count,
the GPU solution equals the oracle's to 1e-10 and the Stage-2 step count,
the truncation decision and the truncated subspace agree.  Closed loop:
whole sequences with truncations meet the tolerance by the oracle's own
residual with the oracle's dimensions and Stage-2/3 counts within one or two.
"""

import numpy as np
import pytest

import oracle
from oracle import three_stage as TS
from problems import Config4Member

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module")
def P():
    import paper_1512_05820_amd as P
    assert torch.cuda.is_available()
    P.load()
    return P


def _ctx(P, cfg, maxit=20000, **ts):
    k = P.PodCG(cfg.n, maxit=maxit)
    k.set_matrix(_dev(cfg.matrix_values(1)), _dev(cfg.rowptr, torch.int32), _dev(cfg.colind, torch.int32))
    k.ts_enable(**ts)
    return k


def _opts(**kw):
    o = TS.TSOptions(**kw)
    return o, {f: getattr(o, f) for f in ("ybar", "y_trunc", "w_max", "w_cap", "stage2_maxit", "cap",
                                          "energy_y", "energy_w", "rho", "stage2_factor", "phi",
                                          "inner_maxit", "inner_rtol")} | {
        "weights": 0 if o.weights == "rbf" else 1,
        "stage3_gram": 0 if o.stage3_gram == "blockdiag" else 1}


def _a_orthonormal(A, Z):
    D = np.stack([oracle.matvec(A, Z[:, k]) for k in range(Z.shape[1])], axis=1)
    G = Z.T @ D
    L = np.linalg.cholesky(0.5 * (G + G.T))
    return Z @ np.linalg.inv(L).T


@pytest.mark.parametrize("case", ["empty", "basis", "truncate", "exact_gram"])
def test_lockstep_one_system(P, case):
    cfg = Config4Member(20, 1020, 1021, 3, 5, 4, 1e-10)
    A = oracle.CSR(cfg.rowptr, cfg.colind, cfg.matrix_values(2))
    b = cfg.rhs(2)
    r = np.random.Generator(np.random.PCG64(80))
    K = 30
    o, kw = _opts(ybar=60, y_trunc=12, w_max=4, stage2_maxit=16,
                  stage3_gram="exact" if case == "exact_gram" else "blockdiag")
    st = TS.TSState(cfg.n)
    if case != "empty":
        m = 40 if case in ("basis", "exact_gram") else 55
        Z = _a_orthonormal(oracle.CSR(cfg.rowptr, cfg.colind, cfg.matrix_values(1)),
                           r.standard_normal((cfg.n, m)))
        st.Y = Z
        st.sel = [0, 1, 2, 3, 4]
        st.eta_acc = r.uniform(0.5, 1.0, m)
    Y0, sel0, eta0 = st.Y.copy(), list(st.sel), st.eta_acc.copy()
    keep = {}
    xo, So = TS.ts_solve(A, b, np.zeros(cfg.n), st, 0.0, K, o, keep)
    ctx = _ctx(P, cfg, maxit=K, **kw)
    ctx.set_matrix(_dev(cfg.matrix_values(2)))
    if case != "empty":
        ctx.ts_set_state(_dev(Y0), sel0, eta0)
    x = _dev(np.zeros(cfg.n))
    Sg = ctx.ts_solve(_dev(b), x, 0.0)
    xg = _host(x)
    e = _relerr(xg, xo)
    print(f"{case}: w {Sg.w}/{So.w} k2 {Sg.k2}/{So.k2} k3 {Sg.k3}/{So.k3} trunc {Sg.truncated}/{So.truncated} "
          f"m_next {Sg.m_next}/{So.m_next} err {e:.2e}")
    assert (Sg.w, Sg.k2, Sg.k3) == (So.w, So.k2, So.k3)
    assert bool(Sg.truncated) == So.truncated and Sg.m_next == So.m_next and Sg.w_next == So.w_next
    assert e <= 1e-10
    Yg, selg = ctx.ts_state()
    Yg = _host(Yg)
    assert selg == st.sel
    if So.truncated:
        D = np.stack([oracle.matvec(A, Yg[:, k]) for k in range(Yg.shape[1])], axis=1)
        assert np.abs(Yg.T @ D - np.eye(Yg.shape[1])).max() <= 1e-9      # A_j-orthonormal
        Po = st.Y @ (st.Y.T @ D)
        Pg = Yg @ (Yg.T @ D)
        assert np.abs(Pg - Po).max() <= 1e-8 * np.abs(Po).max()
    else:
        assert np.abs(Yg - st.Y).max() <= 1e-10 * np.abs(st.Y).max()


@pytest.mark.parametrize("variant", ["rbf_blockdiag", "previous_exact"])
def test_closed_loop_sequence_with_truncations(P, variant):
    cfg = Config4Member(24, 1022, 1023, 8, 5, 4, 1e-10)
    weights, gram = variant.split("_")
    o, kw = _opts(ybar=150, y_trunc=40, w_max=5, rho=1e-3, stage2_maxit=24, weights=weights,
                  stage3_gram=gram)
    orc = TS.run_three_stage(cfg, o, maxit=20000)
    ctx = _ctx(P, cfg, **kw)
    for j, oj in enumerate(orc, start=1):
        if j > 1:
            ctx.set_matrix(_dev(cfg.matrix_values(j)))
        b = cfg.rhs(j)
        x = _dev(np.zeros(cfg.n))
        S = ctx.ts_solve(_dev(b), x, cfg.tol)
        A = oracle.CSR(cfg.rowptr, cfg.colind, cfg.matrix_values(j))
        tr = np.linalg.norm(b - oracle.matvec(A, _host(x))) / np.linalg.norm(b)
        print(f"j={j} w {S.w}/{oj['w']} m {S.m}/{oj['m']} k2 {S.k2}/{oj['k2']} k3 {S.k3}/{oj['k3']} "
              f"trunc {S.truncated}/{oj['truncated']} relres {tr:.2e}")
        assert S.status == 0 and tr <= cfg.tol * 1.01
        assert (S.w, S.m) == (oj["w"], oj["m"])
        assert bool(S.truncated) == oj["truncated"]
        assert abs(S.k2 - oj["k2"]) <= 1 and abs(S.k3 - oj["k3"]) <= 2
    assert any(o_["truncated"] for o_ in orc)


def test_exact_recovery_with_all_new_vectors_in_stage1(P):
    cfg = Config4Member(6, 1006, 1007, 2, 5, 4, 1e-10)
    o, kw = _opts(ybar=400, rho=1.0, w_cap=32, stage2_factor=1e-6, stage2_maxit=32)
    ctx = _ctx(P, cfg, **kw)
    b = _dev(cfg.rhs(1))
    x1 = _dev(np.zeros(cfg.n))
    S1 = ctx.ts_solve(b, x1, cfg.tol)
    x2 = _dev(np.zeros(cfg.n))
    S2 = ctx.ts_solve(b, x2, cfg.tol)
    assert 0 < S1.k3 <= 32 and S2.w == S1.k3 and S2.k3 == 0 and S2.k2 == 0
    assert S2.true_relres <= cfg.tol * 1.01


def test_record_cap_and_errors(P):
    cfg = Config4Member(16, 1024, 1025, 3, 5, 4, 1e-10)
    o, kw = _opts(ybar=30, y_trunc=10, w_max=3, cap=40, stage2_maxit=8)
    orc = TS.run_three_stage(cfg, o, maxit=20000)
    ctx = _ctx(P, cfg, **kw)
    for j, oj in enumerate(orc, start=1):
        if j > 1:
            ctx.set_matrix(_dev(cfg.matrix_values(j)))
        x = _dev(np.zeros(cfg.n))
        S = ctx.ts_solve(_dev(cfg.rhs(j)), x, cfg.tol)
        assert S.status == 0 and (S.m, S.m_next, S.w_next) == (oj["m"], oj["m_next"], oj["w_next"])
    plain = P.PodCG(cfg.n)
    plain.set_matrix(_dev(cfg.matrix_values(1)), _dev(cfg.rowptr, torch.int32), _dev(cfg.colind, torch.int32))
    with pytest.raises(P.PodCGError):
        plain.ts_solve(_dev(cfg.rhs(1)), _dev(np.zeros(cfg.n)), 1e-8)
    with pytest.raises(P.PodCGError):
        plain.ts_enable(ybar=600)
    mixed = P.PodCG(cfg.n, precision="mixed")
    with pytest.raises(P.PodCGError):
        mixed.ts_enable()


@pytest.mark.parametrize("case", ["basis", "truncate"])
def test_lockstep_iterative_stage3(P, case):
    """phi = 1 from identical states with tolerance 0 and the oracle's Stage-3
    count: equal Stage-2, Stage-3 and projection-solve step counts, equal
    truncation decisions, solutions within 1e-10."""
    cfg = Config4Member(20, 1020, 1021, 3, 5, 4, 1e-10)
    A = oracle.CSR(cfg.rowptr, cfg.colind, cfg.matrix_values(2))
    b = cfg.rhs(2)
    r = np.random.Generator(np.random.PCG64(81))
    K = 25
    m = 40 if case == "basis" else 50
    o, kw = _opts(ybar=100 if case == "basis" else 60, y_trunc=12, w_max=4, stage2_maxit=512, phi=1,
                  inner_rtol=1e-10)
    st = TS.TSState(cfg.n)
    st.Y = _a_orthonormal(oracle.CSR(cfg.rowptr, cfg.colind, cfg.matrix_values(1)), r.standard_normal((cfg.n, m)))
    st.sel = [0, 1, 2, 3]
    st.eta_acc = r.uniform(0.5, 1.0, m)
    Y0, sel0, eta0 = st.Y.copy(), list(st.sel), st.eta_acc.copy()
    xo, So = TS.ts_solve(A, b, np.zeros(cfg.n), st, 0.0, K, o)
    ctx = _ctx(P, cfg, maxit=K, **kw)
    ctx.set_matrix(_dev(cfg.matrix_values(2)))
    ctx.ts_set_state(_dev(Y0), sel0, eta0)
    x = _dev(np.zeros(cfg.n))
    Sg = ctx.ts_solve(_dev(b), x, 0.0)
    e = _relerr(_host(x), xo)
    print(f"{case}: w {Sg.w}/{So.w} k2 {Sg.k2}/{So.k2} k3 {Sg.k3}/{So.k3} k_in {Sg.k_in}/{So.k_in} "
          f"trunc {Sg.truncated}/{So.truncated} m_next {Sg.m_next}/{So.m_next} err {e:.2e}")
    assert (Sg.w, Sg.k2, Sg.k3, Sg.k_in) == (So.w, So.k2, So.k3, So.k_in)
    assert Sg.k_in > 0 and Sg.projections == K
    assert bool(Sg.truncated) == So.truncated and Sg.m_next == So.m_next
    assert e <= 1e-10


def test_closed_loop_iterative_stage3_sequence(P):
    cfg = Config4Member(24, 1022, 1023, 6, 5, 4, 1e-10)
    o, kw = _opts(ybar=120, y_trunc=30, w_max=5, rho=1e-3, stage2_maxit=512, phi=1)
    orc = TS.run_three_stage(cfg, o, maxit=20000)
    ctx = _ctx(P, cfg, **kw)
    for j, oj in enumerate(orc, start=1):
        if j > 1:
            ctx.set_matrix(_dev(cfg.matrix_values(j)))
        b = cfg.rhs(j)
        x = _dev(np.zeros(cfg.n))
        S = ctx.ts_solve(_dev(b), x, cfg.tol)
        A = oracle.CSR(cfg.rowptr, cfg.colind, cfg.matrix_values(j))
        tr = np.linalg.norm(b - oracle.matvec(A, _host(x))) / np.linalg.norm(b)
        print(f"j={j} w {S.w}/{oj['w']} m {S.m}/{oj['m']} k2 {S.k2}/{oj['k2']} k3 {S.k3}/{oj['k3']} "
              f"k_in {S.k_in}/{oj['k_in']} trunc {S.truncated}/{oj['truncated']} relres {tr:.2e}")
        assert S.status == 0 and tr <= cfg.tol * 1.01
        assert (S.w, S.m) == (oj["w"], oj["m"]) and bool(S.truncated) == oj["truncated"]
        assert abs(S.k2 - oj["k2"]) <= 1 and abs(S.k3 - oj["k3"]) <= 2
    assert any(o_["truncated"] for o_ in orc) and sum(o_["k_in"] for o_ in orc) > 0


def test_iterative_stage3_with_capped_projection_solves(P):
    # projection solves capped at one step: whenever a solve seeded with kept
    # directions stays above its tolerance it is redone once with none kept
    # (its step then counts twice in k_in; how often that happens depends on
    # rounding, so the count is printed, not asserted).  Over the first
    # systems of this sequence the solves still meet the tolerance by the
    # oracle's own residual; with one step per projection the outer iteration
    # is not guaranteed to converge in general (here it diverges at system 4)
    cfg = Config4Member(24, 1022, 1023, 3, 5, 4, 1e-10)
    o, kw = _opts(ybar=120, y_trunc=30, w_max=5, rho=1e-3, stage2_maxit=512, phi=1)
    kw["inner_maxit"] = 1
    kw["inner_rtol"] = 1e-13
    ctx = _ctx(P, cfg, maxit=400, **kw)
    for j in range(1, cfg.steps + 1):
        if j > 1:
            ctx.set_matrix(_dev(cfg.matrix_values(j)))
        b = cfg.rhs(j)
        x = _dev(np.zeros(cfg.n))
        S = ctx.ts_solve(_dev(b), x, cfg.tol)
        A = oracle.CSR(cfg.rowptr, cfg.colind, cfg.matrix_values(j))
        tr = np.linalg.norm(b - oracle.matvec(A, _host(x))) / np.linalg.norm(b)
        print(f"j={j} status {S.status} k3 {S.k3} k_in {S.k_in} projections {S.projections} "
              f"restarts {S.k_in - S.projections} relres {tr:.2e}")
        assert S.status == 0 and tr <= cfg.tol * 1.01, (j, S.status, tr)
        assert S.k_in <= 2 * S.projections
