"""The one-workgroup solve (option lds_solve: systems of at most 1024
unknowns, slices at most 8 wide, a basis of at most 5 columns) against the
oracle, through the C ABI.

  * lockstep: the GPU runs exactly the oracle's iteration count from the same
    (A, b, xbar, W) and the solutions agree to 1e-10 relative: config 1 at
    every basis dimension the kernel covers, with the oracle's own POD basis
    of the earlier systems, and from a non-zero initial guess;
  * closed loop: the config-1 sequence, every solution meeting the tolerance
    by the oracle's own residual, iteration counts within one, equal ranks;
  * the multi-kernel loop on the same systems gives the same iterations and
    solutions within 1e-10;
  * shapes: one unknown, one full slice, a ragged second slice, 1024 rows;
    offset-table slices of widths 1, 3, 5, 7 and per-entry (16-bit, int32)
    columns up to 8 per row;
  * edge cases: the iteration cap, zero and NaN right-hand sides, an
    indefinite matrix, exact recovery, a dependent basis column, a basis
    wider than the kernel covers (the multi-kernel loop takes it).
Every case checks which path ran (stats.path)."""

import numpy as np
import pytest

import oracle
from problems import config1, tiny

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


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


@pytest.fixture(scope="module")
def P():
    import paper_1512_05820_amd as P
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    P.load()
    return P


def _ctx(P, n, rowptr, colind, vals, **kw):
    c = P.PodCG(n, **kw)
    c.set_matrix(_dev(vals), _dev(rowptr, torch.int32), _dev(colind, torch.int32))
    return c


def _lockstep(P, rowptr, colind, vals, b, xbar, W, tol, lds=True):
    """The oracle to tol, then the GPU for exactly the oracle's iterations."""
    n = len(rowptr) - 1
    A = oracle.CSR(rowptr, colind, vals)
    xo, so = oracle.aug_pcg(A, b, xbar, W, tol=tol, maxit=20000)
    y = 0 if W is None else W.shape[1]
    ctx = _ctx(P, n, rowptr, colind, vals, rank_max=max(y, 1), maxit=so.iters, lds_solve=lds)
    ctx.set_basis(None if W is None else _dev(W))
    x = _dev(xbar)
    st = ctx.solve(_dev(b), x, 0.0)
    return xo, so, _host(x), st


@pytest.mark.parametrize("y", [0, 1, 2, 3, 4, 5])
def test_lockstep_config1_every_basis_dimension(P, y):
    cfg = config1()
    vals = cfg.matrix_values(3)
    b = cfg.rhs(3)
    W = _rng(20 + y).standard_normal((cfg.n, y)) if y else None
    xo, so, xg, st = _lockstep(P, cfg.rowptr, cfg.colind, vals, b, np.zeros(cfg.n), W, cfg.tol)
    assert st.path == 1
    assert so.status == 0 and st.iters == so.iters and st.rank == y
    assert _relerr(xg, xo) <= 1e-10
    assert abs(st.stage1_relres - so.stage1_relres) <= 1e-9 * so.stage1_relres


def test_lockstep_with_the_oracles_pod_basis(P):
    """System 7 of the config-1 sequence with W_7 = the oracle's POD of its
    own solutions of systems 2-6 (rank 4), as the sequence runs it."""
    cfg = config1()
    orc = oracle.run_sequence(cfg, "aug", steps=6, keep_W=True, keep_x=True)
    W = orc[-1]["W"]
    assert W.shape[1] == cfg.rank
    vals = cfg.matrix_values(7)
    b = cfg.rhs(7, orc[-1]["x"])
    xo, so, xg, st = _lockstep(P, cfg.rowptr, cfg.colind, vals, b, np.zeros(cfg.n), W, cfg.tol)
    assert st.path == 1 and st.iters == so.iters and st.rank == cfg.rank
    assert _relerr(xg, xo) <= 1e-10


def test_lockstep_from_a_nonzero_guess(P):
    cfg = config1()
    vals = cfg.matrix_values(5)
    r = _rng(31)
    b = cfg.rhs(5)
    xbar = r.standard_normal(cfg.n) * 0.1
    W = r.standard_normal((cfg.n, 3))
    xo, so, xg, st = _lockstep(P, cfg.rowptr, cfg.colind, vals, b, xbar, W, cfg.tol)
    assert st.path == 1 and st.iters == so.iters
    assert _relerr(xg, xo) <= 1e-10


def _sequence(P, cfg, lds):
    ctx = P.PodCG(cfg.n, omega=cfg.omega, rank_max=cfg.rank, lds_solve=lds)
    rowptr, colind = _dev(cfg.rowptr, torch.int32), _dev(cfg.colind, torch.int32)
    out, x_prev = [], None
    for j in range(1, cfg.steps + 1):
        vals = cfg.matrix_values(j)
        ctx.set_matrix(_dev(vals), rowptr if j == 1 else None, colind if j == 1 else None)
        b = cfg.rhs(j, x_prev)
        x = _dev(np.zeros(cfg.n))
        st = ctx.solve(_dev(b), x, cfg.tol)
        ctx.push_snapshot(x)
        ctx.build_pod()
        xh = _host(x)
        out.append((st.as_dict(), xh, b, vals))
        x_prev = xh
    return out


def test_closed_loop_config1_sequence(P):
    cfg = config1()
    orc = oracle.run_sequence(cfg, "aug")
    gpu = _sequence(P, cfg, True)
    for o, (st, x, b, vals) in zip(orc, gpu):
        A = oracle.CSR(cfg.rowptr, cfg.colind, vals)
        tr = np.linalg.norm(b - oracle.matvec(A, x)) / np.linalg.norm(b)
        assert st["path"] == 1
        assert tr <= cfg.tol * 1.01, (o["j"], tr)
        assert st["status"] in (0, 2)
        assert abs(st["iters"] - o["iters"]) <= 1, (o["j"], st["iters"], o["iters"])
        assert st["rank"] == o["rank"]


def test_agrees_with_the_multikernel_loop(P):
    cfg = config1()
    one = _sequence(P, cfg, True)
    multi = _sequence(P, cfg, False)
    for (s1, x1, _, _), (s2, x2, _, _) in zip(one, multi):
        assert s1["path"] == 1 and s2["path"] == 0
        assert abs(s1["iters"] - s2["iters"]) <= 1 and s1["rank"] == s2["rank"]
        assert _relerr(x1, x2) <= 1e-10


def _banded(n, offsets, seed):
    """Symmetric banded SPD matrix whose rows draw on `offsets` (a symmetric
    list), diagonally dominant with random off-diagonal values."""
    r = _rng(seed)
    A = np.zeros((n, n))
    for d in offsets:
        if d > 0:
            v = -r.uniform(0.2, 1.0, n - d)
            A[np.arange(n - d), np.arange(d, n)] = v
            A[np.arange(d, n), np.arange(n - d)] = v
    A[np.arange(n), np.arange(n)] = np.abs(A).sum(axis=1) + r.uniform(0.1, 1.0, n)
    return A


@pytest.mark.parametrize("n,w", [(1, 1), (64, 3), (65, 5), (1000, 7), (1024, 5), (777, 1)])
def test_shapes_and_table_widths(P, n, w):
    offsets = [d for d in range(-(w // 2), w // 2 + 1)]
    if w == 5:
        offsets = [-8, -1, 0, 1, 8]
    if w == 7:
        offsets = [-30, -5, -1, 0, 1, 5, 30]
    Ad = _banded(n, offsets, 40 + n + w) if n > 1 else np.array([[2.5]])
    rowptr, colind, vals = tiny.dense_to_csr(Ad)
    r = _rng(41 + n)
    b = r.standard_normal(n)
    y = min(3, n)
    W = r.standard_normal((n, y))
    xo, so, xg, st = _lockstep(P, rowptr, colind, vals, b, np.zeros(n), W, 1e-11)
    assert st.path == 1 and st.iters == so.iters
    assert _relerr(xg, xo) <= 1e-10
    xo, so, xg, st = _lockstep(P, rowptr, colind, vals, b, np.zeros(n), None, 1e-11)
    assert st.path == 1 and st.iters == so.iters
    assert _relerr(xg, xo) <= 1e-10


def test_per_entry_columns_up_to_eight_a_row(P):
    """A random symmetric pattern (at most 8 entries a row, rows that differ
    within a slice): the slices keep 16-bit offsets or int32 columns."""
    n = 900
    r = _rng(44)
    A = np.zeros((n, n))
    deg = np.zeros(n, dtype=int)
    for _ in range(4 * n):
        i, j = r.integers(0, n, 2)
        if i != j and deg[i] < 7 and deg[j] < 7 and A[i, j] == 0.0:
            v = -r.uniform(0.1, 1.0)
            A[i, j] = A[j, i] = v
            deg[i] += 1
            deg[j] += 1
    A[np.arange(n), np.arange(n)] = np.abs(A).sum(axis=1) + 0.5
    rowptr, colind, vals = tiny.dense_to_csr(A)
    assert np.diff(rowptr).max() == 8
    b = r.standard_normal(n)
    W = r.standard_normal((n, 5))
    xo, so, xg, st = _lockstep(P, rowptr, colind, vals, b, np.zeros(n), W, 1e-10)
    ctx = _ctx(P, n, rowptr, colind, vals)
    kinds = ctx.format_counts()
    assert kinds["table"] < (n + 63) // 64    # not every slice is an offset table
    assert st.path == 1 and st.iters == so.iters
    assert _relerr(xg, xo) <= 1e-10


def test_edge_cases(P):
    cfg = config1(N=12)
    n = cfg.n
    vals = cfg.matrix_values(1)
    ctx = _ctx(P, n, cfg.rowptr, cfg.colind, vals, maxit=5)
    bn = np.ones(n)
    bn[7] = np.nan
    with pytest.raises(P.PodCGError) as e:
        ctx.solve(_dev(bn), _dev(np.zeros(n)), 1e-8)
    assert e.value.code == -5
    x = _dev(np.zeros(n))
    st = ctx.solve(_dev(np.ones(n)), x, 1e-14)    # cap of 5 iterations
    assert st.path == 1 and st.status == 1 and st.iters == 5
    A = oracle.CSR(cfg.rowptr, cfg.colind, vals)
    assert abs(st.true_relres - np.linalg.norm(np.ones(n) - oracle.matvec(A, _host(x))) / np.sqrt(n)) <= 1e-12
    x = _dev(np.zeros(n))
    st = ctx.solve(_dev(np.zeros(n)), x, 1e-8)    # zero rhs, zero guess
    assert st.path == 1 and st.status == 0 and st.iters == 0
    assert not np.any(_host(x))
    st = ctx.solve_plain(_dev(np.ones(n)), _dev(np.zeros(n)), 1e-14)
    assert st.path == 1 and st.iters == 5


def test_indefinite_matrix(P):
    n = 64
    A = np.eye(n)
    for i in range(n - 1):
        A[i, i + 1] = A[i + 1, i] = 0.9
    A[10, 11] = A[11, 10] = 5.0
    rowptr, colind, vals = tiny.dense_to_csr(A)
    orc = oracle.plain_pcg(oracle.CSR(rowptr, colind, vals), np.ones(n), np.zeros(n), 1e-12, 200)[1]
    assert orc.status == oracle.ERR_NOT_SPD
    ctx = _ctx(P, n, rowptr, colind, vals, maxit=200)
    with pytest.raises(P.PodCGError) as e:
        ctx.solve(_dev(np.ones(n)), _dev(np.zeros(n)), 1e-12)
    assert e.value.code == -4


def test_exact_recovery_dependent_column_and_fallback(P):
    cfg = config1(N=20)
    vals = cfg.matrix_values(2)
    A = oracle.CSR(cfg.rowptr, cfg.colind, vals)
    r = _rng(50)
    W = r.standard_normal((cfg.n, 4))
    c = r.standard_normal(4)
    b = oracle.matvec(A, W @ c)
    ctx = _ctx(P, cfg.n, cfg.rowptr, cfg.colind, vals, rank_max=8)
    ctx.set_basis(_dev(W))
    x = _dev(np.zeros(cfg.n))
    st = ctx.solve(_dev(b), x, 1e-10)
    assert st.path == 1 and st.iters == 0 and st.status == 0
    assert _relerr(_host(x), W @ c) <= 1e-12
    # a dependent column: the factor keeps 3, RANK_REDUCED, still solved
    Wd = W.copy()
    Wd[:, 3] = Wd[:, 0] - 2.0 * Wd[:, 1]
    b = cfg.rhs(2)
    xo, so = oracle.aug_pcg(A, b, np.zeros(cfg.n), Wd, tol=1e-10, maxit=20000)
    ctx.set_basis(_dev(Wd))
    x = _dev(np.zeros(cfg.n))
    st = ctx.solve(_dev(b), x, 1e-10)
    assert st.path == 1 and st.status == 2 and st.rank == 3
    assert abs(st.iters - so.iters) <= 1
    assert np.linalg.norm(b - oracle.matvec(A, _host(x))) / np.linalg.norm(b) <= 1e-10 * 1.01
    # a second solve reuses the factor: bitwise the same solution
    x2 = _dev(np.zeros(cfg.n))
    st2 = ctx.solve(_dev(b), x2, 1e-10)
    assert st2.setup_ms == 0.0 and st2.rank == 3 and np.array_equal(_host(x2), _host(x))
    # six columns: beyond the kernel's registers, the multi-kernel loop runs
    W6 = r.standard_normal((cfg.n, 6))
    xo, so = oracle.aug_pcg(A, b, np.zeros(cfg.n), W6, tol=1e-10, maxit=20000)
    ctx.set_basis(_dev(W6))
    x = _dev(np.zeros(cfg.n))
    st = ctx.solve(_dev(b), x, 1e-10)
    assert st.path == 0 and st.rank == 6 and abs(st.iters - so.iters) <= 1
