"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Protocol:
  * kernels on identical inputs (SpMV, Stage 1, POD basis): relative error
    <= 1e-12, far inside the 1e-10 the method's FP64 path must meet;
  * lockstep: the GPU runs exactly the oracle's iteration count from the same
    (A, b, xbar, W); solutions agree to 1e-10 relative;
  * closed loop: each side runs its own sequence; every GPU solution meets
    the tolerance by the oracle's own residual, and iteration counts agree
    to within one.
"""

import numpy as np
import pytest

import oracle
from problems import config1, config2, tiny

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


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


@pytest.fixture(scope="module")
def P():
    import paper_1512_05820_amd as P
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    P.load()
    return P


def _ctx(P, n, **kw):
    return P.PodCG(n, **kw)


def _set(ctx, rowptr, colind, vals):
    ctx.set_matrix(_dev(vals), _dev(rowptr, torch.int32), _dev(colind, torch.int32))


def _relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# ------------------------------------------------------------------- kernels

@pytest.mark.parametrize("N,dim", [(32, 2), (23, 2), (3, 2), (21, 3), (41, 3)])
def test_matvec_matches_oracle(P, N, dim):
    cfg = config1(N=N) if dim == 2 else config2(N=N, steps=3)
    vals = cfg.matrix_values(2)
    A = oracle.CSR(cfg.rowptr, cfg.colind, vals)
    x = _rng(N).standard_normal(cfg.n)
    ref = oracle.matvec(A, x)
    ctx = _ctx(P, cfg.n)
    _set(ctx, cfg.rowptr, cfg.colind, vals)
    y = torch.empty(cfg.n, dtype=torch.float64, device="cuda")
    ctx.matvec(_dev(x), y)
    assert _relerr(_host(y), ref) <= 1e-14
    # values-only update keeps the pattern
    ctx.set_matrix(_dev(vals * 2.0))
    ctx.matvec(_dev(x), y)
    assert _relerr(_host(y), 2.0 * ref) <= 1e-14


def test_matvec_general_sparsity_ragged_rows(P):
    r = _rng(3)
    n = 300
    A = np.zeros((n, n))
    for i in range(n):
        k = r.integers(0, 40)
        cols = r.choice(n, size=k, replace=False)
        A[i, cols] = r.standard_normal(k)
    A = A + A.T + np.diag(np.full(n, 50.0))
    rowptr, colind, vals = tiny.dense_to_csr(A)
    x = r.standard_normal(n)
    ctx = _ctx(P, n)
    _set(ctx, rowptr, colind, vals)
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx.matvec(_dev(x), y)
    assert _relerr(_host(y), A @ x) <= 1e-13


def _csr_from_triplets(n, rows, cols, vals, keep_order=False):
    rows, cols, vals = np.asarray(rows), np.asarray(cols), np.asarray(vals, dtype=np.float64)
    order = np.arange(len(rows)) if keep_order else np.lexsort((cols, rows))
    order = order[np.argsort(rows[order], kind="stable")]
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    return np.cumsum(rowptr).astype(np.int32), cols.astype(np.int32), vals


def test_matvec_mixes_all_three_column_storages(P):
    """A banded pattern (offsets -301, -1, 0, 1, 301) whose slices take the
    per-slice offset table; slices where two rows carry different extra
    offsets cannot (their offset union is wider than the slice) and keep
    16-bit offsets, or 32-bit columns when an offset exceeds 16 bits; a ragged
    last slice (n = 90,001)."""
    r = _rng(5)
    n = 90_001
    rows, cols, vals = [], [], []
    for i in range(n):
        for d in (-301, -1, 0, 1, 301):
            j = i + d
            if 0 <= j < n:
                rows.append(i)
                cols.append(j)
                vals.append(10.0 if d == 0 else -1.0 + 0.1 * r.standard_normal())

    def couple(i, d, v):                 # symmetric pair (i, i + d), (i + d, i)
        rows.extend([i, i + d])
        cols.extend([i + d, i])
        vals.extend([v, v])

    for t, i in enumerate(range(640, 20_000, 1280)):   # 32-bit: offsets 60,000 and 60,003 in one slice
        couple(i, 60_000, 0.5)
        couple(i + 1, 60_003, 0.25)
    for i in range(30_080, 40_000, 1280):               # 16-bit: offsets 150 and 170 in one slice
        couple(i, 150, 0.5)
        couple(i + 1, 170, 0.25)
    rowptr, colind, vals = _csr_from_triplets(n, rows, cols, vals)
    A = oracle.CSR(rowptr, colind, vals)
    x = r.standard_normal(n)
    ctx = _ctx(P, n)
    _set(ctx, rowptr, colind, vals)
    f = ctx.format_counts()
    print(f)
    assert f["int32"] >= 8 and f["offset16"] >= 8 and f["table"] >= 1000
    assert sum(f.values()) == (n + 63) // 64
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx.matvec(_dev(x), y)
    assert _relerr(_host(y), oracle.matvec(A, x)) <= 1e-14


@pytest.mark.parametrize("N,dim", [(24, 3), (20, 2), (5, 3)])
def test_stencil_slices_use_offset_tables(P, N, dim):
    """Every slice of a 2-D or 3-D stencil stores one offset table (boundary
    rows hold zero-valued slots for their missing neighbours), and the product
    and a full solve are unchanged."""
    cfg = config1(N=N) if dim == 2 else config2(N=N, steps=2)
    vals = cfg.matrix_values(1)
    A = oracle.CSR(cfg.rowptr, cfg.colind, vals)
    ctx = _ctx(P, cfg.n)
    _set(ctx, cfg.rowptr, cfg.colind, vals)
    f = ctx.format_counts()
    assert f == {"int32": 0, "offset16": 0, "table": (cfg.n + 63) // 64}
    x = _rng(N + 7).standard_normal(cfg.n)
    y = torch.empty(cfg.n, dtype=torch.float64, device="cuda")
    ctx.matvec(_dev(x), y)
    assert _relerr(_host(y), oracle.matvec(A, x)) <= 1e-14
    b = cfg.rhs(1, None)
    xo, so = oracle.plain_pcg(A, b, np.zeros(cfg.n), tol=1e-10, maxit=5000)
    xg = _dev(np.zeros(cfg.n))
    st = ctx.solve_plain(_dev(b), xg, 1e-10)
    assert st.status == 0 and abs(st.iters - so.iters) <= 1
    assert _relerr(_host(xg), xo) <= 1e-9


@pytest.mark.parametrize("w", [1, 2, 3, 4, 5, 6, 7, 8])
def test_offset_tables_of_every_width(P, w):
    """Banded matrices whose slices all draw on one list of w offsets (the
    first w of 0, 1, -1, 5, -5, 64, -64, 300), n = 5,000 with a ragged last
    slice: every slice stores an offset table and takes the path of its exact
    width.  The product matches the oracle's; for the symmetric lists (odd w)
    plain and augmented solves (random 3-column basis) match the oracle's
    iterates, which exercises the loop SpMV and the FP32 one of mixed
    precision."""
    n = 5_000
    offs = [0, 1, -1, 5, -5, 64, -64, 300][:w]
    r = _rng(40 + w)
    rows, cols, vals = [], [], []
    sym = {}
    for i in range(n):
        for d in offs:
            j = i + d
            if 0 <= j < n:
                if d == 0:
                    v = 4.0 * len(offs) + r.random()
                else:
                    key = (min(i, j), max(i, j))
                    v = sym.setdefault(key, -0.5 - 0.5 * r.random())
                rows.append(i)
                cols.append(j)
                vals.append(v)
    rowptr, colind, vals = _csr_from_triplets(n, rows, cols, vals)
    A = oracle.CSR(rowptr, colind, vals)
    ctx = _ctx(P, n, rank_max=3)
    _set(ctx, rowptr, colind, vals)
    f = ctx.format_counts()
    assert f == {"int32": 0, "offset16": 0, "table": (n + 63) // 64}
    x = r.standard_normal(n)
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx.matvec(_dev(x), y)
    assert _relerr(_host(y), oracle.matvec(A, x)) <= 1e-14
    if w % 2 == 0:
        return
    b = r.standard_normal(n)
    xo, so = oracle.plain_pcg(A, b, np.zeros(n), tol=1e-10, maxit=5000)
    xg = _dev(np.zeros(n))
    st = ctx.solve_plain(_dev(b), xg, 1e-10)
    assert st.status == 0 and abs(st.iters - so.iters) <= 1
    assert _relerr(_host(xg), xo) <= 1e-9
    W = r.standard_normal((n, 3))
    xa, sa = oracle.aug_pcg(A, b, np.zeros(n), W, 1e-10, 5000)
    ctx.set_basis(_dev(W))
    xg = _dev(np.zeros(n))
    st = ctx.solve(_dev(b), xg, 1e-10)
    assert st.status == 0 and abs(st.iters - sa.iters) <= 1
    assert _relerr(_host(xg), xa) <= 1e-9
    mixed = _ctx(P, n, rank_max=3, precision="mixed")
    _set(mixed, rowptr, colind, vals)
    mixed.set_basis(_dev(W))
    xm = _dev(np.zeros(n))
    st = mixed.solve(_dev(b), xm, 1e-10)
    assert st.status == 0
    assert np.linalg.norm(b - oracle.matvec(A, _host(xm))) / np.linalg.norm(b) <= 1.01e-10


def test_unsorted_and_duplicate_rows_keep_per_entry_columns(P):
    """A row whose columns are out of order, and a row with a repeated column
    (two entries that add up), make their slices keep per-entry columns; the
    product still matches the oracle's."""
    cfg = config1(N=20)
    vals = cfg.matrix_values(1)
    rowptr, colind = cfg.rowptr.copy(), cfg.colind.copy()
    i = 70                                        # reverse the columns of row 70 (slice 1)
    a, b = rowptr[i], rowptr[i + 1]
    colind[a:b] = colind[a:b][::-1].copy()
    vals = vals.copy()
    vals[a:b] = vals[a:b][::-1].copy()
    rows = np.repeat(np.arange(cfg.n), np.diff(rowptr))
    rl, cl, vl = list(rows), list(colind), list(vals)
    j = 300                                       # split the diagonal of row 300 (slice 4) in two
    k = rowptr[j] + list(colind[rowptr[j]:rowptr[j + 1]]).index(j)
    rl.append(j)
    cl.append(j)
    vl.append(0.25 * vl[k])
    vl[k] *= 0.75
    rp, ci, vv = _csr_from_triplets(cfg.n, rl, cl, vl, keep_order=True)
    A = oracle.CSR(rp, ci, vv)
    ctx = _ctx(P, cfg.n)
    _set(ctx, rp, ci, vv)
    f = ctx.format_counts()
    assert f["offset16"] == 2 and f["table"] == (cfg.n + 63) // 64 - 2
    x = _rng(71).standard_normal(cfg.n)
    y = torch.empty(cfg.n, dtype=torch.float64, device="cuda")
    ctx.matvec(_dev(x), y)
    assert _relerr(_host(y), oracle.matvec(A, x)) <= 1e-14


def test_stage1_matches_closed_form_projection(P):
    cfg = config2(N=19, steps=3)
    vals = cfg.matrix_values(1)
    A = oracle.CSR(cfg.rowptr, cfg.colind, vals)
    r = _rng(5)
    W = r.standard_normal((cfg.n, 6))
    b = r.standard_normal(cfg.n)
    xbar = r.standard_normal(cfg.n)
    xo, so = oracle.aug_pcg(A, b, xbar, W, tol=0.0, maxit=0)
    ctx = _ctx(P, cfg.n, rank_max=6, maxit=0)
    _set(ctx, cfg.rowptr, cfg.colind, vals)
    ctx.set_basis(_dev(W))
    x = _dev(xbar)
    st = ctx.solve(_dev(b), x, 0.0)
    assert st.iters == 0 and st.status == 1 and st.rank == 6
    xg = _host(x)
    assert _relerr(xg, xo) <= 1e-12
    res = b - oracle.matvec(A, xg)
    assert np.linalg.norm(W.T @ res) <= 1e-10 * np.linalg.norm(W) * np.linalg.norm(b)
    assert abs(st.stage1_relres - so.stage1_relres) <= 1e-9 * so.stage1_relres


def test_reduced_matrix_and_inverse(P):
    cfg = config2(N=17, steps=3)
    vals = cfg.matrix_values(1)
    A = oracle.CSR(cfg.rowptr, cfg.colind, vals)
    W = _rng(6).standard_normal((cfg.n, 5))
    _, G, R, kept = oracle.reduced_setup(A, W)
    ctx = _ctx(P, cfg.n, rank_max=5)
    _set(ctx, cfg.rowptr, cfg.colind, vals)
    ctx.set_basis(_dev(W))
    Gg, Gi = ctx.get_reduced()
    assert kept == 5 and Gg.shape == (5, 5)
    assert np.allclose(Gg, G, rtol=1e-13, atol=1e-13 * np.abs(G).max())
    assert np.allclose(Gi @ G, np.eye(5), atol=1e-11)


def test_pod_basis_matches_oracle_subspace(P):
    cfg = config2(N=18, steps=4)
    vals = cfg.matrix_values(2)
    A = oracle.CSR(cfg.rowptr, cfg.colind, vals)
    r = _rng(7)
    snaps = [r.standard_normal(cfg.n) for _ in range(7)]     # pushed oldest first
    S_recent_first = np.stack(snaps[::-1], axis=1)
    Wo, lam_o = oracle.pod_evd(A, S_recent_first, oracle.idw_weights(7), 5)
    ctx = _ctx(P, cfg.n, omega=5, rank_max=5)                 # ring keeps the last 5
    _set(ctx, cfg.rowptr, cfg.colind, vals)
    for s in snaps:
        ctx.push_snapshot(_dev(s))
    y = ctx.build_pod()
    Wo5, lam5 = oracle.pod_evd(A, np.stack(snaps[::-1][:5], axis=1), oracle.idw_weights(5), 5)
    assert y == Wo5.shape[1] == 5
    lam_g = ctx.pod_spectrum()
    assert np.allclose(lam_g, lam5, rtol=1e-11, atol=1e-13 * lam5[0])
    Wg = _host(ctx.get_basis())
    for i in range(y):     # columns agree up to the eigenvector sign convention
        s = np.sign(Wg[:, i] @ Wo5[:, i])
        assert _relerr(s * Wg[:, i], Wo5[:, i]) <= 1e-9
    D = cfg.fv.dense(vals)
    assert np.allclose(Wg.T @ D @ Wg, np.eye(y), atol=1e-10)


def test_pod_rank_cut_on_duplicate_snapshots(P):
    cfg = config1(N=16)
    vals = cfg.matrix_values(1)
    r = _rng(8)
    a, b = r.standard_normal(cfg.n), r.standard_normal(cfg.n)
    ctx = _ctx(P, cfg.n, omega=5, rank_max=4)
    _set(ctx, cfg.rowptr, cfg.colind, vals)
    for s in (a, b, a, 2 * b, a + b):
        ctx.push_snapshot(_dev(s))
    assert ctx.build_pod() == 2


# ------------------------------------------------------------------- solves

def _lockstep(P, cfg, vals, b, xbar, W, tol, maxit=20000, projection="implicit"):
    A = oracle.CSR(cfg.rowptr, cfg.colind, vals)
    xo, so = oracle.aug_pcg(A, b, xbar, W, tol=tol, maxit=maxit)
    y = 0 if W is None else W.shape[1]
    ctx = _ctx(P, cfg.n, rank_max=max(y, 1), maxit=so.iters, projection=projection)
    _set(ctx, cfg.rowptr, cfg.colind, vals)
    ctx.set_basis(None if W is None else _dev(W))
    x = _dev(xbar)
    st = ctx.solve(_dev(b), x, 0.0)
    return xo, so, _host(x), st


@pytest.mark.parametrize("use_basis,projection", [(False, "implicit"), (True, "explicit"), (True, "implicit")])
def test_lockstep_config1(P, use_basis, projection):
    cfg = config1()
    vals = cfg.matrix_values(3)
    b = cfg.rhs(3)
    W = _rng(9).standard_normal((cfg.n, 4)) if use_basis else None
    xo, so, xg, st = _lockstep(P, cfg, vals, b, np.zeros(cfg.n), W, cfg.tol, projection=projection)
    assert so.status == 0 and st.iters == so.iters
    assert _relerr(xg, xo) <= 1e-10


@pytest.mark.parametrize("projection", ["explicit", "implicit"])
@pytest.mark.parametrize("N", [24, 33])
def test_lockstep_config2_small(P, N, projection):
    cfg = config2(N=N, steps=4)
    vals = cfg.matrix_values(2)
    r = _rng(N)
    b = cfg.rhs(2, r.standard_normal(cfg.n) * 1e-3)
    W = r.standard_normal((cfg.n, 10))
    xo, so, xg, st = _lockstep(P, cfg, vals, b, np.zeros(cfg.n), W, cfg.tol, projection=projection)
    assert so.status == 0 and st.iters == so.iters
    assert _relerr(xg, xo) <= 1e-10


def _gpu_sequence(P, cfg, steps, method="aug", warm=False, projection="implicit", wait=True):
    ctx = _ctx(P, cfg.n, omega=cfg.omega, rank_max=cfg.rank, projection=projection)
    rowptr, colind = _dev(cfg.rowptr, torch.int32), _dev(cfg.colind, torch.int32)
    out = []
    x_prev = None
    for j in range(1, steps + 1):
        vals = cfg.matrix_values(j)
        if j == 1:
            ctx.set_matrix(_dev(vals), rowptr, colind)
        else:
            ctx.set_matrix(_dev(vals))
        b = cfg.rhs(j, None if x_prev is None else x_prev)
        if method == "aug" or not warm or x_prev is None:
            xbar = np.zeros(cfg.n)
        else:
            xbar = x_prev
        x = _dev(xbar)
        st = ctx.solve(_dev(b), x, cfg.tol) if method == "aug" else ctx.solve_plain(_dev(b), x, cfg.tol)
        xh = _host(x)
        if method == "aug":
            ctx.push_snapshot(_dev(xh - xbar))
            ctx.build_pod(wait=wait)
        out.append((st.as_dict(), xh, b, vals))
        x_prev = xh
    return out


@pytest.mark.parametrize("which", ["c1", "c2_small"])
def test_pod_build_without_waiting_matches(P, which):
    """build_pod with no rank output returns without waiting for the GPU; the
    next solve takes the rank then.  Same kernels in the same order, so the
    sequence must match the waiting build bit for bit (config 1 runs the
    one-workgroup solve, the 26^3 family the multi-kernel loop)."""
    cfg = config1() if which == "c1" else config2(N=26, steps=6)
    a = _gpu_sequence(P, cfg, cfg.steps, wait=True)
    b = _gpu_sequence(P, cfg, cfg.steps, wait=False)
    for (sa, xa, _, _), (sb, xb, _, _) in zip(a, b):
        assert sa["iters"] == sb["iters"] and sa["rank"] == sb["rank"]
        assert np.array_equal(xa, xb)
    assert max(s["rank"] for s, _, _, _ in b) > 0


@pytest.mark.parametrize("which,projection", [("c1", "implicit"), ("c1_r2", "implicit"),
                                              ("c2_small", "explicit"), ("c2_small", "implicit")])
def test_closed_loop_sequence(P, which, projection):
    if which == "c1":
        cfg = config1()
    elif which == "c1_r2":
        cfg = config1(variant="r2", steps=6)
    else:
        cfg = config2(N=26, steps=8)
    orc = oracle.run_sequence(cfg, "aug")
    gpu = _gpu_sequence(P, cfg, cfg.steps, projection=projection)
    for o, (st, x, b, vals) in zip(orc, gpu):
        A = oracle.CSR(cfg.rowptr, cfg.colind, vals)
        tr = np.linalg.norm(b - oracle.matvec(A, x)) / np.linalg.norm(b)
        assert tr <= cfg.tol * 1.01, (o["j"], tr)
        assert st["status"] in (0, 2)
        assert abs(st["iters"] - o["iters"]) <= 1, (o["j"], st["iters"], o["iters"])
        assert st["rank"] == o["rank"]


def test_plain_pcg_warm_and_cold(P):
    cfg = config2(N=20, steps=4)
    for warm in (False, True):
        orc = oracle.run_sequence(cfg, "plain", warm=warm)
        gpu = _gpu_sequence(P, cfg, cfg.steps, method="plain", warm=warm)
        for o, (st, x, b, vals) in zip(orc, gpu):
            assert abs(st["iters"] - o["iters"]) <= 1
            assert st["true_relres"] <= cfg.tol * 1.01


def test_deterministic_bitwise(P):
    cfg = config2(N=22, steps=3)
    vals = cfg.matrix_values(1)
    b = cfg.rhs(1, None)
    W = _rng(10).standard_normal((cfg.n, 8))
    xs = []
    for _ in range(2):
        ctx = _ctx(P, cfg.n, rank_max=8)
        _set(ctx, cfg.rowptr, cfg.colind, vals)
        ctx.set_basis(_dev(W))
        x = _dev(np.zeros(cfg.n))
        ctx.solve(_dev(b), x, 1e-10)
        xs.append(_host(x))
    assert np.array_equal(xs[0], xs[1])


def test_cleared_basis_after_a_sequence_is_plain_pcg(P):
    """Clearing the basis after a sequence must give exactly a fresh plain solve."""
    cfg = config2(N=16, steps=4)
    seq = _gpu_sequence(P, cfg, 4)
    assert seq[-1][0]["rank"] > 0
    vals = cfg.matrix_values(1)
    b = cfg.rhs(1, None)
    fresh = _ctx(P, cfg.n, omega=cfg.omega, rank_max=cfg.rank)
    _set(fresh, cfg.rowptr, cfg.colind, vals)
    x0 = _dev(np.zeros(cfg.n))
    st0 = fresh.solve(_dev(b), x0, cfg.tol)
    ctx = _ctx(P, cfg.n, omega=cfg.omega, rank_max=cfg.rank)
    _set(ctx, cfg.rowptr, cfg.colind, cfg.matrix_values(3))
    W = _rng(14).standard_normal((cfg.n, 3))
    ctx.set_basis(_dev(W))
    ctx.solve(_dev(b), _dev(np.zeros(cfg.n)), cfg.tol)
    ctx.set_basis(None)
    ctx.reset_snapshots()
    ctx.set_matrix(_dev(vals))
    x1 = _dev(np.zeros(cfg.n))
    st1 = ctx.solve(_dev(b), x1, cfg.tol)
    assert st1.rank == 0 and st1.iters == st0.iters
    assert np.array_equal(_host(x1), _host(x0))


# ------------------------------------------------------------------- edge cases

def test_error_paths(P):
    cfg = config1(N=12)
    n = cfg.n
    vals = cfg.matrix_values(1)
    ctx = _ctx(P, n, maxit=5)
    x = _dev(np.zeros(n))
    with pytest.raises(P.PodCGError) as e:
        ctx.solve(_dev(np.ones(n)), x, 1e-8)
    assert e.value.code == -6                     # no matrix
    bad = cfg.colind.copy()
    bad[5] = n + 3
    with pytest.raises(P.PodCGError) as e:
        _set(ctx, cfg.rowptr, bad, vals)
    assert e.value.code == -1                     # column out of range, caught before use
    neg = vals.copy()
    neg[cfg.rowptr[4] + list(cfg.colind[cfg.rowptr[4]:cfg.rowptr[5]]).index(4)] = -1.0
    with pytest.raises(P.PodCGError) as e:
        _set(ctx, cfg.rowptr, cfg.colind, neg)
    assert e.value.code == -4
    _set(ctx, cfg.rowptr, cfg.colind, vals)
    bn = np.ones(n)
    bn[7] = np.nan
    with pytest.raises(P.PodCGError) as e:
        ctx.solve(_dev(bn), x, 1e-8)
    assert e.value.code == -5
    x = _dev(np.zeros(n))
    st = ctx.solve(_dev(np.ones(n)), x, 1e-14)    # cap of 5 iterations
    assert st.status == 1 and st.iters == 5
    x = _dev(np.zeros(n))
    st = ctx.solve(_dev(np.zeros(n)), x, 1e-8)    # zero rhs, zero guess
    assert st.status == 0 and st.iters == 0
    assert not np.any(_host(x))
    assert ctx.build_pod() == 0                   # no snapshots yet


def test_indefinite_matrix_is_reported(P):
    # symmetric, positive diagonal, but indefinite: (A p, p) <= 0 shows up
    n = 64
    A = np.eye(n) * 1.0
    for i in range(n - 1):
        A[i, i + 1] = A[i + 1, i] = 0.9
    A[10, 11] = A[11, 10] = 5.0
    rowptr, colind, vals = tiny.dense_to_csr(A)
    orc = oracle.plain_pcg(oracle.CSR(rowptr, colind, vals), np.ones(n), np.zeros(n), 1e-12, 200)[1]
    import paper_1512_05820_amd as P2
    ctx = P2.PodCG(n, maxit=200)
    ctx.set_matrix(_dev(vals), _dev(rowptr, torch.int32), _dev(colind, torch.int32))
    if orc.status == oracle.ERR_NOT_SPD:
        with pytest.raises(P2.PodCGError) as e:
            ctx.solve(_dev(np.ones(n)), _dev(np.zeros(n)), 1e-12)
        assert e.value.code == -4


def test_exact_recovery_zero_iterations(P):
    cfg = config2(N=15, steps=3)
    vals = cfg.matrix_values(1)
    A = oracle.CSR(cfg.rowptr, cfg.colind, vals)
    W = _rng(11).standard_normal((cfg.n, 4))
    c = _rng(12).standard_normal(4)
    b = oracle.matvec(A, W @ c)
    ctx = _ctx(P, cfg.n, rank_max=4)
    _set(ctx, cfg.rowptr, cfg.colind, vals)
    ctx.set_basis(_dev(W))
    x = _dev(np.zeros(cfg.n))
    st = ctx.solve(_dev(b), x, 1e-10)
    assert st.iters == 0 and st.status == 0
    assert _relerr(_host(x), W @ c) <= 1e-12


def test_implicit_and_explicit_direction_forms_agree(P):
    """The implicit form (p = pt - W nu, x = xt - W xi) against the explicit
    form of Alg. 1 on a POD basis built from a sequence: same iteration
    counts, solutions within 1e-12; a solve stopped by the iteration cap
    returns a consistent x (the reported true residual is the oracle's
    residual of the returned x)."""
    cfg = config2(N=30, steps=6)
    rp, ci = _dev(cfg.rowptr, torch.int32), _dev(cfg.colind, torch.int32)
    ctx = {f: _ctx(P, cfg.n, omega=cfg.omega, rank_max=cfg.rank, projection=f) for f in ("explicit", "implicit")}
    capped = {f: _ctx(P, cfg.n, omega=cfg.omega, rank_max=cfg.rank, projection=f, maxit=7)
              for f in ("explicit", "implicit")}
    x_prev = None
    for j in range(1, cfg.steps + 1):
        vals = cfg.matrix_values(j)
        A = oracle.CSR(cfg.rowptr, cfg.colind, vals)
        b = cfg.rhs(j, x_prev)
        out, cap = {}, {}
        for f in ("explicit", "implicit"):
            for c in (ctx[f], capped[f]):
                if j == 1:
                    c.set_matrix(_dev(vals), rp, ci)
                else:
                    c.set_matrix(_dev(vals))
            x = _dev(np.zeros(cfg.n))
            out[f] = (ctx[f].solve(_dev(b), x, cfg.tol), _host(x))
            xc = _dev(np.zeros(cfg.n))
            cap[f] = (capped[f].solve(_dev(b), xc, 0.0), _host(xc))
        (se, xe), (si, xi) = out["explicit"], out["implicit"]
        assert se.rank == si.rank and se.iters == si.iters, (j, se.iters, si.iters)
        assert _relerr(xi, xe) <= 1e-12
        assert si.true_relres <= cfg.tol * 1.01
        (ce, xce), (ci_, xci) = cap["explicit"], cap["implicit"]
        if si.rank > 0:
            assert ci_.status == 1 and ci_.iters == 7
        assert _relerr(xci, xce) <= 1e-12
        res = np.linalg.norm(b - oracle.matvec(A, xci)) / np.linalg.norm(b)
        assert abs(res - ci_.true_relres) <= 1e-6 * res
        for f in ("explicit", "implicit"):
            ctx[f].push_snapshot(_dev(out[f][1]))
            ctx[f].build_pod()
            capped[f].push_snapshot(_dev(out[f][1]))
            capped[f].build_pod()
        x_prev = xe


@pytest.mark.parametrize("projection", ["implicit", "explicit"])
def test_small_loop_grids_match_the_default_grids(P, projection):
    """Tiny launch grids (SpMV 4, update 3, direction 2 workgroups) make every
    loop kernel walk many slices or load blocks per thread and run the
    direction kernels' remainder loops; along a POD sequence (and for warm
    plain PCG) the solutions agree with the default grids' to rounding, with
    iteration counts within one, and meet the tolerance by the oracle's
    residual."""
    cfg = config2(N=24, steps=4)
    rp, ci = _dev(cfg.rowptr, torch.int32), _dev(cfg.colind, torch.int32)
    kw = dict(omega=cfg.omega, rank_max=cfg.rank, projection=projection)
    ctx = {"default": _ctx(P, cfg.n, **kw),
           "small": _ctx(P, cfg.n, spmv_grid=4, update_grid=3, dir_grid=2, **kw)}
    x_prev = None
    for j in range(1, cfg.steps + 1):
        vals = cfg.matrix_values(j)
        A = oracle.CSR(cfg.rowptr, cfg.colind, vals)
        b = cfg.rhs(j, x_prev)
        out, outp = {}, {}
        for name, c in ctx.items():
            if j == 1:
                c.set_matrix(_dev(vals), rp, ci)
            else:
                c.set_matrix(_dev(vals))
            x = _dev(np.zeros(cfg.n))
            out[name] = (c.solve(_dev(b), x, cfg.tol), _host(x))
            xp = _dev(np.zeros(cfg.n) if x_prev is None else x_prev)
            outp[name] = (c.solve_plain(_dev(b), xp, cfg.tol), _host(xp))
        for o in (out, outp):
            (sd, xd), (ss, xs) = o["default"], o["small"]
            assert sd.status == 0 and ss.status == 0
            assert abs(sd.iters - ss.iters) <= 1 and sd.rank == ss.rank
            assert _relerr(xs, xd) <= 1e-9
            assert np.linalg.norm(b - oracle.matvec(A, xs)) / np.linalg.norm(b) <= cfg.tol * 1.01
        for name, c in ctx.items():
            c.push_snapshot(_dev(out[name][1]))
            c.build_pod()
        x_prev = out["default"][1]


# ------------------------------------------------------------------- full size

def test_full_size_config2_matvec_and_first_solves(P):
    """128^3 (n = 2,097,152): every row of A p against the oracle, then two
    systems of the sequence: the GPU answers meet 1e-10 by the oracle's own
    residual, and the iteration counts agree with the oracle's."""
    cfg = config2()
    vals1 = cfg.matrix_values(1)
    A1 = oracle.CSR(cfg.rowptr, cfg.colind, vals1)
    x = _rng(13).standard_normal(cfg.n)
    ctx = _ctx(P, cfg.n, omega=cfg.omega, rank_max=cfg.rank)
    _set(ctx, cfg.rowptr, cfg.colind, vals1)
    y = torch.empty(cfg.n, dtype=torch.float64, device="cuda")
    ctx.matvec(_dev(x), y)
    assert _relerr(_host(y), oracle.matvec(A1, x)) <= 1e-14

    orc = oracle.run_sequence(cfg, "aug", steps=2)
    b = cfg.rhs(1, None)
    xg = _dev(np.zeros(cfg.n))
    st = ctx.solve(_dev(b), xg, cfg.tol)
    x1 = _host(xg)
    assert abs(st.iters - orc[0]["iters"]) <= 1
    assert np.linalg.norm(b - oracle.matvec(A1, x1)) <= cfg.tol * np.linalg.norm(b) * 1.01
    ctx.push_snapshot(xg)
    assert ctx.build_pod() == 1
    vals2 = cfg.matrix_values(2)
    ctx.set_matrix(_dev(vals2))
    b2 = cfg.rhs(2, x1)
    xg2 = _dev(np.zeros(cfg.n))
    st2 = ctx.solve(_dev(b2), xg2, cfg.tol)
    A2 = oracle.CSR(cfg.rowptr, cfg.colind, vals2)
    x2 = _host(xg2)
    assert st2.rank == 1 and abs(st2.iters - orc[1]["iters"]) <= 1
    assert np.linalg.norm(b2 - oracle.matvec(A2, x2)) <= cfg.tol * np.linalg.norm(b2) * 1.01
