"""Edge cases of the GPU path against the oracle: the widest basis tiers
(17..32 columns), the largest snapshot memory (32), systems of one, two and
a ragged slice of unknowns, and a basis with a dependent column (the Cholesky
pivot rule truncates it and the solve reports RANK_REDUCED)."""

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


def _relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module")
def P():
    import paper_1512_05820_amd as P
    assert torch.cuda.is_available()
    P.load()
    return P


def _ctx(P, n, rowptr, colind, vals, **kw):
    c = P.PodCG(n, **kw)
    c.set_matrix(_dev(vals), _dev(rowptr, torch.int32), _dev(colind, torch.int32))
    return c


@pytest.mark.parametrize("y,projection", [(17, "implicit"), (24, "implicit"), (32, "explicit"), (32, "implicit")])
def test_lockstep_wide_basis_tiers(P, y, projection):
    cfg = config2(N=16, steps=3)
    vals = cfg.matrix_values(2)
    A = oracle.CSR(cfg.rowptr, cfg.colind, vals)
    r = np.random.Generator(np.random.PCG64(90 + y))
    W = r.standard_normal((cfg.n, y))
    b = cfg.rhs(2, r.standard_normal(cfg.n) * 1e-3)
    xo, so = oracle.aug_pcg(A, b, np.zeros(cfg.n), W, tol=1e-10, maxit=20000)
    ctx = _ctx(P, cfg.n, cfg.rowptr, cfg.colind, vals, rank_max=32, maxit=so.iters, projection=projection)
    ctx.set_basis(_dev(W))
    x = _dev(np.zeros(cfg.n))
    st = ctx.solve(_dev(b), x, 0.0)
    print(f"y={y}: iters {st.iters} (oracle {so.iters}) err {_relerr(_host(x), xo):.2e}")
    assert so.status == 0 and st.iters == so.iters and st.rank == y
    assert _relerr(_host(x), xo) <= 1e-10


def test_pod_with_32_snapshots_and_rank_32(P):
    cfg = config1(N=20)
    vals = cfg.matrix_values(1)
    A = oracle.CSR(cfg.rowptr, cfg.colind, vals)
    r = np.random.Generator(np.random.PCG64(95))
    S = r.standard_normal((cfg.n, 32)) @ np.diag(np.logspace(0, -3, 32))
    ctx = _ctx(P, cfg.n, cfg.rowptr, cfg.colind, vals, omega=32, rank_max=32)
    for k in range(32):                        # oldest first: column 31 is the newest
        ctx.push_snapshot(_dev(S[:, k]))
    y = ctx.build_pod()
    w = oracle.idw_weights(32)[::-1].copy()    # weights 2^{1-age}, age 1 = newest
    Wo, lam_o = oracle.pod_evd(A, S, w, 32)
    lam_g = ctx.pod_spectrum()
    assert y == Wo.shape[1]
    assert np.allclose(lam_g[:y], lam_o[:y], rtol=1e-10, atol=1e-12 * lam_o[0])
    Wg = _host(ctx.get_basis())
    D = np.stack([oracle.matvec(A, Wo[:, k]) for k in range(y)], axis=1)
    k = min(y, 6)                               # well-separated leading subspace
    Po = Wo[:, :k] @ (D[:, :k].T)
    Pg = Wg[:, :k] @ (np.stack([oracle.matvec(A, Wg[:, i]) for i in range(k)], axis=1).T)
    assert np.abs(Pg - Po).max() <= 1e-8 * np.abs(Po).max()


@pytest.mark.parametrize("n", [1, 2, 63, 65])
def test_tiny_systems(P, n):
    Ad = tiny.random_spd(n, 50.0, 96 + n) if n > 1 else np.array([[3.0]])
    rowptr, colind, vals = tiny.dense_to_csr(Ad)
    A = oracle.CSR(rowptr, colind, vals)
    r = np.random.Generator(np.random.PCG64(97 + n))
    b = r.standard_normal(n)
    xd = np.linalg.solve(Ad, b)
    ctx = _ctx(P, n, rowptr, colind, vals, omega=3, rank_max=2)
    x = _dev(np.zeros(n))
    st = ctx.solve(_dev(b), x, 1e-12)
    assert st.status == 0 and _relerr(_host(x), xd) <= 1e-10
    # with a one-column basis (the solution itself when n = 1: Stage 1 is exact)
    W = (xd if n == 1 else r.standard_normal(n)).reshape(n, 1)
    ctx.set_basis(_dev(W))
    x = _dev(np.zeros(n))
    st = ctx.solve(_dev(b), x, 1e-12)
    xo, so = oracle.aug_pcg(A, b, np.zeros(n), W, tol=1e-12, maxit=1000)
    assert st.status == 0
    # Alg. 1 ends in at most n - dim(W) steps in exact arithmetic; counts past
    # that bound are set by rounding (loss of orthogonality), so they are
    # compared exactly up to the bound and within a few steps beyond it
    bound = n - 1
    if so.iters <= bound:
        assert abs(st.iters - so.iters) <= 1
    else:
        assert st.iters > bound - 1 and abs(st.iters - so.iters) <= 4
    assert _relerr(_host(x), xd) <= 1e-10
    if n == 1:
        assert st.iters == 0


def test_dependent_basis_column_is_truncated(P):
    cfg = config1(N=16)
    vals = cfg.matrix_values(1)
    A = oracle.CSR(cfg.rowptr, cfg.colind, vals)
    r = np.random.Generator(np.random.PCG64(98))
    W = r.standard_normal((cfg.n, 4))
    W[:, 3] = W[:, 0] - 2.0 * W[:, 1]           # dependent last column
    b = cfg.rhs(1)
    _, G, R, kept = oracle.reduced_setup(A, W)
    assert kept == 3
    xo, so = oracle.aug_pcg(A, b, np.zeros(cfg.n), W, tol=1e-10, maxit=20000)
    ctx = _ctx(P, cfg.n, cfg.rowptr, cfg.colind, vals, rank_max=4)
    ctx.set_basis(_dev(W))
    x = _dev(np.zeros(cfg.n))
    st = ctx.solve(_dev(b), x, 1e-10)
    assert st.status == 2 and st.rank == 3         # RANK_REDUCED, still solved
    assert abs(st.iters - so.iters) <= 1
    res = np.linalg.norm(b - oracle.matvec(A, _host(x))) / np.linalg.norm(b)
    assert res <= 1e-10 * 1.01
