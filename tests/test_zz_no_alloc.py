"""podcg_solve_noalloc (the small-system solve whose scratch is a static
device array of the library) through the C ABI, against podcg_solve on the
same context and inputs: two calls in a row, the second on a smaller system,
then one with no basis.  Both take the one-workgroup path with the same
kernels, so the solutions and statistics agree bitwise; the solutions also
meet the tolerance by the oracle's own residual.  Sizes beyond the limit
are refused with PODCG_ERR_SIZE before anything runs."""

import ctypes as C

import numpy as np
import pytest

import oracle
from problems import config1

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


@pytest.fixture(scope="module")
def P():
    import paper_1512_05820_amd as P
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    P.load()
    return P


def _noalloc(P, ctx, b, x, rtol):
    """Calls podcg_solve_noalloc through the ctypes declaration of the ABI."""
    L = P.load()
    st = P._lib.Stats()
    torch.cuda.synchronize()
    rc = L.podcg_solve_noalloc(ctx._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), float(rtol),
                               C.byref(st))
    return rc, st


def _case(P, N, y, j, seed):
    cfg = config1(N=N)
    vals = cfg.matrix_values(j)
    ctx = P.PodCG(cfg.n, omega=cfg.omega, rank_max=5)
    ctx.set_matrix(_dev(vals), _dev(cfg.rowptr, torch.int32), _dev(cfg.colind, torch.int32))
    W = np.random.Generator(np.random.PCG64(seed)).standard_normal((cfg.n, y)) if y else None
    ctx.set_basis(None if W is None else _dev(W))
    b = _dev(cfg.rhs(j))
    return cfg, vals, ctx, b


@pytest.mark.parametrize("order", ["noalloc_first", "solve_first"])
def test_noalloc_matches_solve_on_two_calls(P, order):
    for N, y, j, seed in ((32, 4, 3, 61), (15, 2, 2, 62), (15, 0, 4, 63)):
        cfg, vals, ctx, b = _case(P, N, y, j, seed)
        x_ref = _dev(np.zeros(cfg.n))
        x_na = _dev(np.zeros(cfg.n))
        if order == "solve_first":
            st_ref = ctx.solve(b, x_ref, cfg.tol)
            rc, st = _noalloc(P, ctx, b, x_na, cfg.tol)
        else:
            rc, st = _noalloc(P, ctx, b, x_na, cfg.tol)
            st_ref = ctx.solve(b, x_ref, cfg.tol)
        assert rc == st_ref.status == 0, (rc, st_ref.status)
        assert st.path == 1 and st_ref.path == 1
        assert (st.iters, st.rank) == (st_ref.iters, st_ref.rank) and st.rank == y
        assert st.true_relres == st_ref.true_relres and st.stage1_relres == st_ref.stage1_relres
        xa, xr = x_na.cpu().numpy(), x_ref.cpu().numpy()
        assert np.array_equal(xa, xr)
        A = oracle.CSR(cfg.rowptr, cfg.colind, vals)
        bh = b.cpu().numpy()
        assert np.linalg.norm(bh - oracle.matvec(A, xa)) / np.linalg.norm(bh) <= cfg.tol * 1.01
        ctx.close()


def test_noalloc_refuses_sizes_beyond_its_limit(P):
    cfg = config1(N=40)                        # 1600 unknowns
    ctx = P.PodCG(cfg.n, rank_max=5)
    ctx.set_matrix(_dev(cfg.matrix_values(1)), _dev(cfg.rowptr, torch.int32), _dev(cfg.colind, torch.int32))
    x = _dev(np.zeros(cfg.n))
    rc, _ = _noalloc(P, ctx, _dev(cfg.rhs(1)), x, cfg.tol)
    assert rc == -7 and "at most 1024 unknowns" in P.load().podcg_last_error(ctx._h).decode()
    assert not torch.any(x).item()
    cfg, vals, ctx, b = _case(P, 16, 0, 1, 64)
    ctx2 = P.PodCG(cfg.n, rank_max=6)
    ctx2.set_matrix(_dev(vals), _dev(cfg.rowptr, torch.int32), _dev(cfg.colind, torch.int32))
    ctx2.set_basis(_dev(np.random.Generator(np.random.PCG64(65)).standard_normal((cfg.n, 6))))
    rc, _ = _noalloc(P, ctx2, b, _dev(np.zeros(cfg.n)), cfg.tol)
    assert rc == -7
