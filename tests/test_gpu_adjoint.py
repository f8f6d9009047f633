"""Differentiation of a recycled diffusion sequence on the GPU (config-5 family).

The gradient of J = sum_j w_j . (C x_j) with respect to the log-coefficient
field theta and the source s comes from adjoint solves in libpodcg (Stage 1 +
augmented PCG with the same recycled bases, recovered by checkpoint replay)
and torch autograd of the differentiable assembly.  It is checked against
the oracle's dense adjoint and against central finite differences.
"""

import numpy as np
import pytest

from oracle.adjoint import sequence_gradient
from problems import config5
from problems.fv_torch import FVDiffusionTorch

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _setup(N, steps, ce, tol=1e-12, n_out=64, basis="forward"):
    import paper_1512_05820_amd as P
    from paper_1512_05820_amd.adjoint import RecycledSequence, SequenceSpec
    cfg = config5(N=N, steps=steps, checkpoint_every=ce, n_outputs=n_out, omega=5, rank=4, tol=tol)
    fvt = FVDiffusionTorch(cfg.fv, "cuda")
    outs = torch.from_numpy(cfg.outputs).cuda()

    def assemble(j, params):
        th = params[0]
        return fvt.values(torch.exp(th[cfg.window(j)]), shift=1.0 / cfg.dt)

    def rhs(j, x_prev, params):
        s = params[1]
        return s.clone() if x_prev is None else s + x_prev / cfg.dt

    def output(j, x):
        return x[outs]

    spec = SequenceSpec(steps, assemble, rhs, output, tol, ce, adjoint_basis=basis)
    mk = lambda: P.PodCG(cfg.n, omega=cfg.omega, rank_max=cfg.rank, maxit=50000)
    solver, adj = mk(), mk()
    v0 = torch.from_numpy(cfg.matrix_values(1)).cuda()
    rp, ci = torch.from_numpy(cfg.rowptr).cuda(), torch.from_numpy(cfg.colind).cuda()
    solver.set_matrix(v0, rp, ci)
    adj.set_matrix(v0, rp, ci)
    return cfg, spec, solver, adj, RecycledSequence


def _run(cfg, spec, solver, adj, RS, theta, s, w):
    th = torch.from_numpy(theta).cuda().requires_grad_(True)
    sv = torch.from_numpy(s).cuda().requires_grad_(True)
    q = RS.apply(solver, adj, spec, th, sv)
    J = (q * torch.from_numpy(w).cuda()).sum()
    J.backward()
    return float(J), th.grad.cpu().numpy(), sv.grad.cpu().numpy()


@pytest.mark.parametrize("basis", ["forward", "adjoint", "none"])
def test_gradient_matches_dense_adjoint_16cube(basis):
    cfg, spec, solver, adj, RS = _setup(16, 8, 3, basis=basis)
    r = np.random.Generator(np.random.PCG64(21))
    w = r.standard_normal((cfg.steps, cfg.outputs.size))
    s = np.full(cfg.n, 1.0)
    J, gth, gs = _run(cfg, spec, solver, adj, RS, cfg.theta, s, w)
    Jo, gth_o, gs_o, _ = sequence_gradient(cfg, cfg.theta, s, w, cfg.steps)
    e_t = np.linalg.norm(gth - gth_o) / np.linalg.norm(gth_o)
    e_s = np.linalg.norm(gs - gs_o) / np.linalg.norm(gs_o)
    print(f"[{basis}] J {J:.12e} oracle {Jo:.12e}; dJ/dtheta rel err {e_t:.2e}; dJ/ds rel err {e_s:.2e}")
    assert abs(J - Jo) <= 1e-10 * abs(Jo)
    assert e_t <= 1e-8 and e_s <= 1e-8


def test_gradient_matches_central_differences():
    cfg, spec, solver, adj, RS = _setup(12, 6, 4)
    r = np.random.Generator(np.random.PCG64(22))
    w = r.standard_normal((cfg.steps, cfg.outputs.size))
    s = np.full(cfg.n, 1.0)
    J, gth, gs = _run(cfg, spec, solver, adj, RS, cfg.theta, s, w)
    h = 1e-6
    for trial in range(2):
        dth = r.standard_normal(cfg.theta.shape)
        ds = r.standard_normal(cfg.n)
        Jp = _run(cfg, spec, solver, adj, RS, cfg.theta + h * dth, s + h * ds, w)[0]
        Jm = _run(cfg, spec, solver, adj, RS, cfg.theta - h * dth, s - h * ds, w)[0]
        fd = (Jp - Jm) / (2 * h)
        an = float(np.sum(gth * dth) + gs @ ds)
        print(f"directional derivative: adjoint {an:.10e} central FD {fd:.10e}")
        assert abs(fd - an) <= 1e-5 * abs(an)


def test_checkpoint_interval_does_not_change_the_gradient():
    res = []
    for ce in (2, 5, 100):
        cfg, spec, solver, adj, RS = _setup(10, 6, ce)
        w = np.ones((cfg.steps, cfg.outputs.size))
        res.append(_run(cfg, spec, solver, adj, RS, cfg.theta, np.ones(cfg.n), w))
    for J, gth, gs in res[1:]:
        assert abs(J - res[0][0]) <= 1e-12 * abs(res[0][0])
        assert np.linalg.norm(gth - res[0][1]) <= 1e-9 * np.linalg.norm(res[0][1])
        assert np.linalg.norm(gs - res[0][2]) <= 1e-9 * np.linalg.norm(res[0][2])
