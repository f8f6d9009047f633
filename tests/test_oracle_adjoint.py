"""Pin of the oracle's dense adjoint: central finite differences of the
dense forward (exact solves) agree with the hand-derived gradient."""

import numpy as np

from oracle.adjoint import sequence_gradient
from problems import config5


def _J(cfg, theta, s, w, steps):
    return sequence_gradient(cfg, theta, s, w, steps)[0]


def test_dense_adjoint_matches_finite_differences():
    cfg = config5(N=6, steps=4, n_outputs=20)
    r = np.random.Generator(np.random.PCG64(11))
    w = r.standard_normal((cfg.steps, cfg.outputs.size))
    s = np.full(cfg.n, 1.0) + 0.1 * r.standard_normal(cfg.n)
    J, gth, gs, _ = sequence_gradient(cfg, cfg.theta, s, w, cfg.steps)
    h = 1e-6
    for trial in range(3):
        dth = r.standard_normal(cfg.theta.shape)
        ds = r.standard_normal(cfg.n)
        fd = (_J(cfg, cfg.theta + h * dth, s + h * ds, w, cfg.steps)
              - _J(cfg, cfg.theta - h * dth, s - h * ds, w, cfg.steps)) / (2 * h)
        an = float(np.sum(gth * dth) + gs @ ds)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-12), (fd, an)


def test_only_windowed_cells_receive_gradient():
    cfg = config5(N=5, steps=3, n_outputs=10)
    w = np.ones((cfg.steps, cfg.outputs.size))
    _, gth, _, _ = sequence_gradient(cfg, cfg.theta, np.ones(cfg.n), w, cfg.steps)
    used = np.zeros(cfg.theta.shape, dtype=bool)
    for j in range(1, cfg.steps + 1):
        used[cfg.window(j)] = True
    assert np.all(gth[~used] == 0) and np.any(gth[used] != 0)
