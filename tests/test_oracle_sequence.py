"""Pins of the oracle's sequence driver: which snapshots feed each POD, in
which order, with which weight, centred how.

The expected basis W_{j+1} is rebuilt here without the oracle.  Each system
is solved densely (numpy.linalg.solve), the snapshots are the last omega
centred solutions s_i = x_{j+1-i} - xbar_{j+1-i} (i = 1 the newest), weighted by
the inverse-distance weights 2^{1-i} (Section 3.3), and the POD in the metric
A_j follows its definition (Eqs. (podOpt)-(podOrth)): the eigenvectors of
diag(g) S^T A_j S diag(g) by numpy.linalg.eigh, W = S diag(g) V Sigma^{-1}.
The A_j-orthogonal projectors W W^T A_j of the two bases must agree.

The sequence has omega = 3 and 6 systems, so the ring evicts, and rank 2 <
omega, so the weights decide the kept subspace.  Altered copies of the driver
(weights reversed, a ring of omega + 1, snapshots not centred, oldest snapshot
weighted most) must fail the pin.
"""

import os
import types

import numpy as np
import pytest

import oracle
from problems.exact import exact2d

SEQ_SRC = os.path.join(os.path.dirname(oracle.__file__), "sequence.py")


def _cfg():
    return exact2d(N=10, steps=6, omega=3, rank=2, tol=1e-13)


def _expected_bases(cfg, xbar_mode):
    """W_{j+1} for j = 1..steps from dense solves and the POD definition."""
    out = []
    snaps = []
    x_prev = None
    for j in range(1, cfg.steps + 1):
        A = cfg.fv.dense(cfg.matrix_values(j))
        b = cfg.rhs(j, x_prev)
        x = np.linalg.solve(A, b)
        xbar = x_prev if (xbar_mode == "prev" and x_prev is not None) else np.zeros(cfg.n)
        snaps = [x - xbar] + snaps
        snaps = snaps[: cfg.omega]
        S = np.stack(snaps, axis=1)
        g = np.array([2.0 ** (1 - i) for i in range(1, S.shape[1] + 1)])
        Sg = S * g
        lam, V = np.linalg.eigh(Sg.T @ A @ Sg)
        lam, V = lam[::-1], V[:, ::-1]
        y = min(cfg.rank, int(np.sum(lam > 1e-12 * lam[0])))
        out.append((A, Sg @ (V[:, :y] / np.sqrt(lam[:y])), lam))
        x_prev = x
    return out


def _projector_gap(run_sequence, cfg, xbar_mode):
    rows = run_sequence(cfg, "aug", keep_W=True, aug_xbar=xbar_mode)
    worst = 0.0
    for rec, (A, We, lam) in zip(rows, _expected_bases(cfg, xbar_mode)):
        Wo = rec["W"]
        if Wo.shape[1] != We.shape[1]:
            return np.inf
        Pe, Po = We @ We.T @ A, Wo @ Wo.T @ A
        worst = max(worst, np.linalg.norm(Po - Pe) / np.linalg.norm(Pe))
    return worst


@pytest.mark.parametrize("xbar_mode", ["zero", "prev"])
def test_sequence_bases_follow_the_pod_definition(xbar_mode):
    cfg = _cfg()
    rows = oracle.run_sequence(cfg, "aug", keep_W=True, aug_xbar=xbar_mode)
    assert [r["rank_next"] for r in rows] == [1, 2, 2, 2, 2, 2]
    assert _projector_gap(oracle.run_sequence, cfg, xbar_mode) <= 1e-7
    # the oracle's basis is A_j-orthonormal (Eq. (podOrth)) for the matrix of its system
    for j, rec in enumerate(rows, start=1):
        A = cfg.fv.dense(cfg.matrix_values(j))
        W = rec["W"]
        assert np.allclose(W.T @ A @ W, np.eye(W.shape[1]), atol=1e-10)


MUTANTS = {
    "reversed_weights": ("idw_weights(len(snaps))", "idw_weights(len(snaps))[::-1]"),
    "ring_of_omega_plus_one": ("del snaps[cfg.omega:]", "del snaps[cfg.omega + 1:]"),
    "uncentred_snapshots": ("snaps.insert(0, x - xbar)", "snaps.insert(0, x)"),
    "oldest_weighted_most": ("snaps.insert(0, x - xbar)\n            del snaps[cfg.omega:]",
                             "snaps.append(x - xbar)\n            del snaps[:-cfg.omega]"),
}


def _load_mutant(text):
    mod = types.ModuleType("oracle._sequence_mutant")
    mod.__package__ = "oracle"
    exec(compile(text, "sequence_mutant.py", "exec"), mod.__dict__)
    return mod.run_sequence


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_sequence_mutant_is_caught(name):
    old, new = MUTANTS[name]
    text = open(SEQ_SRC).read()
    assert text.count(old) == 1, f"mutation site for {name} not found"
    run = _load_mutant(text.replace(old, new))
    cfg = _cfg()
    gaps = [_projector_gap(run, cfg, mode) for mode in ("zero", "prev")]
    assert max(gaps) > 1e-3, (name, gaps)
