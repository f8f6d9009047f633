"""Sequence driver of the oracle (test infrastructure only).

Follows the loop of Alg. 3 with the POD basis rebuilt after every system:
for j = 1..p:  solve A_j x_j = b_j from xbar_j with the current basis W_j
(Stage 1 + augmented PCG; W_1 is empty, so the first solve is plain PCG),
push the centred solution x_j - xbar_j into a memory of the last omega
snapshots, and build W_{j+1} = pod_evd(S, inverse-distance weights, A_j).
The plain baseline solves every system with Jacobi PCG, cold (xbar = 0) or
warm (xbar = x_{j-1}).
"""

from __future__ import annotations

import time

import numpy as np


def run_sequence(cfg, method: str = "aug", steps: int | None = None, warm: bool = False,
                 maxit: int = 100000, rank_rtol: float = 1e-12, keep_x: bool = False,
                 keep_W: bool = False, aug_xbar: str = "zero", on_system=None):
    """One pass over the sequence.  aug_xbar chooses the augmented solves'
    initial guess: "zero" (xbar_j = 0, the snapshots are the solutions) or
    "prev" (xbar_j = x_{j-1}, the snapshots are the increments).  keep_W adds
    to each record the basis W_{j+1} built after system j ((n, y) array).
    on_system, if given, is called with each system's record as it is done."""
    from . import CSR, aug_pcg, idw_weights, plain_pcg, pod_evd

    if aug_xbar not in ("zero", "prev"):
        raise ValueError("aug_xbar must be 'zero' or 'prev'")

    steps = cfg.steps if steps is None else steps
    W = None
    snaps: list[np.ndarray] = []
    x_prev = None
    out = []
    for j in range(1, steps + 1):
        A = CSR(cfg.rowptr, cfg.colind, cfg.matrix_values(j))
        b = cfg.rhs(j, x_prev)
        if method == "aug":
            xbar = x_prev.copy() if (aug_xbar == "prev" and x_prev is not None) else np.zeros(cfg.n)
        else:
            xbar = x_prev.copy() if (warm and x_prev is not None) else np.zeros(cfg.n)
        t0 = time.perf_counter()
        if method == "aug":
            x, st = aug_pcg(A, b, xbar, W, cfg.tol, maxit)
        else:
            x, st = plain_pcg(A, b, xbar, cfg.tol, maxit)
        t1 = time.perf_counter()
        rank_next = 0
        if method == "aug":
            snaps.insert(0, x - xbar)
            del snaps[cfg.omega:]
            S = np.stack(snaps, axis=1)
            W, _ = pod_evd(A, S, idw_weights(len(snaps)), cfg.rank, rank_rtol)
            rank_next = W.shape[1]
            if rank_next == 0:
                W = None
        t2 = time.perf_counter()
        rec = {"j": j, "iters": st.iters, "matvecs": st.matvecs, "status": st.status,
               "rank": st.rank, "rank_next": rank_next, "stage1_relres": st.stage1_relres,
               "relres": st.relres, "true_relres": st.true_relres, "cond_G": st.cond_G,
               "solve_s": t1 - t0, "pod_s": t2 - t1}
        if keep_x:
            rec["x"] = x
            rec["b"] = b
        if keep_W and method == "aug":
            rec["W"] = np.zeros((cfg.n, 0)) if W is None else W
        out.append(rec)
        if on_system is not None:
            on_system(rec)
        x_prev = x
    return out
