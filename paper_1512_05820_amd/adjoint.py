"""Differentiable sequences of recycled solves (outputs q_j = C x_j of Section 2).

A sequence A_j(p) x_j = b_j(x_{j-1}, p), j = 1..m, with parameters p, is run
with the POD-augmented solver; `RecycledSequence` makes the stacked outputs
q_j differentiable in p.  The gradient of a solve is the adjoint solve

    A_j lambda_j = xbar_j          (A_j symmetric; same basis W_j, Stage 1 +
                                    augmented PCG in the library),
    bbar_j = lambda_j,   (dA_j)bar = -lambda_j x_j^T on the stored pattern,

and the rest of the chain (how A_j and b_j depend on p and on x_{j-1}, how q_j
depends on x_j) is differentiated by torch autograd of the caller's
callbacks.  Checkpointing: the forward keeps every solution x_j (n values
each) but not the bases; the backward replays, segment by segment, only the
POD builds from the stored solutions to recover each W_j, then runs the
adjoint solves of that segment in reverse.  All arithmetic of the solves,
POD builds and the pattern outer product runs in libpodcg's HIP kernels.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, Sequence

import torch


@dataclass
class SequenceSpec:
    steps: int
    assemble: Callable[[int, Sequence[torch.Tensor]], torch.Tensor]    # j, params -> CSR values
    rhs: Callable[[int, torch.Tensor | None, Sequence[torch.Tensor]], torch.Tensor]  # j, x_{j-1}, params -> b_j
    output: Callable[[int, torch.Tensor], torch.Tensor]                # j, x_j -> q_j
    rtol: float
    checkpoint_every: int = 20
    # basis of the adjoint solves: "forward" = the forward sequence's W_j
    # (replayed from checkpoints), "adjoint" = POD of the adjoint solutions
    # lambda_{j+1}, lambda_{j+2}, ... themselves (the adjoint run is itself a
    # sequence of SPD systems, recycled the same way; no replay needed),
    # "none" = plain Jacobi PCG
    adjoint_basis: str = "forward"


class RecycledSequence(torch.autograd.Function):
    """q = RecycledSequence.apply(solver, adjoint_solver, spec, *params) -> (m, k) outputs.

    `solver` and `adjoint_solver` are PodCG contexts for the same pattern
    (already set with set_matrix(vals, rowptr, colind)); the first runs the
    forward sequence (and the POD replays), the second the adjoint solves."""

    @staticmethod
    def forward(ctx, solver, adjoint_solver, spec: SequenceSpec, *params):
        xs, qs, stats = [], [], []
        solver.reset_snapshots()
        solver.set_basis(None)
        x_prev = None
        with torch.no_grad():
            for j in range(1, spec.steps + 1):
                vals = spec.assemble(j, params).contiguous()
                b = spec.rhs(j, x_prev, params).contiguous()
                solver.set_matrix(vals)
                x = torch.zeros_like(b)
                st = solver.solve(b, x, spec.rtol)
                if st.status not in (0, 2):
                    raise RuntimeError(f"forward solve {j} failed with status {st.status}")
                solver.push_snapshot(x)
                solver.build_pod(wait=False)
                xs.append(x)
                qs.append(spec.output(j, x))
                stats.append(st.as_dict())
                x_prev = x
        ctx.solver, ctx.adj, ctx.spec = solver, adjoint_solver, spec
        ctx.xs = xs
        ctx.forward_stats = stats
        ctx.save_for_backward(*params)
        return torch.stack(qs)

    @staticmethod
    def backward(ctx, qbar):
        spec, solver, adj = ctx.spec, ctx.solver, ctx.adj
        params = ctx.saved_tensors
        xs = ctx.xs
        m = spec.steps
        omega = solver.omega
        grads = [None] * len(params)
        carry = None                     # xbar_{j} contribution from b_{j+1}
        adj_stats = []
        mode = spec.adjoint_basis
        if mode not in ("forward", "adjoint", "none"):
            raise ValueError(f"adjoint_basis must be forward, adjoint or none, not {mode!r}")
        if mode != "forward":
            adj.reset_snapshots()
            adj.set_basis(None)
        starts = list(range(1, m + 1, spec.checkpoint_every)) if mode == "forward" else [1]
        for k in reversed(starts):
            end = min(k + spec.checkpoint_every, m + 1) if mode == "forward" else m + 1
            # replay the POD builds of this segment: W_k .. W_{end-1}
            with torch.no_grad():
                if mode != "forward":
                    Ws = None
                else:
                    solver.reset_snapshots()
                    solver.set_basis(None)
                    if k > 1:
                        solver.set_matrix(spec.assemble(k - 1, params).contiguous())
                        for x in xs[max(0, k - 1 - omega):k - 1]:
                            solver.push_snapshot(x)
                        solver.build_pod()
                    Ws = {}
                    for j in range(k, end):
                        Ws[j] = solver.get_basis().clone()
                        if j + 1 < end:
                            solver.set_matrix(spec.assemble(j, params).contiguous())
                            solver.push_snapshot(xs[j - 1])
                            solver.build_pod()
            for j in range(end - 1, k - 1, -1):
                xj = xs[j - 1]
                with torch.enable_grad():
                    xl = xj.detach().requires_grad_(True)
                    qj = spec.output(j, xl)
                    (xbar,) = torch.autograd.grad(qj, xl, qbar[j - 1], allow_unused=True)
                if xbar is None:
                    xbar = torch.zeros_like(xj)
                if carry is not None:
                    xbar = xbar + carry
                xbar = xbar.contiguous()
                with torch.no_grad():
                    vals = spec.assemble(j, params).contiguous()
                    adj.set_matrix(vals)
                    if mode == "forward":
                        W = Ws[j]
                        adj.set_basis(W if W.numel() else None)
                    lam = torch.zeros_like(xbar)
                    if torch.any(xbar != 0):
                        st = adj.solve(xbar, lam, spec.rtol)
                        if st.status not in (0, 2):
                            raise RuntimeError(f"adjoint solve {j} failed with status {st.status}")
                        adj_stats.append(st.as_dict())
                        if mode == "adjoint":
                            # metric A_j for the basis of system j-1
                            adj.push_snapshot(lam)
                            adj.build_pod(wait=False)
                    vbar = adj.pattern_outer(lam, xj, -1.0, torch.empty_like(vals))
                with torch.enable_grad():
                    p_req = [p for p in params if p.requires_grad]
                    vals_g = spec.assemble(j, params)
                    xp = xs[j - 2].detach().requires_grad_(True) if j > 1 else None
                    b_g = spec.rhs(j, xp, params)
                    inputs = p_req + ([xp] if xp is not None else [])
                    outs, gouts = [], []
                    if vals_g.requires_grad:
                        outs.append(vals_g)
                        gouts.append(vbar)
                    if b_g.requires_grad:
                        outs.append(b_g)
                        gouts.append(lam)
                    g = torch.autograd.grad(outs, inputs, gouts, allow_unused=True) if outs else \
                        [None] * len(inputs)
                it = iter(g)
                for i, p in enumerate(params):
                    if p.requires_grad:
                        gi = next(it)
                        if gi is not None:
                            grads[i] = gi if grads[i] is None else grads[i] + gi
                carry = next(it) if xp is not None else None
        ctx.adjoint_stats = adj_stats
        ctx.xs = None
        return (None, None, None, *grads)
