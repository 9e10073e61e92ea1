"""Differentiable rollout of N Heun steps at frozen time steps, with
checkpoint-and-recompute over the time steps.

Forward: N calls of ``lf_step`` with the given dts; the state at every
``ckpt_every``-th step is kept (those are the outputs of the step calls,
not copies).  The last segment runs ``lf_step_save`` instead, which gives
the same states and also each step's predictor state U*, and keeps them
all: the backward pass starts there without recomputing it.  Backward: for
each segment, last to first, the segment's states are recomputed from its
checkpoint with ``lf_step_save`` (the last step of the segment needs only
its predictor stage), and the adjoint is carried back through the segment
with ``lf_adjoint_step_ustar`` (the discrete adjoint of the step map at
that U*).

Peak device memory: the checkpoints plus one segment of states and of
predictor states (the last segment's are held from the forward pass to
the backward pass).
"""
from __future__ import annotations

from typing import Sequence

import torch


class LagrangeFluxRollout(torch.autograd.Function):
    """U_N = S_{dt_{N-1}} o ... o S_{dt_0} (U_0), differentiable in U_0."""

    @staticmethod
    def forward(ctx, U0: torch.Tensor, solver, dts: Sequence[float], ckpt_every: int = 20):
        dts = [float(d) for d in dts]
        C = max(1, int(ckpt_every))
        N = len(dts)
        last0 = ((N - 1) // C) * C if N else 0  # first step of the last segment
        ckpts = [U0.detach()]
        U = U0.detach()
        A, B = solver.empty_state(), solver.empty_state()  # ping-pong for the other steps
        tail_states, tail_ustars = [], []  # U^n and U* of the last segment's steps
        for n, dt in enumerate(dts):
            if n >= last0:
                out, us = solver.empty_state(), solver.empty_state()
                solver.step_save(U, out, us, dt)
                tail_states.append(U)
                tail_ustars.append(us)
            else:
                keep = (n + 1) % C == 0
                out = solver.empty_state() if keep else (A if U is not A else B)
                solver.step(U, out, dt)
                if keep:
                    ckpts.append(out)
            U = out
        if not dts:
            U = U0.detach().clone()
        ctx.solver = solver
        ctx.dts = dts
        ctx.C = C
        ctx.tail = (tail_states, tail_ustars)
        ctx.save_for_backward(*ckpts)
        return U

    @staticmethod
    def backward(ctx, gN: torch.Tensor):
        solver, dts, C = ctx.solver, ctx.dts, ctx.C
        ckpts = ctx.saved_tensors
        N = len(dts)
        # a copy: the adjoint steps below ping-pong between lam and lam_next,
        # and the caller's output gradient must come back unchanged
        lam = gN.to(solver.torch_dtype, copy=True).contiguous()
        if N == 0:  # U_N = U_0
            return lam, None, None, None
        nseg = len(ckpts)
        lam_next = torch.empty_like(lam)
        for s in reversed(range(nseg)):
            n0 = s * C
            n1 = min(N, n0 + C)
            if s == nseg - 1:
                states, ustars = ctx.tail  # kept by the forward pass
                ctx.tail = None
            else:
                states = [ckpts[s]]
                ustars = []
                for n in range(n0, n1 - 1):
                    out, us = solver.empty_state(), solver.empty_state()
                    solver.step_save(states[-1], out, us, dts[n])
                    states.append(out)
                    ustars.append(us)
                us = solver.empty_state()
                solver.stage(1, states[-1], us, dts[n1 - 1])
                ustars.append(us)
            for n in reversed(range(n0, n1)):
                solver.adjoint_step_ustar(states[n - n0], ustars[n - n0], dts[n], lam, lam_next)
                lam, lam_next = lam_next, lam
            del states, ustars
        return lam, None, None, None


def rollout(U0: torch.Tensor, solver, dts: Sequence[float], ckpt_every: int = 20) -> torch.Tensor:
    return LagrangeFluxRollout.apply(U0, solver, dts, ckpt_every)
