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
the backward pass).  With ``ckpt_every`` at least the step count the whole
run is one segment, kept from the forward pass: nothing is recomputed.
``ckpt_every="auto"`` takes the largest spacing whose peak fits in the
free device memory (``checkpoint_spacing``): on a GPU with room for every
state and predictor state of the run, that is the whole run.
"""
from __future__ import annotations

import math
from typing import Sequence, Union

import torch


def checkpoint_spacing(n_steps: int, state_bytes: int, free_bytes: int, margin: float = 0.85) -> int:
    """Largest checkpoint spacing C whose peak memory fits in ``margin``
    of ``free_bytes``.  With spacing C the rollout holds about n/C
    checkpoints plus one segment of C states and C predictor states, n/C +
    2C states in all; C = n (the whole run kept, no recompute) needs 2n + 1.
    When not even the smallest peak fits, returns the spacing of the
    smallest peak, sqrt(n/2)."""
    n = int(n_steps)
    if n <= 1:
        return 1
    m = math.floor(margin * free_bytes / state_bytes)  # states that fit
    if m >= 2 * n + 1:
        return n
    disc = m * m - 8 * n
    if disc < 0:
        return max(1, round(math.sqrt(n / 2)))
    c = math.floor((m + math.sqrt(disc)) / 4)  # largest root of 2C^2 - mC + n = 0
    while c > 1 and math.ceil(n / c) + 2 * c > m:  # rounding of the root
        c -= 1
    return max(1, min(n, c))


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


def rollout(U0: torch.Tensor, solver, dts: Sequence[float], ckpt_every: Union[int, str] = 20,
            free_bytes: int = None) -> torch.Tensor:
    """U_N of the steps at the given dts, differentiable in U0.  ckpt_every:
    checkpoint spacing, or "auto" for the largest one that fits in
    ``free_bytes`` (default: the free memory of U0's device)."""
    if ckpt_every == "auto":
        if free_bytes is None:
            if U0.device.type != "cuda":
                raise ValueError('ckpt_every="auto" needs free_bytes for a tensor off the GPU')
            free_bytes = torch.cuda.mem_get_info(U0.device)[0]
        ckpt_every = checkpoint_spacing(len(dts), U0.numel() * U0.element_size(), free_bytes)
    return LagrangeFluxRollout.apply(U0, solver, dts, int(ckpt_every))
