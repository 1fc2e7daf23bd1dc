"""Differentiable rollouts: torch.autograd.Function wrappers around the
forward step and the hand-written reverse sweep of libbgk.so.

Parameters that the C library takes at bgk_init (Kn, the wall temperature)
enter as scalar tensors so that autograd can return their gradients; their
values must equal the ones the Context was built with.

The backward pass recomputes states from checkpoints: the forward pass keeps
f every `every` steps, and the backward pass re-runs each segment forward
(storing its states) before sweeping back through it, so memory is
(nsteps / every + every) states instead of nsteps.  With every = None the
interval is picked from the free device memory: 1 (every state kept, no
recomputation) when the whole trajectory fits the budget, which on a
288 GB device is the common case (200 states of a 64^2 x 24^3 cavity take
45 GB in FP32), else the smallest interval whose checkpoints and one
recomputed segment fit.

The recomputed states are the forward pass's own, bit for bit.  A call of n
steps keeps the relaxations between its streaming passes fused and
materialises only its final state (in FP32 rounded stochastically, with
random bits keyed by the context's rounding counter).  So the forward pass
advances one step per call, as the recomputation does, and records the
rounding seed at each checkpoint; the backward pass sets that seed before it
recomputes a segment and restores the caller's seed at the end.
"""
from __future__ import annotations

import math

import torch

from .binding import Context


def _check_param(value: torch.Tensor, expected: float, name: str):
    v = float(value.detach().reshape(-1)[0])
    if abs(v - expected) > 1e-12 * max(1.0, abs(expected)):
        raise ValueError(f"{name}={v} differs from the Context's {expected}; build a Context for it")


def auto_every(f0: torch.Tensor, nsteps: int, fraction: float = 0.5, free_bytes: int | None = None) -> int:
    """Checkpoint interval for a rollout of nsteps steps from f0: the smallest
    `every` whose ceil(nsteps / every) stored states plus the `every` states
    of one recomputed segment (every = 1: the nsteps + 1 states of the whole
    trajectory) fit in `fraction` of the device's free memory (free_bytes
    overrides the query); ceil(sqrt(nsteps)) if none does."""
    state = f0.numel() * f0.element_size()
    if free_bytes is None:
        free_bytes = torch.cuda.mem_get_info(f0.device)[0]
    budget = fraction * free_bytes
    for every in range(1, nsteps + 1):
        held = nsteps + 1 if every == 1 else -(-nsteps // every) + every
        if held * state <= budget:
            return every
    return max(1, math.isqrt(nsteps - 1) + 1)


def forward_checkpoints(solver: Context, f0: torch.Tensor, nsteps: int, every: int):
    """Steps f0 forward nsteps times; returns (f_N, the state at the start of
    every segment of `every` steps, the rounding seed at each of them)."""
    checkpoints, seeds = [], []
    f = f0
    done = 0
    while done < nsteps:
        checkpoints.append(f)
        seeds.append(solver.seed())
        k = min(every, nsteps - done)
        for _ in range(k):
            f = solver.step(f, n=1)
        done += k
    return f, checkpoints, seeds


def recompute_segment(solver: Context, start: torch.Tensor, seed: int, k: int):
    """The states f^0 .. f^(k-1) of a segment from its checkpoint and seed,
    as the forward pass computed them (one step per call)."""
    solver.set_seed(seed)
    states = [start]
    for _ in range(k - 1):
        states.append(solver.step(states[-1], n=1))
    return states


class Rollout(torch.autograd.Function):
    """f_N = step^nsteps(f_0) for a single-instance Context."""

    @staticmethod
    def forward(ctx, f0, kn, tw, solver: Context, nsteps: int, every: int | None):
        p = solver.problems[0]
        _check_param(kn, p["kn"], "kn")
        _check_param(tw, p.get("t_wall", 1.0), "t_wall")
        if every is None:
            every = auto_every(f0, nsteps)
        solver.last_checkpoint_every = every
        f, checkpoints, seeds = forward_checkpoints(solver, f0.detach().contiguous(), nsteps, every)
        ctx.solver, ctx.nsteps, ctx.every = solver, nsteps, every
        ctx.checkpoints, ctx.seeds = checkpoints, seeds
        ctx.shapes = (kn.shape, tw.shape)
        ctx.devices = (kn.device, tw.device)
        return f

    @staticmethod
    def backward(ctx, lam):
        solver, every, nsteps = ctx.solver, ctx.every, ctx.nsteps
        # own copy: the incoming gradient may be shared with other graph nodes
        lam = lam.to(solver.dtype).contiguous().clone()
        grad = solver.grad_buffer(lam.device)
        other = torch.empty_like(lam)
        caller_seed = solver.seed()
        for seg in range(len(ctx.checkpoints) - 1, -1, -1):
            k = min(every, nsteps - seg * every)
            states = recompute_segment(solver, ctx.checkpoints[seg], ctx.seeds[seg], k)
            ctx.checkpoints[seg] = None  # held by `states` until the segment is swept
            for i in range(k - 1, -1, -1):
                solver.step_adjoint(states[i], lam, other, grad)
                lam, other = other, lam
        solver.set_seed(caller_seed)
        ctx.checkpoints = ctx.seeds = None
        g = grad[0]
        return (lam, g[0].reshape(ctx.shapes[0]).to(ctx.devices[0]), g[1].reshape(ctx.shapes[1]).to(ctx.devices[1]),
                None, None, None)


class LidShear(torch.autograd.Function):
    """Integrated lid shear of a single-instance cavity Context (float64 scalar)."""

    @staticmethod
    def forward(ctx, f, tw, solver: Context):
        _check_param(tw, solver.problems[0].get("t_wall", 1.0), "t_wall")
        ctx.solver = solver
        ctx.tw_shape, ctx.tw_device = tw.shape, tw.device
        ctx.save_for_backward(f)
        return solver.lid_shear(f.detach().contiguous())[0]

    @staticmethod
    def backward(ctx, gL):
        (f,) = ctx.saved_tensors
        lam, grad = ctx.solver.lid_shear_grad(f.detach().contiguous())
        s = gL.reshape(-1)[0]
        return lam * s.to(lam.dtype), (grad[0, 1] * s).reshape(ctx.tw_shape).to(ctx.tw_device), None


def rollout(f0, kn, tw, solver: Context, nsteps: int, every: int | None = None):
    """f_N of nsteps steps from f0, differentiable in f0, kn and tw; every:
    checkpoint interval (None: picked by auto_every from the free memory)."""
    return Rollout.apply(f0, kn, tw, solver, nsteps, every)


def lid_shear(f, tw, solver: Context):
    return LidShear.apply(f, tw, solver)
