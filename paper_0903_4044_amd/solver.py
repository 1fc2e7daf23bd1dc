"""Differentiable rollouts: torch.autograd.Function wrappers around the
forward step and the hand-written reverse sweep of libbgk.so.

Parameters that the C library takes at bgk_init (Kn, the wall temperature)
enter as scalar tensors so that autograd can return their gradients; their
values must equal the ones the Context was built with.

The backward pass recomputes states from checkpoints: the forward pass keeps
f every `every` steps, and the backward pass re-runs each segment forward
(storing its states) before sweeping back through it, so memory is
(nsteps / every + every) states instead of nsteps.

The recomputed states are the forward pass's own, bit for bit.  A call of n
steps keeps the relaxations between its streaming passes fused and
materialises only its final state (in FP32 rounded stochastically, with
random bits keyed by the context's rounding counter).  So the forward pass
advances one step per call, as the recomputation does, and records the
rounding seed at each checkpoint; the backward pass sets that seed before it
recomputes a segment and restores the caller's seed at the end.
"""
from __future__ import annotations

import torch

from .binding import Context


def _check_param(value: torch.Tensor, expected: float, name: str):
    v = float(value.detach().reshape(-1)[0])
    if abs(v - expected) > 1e-12 * max(1.0, abs(expected)):
        raise ValueError(f"{name}={v} differs from the Context's {expected}; build a Context for it")


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
    def forward(ctx, f0, kn, tw, solver: Context, nsteps: int, every: int):
        p = solver.problems[0]
        _check_param(kn, p["kn"], "kn")
        _check_param(tw, p.get("t_wall", 1.0), "t_wall")
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


def rollout(f0, kn, tw, solver: Context, nsteps: int, every: int = 20):
    return Rollout.apply(f0, kn, tw, solver, nsteps, every)


def lid_shear(f, tw, solver: Context):
    return LidShear.apply(f, tw, solver)
