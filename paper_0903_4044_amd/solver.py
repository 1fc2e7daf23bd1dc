"""Differentiable rollouts: torch.autograd.Function wrappers around the
forward step and the hand-written reverse sweep of libbgk.so.

Parameters that the C library takes at bgk_init (Kn, the wall temperature)
enter as scalar tensors so that autograd can return their gradients; their
values must equal the ones the Context was built with.

The backward pass recomputes states from checkpoints: the forward pass keeps
f every `every` steps, and the backward pass re-runs each segment forward
(storing its states) before sweeping back through it, so memory is
(nsteps / every + every) states instead of nsteps.

Where memory allows, the rollout instead keeps every state together with
its step record (bgk_step_record: the step's streamed intermediate, its
moment sums and its limiter branches), and each reverse step reads the
record instead of recomputing the forward pass (bgk_step_adjoint_record).
mode = "auto" takes records when nsteps states and records fit in 60% of
the free device memory (200 steps of a 64^2 x 24^3 cavity: 102 GB in FP32,
193 GB in FP64, of a 288 GB device), else checkpoints with the smallest
interval whose states fit half of it (every = 1 keeps every state and
recomputes one streaming pass per reverse step).

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
        free_bytes = _free_bytes(f0.device)
    budget = fraction * free_bytes
    for every in range(1, nsteps + 1):
        held = nsteps + 1 if every == 1 else -(-nsteps // every) + every
        if held * state <= budget:
            return every
    return max(1, math.isqrt(nsteps - 1) + 1)


def _free_bytes(device) -> int:
    """Free device memory plus what torch's caching allocator holds unused."""
    free = torch.cuda.mem_get_info(device)[0]
    return free + torch.cuda.memory_reserved(device) - torch.cuda.memory_allocated(device)


def auto_mode(f0: torch.Tensor, nsteps: int, record_bytes: int, fraction: float = 0.6,
              free_bytes: int | None = None) -> str:
    """"record" when the nsteps states and step records of a rollout from f0
    fit in `fraction` of the device's free memory, else "checkpoint"."""
    state = f0.numel() * f0.element_size()
    if free_bytes is None:
        free_bytes = _free_bytes(f0.device)
    return "record" if (nsteps + 1) * state + nsteps * record_bytes <= fraction * free_bytes else "checkpoint"


def forward_records(solver: Context, f0: torch.Tensor, nsteps: int):
    """Steps f0 forward nsteps times keeping every state and step record;
    returns (f_N, states f^0 .. f^(N-1), their records)."""
    states, records = [], []
    f = f0
    for _ in range(nsteps):
        states.append(f)
        f, rec = solver.step_record(f)
        records.append(rec)
    return f, states, records


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
    def forward(ctx, f0, kn, tw, solver: Context, nsteps: int, every: int | None, mode: str):
        p = solver.problems[0]
        _check_param(kn, p["kn"], "kn")
        _check_param(tw, p.get("t_wall", 1.0), "t_wall")
        f0 = f0.detach().contiguous()
        if mode == "auto":
            mode = "checkpoint" if every is not None else auto_mode(f0, nsteps, solver.record_bytes)
        if mode not in ("record", "checkpoint"):
            raise ValueError(f"mode {mode!r}: auto, record or checkpoint")
        ctx.solver, ctx.nsteps, ctx.mode = solver, nsteps, mode
        ctx.shapes = (kn.shape, tw.shape)
        ctx.devices = (kn.device, tw.device)
        if mode == "record":
            f, ctx.states, ctx.records = forward_records(solver, f0, nsteps)
            solver.last_rollout = {"mode": "record", "every": 1}
            return f
        if every is None:
            every = auto_every(f0, nsteps)
        f, checkpoints, seeds = forward_checkpoints(solver, f0, nsteps, every)
        ctx.every, ctx.checkpoints, ctx.seeds = every, checkpoints, seeds
        solver.last_rollout = {"mode": "checkpoint", "every": every}
        return f

    @staticmethod
    def backward(ctx, lam):
        solver, nsteps = ctx.solver, ctx.nsteps
        # own copy: the incoming gradient may be shared with other graph nodes
        lam = lam.to(solver.dtype).contiguous().clone()
        grad = solver.grad_buffer(lam.device)
        other = torch.empty_like(lam)
        if ctx.mode == "record":
            # one call for the whole sweep (each step's close pass forms the
            # sums of the step before it)
            lam, _ = solver.adjoint_sweep_record(ctx.states, ctx.records, lam, other, grad)
            ctx.states = ctx.records = None
        else:
            every = ctx.every
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
                None, None, None, None)


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


def rollout(f0, kn, tw, solver: Context, nsteps: int, every: int | None = None, mode: str = "auto"):
    """f_N of nsteps steps from f0, differentiable in f0, kn and tw.  mode:
    "record" (every state and step record kept), "checkpoint" (states every
    `every` steps; None: auto_every's interval) or "auto" (checkpoints if
    `every` is given, else records when they fit the free memory)."""
    return Rollout.apply(f0, kn, tw, solver, nsteps, every, mode)


def lid_shear(f, tw, solver: Context):
    return LidShear.apply(f, tw, solver)
