"""Runs to a steady state, judged by the cavity metrics of the Table of
Sec. 5.2 (mean lid shear stress D and main-vortex flow rate G).

Stepping and metrics run in libbgk.so; this module only decides when to
stop: after every chunk of steps it reads (D, G) and stops once neither
changed by more than ``rtol`` (relative) over the last chunk.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from .binding import Context


def run_to_steady(ctx: Context, f: torch.Tensor, chunk: int, rtol: float = 1e-5, max_steps: int = 400000,
                  log=None) -> dict:
    """Step f (the context's initial state, or any state) until the metrics of
    every instance settle.  Returns the final state, the metrics [ninst, 2],
    the step count, the simulated time per instance and the metric history."""
    a, b = f, torch.empty_like(f)
    steps, prev, hist = 0, None, []
    t0 = time.perf_counter()
    while steps < max_steps:
        n = min(chunk, max_steps - steps)
        ctx.step(a, b, n=n)
        a, b = b, a
        steps += n
        m = ctx.cavity_metrics(a)
        hist.append((steps, m.copy()))
        if log:
            log(steps, m)
        if prev is not None and np.all(np.abs(m - prev) <= rtol * np.abs(m)):
            break
        prev = m
    torch.cuda.synchronize()
    return {"f": a, "metrics": hist[-1][1], "steps": steps, "seconds": time.perf_counter() - t0,
            "time": [steps * dt for dt in ctx.dts], "converged": steps < max_steps, "history": hist}
