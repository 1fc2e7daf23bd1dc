"""Benchmark of the BGK step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Times K BGK time steps (one bgk_step call; every step is the whole hot path:
relaxation, moments, Maxwellian, minmod streaming with boundary fluxes) of the
largest single-GPU workload, the seeded batch of 64 lid-driven cavities of
uneven size (sides from {32, 48, 64, 96, 128}, 24^3 velocities, FP32 f, FP64
moments, 5.88e9 phase-space points), launched as one graph per call with the
tuned launch shape, the state resident in HBM.  Prints one JSON line with
  value     phase-space point updates per second (points x steps / s),
  roofline  algorithmic HBM bytes of the streaming kernel / its average
            duration (HIP event pairs inside the replayed graph), against 8 TB/s,
  error     moments after the workload's full step count against the stored
            FP64 oracle runs (tests/golden/),
  cpu_baseline  the FP64 oracle timed on the host cores on a bounded sample,
  extras    the other single-GPU workloads (FP64 and FP32 shocks, the 128^2
            cavity, the adjoint rollout, the paper's shock runs, variants),
            each with its rate, roofline fraction and error where stored.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")

GOLDEN = os.path.join(ROOT, "tests", "golden")
GAMMA = 5.0 / 3.0
BATCH = "batch_64_cavities_fp32"

DESCRIPTIONS = {
    BATCH: "64 independent 2D lid-driven cavities in one context (seed 9034044: sides uniform from "
           "{32,48,64,96,128}, Kn log-uniform on [0.01,1], lid Mach uniform on [0.05,0.3]), 24^3 velocities on "
           "[-5,5]^3, diffuse walls, T_w 1, Strang + minmod upwind, CFL 0.5; f FP32, moments FP64; one graph "
           "per bgk_step call, tuned launch shape",
    "shock_m3_fp32": "1D normal shock, Mach 3, Kn 1, Nx 1024 on [-20,20], 48^3 velocities on [-8,8]^3, "
                     "RH step initial state, Strang + minmod upwind, CFL 0.5; f FP32, moments FP64",
    "shock_m1.5_fp64": "1D normal shock, Mach 1.5, Kn 1, Nx 256 on [-20,20], 32^3 velocities on [-6,6]^3, "
                       "FP64 throughout, Strang + minmod upwind, CFL 0.5",
    "cavity_128_fp32": "2D lid-driven cavity 128x128, lid Mach 0.1, Kn 0.1, T_w 1, 24^3 velocities on [-5,5]^3, "
                       "diffuse walls; f FP32, moments FP64",
    "cube_48_fp32": "3D lid-driven cube 48^3, lid Mach 0.1 along x on the y = 1 face, Kn 0.1, T_w 1, six diffuse "
                    "walls, 16^3 velocities on [-4.5,4.5]^3; f FP32, moments FP64",
    "batch_mixed_fp32": "the 64-cavity batch with 8 seeded normal shocks (Nx from {256,512,1024}, Mach U(1.2,2)) "
                        "on the same 24^3 grid, one context: 2D kernels with the shocks streaming along x only",
    "shock_m3_fp32_conservative": "the Mach-3 shock above with every relaxation towards the effective "
                                  "Maxwellian (per-cell Newton solve, exact conservation on the grid)",
    "cavity_128_fp32_conservative": "the 128^2 cavity above with every relaxation towards the effective "
                                    "Maxwellian (per-cell Newton solve, exact conservation on the grid)",
}


def kernel_source_hash() -> str:
    """sha256 of the source of the streaming kernel (bgk_device.h holds
    k_stream and everything it inlines): traffic counters are reported only
    while the kernel is the one they were taken from."""
    with open(os.path.join(ROOT, "paper_0903_4044_amd", "csrc", "bgk_device.h"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def read_traffic(workload: str, kname: str = "k_stream"):
    """HBM bytes per streaming launch from a committed counter summary
    (profiles/<kernel>_<workload>_counters.txt), if taken from these kernels."""
    path = os.path.join(PROFILES, f"{kname}_{workload}_counters.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def bytes_per_update(precision: str) -> int:
    # the streaming kernel reads h once and writes it once per time step
    return 8 if precision == "fp32" else 16


def speed_scale(p) -> float:
    """Velocity scale of the moment errors: the upstream speed of a shock,
    the lid speed of a cavity."""
    if p["kind"] == "shock":
        return p["mach"] * (GAMMA / 2) ** 0.5
    if p["kind"] in ("cavity", "cavity3d") and p.get("lid_mach", 0.0) != 0.0:
        return abs(p["lid_mach"]) * (GAMMA / 2) ** 0.5
    return 1.0


def moment_errors(got, ref, p):
    """(e_n, e_V, e_T): max relative density and temperature errors, max
    velocity error over the problem's speed scale."""
    import numpy as np
    got, ref = np.asarray(got), np.asarray(ref)
    e_n = float(np.max(np.abs(got[:, 0] - ref[:, 0]) / np.abs(ref[:, 0])))
    e_T = float(np.max(np.abs(got[:, 4] - ref[:, 4]) / np.abs(ref[:, 4])))
    e_V = float(np.max(np.abs(got[:, 1:4] - ref[:, 1:4])) / speed_scale(p))
    return e_n, e_V, e_T


def goldens(name: str, problems):
    """Stored FP64 oracle moments for a workload: [(instance, marks, file)]."""
    import numpy as np
    out = []
    if name == BATCH:
        for i in range(len(problems)):
            path = os.path.join(GOLDEN, f"batch_cavity_{i}_oracle.npz")
            if os.path.exists(path):
                out.append((i, np.load(path)))
    else:
        path = os.path.join(GOLDEN, f"{name}_oracle.npz")
        if os.path.exists(path):
            out.append((0, np.load(path)))
    return out


def error_vs_oracle(binding, torch, name, problems, precision, shape):
    """Runs the workload from its initial state (launch shape as timed) to
    the step counts the stored oracle runs hold and reports the moment
    errors at each and at the last (None if nothing is stored)."""
    gold = goldens(name, problems)
    if not gold:
        return None
    marks = sorted(set(int(m) for _, G in gold for m in G["steps"]))
    ctx = binding.Context(problems, precision, tune="off")
    ctx.set_launch(shape["vec"], shape["unroll"], shape["vsplit"], shape["persist"])
    f = ctx.initial_state()
    per_mark, done = {}, 0
    for m in marks:
        g = ctx.step(f, n=m - done)
        del f
        f, done = g, m
        mom = ctx.moments(f).cpu().numpy()
        worst = [0.0, 0.0, 0.0]
        for i, G in gold:
            if f"moments_{m}" not in G.files:
                continue
            c0 = ctx.cell_offsets[i]
            n = G[f"moments_{m}"].shape[0]
            e = moment_errors(mom[c0:c0 + n], G[f"moments_{m}"], problems[i])
            worst = [max(a, b) for a, b in zip(worst, e)]
        per_mark[m] = {"e_n": worst[0], "e_V": worst[1], "e_T": worst[2]}
    ctx.close()
    del f
    torch.cuda.empty_cache()
    last = per_mark[marks[-1]]
    return dict(last, steps=marks[-1], marks=per_mark, instances=[i for i, _ in gold],
                tolerance=1e-12 if precision == "fp64" else 1e-5,
                reference="FP64 oracle moments stored by tests/golden/make_golden.py and make_batch_golden.py")


def run_workload(binding, torch, problems, precision, steps, warmup, kernel_timing=True, tune=True, graph=False):
    """Times one bgk_step call of `steps` steps.  Eagerly, with a HIP event
    pair around every streaming launch on the launch stream; or, with graph
    replay, as one replay of the graph that an untimed call of the same step
    count captured after the warm-up (wall clock only: HIP reports no
    elapsed time for events that graph nodes record).  Returns (seconds for
    `steps`, kernel ms per launch or NaN, points, launch shape)."""
    ctx = binding.Context(problems, precision)
    points = ctx.f_elems
    x = ctx.initial_state()
    y = ctx.empty()
    torch.cuda.synchronize()
    if tune:
        ctx.autotune(x)
    shape = ctx.launch()
    stream = torch.cuda.Stream() if graph else torch.cuda.current_stream()  # graphs need a capturable stream
    with torch.cuda.stream(stream):
        ctx.set_graph(graph)
        kernel_timing = kernel_timing and not graph
        ctx.set_timing(steps + warmup + 4 if kernel_timing else 0)
        if warmup:
            ctx.step(x, y, n=warmup)
        if graph:
            ctx.step(x, y, n=steps)  # capture the timed call's graph (untimed)
        torch.cuda.synchronize()
        ctx.timing()  # reset
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(x, y, n=steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ms, launches = ctx.timing()
        if not kernel_timing or launches != steps:
            ms, launches = float("nan"), 1
        ctx.set_timing(0)
        ctx.set_graph(False)
        rc = ctx.check(y)
    ctx.close()
    del x, y
    torch.cuda.empty_cache()
    if rc != 0:
        raise RuntimeError(f"state check failed after the timed run (status {rc})")
    return t1 - t0, ms / max(launches, 1), points, shape


def run_adjoint(binding, torch, cfg, precision, every=None, mode="auto"):
    """Differentiated rollout of the adjoint workload: forward keeping step
    records (mode "record"; "auto" takes them when they fit the free device
    memory) or checkpoints every `every` steps, then the reverse sweep down to
    dL/df0, dL/dKn and dL/dT_w.  Returns (forward s, backward s, points,
    steps, gradient errors against the stored FP64 oracle sweep or None, the
    rollout plan used)."""
    import numpy as np

    from paper_0903_4044_amd import inputs, solver
    ctx = binding.Context(cfg, precision)
    nsteps = cfg["steps"]
    xi = torch.tensor(inputs.noise((ctx.f_elems,)), dtype=ctx.dtype, device="cuda")
    f0 = ctx.initial_state() * (1 + 1e-3 * xi)
    del xi
    ctx.autotune(f0)

    def once(n):
        ctx.set_seed(0)  # the warm-up and the timed rollout take the same trajectory
        x = f0.clone().requires_grad_(True)
        kn = torch.tensor(cfg["kn"], dtype=torch.float64, requires_grad=True)
        tw = torch.tensor(cfg["t_wall"], dtype=torch.float64, requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L = solver.lid_shear(solver.rollout(x, kn, tw, ctx, n, every=every, mode=mode), tw, ctx)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if not all(torch.isfinite(t.grad).all() for t in (x, kn, tw)):
            raise RuntimeError("non-finite gradient in the adjoint run")
        return t1 - t0, t2 - t1, float(L.detach()), float(kn.grad), float(tw.grad)

    once(nsteps)  # warm-up: the same rollout, so that its buffers come from torch's cache when timed
    fwd, bwd, L, gkn, gtw = once(nsteps)
    used = ctx.last_rollout
    err = None
    path = os.path.join(GOLDEN, "cavity_64_adjoint_oracle.npz")
    if os.path.exists(path):
        G = np.load(path)
        err = {"L": abs(L / float(G["L"]) - 1), "dL_dKn": abs(gkn / float(G["grad"][0]) - 1),
               "dL_dTw": abs(gtw / float(G["grad"][1]) - 1),
               "reference": "FP64 oracle reverse sweep (tests/golden/make_adjoint_golden.py), relative errors"}
    points = ctx.f_elems
    ctx.close()
    del f0
    torch.cuda.empty_cache()
    return fwd, bwd, points, nsteps, err, used


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(problems, budget_s: float):
    """The FP64 oracle on the same workload, on all host threads: one untimed
    step of the first instance, then one step of each instance in turn (a
    single instance steps repeatedly) until the budget is spent; then one
    step of the first instance on one thread, the paper's CPU comparison.
    Returns updates/s and the sample description."""
    import ctypes
    import oracle
    Os = [oracle.Oracle(p) for p in problems]
    f = Os[0].step(Os[0].initial_state(), 1)  # untimed
    points, t, steps = 0, 0.0, 0
    while t < budget_s and (len(Os) == 1 or steps < len(Os)):
        O = Os[0] if len(Os) == 1 else Os[steps]
        if len(Os) > 1:
            f = O.initial_state()
        t0 = time.perf_counter()
        g = O.step(f, 1)
        t += time.perf_counter() - t0
        f = g if len(Os) == 1 else None
        points += O.ncell * O.nvel
        steps += 1
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0))
    what = (f"{steps} time steps of the full {Os[0].ncell} x {Os[0].nvel} grid" if len(Os) == 1 else
            f"one time step of each of the first {min(steps, len(Os))} instances of the batch "
            f"({steps} instance-steps, {points} point updates)")
    out = {"value": points / t, "unit": "updates/s", "cores": threads, "kind": "oracle",
           "sample": f"{what} in FP64 after one untimed step ({t:.1f} s)", "cpu_model": _cpu_model(),
           "nproc": os.cpu_count()}
    try:  # the oracle's OpenMP runtime: same library in this process
        gomp = ctypes.CDLL("libgomp.so.1")
        gomp.omp_set_num_threads(1)
        f = Os[0].initial_state()
        t0 = time.perf_counter()
        Os[0].step(f, 1)
        t1 = time.perf_counter() - t0
        gomp.omp_set_num_threads(threads)
        out["single_thread"] = {"value": Os[0].ncell * Os[0].nvel / t1, "unit": "updates/s",
                                "sample": f"1 time step of the first instance ({Os[0].ncell} x {Os[0].nvel}) "
                                          f"on 1 thread ({t1:.1f} s)"}
    except OSError:
        pass
    return out


# The Table of Sec. 5.2: per rarefaction parameter delta, the paper's D and G
# and the range of the reference values it quotes.
TABLE1 = {0.1: (0.675, (0.676, 0.678), 0.0975, (0.0973, 0.0976)),
          1.0: (0.624, (0.625, 0.631), 0.103, (0.104, 0.105)),
          10.0: (0.393, (0.412, 0.415), 0.143, (0.145, 0.145))}


def table1(binding, torch, inputs) -> dict:
    """Steady driven-cavity runs at the paper's settings, from rest until D
    and G change by less than 1e-5 over two time units, for this library's
    scheme (Strang, minmod) and the paper's (Lie, first-order upwind), both
    with the conservative Maxwellian, and for the first in the reduced
    velocity space (v_z integrated out); and the drift of D with the
    point-value Maxwellian (whose mass defect on this grid slowly drains the
    cavity)."""
    from paper_0903_4044_amd.steady import run_to_steady
    rows = []
    for scheme, spl, lim, red in (("strang-minmod", "strang", "minmod", False), ("lie-upwind", "lie", "none", False),
                                  ("strang-minmod-reduced", "strang", "minmod", True)):
        for delta in inputs.TABLE_DELTAS:
            cfg = inputs.table_cavity(delta, splitting=spl, limiter=lim)
            if red:  # v_z integrated out: the g and h planes on the 20^2 (v_x, v_y) grid
                cfg = dict(cfg, nv=(20, 20, 2), reduced=True)
            C = binding.Context(cfg, "fp32")
            C.autotune(C.initial_state())
            f = C.initial_state()
            chunk = int(round(2.0 / C.dts[0]))
            r = run_to_steady(C, f, chunk, rtol=1e-5, max_steps=40 * chunk)
            D, G = (float(x) for x in r["metrics"][0])
            Dp, Dr, Gp, Gr = TABLE1[delta]
            pts = inputs.ncells(cfg) * inputs.nvel(cfg)
            rows.append({"delta": delta, "scheme": scheme, "D": D, "G": G, "D_paper": Dp, "D_ref": Dr,
                         "G_paper": Gp, "G_ref": Gr, "G_ref_over_G": Gr[0] / G, "steps": r["steps"],
                         "t": r["time"][0],
                         "converged": r["converged"], "seconds": r["seconds"],
                         "updates_per_s": pts * r["steps"] / r["seconds"]})
            print(f"# delta {delta} {scheme}: D {D:.4f} (paper {Dp}, ref {Dr[0]}-{Dr[1]}), "
                  f"G {G:.4f} (paper {Gp}, ref {Gr[0]}-{Gr[1]}), {r['steps']} steps, {r['seconds']:.1f} s",
                  file=sys.stderr, flush=True)
            C.close()
    # point-value Maxwellian: D after 10 and 20 time units at delta = 10
    cfg = inputs.table_cavity(10.0, maxwellian="point")
    C = binding.Context(cfg, "fp32")
    C.autotune(C.initial_state())
    chunk = int(round(10.0 / C.dts[0]))
    r = run_to_steady(C, C.initial_state(), chunk, rtol=0.0, max_steps=2 * chunk)
    (s1, m1), (s2, m2) = r["history"]
    drift = {"delta": 10.0, "D_t10": float(m1[0, 0]), "D_t20": float(m2[0, 0]), "G_t10": float(m1[0, 1]),
             "G_t20": float(m2[0, 1])}
    print(f"# point Maxwellian, delta 10: D {drift['D_t10']:.5f} at t = 10, {drift['D_t20']:.5f} at t = 20",
          file=sys.stderr, flush=True)
    return {"table": "Sec. 5.2 driven cavity, 160^2 cells, 20^3 velocities on [-3,3]^3, lid 0.01, FP32 f",
            "G_normalisation": "unpinned: G is the integral Sec. 5.2 defines (V_x / U_W along the centre line "
                               "from the top vortex's centre to the lid, over the height); the Table's values "
                               "follow a normalisation from its cited reference that the paper does not give "
                               "(G_ref_over_G reports the ratio)",
            "rows": rows, "point_maxwellian_drift": drift}


def workload(inputs, name: str):
    """(problems, precision) of a named workload."""
    if name == BATCH:
        return inputs.batch_cavities(), "fp32"
    if name == "batch_mixed_fp32":
        return inputs.batch_mixed(), "fp32"
    cfg = inputs.config(name)
    return [cfg], cfg["precision"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default=BATCH)
    ap.add_argument("--graph", action="store_true",
                    help="time the headline by graph replay (wall clock; no kernel events, so no roofline)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-errors", action="store_true", help="skip the runs against the stored oracle moments")
    ap.add_argument("--extras", default="",
                    help="comma-separated subset of the extra workloads to run (default: all)")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="no HIP events around the streaming launches (roofline not reported)")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch shape (no autotuning)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first copy a buffer of this size 3 times (HBM counter calibration)")
    ap.add_argument("--table1", action="store_true",
                    help="instead of the throughput line: the steady driven-cavity runs of the Sec. 5.2 Table")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the stepper has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_0903_4044_amd import binding, inputs

    torch.cuda.set_device(0)
    if args.copy_calibration_mib:
        n = args.copy_calibration_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.table1:
        print(json.dumps(table1(binding, torch, inputs)), flush=True)
        return
    probs, prec = workload(inputs, args.workload)
    graph = args.graph
    secs, kms, points, shape = run_workload(binding, torch, probs, prec, args.steps, args.warmup,
                                            not args.no_kernel_timing, not args.no_tune, graph)
    value = points * args.steps / secs
    bpu = bytes_per_update(prec)
    achieved = bpu * points / (kms * 1e-3) / 1e9
    kname = "k_shift" if probs[0].get("limiter") == "shift" else "k_stream"  # the streaming kernel of this workload
    traffic = read_traffic(args.workload, kname)
    cells = sum(inputs.ncells(q) for q in probs)
    out = {
        "metric": "phase-space point updates/s",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == "fp32" else "f64",
        "data": "synthetic: analytic initial states (gas at rest, Rankine-Hugoniot step) and seeded parameter "
                "draws, no dataset",
        "config": {"workload": args.workload, "description": DESCRIPTIONS.get(args.workload, ""),
                   "instances": len(probs), "cells": cells, "velocities": inputs.nvel(probs[0]), "points": points,
                   "moments": "f64", "launch": shape, "graph_replay": graph},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "kernel": kname, "kernel_ms": kms, "bytes_per_update": bpu,
                     "timing": "HIP event pairs around every streaming launch of the timed call, on its stream"
                               if kms == kms else "none (graph replay)"},
    }
    print(f"# {args.workload}: {value:.4g} updates/s, {kname} {kms * 1e3:.1f} us, "
          f"{achieved:.0f} GB/s", file=sys.stderr, flush=True)
    if not args.no_errors:
        err = error_vs_oracle(binding, torch, args.workload, probs, prec, shape)
        if err:
            out["error_vs_oracle"] = err
            print(f"# {args.workload} vs oracle after {err['steps']} steps: e_n {err['e_n']:.2e} "
                  f"e_V {err['e_V']:.2e} e_T {err['e_T']:.2e}", file=sys.stderr, flush=True)

    if not args.no_extras:
        extras = {}
        runs = [("shock_m1.5_fp64", "fp64", 200, 10, False),
                ("shock_m3_fp32", "fp32", 200, 10, False),
                ("cavity_128_fp32", "fp32", 200, 10, False),
                # three dimensions: the lid-driven cube
                ("cube_48_fp32", "fp32", 20, 3, False),
                # shocks batched with the cavities in one context
                ("batch_mixed_fp32", "fp32", 20, 3, False),
                # the headline batch again, one replayed graph per call (wall clock)
                (BATCH + "_graph", "fp32", 20, 2, True),
                # the paper's own shock runs: translation streaming, Courant numbers up to ~150
                ("shock_m1.5_paper", "fp32", 100, 10, False),
                ("shock_m3_paper", "fp32", 50, 5, False),
                # relaxation towards the effective Maxwellian (exact conservation on the grid)
                ("shock_m3_fp32_conservative", "fp32", 500, 20, False),
                ("cavity_128_fp32_conservative", "fp32", 200, 10, False),
                # the paper's shock runs with v_y and v_z integrated out (16 x 2 and 30 x 2 values per cell)
                ("shock_m1.5_paper_reduced", "fp32", 400, 20, False),
                ("shock_m3_paper_reduced", "fp32", 200, 10, False)]
        wanted = set(x for x in args.extras.split(",") if x)
        for name, p, steps, warm, graph_x in runs:
            if wanted and name not in wanted:
                continue
            if name == args.workload or (name.startswith(BATCH) and name.endswith("_graph") == graph and
                                         args.workload == BATCH):
                continue
            wname = BATCH if name.startswith(BATCH) else name
            wprobs, _ = workload(inputs, wname)
            s, k, pts, shp = run_workload(binding, torch, wprobs, p, steps, warm, True, True, graph_x)
            cells_x = sum(inputs.ncells(q) for q in wprobs)
            e = {"updates_per_s": pts * steps / s, "ns_per_update": s / (pts * steps) * 1e9, "steps": steps,
                 "points": pts, "cell_steps_per_s": cells_x * steps / s, "launch": shp, "precision": p,
                 "graph": graph_x, "kernel": "k_shift" if wprobs[0].get("limiter") == "shift" else "k_stream"}
            if k == k:  # timed kernels (not NaN)
                a = bytes_per_update(p) * pts / (k * 1e-3) / 1e9
                e.update({"kernel_ms": k, "achieved_GBs": a, "frac": a / PEAK_HBM_GBS})
            if not args.no_errors and not name.startswith(BATCH):
                err = error_vs_oracle(binding, torch, wname, wprobs, p, shp)
                if err:
                    e["error_vs_oracle"] = err
            extras[name] = e
            print(f"# {name}: {e['updates_per_s']:.4g} updates/s" +
                  (f", {e['achieved_GBs']:.0f} GB/s" if "achieved_GBs" in e else "") +
                  (f", e_n {e['error_vs_oracle']['e_n']:.1e} e_V {e['error_vs_oracle']['e_V']:.1e} "
                   f"e_T {e['error_vs_oracle']['e_T']:.1e} at step {e['error_vs_oracle']['steps']}"
                   if "error_vs_oracle" in e else ""), file=sys.stderr, flush=True)
        for p in ("fp32", "fp64"):
            if wanted and f"adjoint_cavity_64_{p}" not in wanted:
                continue
            fwd, bwd, pts, n, gerr, plan = run_adjoint(binding, torch, inputs.config("cavity_64_adjoint"), p)
            e = {"updates_per_s": pts * n / (fwd + bwd), "steps": n, "points": pts, "precision": p,
                 "forward_s": fwd, "reverse_s": bwd, "reverse_updates_per_s": pts * n / bwd,
                 "rollout": plan,
                 "note": "updates/s counts each of the rollout's steps once over forward + reverse sweep; "
                         "rollout mode record: every state and step record kept in HBM, nothing recomputed; "
                         "checkpoint: states every k steps, one streaming pass recomputed per reverse step"}
            if gerr:
                e["error_vs_oracle"] = gerr
            extras[f"adjoint_cavity_64_{p}"] = e
            print(f"# adjoint_cavity_64_{p}: {e['updates_per_s']:.4g} updates/s (forward {fwd * 1e3:.1f} ms, "
                  f"reverse {bwd * 1e3:.1f} ms)", file=sys.stderr, flush=True)
        if "shock_m1.5_fp64" in extras:
            plain = extras["shock_m1.5_fp64"]["updates_per_s"]
            extras["plain_fp64_updates_per_s"] = plain
            ratios = {k: v["updates_per_s"] / plain for k, v in extras.items()
                      if isinstance(v, dict) and "updates_per_s" in v}
            ratios[args.workload] = value / plain
            extras["ratio_vs_plain_fp64"] = ratios
        out["extras"] = extras

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(probs, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
