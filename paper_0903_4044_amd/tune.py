"""Autotune the streaming kernel for the standard workloads on this GPU and
record the shapes in tuned.json (read by binding.Context(tune="table")).

    python -m paper_0903_4044_amd.tune [--out PATH]
"""
from __future__ import annotations

import argparse
import json
import sys

import torch

from . import binding, inputs


def workloads():
    yield "shock_m1.5_fp64", [inputs.config("shock_m1.5_fp64")], "fp64"
    yield "shock_m3_fp32", [inputs.config("shock_m3_fp32")], "fp32"
    yield "cavity_128_fp32", [inputs.config("cavity_128_fp32")], "fp32"
    yield "cavity_128_fp64", [inputs.config("cavity_128_fp32")], "fp64"
    yield "cavity_64_fp32", [inputs.config("cavity_64_adjoint")], "fp32"
    yield "batch_64_fp32", inputs.batch_cavities(), "fp32"
    yield "shock_m1.5_paper_fp32", [inputs.config("shock_m1.5_paper")], "fp32"
    yield "shock_m3_paper_fp32", [inputs.config("shock_m3_paper")], "fp32"
    yield "shock_m1.5_paper_reduced_fp32", [inputs.config("shock_m1.5_paper_reduced")], "fp32"
    yield "shock_m3_paper_reduced_fp32", [inputs.config("shock_m3_paper_reduced")], "fp32"
    yield "table_cavity_160_fp32", [inputs.table_cavity(1.0)], "fp32"
    yield "table_cavity_160_reduced_fp32", [inputs.table_cavity(1.0, nv=(20, 20, 2), reduced=True)], "fp32"


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=binding.TUNED_PATH, help="where to write the table")
    ap.add_argument("--only", default="", help="comma-separated workload names (default: all)")
    args = ap.parse_args()
    only = {w for w in args.only.split(",") if w}
    torch.cuda.set_device(0)
    table = binding.load_tuned()
    for name, probs, prec in workloads():
        if only and name not in only:
            continue
        ctx = binding.Context(probs, prec, tune="off")
        f = ctx.initial_state()
        torch.cuda.synchronize()
        shape = ctx.autotune(f)
        table[ctx.key] = {k: shape[k] for k in ("vec", "unroll", "vsplit", "persist")} | {"us": round(shape["tuned_us"], 2),
                                                                                "workload": name}
        print(f"{name}: {ctx.key} -> {table[ctx.key]}", flush=True)
        del f
        ctx.close()
        torch.cuda.empty_cache()
    with open(args.out, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
