"""Write the oracle's moments of long full-size runs to tests/golden/.

Calls only the FP64 oracle and the problem statements; the stored values are
what the parity tests compare the HIP path with at full size and full step
count, where running the oracle inside a test would take too long.  The file
is rewritten after every mark, so a long run leaves the marks it reached.

    python tests/golden/make_golden.py shock_m3_fp32 1,10,100,500,1000,2000
    python tests/golden/make_golden.py cavity_128_fp32 1,10,100,1000,2500,5000 [OUT.npz]

(OUT.npz: where to write instead of tests/golden/<name>_oracle.npz.)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_0903_4044_amd import inputs  # noqa: E402


def save(path: str, out: dict):
    tmp = path + ".tmp.npz"
    np.savez_compressed(tmp, **out)
    os.replace(tmp, path)


def main(name: str, marks: list[int], path: str | None = None):
    cfg = inputs.config(name)
    O = oracle.Oracle(cfg)
    f = O.initial_state()
    path = path or os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_oracle.npz")
    out = {"dt": np.array(O.dt), "steps": np.array([], dtype=np.int64)}
    done = 0
    t0 = time.time()
    for m in marks:
        f = O.step(f, m - done) if m > done else f
        done = m
        out[f"moments_{m}"] = O.moments(f)
        out[f"totals_{m}"] = O.totals(f)
        out["steps"] = np.append(out["steps"], m)
        save(path, out)
        print(f"{name}: step {m} ({time.time() - t0:.0f} s)", flush=True)
    print("wrote", path)


if __name__ == "__main__":
    main(sys.argv[1], [int(s) for s in sys.argv[2].split(",")], sys.argv[3] if len(sys.argv) > 3 else None)
