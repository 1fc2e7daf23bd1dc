"""Write the oracle's reverse-sweep results for the full adjoint workload
(64^2 cavity, 24^3 velocities, Kn 0.1, lid Mach 0.1, 200 steps, loss = lid
shear at the final step, f0 = rest Maxwellian times (1 + 1e-3 xi)).

Calls only the FP64 oracle and the seeded inputs.  Checkpoints every 20 steps
and recomputes inside segments (all 201 states would need 91 GB).

    python tests/golden/make_adjoint_golden.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_0903_4044_amd import inputs  # noqa: E402

CELLS = (0, 63, 2016, 4095)  # sampled cells whose lambda^0 is stored
DIRS = (101, 102, 103)       # seeds of the stored projections <lambda^0, xi f0>


def main(every: int = 20):
    cfg = inputs.config("cavity_64_adjoint")
    nsteps = cfg["steps"]
    O = oracle.Oracle(cfg)
    f0 = O.initial_state() * (1.0 + 1e-3 * inputs.noise(O.shape))
    t0 = time.time()
    ckpt, f = [], f0
    for s in range(0, nsteps, every):
        ckpt.append(f)
        f = O.step(f, min(every, nsteps - s))
        print(f"forward {s + every} ({time.time() - t0:.0f} s)", flush=True)
    L = O.lid_shear(f)
    lam, grad = O.lid_shear_grad(f)
    del f
    for seg in range(len(ckpt) - 1, -1, -1):
        k = min(every, nsteps - seg * every)
        states = [ckpt[seg]]
        for _ in range(k - 1):
            states.append(O.step(states[-1]))
        for i in range(k - 1, -1, -1):
            lam, g = O.step_adjoint(states[i], lam)
            grad = grad + g
        print(f"reverse to step {seg * every} ({time.time() - t0:.0f} s)", flush=True)
    proj = np.array([np.sum(lam * inputs.noise(O.shape, seed=s) * f0) for s in DIRS])
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cavity_64_adjoint_oracle.npz")
    np.savez_compressed(path, L=L, grad=grad, proj=proj, dirs=np.array(DIRS), cells=np.array(CELLS),
                        lam0_cells=lam[list(CELLS)], dt=O.dt, every=every)
    print("wrote", path, "L", L, "grad", grad, "proj", proj)


if __name__ == "__main__":
    main()
