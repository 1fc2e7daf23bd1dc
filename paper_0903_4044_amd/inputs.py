"""Problem statements and seeded synthetic inputs.

This module holds parameter sets and random draws only: it contains none of
the solver's arithmetic (no Maxwellian, no moment, no streaming formula), so
that the HIP library and the FP64 oracle can both be driven from it without
sharing any code of the method.

A problem is a plain ``dict`` with the keys below (units are the normalised
ones of Sec. 4.1 of the paper: velocity in sqrt(2 R T_r), temperature in T_r,
density in n_r, length in the domain unit, time in length / sqrt(2 R T_r)):

    kind       'shock' (1D, far-field Maxwellian ghosts, Sec. 4.1),
               'cavity' (2D, diffuse walls, Sec. 5.1),
               'cavity3d' (3D: six diffuse walls, the lid at y = y1 moving along x;
               Sec. 2.1 carries the method over to three directions),
               'periodic1d' / 'periodic2d' / 'periodic3d' (test problems)
    nx, ny, nz spatial cells (ny = 1 for 1D kinds, nz = 1 for 1D and 2D kinds)
    x0, x1, y0, y1, z0, z1   spatial box
    nv         (Nvx, Nvy, Nvz) velocity cells (Sec. 2.1)
    vlo, vhi   velocity box per component
    kn, omega  collision frequency nu = n T^(1-omega) / Kn
    cfl, dt    dt > 0 fixes the time step, else dt comes from cfl
    mach       shock: upstream Mach number (Eq. RH)
    lid_mach   cavity: lid speed as a Mach number at the wall temperature
    t_wall     cavity: wall temperature
    splitting  'strang' (R_{dt/2} S_dt R_{dt/2}) or 'lie' (R_dt S_dt, Sec. 2.1)
    limiter    'minmod' (second order), 'none' (first-order upwind, Eq. upwind) or
               'shift' (Sec. 2.1 translation form: integer part of the Courant
               number as a shift, Eq. upwind over the fraction; 1D kinds)
    maxwellian 'point' (Eq. Maxw at the cell's moments) or 'conservative'
               (Eq. Maxw at the effective parameters whose grid moments are the
               cell's, Sec. 2.1, the remark after Eq. exact)
    reduced    True: two-dimensional kinds with v_z integrated out (nv[2] = 2,
               planes g = int f dv_z and h = int v_z^2 f dv_z)
    steps      number of time steps of the workload
    precision  'fp64' or 'fp32' (storage/streaming precision of f)
"""
from __future__ import annotations

import copy

import numpy as np

BATCH_SEED = 9034044
NOISE_SEED = 9034045


def _base(**kw):
    d = dict(kind="shock", nx=1, ny=1, nz=1, x0=0.0, x1=1.0, y0=0.0, y1=1.0, z0=0.0, z1=1.0,
             nv=(8, 8, 8), vlo=(-4.0, -4.0, -4.0), vhi=(4.0, 4.0, 4.0),
             kn=1.0, omega=0.5, cfl=0.5, dt=0.0, mach=0.0, lid_mach=0.0,
             t_wall=1.0, splitting="strang", limiter="minmod", maxwellian="point",
             steps=1, precision="fp64")
    d.update(kw)
    return d


# The five workloads.  Sizes follow the paper's two problems (Sec. 4.1 and
# Sec. 5.1) at the resolutions this library is measured on.
CONFIGS = {
    # 1D normal shock, Mach 1.5, FP64 throughout, 200 Strang steps.
    "shock_m1.5_fp64": _base(kind="shock", nx=256, x0=-20.0, x1=20.0,
                             nv=(32, 32, 32), vlo=(-6.0,) * 3, vhi=(6.0,) * 3,
                             kn=1.0, mach=1.5, steps=200, precision="fp64"),
    # 1D normal shock, Mach 3, FP32 f with FP64 moments, 2000 steps.
    "shock_m3_fp32": _base(kind="shock", nx=1024, x0=-20.0, x1=20.0,
                           nv=(48, 48, 48), vlo=(-8.0,) * 3, vhi=(8.0,) * 3,
                           kn=1.0, mach=3.0, steps=2000, precision="fp32"),
    # 2D lid-driven cavity 128^2, lid Mach 0.1, Kn 0.1, 5000 steps.
    "cavity_128_fp32": _base(kind="cavity", nx=128, ny=128, nv=(24, 24, 24),
                             vlo=(-5.0,) * 3, vhi=(5.0,) * 3, kn=0.1,
                             lid_mach=0.1, t_wall=1.0, steps=5000,
                             precision="fp32"),
    # The paper's own shock runs (Sec. 4.1): L = 70 mean free paths, Nx up to
    # 18432, dt = 0.05, Lie splitting, translation-form first-order streaming
    # (Courant numbers up to ~150 here), viscosity exponent 0.74, the paper's
    # velocity boxes (16^3 for Mach 1.5, 30^3 for Mach 3), FP32 f.
    "shock_m1.5_paper": _base(kind="shock", nx=18432, x0=-35.0, x1=35.0,
                              nv=(16, 16, 16), vlo=(-5.0, -6.0, -6.0), vhi=(7.0, 6.0, 6.0),
                              kn=1.0, omega=0.74, dt=0.05, mach=1.5, splitting="lie",
                              limiter="shift", steps=400, precision="fp32"),
    "shock_m3_paper": _base(kind="shock", nx=18432, x0=-35.0, x1=35.0,
                            nv=(30, 30, 30), vlo=(-10.0, -11.0, -11.0), vhi=(12.0, 11.0, 11.0),
                            kn=1.0, omega=0.74, dt=0.05, mach=3.0, splitting="lie",
                            limiter="shift", steps=200, precision="fp32"),
    # The Mach-3 shock and the 128^2 cavity relaxing towards the effective
    # Maxwellian (Sec. 2.1, the remark after Eq. exact).
    "shock_m3_fp32_conservative": _base(kind="shock", nx=1024, x0=-20.0, x1=20.0,
                                        nv=(48, 48, 48), vlo=(-8.0,) * 3, vhi=(8.0,) * 3,
                                        kn=1.0, mach=3.0, steps=2000, precision="fp32",
                                        maxwellian="conservative"),
    "cavity_128_fp32_conservative": _base(kind="cavity", nx=128, ny=128, nv=(24, 24, 24),
                                          vlo=(-5.0,) * 3, vhi=(5.0,) * 3, kn=0.1,
                                          lid_mach=0.1, t_wall=1.0, steps=5000,
                                          precision="fp32", maxwellian="conservative"),
    # The paper's shock runs in the reduced velocity space (v_y, v_z
    # integrated out: g and h on the v_x grid of the boxes above).
    "shock_m1.5_paper_reduced": _base(kind="shock", nx=18432, x0=-35.0, x1=35.0,
                                      nv=(16, 1, 2), vlo=(-5.0, -1.0, -1.0), vhi=(7.0, 1.0, 1.0),
                                      kn=1.0, omega=0.74, dt=0.05, mach=1.5, splitting="lie",
                                      limiter="shift", steps=400, precision="fp32", reduced=True),
    "shock_m3_paper_reduced": _base(kind="shock", nx=18432, x0=-35.0, x1=35.0,
                                    nv=(30, 1, 2), vlo=(-10.0, -1.0, -1.0), vhi=(12.0, 1.0, 1.0),
                                    kn=1.0, omega=0.74, dt=0.05, mach=3.0, splitting="lie",
                                    limiter="shift", steps=200, precision="fp32", reduced=True),
    # The lid-driven cube: 48^3 cells, 16^3 velocities on [-4.5, 4.5]^3
    # (v_z changes sign at plane 8), lid Mach 0.1, Kn 0.1, six diffuse walls.
    "cube_48_fp32": _base(kind="cavity3d", nx=48, ny=48, nz=48, z0=0.0, z1=1.0, nv=(16, 16, 16),
                          vlo=(-4.5,) * 3, vhi=(4.5,) * 3, kn=0.1, lid_mach=0.1, t_wall=1.0, steps=200,
                          precision="fp32"),
    # Adjoint workload: 64^2 cavity, 200 steps.
    "cavity_64_adjoint": _base(kind="cavity", nx=64, ny=64, nv=(24, 24, 24),
                               vlo=(-5.0,) * 3, vhi=(5.0,) * 3, kn=0.1,
                               lid_mach=0.1, t_wall=1.0, steps=200,
                               precision="fp32"),
}

# The driven-cavity runs of the Table of Sec. 5.2: rarefaction parameter
# delta = 1 / Kn on the unit square, 160 x 160 cells, 20^3 velocities on
# [-3, 3]^3, a lid speed of 0.01 sqrt(2 R T_w) (lid_mach = 0.01 / sqrt(5/6)),
# walls at T_w = 1, run from rest to a steady state.
TABLE_DELTAS = (0.1, 1.0, 10.0)


def table_cavity(delta: float, **override) -> dict:
    d = _base(kind="cavity", nx=160, ny=160, nv=(20, 20, 20), vlo=(-3.0,) * 3, vhi=(3.0,) * 3,
              kn=1.0 / delta, lid_mach=0.01 / (5.0 / 6.0) ** 0.5, t_wall=1.0, steps=0,
              maxwellian="conservative", precision="fp32")
    d.update(override)
    return d


SIDES = (32, 48, 64, 96, 128)


def config(name: str, **override) -> dict:
    """A deep copy of a named workload, with keyword overrides."""
    d = copy.deepcopy(CONFIGS[name])
    d.update(override)
    return d


def batch_cavities(n: int = 64, seed: int = BATCH_SEED, steps: int = 1000,
                   precision: str = "fp32") -> list[dict]:
    """Seeded draw of ``n`` independent lid-driven cavities.

    Per instance, in order: side from {32, 48, 64, 96, 128} (uniform),
    Kn = 10**U(-2, 0) (log-uniform on [0.01, 1]), lid Mach U(0.05, 0.3).
    All share a 24^3 velocity grid on [-5, 5]^3 and T_wall = 1.
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        side = int(rng.choice(SIDES))
        kn = float(10.0 ** rng.uniform(-2.0, 0.0))
        ma = float(rng.uniform(0.05, 0.3))
        out.append(_base(kind="cavity", nx=side, ny=side, nv=(24, 24, 24),
                         vlo=(-5.0,) * 3, vhi=(5.0,) * 3, kn=kn,
                         lid_mach=ma, t_wall=1.0, steps=steps,
                         precision=precision))
    return out


def batch_mixed(seed: int = BATCH_SEED + 2, precision: str = "fp32") -> list[dict]:
    """The 64-cavity batch and 8 seeded normal shocks on the same 24^3 grid
    on [-5, 5]^3, stepped together: per shock, in order, Nx from {256, 512,
    1024} (uniform) on [-20, 20] and Mach U(1.2, 2.0), Kn 1."""
    rng = np.random.default_rng(seed)
    out = batch_cavities(precision=precision)
    for _ in range(8):
        nx = int(rng.choice((256, 512, 1024)))
        mach = float(rng.uniform(1.2, 2.0))
        out.append(_base(kind="shock", nx=nx, x0=-20.0, x1=20.0, nv=(24, 24, 24), vlo=(-5.0,) * 3,
                         vhi=(5.0,) * 3, kn=1.0, mach=mach, steps=1000, precision=precision))
    return out


def noise(shape, seed: int = NOISE_SEED) -> np.ndarray:
    """Standard normal draws (FP64, C order) for the seeded perturbation."""
    return np.random.default_rng(seed).standard_normal(shape)


def uniform(shape, seed: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """Uniform draws (FP64, C order) for test inputs."""
    return np.random.default_rng(seed).uniform(lo, hi, shape)


def ndim(p: dict) -> int:
    """Streaming directions of a problem."""
    return 3 if p["kind"] in ("cavity3d", "periodic3d") else 2 if p["kind"] in ("cavity", "periodic2d") else 1


def ncells(p: dict) -> int:
    d = ndim(p)
    return int(p["nx"]) * (int(p["ny"]) if d >= 2 else 1) * (int(p.get("nz", 1)) if d == 3 else 1)


def nvel(p: dict) -> int:
    a, b, c = p["nv"]
    return int(a) * int(b) * int(c)


def is_2d(p: dict) -> bool:
    return p["kind"] in ("cavity", "periodic2d")


def is_3d(p: dict) -> bool:
    return p["kind"] in ("cavity3d", "periodic3d")
