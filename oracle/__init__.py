"""FP64 CPU oracle of the BGK discrete-velocity step (test infrastructure).

This package is the independent reference the HIP library is checked
against.  Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it.  It shares no code with the
library under ``paper_0903_4044_amd/``; both read problem statements from
``paper_0903_4044_amd.inputs`` (parameters and seeded draws only).

The arithmetic lives in ``bgk_oracle.c`` (plain C, FP64, OpenMP over spatial
cells), compiled with gcc by :func:`build`.  ``twin.py`` is a second, NumPy
implementation written separately, used only to cross-check the C code on
tiny inputs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bgk_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

KINDS = {"shock": 0, "cavity": 1, "periodic1d": 2, "periodic2d": 3, "cavity3d": 4, "periodic3d": 5}


class Problem(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("x0", ctypes.c_double), ("x1", ctypes.c_double),
        ("y0", ctypes.c_double), ("y1", ctypes.c_double),
        ("nv", ctypes.c_int * 3),
        ("vlo", ctypes.c_double * 3), ("vhi", ctypes.c_double * 3),
        ("kn", ctypes.c_double), ("omega", ctypes.c_double),
        ("cfl", ctypes.c_double), ("dt", ctypes.c_double),
        ("mach", ctypes.c_double), ("lid_mach", ctypes.c_double),
        ("t_wall", ctypes.c_double),
        ("strang", ctypes.c_int), ("minmod", ctypes.c_int),
        ("conservative", ctypes.c_int),
        ("reduced", ctypes.c_int),
        ("nz", ctypes.c_int),
        ("z0", ctypes.c_double), ("z1", ctypes.c_double),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fno-fast-math", "-ffp-contract=off",
                               "-shared", "-fPIC", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=False)
        L = ctypes.CDLL(LIB)
        P = ctypes.POINTER(Problem)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_dt.argtypes = [P]
        L.orc_dt.restype = ctypes.c_double
        L.orc_velocity_nodes.argtypes = [P, dp, dp, dp]
        L.orc_maxwellian.argtypes = [P, ctypes.c_double, dp, ctypes.c_double, dp]
        L.orc_moments.argtypes = [P, dp, dp]
        L.orc_collision_frequency.argtypes = [P, ctypes.c_double, ctypes.c_double]
        L.orc_collision_frequency.restype = ctypes.c_double
        L.orc_relax.argtypes = [P, dp, dp, ctypes.c_double]
        L.orc_effective_parameters.argtypes = [P, ctypes.c_double, dp, ctypes.c_double, dp]
        L.orc_effective_parameters.restype = ctypes.c_int
        L.orc_rankine_hugoniot.argtypes = [ctypes.c_double, dp, dp]
        L.orc_wall_density.argtypes = [P, dp, dp]
        L.orc_stream.argtypes = [P, dp, dp, ctypes.c_double]
        L.orc_step.argtypes = [P, dp, dp]
        L.orc_run.argtypes = [P, dp, ctypes.c_int]
        L.orc_initial_state.argtypes = [P, dp]
        L.orc_totals.argtypes = [P, dp, dp]
        L.orc_lid_shear.argtypes = [P, dp]
        L.orc_lid_shear.restype = ctypes.c_double
        L.orc_cavity_metrics.argtypes = [P, dp, dp]
        L.orc_relax_adjoint.argtypes = [P, dp, dp, dp, ctypes.c_double, dp]
        L.orc_stream_adjoint.argtypes = [P, dp, dp, dp, ctypes.c_double, dp]
        L.orc_step_adjoint.argtypes = [P, dp, dp, dp, dp]
        L.orc_lid_shear_grad.argtypes = [P, dp, dp, dp]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_problem(cfg: dict) -> Problem:
    p = Problem()
    p.kind = KINDS[cfg["kind"]]
    p.nx = int(cfg["nx"])
    p.ny = int(cfg.get("ny", 1))
    p.x0, p.x1 = float(cfg["x0"]), float(cfg["x1"])
    p.y0, p.y1 = float(cfg.get("y0", 0.0)), float(cfg.get("y1", 1.0))
    for a in range(3):
        p.nv[a] = int(cfg["nv"][a])
        p.vlo[a] = float(cfg["vlo"][a])
        p.vhi[a] = float(cfg["vhi"][a])
    p.kn, p.omega = float(cfg["kn"]), float(cfg["omega"])
    p.cfl, p.dt = float(cfg.get("cfl", 0.5)), float(cfg.get("dt", 0.0))
    p.mach = float(cfg.get("mach", 0.0))
    p.lid_mach = float(cfg.get("lid_mach", 0.0))
    p.t_wall = float(cfg.get("t_wall", 1.0))
    p.strang = 1 if cfg.get("splitting", "strang") == "strang" else 0
    p.minmod = {"minmod": 1, "none": 0, "shift": 2}[cfg.get("limiter", "minmod")]
    p.conservative = {"point": 0, "conservative": 1}[cfg.get("maxwellian", "point")]
    p.reduced = 1 if cfg.get("reduced", False) else 0
    p.nz = int(cfg.get("nz", 1))
    p.z0, p.z1 = float(cfg.get("z0", 0.0)), float(cfg.get("z1", 1.0))
    if cfg["kind"] in ("cavity3d", "periodic3d") and p.reduced:
        raise ValueError("the reduced velocity space is defined for one- and two-dimensional kinds")
    two = cfg["kind"] in ("cavity", "periodic2d")
    if p.reduced and (int(cfg["nv"][2]) != 2 or (not two and int(cfg["nv"][1]) != 1)):
        raise ValueError("the reduced velocity space takes nv[2] = 2 (and nv[1] = 1 for one-dimensional kinds)")
    return p


class Oracle:
    """FP64 reference stepper for one problem (a dict of ``inputs``)."""

    def __init__(self, cfg: dict):
        self.cfg = dict(cfg)
        self.p = make_problem(cfg)
        self.L = lib()
        self.three_d = cfg["kind"] in ("cavity3d", "periodic3d")
        self.two_d = cfg["kind"] in ("cavity", "periodic2d")
        self.nx = self.p.nx
        self.ny = self.p.ny if (self.two_d or self.three_d) else 1
        self.nz = self.p.nz if self.three_d else 1
        self.ncell = self.nx * self.ny * self.nz
        self.nv = tuple(int(v) for v in cfg["nv"])
        self.nvel = self.nv[0] * self.nv[1] * self.nv[2]
        self.shape = (self.ncell, self.nvel)

    @property
    def dt(self) -> float:
        return self.L.orc_dt(ctypes.byref(self.p))

    def velocity_nodes(self):
        vx, vy, vz = (np.empty(self.nvel) for _ in range(3))
        self.L.orc_velocity_nodes(ctypes.byref(self.p), _ptr(vx), _ptr(vy), _ptr(vz))
        return vx, vy, vz

    def _f(self, f) -> np.ndarray:
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.shape)
        return f

    def initial_state(self) -> np.ndarray:
        f = np.empty(self.shape)
        self.L.orc_initial_state(ctypes.byref(self.p), _ptr(f))
        return f

    def maxwellian(self, n, V, T) -> np.ndarray:
        out = np.empty(self.nvel)
        Va = np.ascontiguousarray(V, dtype=np.float64)
        self.L.orc_maxwellian(ctypes.byref(self.p), float(n), _ptr(Va), float(T), _ptr(out))
        return out

    def moments(self, f) -> np.ndarray:
        f = self._f(f)
        m = np.empty((self.ncell, 5))
        self.L.orc_moments(ctypes.byref(self.p), _ptr(f), _ptr(m))
        return m

    def collision_frequency(self, n, T) -> float:
        return self.L.orc_collision_frequency(ctypes.byref(self.p), float(n), float(T))

    def effective_parameters(self, n, V, T):
        """(n~, V~, T~) whose discretized Maxwellian has the grid moments
        (n, V, T), and the number of Newton steps taken."""
        q = np.empty(5)
        Va = np.ascontiguousarray(V, dtype=np.float64)
        it = self.L.orc_effective_parameters(ctypes.byref(self.p), float(n), _ptr(Va), float(T), _ptr(q))
        return q, it

    def relax(self, f, tau) -> np.ndarray:
        f = self._f(f)
        out = np.empty(self.shape)
        self.L.orc_relax(ctypes.byref(self.p), _ptr(f), _ptr(out), float(tau))
        return out

    def stream(self, g, dt=None) -> np.ndarray:
        g = self._f(g)
        out = np.empty(self.shape)
        self.L.orc_stream(ctypes.byref(self.p), _ptr(g), _ptr(out), float(self.dt if dt is None else dt))
        return out

    def step(self, f, n: int = 1) -> np.ndarray:
        f = self._f(f).copy()
        if n == 1:
            out = np.empty(self.shape)
            self.L.orc_step(ctypes.byref(self.p), _ptr(f), _ptr(out))
            return out
        self.L.orc_run(ctypes.byref(self.p), _ptr(f), int(n))
        return f

    def wall_density(self, g) -> np.ndarray:
        g = self._f(g)
        L = max(self.nx, self.ny)
        out = np.zeros((4, L))
        self.L.orc_wall_density(ctypes.byref(self.p), _ptr(g), _ptr(out))
        return out

    def totals(self, f) -> np.ndarray:
        f = self._f(f)
        out = np.empty(6)
        self.L.orc_totals(ctypes.byref(self.p), _ptr(f), _ptr(out))
        return out

    def lid_shear(self, f) -> float:
        f = self._f(f)
        return self.L.orc_lid_shear(ctypes.byref(self.p), _ptr(f))

    def cavity_metrics(self, f) -> np.ndarray:
        """(D, G) of the Table of Sec. 5.2: mean lid shear stress over
        p0 U_W and twice the main vortex's centre-line flow rate."""
        f = self._f(f)
        out = np.empty(2)
        self.L.orc_cavity_metrics(ctypes.byref(self.p), _ptr(f), _ptr(out))
        return out

    # -- reverse sweep (hand-derived adjoint) -----------------------------
    def _no_conservative(self):
        if self.p.conservative or self.p.reduced or self.three_d:
            raise NotImplementedError("the reverse sweep covers the point-value Maxwellian in full velocity space, "
                                      "one- and two-dimensional kinds")

    def relax_adjoint(self, x, mu, tau):
        """(dR_tau/dx)^T mu at x, and dL/dKn."""
        self._no_conservative()
        x, mu = self._f(x), self._f(mu)
        out, g = np.empty(self.shape), np.zeros(1)
        self.L.orc_relax_adjoint(ctypes.byref(self.p), _ptr(x), _ptr(mu), _ptr(out), float(tau), _ptr(g))
        return out, float(g[0])

    def stream_adjoint(self, g_in, mu, dt=None):
        """(dS/dg)^T mu at g_in, and dL/dT_w."""
        self._no_conservative()
        g_in, mu = self._f(g_in), self._f(mu)
        out, gt = np.empty(self.shape), np.zeros(1)
        self.L.orc_stream_adjoint(ctypes.byref(self.p), _ptr(g_in), _ptr(mu), _ptr(out),
                                  float(self.dt if dt is None else dt), _ptr(gt))
        return out, float(gt[0])

    def step_adjoint(self, f, lam_next):
        """lam_n = (d step/df)^T lam_next and (dL/dKn, dL/dT_w) of this step."""
        self._no_conservative()
        f, lam_next = self._f(f), self._f(lam_next)
        out, grad = np.empty(self.shape), np.zeros(2)
        self.L.orc_step_adjoint(ctypes.byref(self.p), _ptr(f), _ptr(lam_next), _ptr(out), _ptr(grad))
        return out, grad

    def lid_shear_grad(self, f):
        """dL/df of the lid shear and its explicit (dL/dKn, dL/dT_w)."""
        self._no_conservative()
        f = self._f(f)
        lam, grad = np.empty(self.shape), np.zeros(2)
        self.L.orc_lid_shear_grad(ctypes.byref(self.p), _ptr(f), _ptr(lam), _ptr(grad))
        return lam, grad

    def rollout_gradient(self, f0, nsteps):
        """Loss = lid shear of f^nsteps; returns (L, dL/df0, dL/dKn, dL/dT_w)
        by storing every state and sweeping back."""
        states = [self._f(f0).copy()]
        for _ in range(nsteps):
            states.append(self.step(states[-1]))
        L = self.lid_shear(states[-1])
        lam, grad = self.lid_shear_grad(states[-1])
        for n in range(nsteps - 1, -1, -1):
            lam, gs = self.step_adjoint(states[n], lam)
            grad = grad + gs
        return L, lam, grad[0], grad[1]

    @staticmethod
    def rankine_hugoniot(mach):
        up, dn = np.empty(3), np.empty(3)
        lib().orc_rankine_hugoniot(float(mach), _ptr(up), _ptr(dn))
        return up, dn
