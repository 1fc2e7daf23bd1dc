"""NumPy twin of the FP64 oracle, for tiny inputs only (test infrastructure).

Written separately from ``bgk_oracle.c`` and in a different style (whole-array
operations on f shaped (ny, nx, Nvz, Nvy, Nvx), face arrays built by slicing)
so that a slip in one is unlikely to be repeated in the other.  It follows the
same passages of the paper: Eqs. (Maxw), (macroscopic), (frequency) of Sec. 2,
the splitting and Eqs. (upwind), (relaxation) of Sec. 2.1, Eqs. (bc_shock),
(RH) of Sec. 4.1 and Eq. (bc_cavity) of Sec. 5.1, with the same readings
(minmod flux-form streaming, Strang or Lie composition, two ghost layers,
discrete zero-mass-flux wall density, lid Mach number at T_r), and the same
variants (translation-form streaming, effective Maxwellian parameters, the
reduced velocity space).
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = 5.0 / 3.0


class Twin:
    def __init__(self, cfg: dict):
        self.cfg = cfg
        self.kind = cfg["kind"]
        self.two = self.kind in ("cavity", "periodic2d")
        self.nx = int(cfg["nx"])
        self.ny = int(cfg["ny"]) if self.two else 1
        nvx, nvy, nvz = (int(k) for k in cfg["nv"])
        self.nvs = (nvz, nvy, nvx)
        axes = []
        for a, k in enumerate((nvx, nvy, nvz)):
            lo, hi = float(cfg["vlo"][a]), float(cfg["vhi"][a])
            h = (hi - lo) / k
            axes.append(lo + h * (np.arange(k) + 0.5))
        self.dv = [(float(cfg["vhi"][a]) - float(cfg["vlo"][a])) / int(cfg["nv"][a]) for a in range(3)]
        # reduced velocity space: the components the problem does not stream
        # along are integrated out; the z axis then holds two planes, the
        # integral g and the moment h of the transverse speed squared
        self.out = (1 if self.two else 2) if cfg.get("reduced", False) else 0
        if self.out:
            axes[2] = np.zeros(2)
            self.dv[2] = 1.0
        if self.out == 2:
            axes[1] = np.zeros(1)
            self.dv[1] = 1.0
        self.dV = self.dv[0] * self.dv[1] * self.dv[2]
        # broadcastable velocity components over (jz, jy, jx)
        self.VZ, self.VY, self.VX = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
        # per node: share in mass and momentum, extra energy term
        self.W = np.ones_like(self.VX)
        self.E = np.zeros_like(self.VX)
        if self.out:
            self.W[1] = 0.0
            self.E[1] = 1.0
        self.dx = (float(cfg["x1"]) - float(cfg["x0"])) / self.nx
        self.dy = (float(cfg["y1"]) - float(cfg["y0"])) / self.ny if self.two else 1.0
        self.kn = float(cfg["kn"])
        self.omega = float(cfg["omega"])
        self.strang = cfg.get("splitting", "strang") == "strang"
        self.limited = cfg.get("limiter", "minmod") == "minmod"

    # -- shapes ---------------------------------------------------------
    def to5(self, f):
        return np.asarray(f, dtype=np.float64).reshape((self.ny, self.nx) + self.nvs)

    def to2(self, f5):
        return f5.reshape(self.ny * self.nx, -1)

    @property
    def dt(self):
        if float(self.cfg.get("dt", 0.0)) > 0:
            return float(self.cfg["dt"])
        rate = np.abs(self.VX) / self.dx
        if self.two:
            rate = rate + np.abs(self.VY) / self.dy
        return float(self.cfg["cfl"]) / rate.max()

    # -- physics --------------------------------------------------------
    def maxwell(self, n, u, T):
        """Maxwellian(s); n, T of shape S, u of shape S+(3,) -> S+(Nvz,Nvy,Nvx)."""
        n = np.asarray(n, dtype=float)[..., None, None, None]
        T = np.asarray(T, dtype=float)[..., None, None, None]
        u = np.asarray(u, dtype=float)
        c2 = ((self.VX - u[..., 0, None, None, None]) ** 2
              + (self.VY - u[..., 1, None, None, None]) ** 2
              + (self.VZ - u[..., 2, None, None, None]) ** 2)
        if self.out:
            # integrals over the components out of the Maxwellian (g) and of
            # it times their speed squared (h = out * T / 2 times g)
            g = n / (math.pi * T) ** (1.5 - 0.5 * self.out) * np.exp(-c2 / T)
            return np.where(self.W > 0, g, 0.5 * self.out * T * g)
        return n / (math.pi * T) ** 1.5 * np.exp(-c2 / T)

    def macro(self, f5):
        ax = (-3, -2, -1)
        mf = f5 * self.W
        n = mf.sum(axis=ax) * self.dV
        u = np.stack([(mf * V).sum(axis=ax) for V in (self.VX, self.VY, self.VZ)], -1) * self.dV / n[..., None]
        c2 = ((self.VX - u[..., 0, None, None, None]) ** 2 + (self.VY - u[..., 1, None, None, None]) ** 2
              + (self.VZ - u[..., 2, None, None, None]) ** 2)
        T = ((c2 * self.W + self.E) * f5).sum(axis=ax) * self.dV / n * (2.0 / 3.0)
        return n, u, T

    def effective(self, n, u, T):
        """Effective parameters of one cell (Sec. 2.1, the remark on
        conservation after Eq. (exact)): the (n~, u~, T~) whose Maxwellian on
        the grid has the grid moments (n, u, T).  Found with SciPy's hybrid
        Powell root finder on those five equations (residuals scaled by n,
        sqrt(T), T), started at (n, u, T)."""
        from scipy.optimize import root

        target = np.array([n, u[0], u[1], u[2], T], dtype=float)
        scale = np.array([n, math.sqrt(T), math.sqrt(T), math.sqrt(T), T])
        free = [0, 1, 2, 3, 4] if not self.out else ([0, 1, 2, 4] if self.out == 1 else [0, 1, 4])

        def resid(x):
            q = target.copy()
            q[free] = x
            m = self.macro(self.maxwell(q[0], q[1:4], q[4]))
            return ((np.array([m[0], *m[1], m[2]]) - target) / scale)[free]

        sol = root(resid, target[free].copy(), method="hybr", options={"xtol": 1e-15})
        q = target.copy()
        q[free] = sol.x
        return q

    def relax(self, f5, tau):
        n, u, T = self.macro(f5)
        if self.cfg.get("maxwellian", "point") == "conservative":
            q = np.array([self.effective(float(a), b, float(c)) for a, b, c in
                          zip(n.ravel(), u.reshape(-1, 3), T.ravel())]).reshape(n.shape + (5,))
            M = self.maxwell(q[..., 0], q[..., 1:4], q[..., 4])
        else:
            M = self.maxwell(n, u, T)
        nu = n * T ** (1.0 - self.omega) / self.kn
        k = np.exp(-nu * tau)[..., None, None, None]
        return M + (f5 - M) * k

    # -- boundaries -----------------------------------------------------
    def _far_field(self):
        M = float(self.cfg["mach"])
        r = 4 * M * M / (M * M + 3)
        Vu = M * math.sqrt(GAMMA / 2)
        Tr = (5 * M * M - 1) * (M * M + 3) / (16 * M * M)
        left = self.maxwell(1.0, np.array([Vu, 0, 0]), 1.0)
        right = self.maxwell(r, np.array([Vu / r, 0, 0]), Tr)
        return left, right

    def _wall(self, g_adj, vn_inward, uw):
        """Ghost values of one wall face. g_adj: (..., vel); vn_inward: v.n."""
        phiw = self.maxwell(1.0, np.array([uw, 0.0, 0.0]), float(self.cfg["t_wall"]))
        out_mask = vn_inward > 0
        in_mask = vn_inward < 0
        arrive = (np.where(in_mask, -vn_inward, 0.0) * self.W * g_adj).sum(axis=(-3, -2, -1))
        leave = (np.where(out_mask, vn_inward, 0.0) * self.W * phiw).sum()
        nw = arrive / leave
        return np.where(out_mask, nw[..., None, None, None] * phiw, g_adj)

    def padded(self, g5):
        ny, nx = self.ny, self.nx
        if self.two:
            P = np.zeros((ny + 4, nx + 4) + self.nvs)
            P[2:-2, 2:-2] = g5
            core = (slice(2, -2),)
        else:
            P = np.zeros((1, nx + 4) + self.nvs)
            P[:, 2:-2] = g5
            core = (slice(None),)
        if self.kind == "shock":
            left, right = self._far_field()
            P[:, 0] = P[:, 1] = left
            P[:, -1] = P[:, -2] = right
        elif self.kind.startswith("periodic"):
            P[core + (slice(0, 2),)] = g5[:, -2:]
            P[core + (slice(-2, None),)] = g5[:, :2]
            if self.two:
                P[0:2, 2:-2] = g5[-2:]
                P[-2:, 2:-2] = g5[:2]
        else:
            uw = float(self.cfg["lid_mach"]) * math.sqrt(GAMMA / 2)
            gl = self._wall(g5[:, 0], self.VX, 0.0)
            gr = self._wall(g5[:, -1], -self.VX, 0.0)
            gb = self._wall(g5[0, :], self.VY, 0.0)
            gt = self._wall(g5[-1, :], -self.VY, uw)
            P[2:-2, 0] = P[2:-2, 1] = gl
            P[2:-2, -1] = P[2:-2, -2] = gr
            P[0, 2:-2] = P[1, 2:-2] = gb
            P[-1, 2:-2] = P[-2, 2:-2] = gt
        return P

    # -- streaming ------------------------------------------------------
    def _fluxdiff(self, P, axis, C):
        """C*(face_{i+1/2} - face_{i-1/2}) along spatial axis (0=y, 1=x) of P."""
        n = P.shape[axis] - 4

        def sl(a, b):
            idx = [slice(None)] * P.ndim
            idx[axis] = slice(a, P.shape[axis] + b if b <= 0 else b)
            return P[tuple(idx)]

        d = sl(1, 0) - sl(0, -1)  # d[k] = P[k+1] - P[k], k = 0..n+2
        if self.limited:
            a, b = d[tuple(self._cut(axis, 1, None, P.ndim))], d[tuple(self._cut(axis, 0, -1, P.ndim))]
            s = np.where(a * b > 0, np.where(np.abs(a) < np.abs(b), a, b), 0.0)  # slopes, cells 1..n+2
        else:
            s = np.zeros_like(sl(1, -1))
        # faces k+1/2 for padded k = 1..n+1 (i.e. interior faces -1/2 .. n-1/2)
        vals = sl(1, -1)  # padded cells 1..n+2
        left_state = self._take(vals, axis, 0, n + 1) + 0.5 * (1 - C) * self._take(s, axis, 0, n + 1)
        right_state = self._take(vals, axis, 1, n + 2) - 0.5 * (1 + C) * self._take(s, axis, 1, n + 2)
        face = np.where(C > 0, left_state, np.where(C < 0, right_state, 0.0))
        return C * (self._take(face, axis, 1, n + 1) - self._take(face, axis, 0, n))

    @staticmethod
    def _cut(axis, a, b, nd):
        idx = [slice(None)] * nd
        idx[axis] = slice(a, b)
        return idx

    @staticmethod
    def _take(x, axis, a, b):
        idx = [slice(None)] * x.ndim
        idx[axis] = slice(a, b)
        return x[tuple(idx)]

    def _shift_stream(self, g5, dt):
        """Translation form of free streaming (Sec. 2.1, below Eq. (exact)):
        per v_x column, the values |C| = m + th cells upwind, gathered by
        index arithmetic on the cell axis (far-field states or periodic
        images outside the box) and blended over the fraction th."""
        out = np.empty_like(g5)
        nx = self.nx
        base = g5[0]  # (nx, nvz, nvy, nvx)
        if self.kind == "shock":
            left, right = self._far_field()
        for jx, vx in enumerate(self.VX[0, 0, :]):
            C = vx * dt / self.dx
            s = 1 if C > 0 else -1
            m = int(math.floor(abs(C)))
            th = abs(C) - m
            src = []
            for k in (0, 1):
                pos = np.arange(nx) - s * (m + k)
                if self.kind == "shock":
                    col = base[np.clip(pos, 0, nx - 1)][..., jx]
                    col = np.where((pos < 0)[:, None, None], left[..., jx][None], col)
                    col = np.where((pos >= nx)[:, None, None], right[..., jx][None], col)
                else:
                    col = base[np.mod(pos, nx)][..., jx]
                src.append(col)
            out[0, :, :, :, jx] = (1 - th) * src[0] + th * src[1]
        return out

    def stream(self, g5, dt):
        if self.cfg.get("limiter", "minmod") == "shift":
            return self._shift_stream(g5, dt)
        P = self.padded(g5)
        if self.two:
            Cx = self.VX * dt / self.dx
            Cy = self.VY * dt / self.dy
            dxf = self._fluxdiff(P[2:-2], 1, Cx)
            dyf = self._fluxdiff(P[:, 2:-2], 0, Cy)
            return g5 - dxf - dyf
        Cx = self.VX * dt / self.dx
        return g5 - self._fluxdiff(P, 1, Cx)

    def step(self, f, nsteps=1):
        f5 = self.to5(f).copy()
        dt = self.dt
        for _ in range(nsteps):
            if self.strang:
                f5 = self.relax(self.stream(self.relax(f5, dt / 2), dt), dt / 2)
            else:
                f5 = self.relax(self.stream(f5, dt), dt)
        return self.to2(f5)
