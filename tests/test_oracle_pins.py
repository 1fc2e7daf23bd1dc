"""Pins of the FP64 oracle against facts fixed by the paper or by mathematics.

None of these re-types the oracle's own formulas: each checks a closed form,
an invariant, a textbook special case or an independent implementation, chosen
so that a plausible slip in the oracle (a dropped factor in the Maxwellian or
in T, a wrong sign or index in the streaming, the wrong wall in n_W, a
transposed axis) makes at least one of them fail.
"""
import math

import numpy as np
import pytest

from paper_0903_4044_amd import inputs

GAMMA = 5.0 / 3.0


def prob(**kw):
    d = dict(kind="periodic1d", nx=4, ny=1, x0=0.0, x1=1.0, y0=0.0, y1=1.0,
             nv=(32, 32, 32), vlo=(-8.0,) * 3, vhi=(8.0,) * 3, kn=1.0, omega=0.5,
             cfl=0.5, dt=0.0, mach=0.0, lid_mach=0.0, t_wall=1.0,
             splitting="strang", limiter="minmod")
    d.update(kw)
    return d


def gauss(O, n, V, T):
    """Maxwellian point values written from the Gaussian integral, as the test's
    own closed form: n * prod_a exp(-(v_a - V_a)^2 / T) / sqrt(pi T)."""
    vx, vy, vz = O.velocity_nodes()
    out = np.full(vx.shape, float(n))
    for v, c in zip((vx, vy, vz), V):
        out *= np.exp(-((v - c) ** 2) / T) / math.sqrt(math.pi * T)
    return out


# --------------------------------------------------------------- Maxwellian


def test_maxwellian_discrete_moments(oracle_mod):
    """Sec. 2, Eqs. (Maxw) and (macroscopic): on a resolving grid the moments of
    the sampled Maxwellian are its parameters (midpoint rule on a Gaussian is
    spectrally accurate).  Pins the (pi T)^(-3/2) prefactor, the exponent and
    the 2/(3n) temperature factor."""
    O = oracle_mod.Oracle(prob(nv=(40, 40, 40), vlo=(-9,) * 3, vhi=(9,) * 3))
    for (n, V, T) in [(1.0, (0, 0, 0), 1.0), (2.5, (0.7, -0.3, 0.2), 1.7), (0.4, (1.2, 0.1, -0.5), 0.6)]:
        phi = O.maxwellian(n, np.array(V, float), T)
        np.testing.assert_allclose(phi, gauss(O, n, V, T), rtol=1e-13, atol=0)
        m = O.moments(np.tile(phi, (O.ncell, 1)))
        np.testing.assert_allclose(m[0], [n, *V, T], rtol=1e-11, atol=1e-12)


def test_rankine_hugoniot_fluxes(oracle_mod):
    """Sec. 4.1, Eq. (RH): the two far-field states carry equal fluxes of mass
    nV, momentum nV^2 + nT/2 and energy nV(V^2 + 5T/2) (moments of a drifting
    Maxwellian in sqrt(2RT) units), and the upstream Mach number is M."""
    for M in (1.5, 3.0):
        up, dn = oracle_mod.Oracle.rankine_hugoniot(M)
        assert up[1] / math.sqrt(GAMMA * up[2] / 2) == pytest.approx(M, rel=1e-15)

        def fl(s):
            n, V, T = s
            return np.array([n * V, n * V * V + n * T / 2, n * V * (V * V + 2.5 * T)])
        np.testing.assert_allclose(fl(dn), fl(up), rtol=1e-14)
    up, dn = oracle_mod.Oracle.rankine_hugoniot(1.5)
    # M = 1.5: n+ = 9/5.25 = 12/7, V+ = V-/n+, T+ = 10.25 * 5.25 / 36
    np.testing.assert_allclose(dn, [12 / 7, 1.5 * math.sqrt(5 / 6) * 7 / 12, 10.25 * 5.25 / 36], rtol=1e-14)


def test_discrete_shock_fluxes_match_closed_form(oracle_mod):
    """The velocity-grid flux sums of a far-field Maxwellian reproduce the
    closed-form fluxes above (pins the grid nodes and dV)."""
    O = oracle_mod.Oracle(prob(nv=(64, 64, 64), vlo=(-12,) * 3, vhi=(12,) * 3))
    vx, vy, vz = O.velocity_nodes()
    dV = (24 / 64) ** 3
    up, dn = oracle_mod.Oracle.rankine_hugoniot(3.0)
    for n, V, T in (up, dn):
        phi = O.maxwellian(n, np.array([V, 0, 0]), T)
        got = [np.sum(vx * phi) * dV, np.sum(vx * vx * phi) * dV,
               np.sum(vx * (vx * vx + vy * vy + vz * vz) * phi) * dV]
        want = [n * V, n * V * V + n * T / 2, n * V * (V * V + 2.5 * T)]
        np.testing.assert_allclose(got, want, rtol=1e-11)


# --------------------------------------------------------------- relaxation


def test_relaxation_fixed_point(oracle_mod):
    """Uniform Maxwellian is a fixed point of the relaxation (Sec. 2.1): it
    changes only by the discrete moment defect, far below 1e-12 here."""
    O = oracle_mod.Oracle(prob(nv=(40, 40, 40), vlo=(-9,) * 3, vhi=(9,) * 3))
    phi = O.maxwellian(1.3, np.array([0.4, -0.2, 0.1]), 1.4)
    f = np.tile(phi, (O.ncell, 1))
    out = O.relax(f, 0.37)
    assert np.max(np.abs(out - f)) <= 1e-12 * np.max(f)


def test_homogeneous_relaxation_closed_form(oracle_mod):
    """Sec. 2.1, Eq. (relaxation): with f uniform in space, streaming is the
    identity and f(t) = Phi_inf + (f0 - Phi_inf) exp(-nu t), Phi_inf carrying
    the (conserved) moments of f0.  f0 is two Maxwellians of density 1/2,
    velocities +-u e_x, temperature T0, whose mixture has n = 1, V = 0 and
    T = T0 + (2/3) u^2 in closed form; nu = n T^(1-omega) / Kn."""
    u, T0, kn, omega = 0.5, 0.8, 0.7, 0.74  # omega of Eq. (viscosity)
    for splitting in ("strang", "lie"):
        cfg = prob(nv=(40, 40, 40), kn=kn, omega=omega, splitting=splitting, dt=0.01)
        O = oracle_mod.Oracle(cfg)
        f0 = 0.5 * gauss(O, 1.0, (u, 0, 0), T0) + 0.5 * gauss(O, 1.0, (-u, 0, 0), T0)
        Tinf = T0 + 2.0 / 3.0 * u * u
        nu = 1.0 * Tinf ** (1 - omega) / kn
        nsteps = 25
        f = O.step(np.tile(f0, (O.ncell, 1)), nsteps)
        t = nsteps * 0.01
        Pinf = gauss(O, 1.0, (0, 0, 0), Tinf)
        want = Pinf + (f0 - Pinf) * math.exp(-nu * t)
        assert np.max(np.abs(f - want)) <= 1e-12 * np.max(f0)


def test_collisions_conserve(oracle_mod):
    """Relaxation conserves mass, momentum and energy (Sec. 2) up to the
    discrete Maxwellian's moment defect, which is below 1e-13 on this grid."""
    O = oracle_mod.Oracle(prob(nx=3, nv=(36, 36, 36), vlo=(-9,) * 3, vhi=(9,) * 3))
    base = gauss(O, 1.0, (0.3, -0.1, 0.2), 1.2)
    xi = inputs.uniform((O.ncell, O.nvel), seed=11, lo=0.5, hi=1.5)
    f = base[None, :] * xi
    before = O.totals(f)
    after = O.totals(O.relax(f, 0.9))
    np.testing.assert_allclose(after[:5], before[:5], rtol=1e-13, atol=1e-14)


def test_entropy_decreases_under_relaxation(oracle_mod):
    """H = sum f ln f is non-increasing under relaxation (convexity)."""
    O = oracle_mod.Oracle(prob(nx=2, nv=(24, 24, 24)))
    base = gauss(O, 1.0, (0.0, 0.0, 0.0), 1.5)
    f = base[None, :] * inputs.uniform((O.ncell, O.nvel), seed=3, lo=0.2, hi=1.8)
    h0 = O.totals(f)[5]
    g = O.relax(f, 0.1)
    h1 = O.totals(g)[5]
    h2 = O.totals(O.relax(g, 0.5))[5]
    assert h1 < h0 and h2 < h1


# ------------------------------------------------- conservative Maxwellian
# Sec. 2.1, the remark after Eq. (exact): the relaxation may use effective
# (n~, V~, T~) chosen so that the discretized Maxwellian has exactly the grid
# moments of the cell.


def coarse(**kw):
    return prob(nx=3, nv=(8, 8, 8), vlo=(-3,) * 3, vhi=(3,) * 3, maxwellian="conservative", **kw)


def test_effective_parameters_invert_the_discretization(oracle_mod):
    """A Maxwellian sampled with known (n0, V0, T0) on a coarse grid has grid
    moments off by ~1e-4; the effective parameters of those moments are
    (n0, V0, T0) again, and that Maxwellian is a fixed point of the
    conservative relaxation (but not of the point-value one)."""
    O = oracle_mod.Oracle(coarse())
    P = oracle_mod.Oracle(dict(coarse(), maxwellian="point"))
    for n0, V0, T0 in [(1.3, (0.3, -0.2, 0.1), 0.8), (0.6, (-0.5, 0.0, 0.4), 1.1)]:
        phi = gauss(O, n0, V0, T0)
        m = O.moments(np.tile(phi, (O.ncell, 1)))[0]
        assert np.max(np.abs(m - [n0, *V0, T0])) > 1e-5
        q, it = O.effective_parameters(m[0], m[1:4], m[4])
        assert it <= 8
        np.testing.assert_allclose(q, [n0, *V0, T0], rtol=0, atol=2e-14)
        f = np.tile(phi, (O.ncell, 1))
        assert np.max(np.abs(O.relax(f, 0.6) - f)) <= 1e-13 * phi.max()
        assert np.max(np.abs(P.relax(f, 0.6) - f)) > 1e-6 * phi.max()


def test_effective_parameters_newton_is_quadratic(oracle_mod):
    """On a very coarse grid (6^3 nodes on [-2.5, 2.5]^3, moment defects near
    1e-2) Newton's method with the exact Jacobian reaches the 1e-14 stop in at
    most 4 steps plus the closing one; a Jacobian with a slipped term
    converges only linearly and needs 6 or more."""
    O = oracle_mod.Oracle(prob(nx=3, nv=(6, 6, 6), vlo=(-2.5,) * 3, vhi=(2.5,) * 3, maxwellian="conservative"))
    for V, T in [((0.5, 0.1, 0.0), 1.0), ((-0.7, 0.3, 0.2), 0.6), ((0.0, 0.0, 0.0), 1.5)]:
        q, it = O.effective_parameters(1.0, np.array(V, float), T)
        assert abs(q[4] - T) > 5e-4 and it <= 5


def test_effective_parameters_resolved_grid_limit(oracle_mod):
    """On a grid that resolves the Maxwellian the moment defect vanishes, so
    the effective parameters are the moments themselves."""
    O = oracle_mod.Oracle(prob(nv=(40, 40, 40), vlo=(-9,) * 3, vhi=(9,) * 3, maxwellian="conservative"))
    for n, V, T in [(1.0, (0.0, 0.0, 0.0), 1.0), (2.5, (0.7, -0.3, 0.2), 1.7)]:
        q, _ = O.effective_parameters(n, np.array(V, float), T)
        np.testing.assert_allclose(q, [n, *V, T], rtol=0, atol=1e-12)


def test_effective_parameters_mirror_symmetry(oracle_mod):
    """On a grid symmetric about 0 the map (n, V, T) -> (n~, V~, T~) commutes
    with reflecting a velocity component, and V = 0 gives V~ = 0."""
    O = oracle_mod.Oracle(coarse())
    q, _ = O.effective_parameters(1.0, np.array([0.4, -0.25, 0.1]), 0.9)
    r, _ = O.effective_parameters(1.0, np.array([-0.4, -0.25, -0.1]), 0.9)
    np.testing.assert_allclose(r, q * [1, -1, 1, -1, 1], rtol=1e-14, atol=1e-15)
    z, _ = O.effective_parameters(1.0, np.zeros(3), 0.9)
    assert np.max(np.abs(z[1:4])) < 1e-15 and abs(z[4] - 0.9) > 1e-5


def test_conservative_relaxation_conserves_exactly(oracle_mod):
    """With the effective parameters the relaxation conserves mass, momentum
    and energy to rounding on a coarse grid, where the point-value
    Maxwellian's defect is above 1e-7."""
    O = oracle_mod.Oracle(coarse())
    P = oracle_mod.Oracle(dict(coarse(), maxwellian="point"))
    base = gauss(O, 1.0, (0.3, -0.1, 0.2), 1.2)
    f = base[None, :] * inputs.uniform((O.ncell, O.nvel), seed=11, lo=0.5, hi=1.5)
    before = O.totals(f)[:5]
    np.testing.assert_allclose(O.totals(O.relax(f, 0.9))[:5], before, rtol=1e-14, atol=1e-15)
    assert np.max(np.abs(P.totals(P.relax(f, 0.9))[:5] - before)) > 1e-7


@pytest.mark.parametrize("splitting", ["strang", "lie"])
def test_conservative_periodic_run_conserves(oracle_mod, splitting):
    """On a periodic box streaming in flux form conserves every velocity sum,
    so with the conservative relaxation whole steps conserve mass, momentum
    and energy to rounding; with the point-value Maxwellian energy drifts."""
    cfg = prob(kind="periodic2d", nx=4, ny=3, nv=(8, 8, 6), vlo=(-3, -3, -3), vhi=(3, 3, 3), kn=0.3,
               splitting=splitting, maxwellian="conservative")
    O, P = oracle_mod.Oracle(cfg), oracle_mod.Oracle(dict(cfg, maxwellian="point"))
    f = np.tile(gauss(O, 1.0, (0.2, 0.0, 0.0), 1.0), (O.ncell, 1))
    f *= 1 + 0.4 * inputs.uniform(O.shape, seed=41, lo=-1, hi=1)
    t0 = O.totals(f)[:5]
    np.testing.assert_allclose(O.totals(O.step(f, 6))[:5], t0, rtol=1e-13, atol=1e-14)
    assert abs(P.totals(P.step(f, 6))[4] - t0[4]) > 1e-7 * abs(t0[4])


@pytest.mark.parametrize("kind", ["shock", "periodic2d", "cavity"])
def test_twin_agrees_conservative(oracle_mod, kind):
    """The C oracle's Newton solve and the twin's SciPy root finder on the
    same defining equations give the same three steps to rounding."""
    from oracle.twin import Twin
    cfg = prob(kind=kind, nx=4, ny=3, nv=(6, 4, 4), vlo=(-3, -3, -3), vhi=(3, 3, 3), kn=0.4,
               mach=1.5, x0=-1.0 if kind == "shock" else 0.0, lid_mach=0.25, t_wall=1.2,
               maxwellian="conservative")
    O, W = oracle_mod.Oracle(cfg), Twin(cfg)
    f = O.initial_state() * (1 + 0.3 * inputs.uniform(O.shape, seed=53, lo=-1, hi=1))
    np.testing.assert_allclose(O.step(f, 3), W.step(f, 3), rtol=1e-12, atol=1e-15)


# --------------------------------------------------------------- streaming


def test_first_order_upwind_is_eq_upwind(oracle_mod):
    """Limiter off: streaming is the donor-cell formula of Sec. 2.1, Eq. (upwind):
    f_i <- (1 - C) f_i + C f_{i-1} for C > 0, (1 + C) f_i - C f_{i+1} for C < 0."""
    cfg = prob(kind="periodic1d", nx=9, nv=(6, 2, 2), vlo=(-3,) * 3, vhi=(3,) * 3, limiter="none")
    O = oracle_mod.Oracle(cfg)
    g = inputs.uniform(O.shape, seed=5, lo=0.1, hi=1.0)
    dt = O.dt
    out = O.stream(g, dt)
    vx, _, _ = O.velocity_nodes()
    C = vx * dt / (1.0 / 9)
    left, right = np.roll(g, 1, axis=0), np.roll(g, -1, axis=0)
    want = np.where(C > 0, (1 - C) * g + C * left, (1 + C) * g - C * right)
    np.testing.assert_allclose(out, want, rtol=1e-14, atol=1e-16)


def test_unit_courant_number_is_exact_shift(oracle_mod):
    """Sec. 2.1, Eq. (exact): at |C| = 1 the scheme moves f by one cell,
    whatever the limiter does (the slope term carries a factor 1 - |C|)."""
    cfg = prob(kind="periodic1d", nx=10, nv=(2, 2, 2), vlo=(-1,) * 3, vhi=(1,) * 3, dt=0.2)
    O = oracle_mod.Oracle(cfg)  # v_x = +-0.5, dx = 0.1 -> C = +-1
    g = inputs.uniform(O.shape, seed=7, lo=0.0, hi=1.0)
    out = O.stream(g, 0.2)
    vx, _, _ = O.velocity_nodes()
    want = np.where(vx > 0, np.roll(g, 1, axis=0), np.roll(g, -1, axis=0))
    np.testing.assert_allclose(out, want, rtol=0, atol=1e-15)


def test_linear_profile_translates_exactly(oracle_mod):
    """Second-order reading: minmod keeps the exact slope of linear data, so a
    linear profile moves by v dt exactly in cells whose stencil is interior."""
    cfg = prob(kind="shock", nx=16, x0=-1.0, x1=1.0, nv=(4, 2, 2), vlo=(-2,) * 3, vhi=(2,) * 3,
               mach=1.2, cfl=0.45)
    O = oracle_mod.Oracle(cfg)
    x = -1.0 + (np.arange(16) + 0.5) * (2.0 / 16)
    vx, _, _ = O.velocity_nodes()
    a, b = 0.3 + np.arange(O.nvel) * 0.01, 0.2 + np.arange(O.nvel) * 0.005
    g = a[None, :] + b[None, :] * x[:, None]
    dt = O.dt
    out = O.stream(g, dt)
    want = a[None, :] + b[None, :] * (x[:, None] - vx[None, :] * dt)
    np.testing.assert_allclose(out[3:-3], want[3:-3], rtol=1e-13)


@pytest.mark.parametrize("kind", ["periodic1d", "periodic2d", "cavity"])
def test_streaming_conserves_mass(oracle_mod, kind):
    """Flux form telescopes; periodic ghosts wrap and the wall density makes the
    net wall mass flux zero (Sec. 5.1), so sum f is kept to rounding."""
    cfg = prob(kind=kind, nx=7, ny=5, nv=(8, 8, 4), vlo=(-4,) * 3, vhi=(4,) * 3, lid_mach=0.3, t_wall=1.3)
    O = oracle_mod.Oracle(cfg)
    base = gauss(O, 1.0, (0.1, 0.0, 0.0), 1.0)
    g = base[None, :] * inputs.uniform(O.shape, seed=13, lo=0.3, hi=1.7)
    out = O.stream(g)
    assert abs(out.sum() - g.sum()) <= 1e-14 * g.sum()
    if kind.startswith("periodic"):  # per velocity as well
        np.testing.assert_allclose(out.sum(axis=0), g.sum(axis=0), rtol=1e-13)


@pytest.mark.parametrize("kind", ["periodic2d", "cavity"])
def test_streaming_positivity(oracle_mod, kind):
    """Courant sum 2/3 keeps every value non-negative (each update is a convex
    combination of neighbours under minmod), also for rough data."""
    cfg = prob(kind=kind, nx=6, ny=6, nv=(6, 6, 2), vlo=(-3,) * 3, vhi=(3,) * 3, cfl=2.0 / 3.0,
               lid_mach=0.3)
    O = oracle_mod.Oracle(cfg)
    g = inputs.uniform(O.shape, seed=17, lo=0.0, hi=1.0) ** 4
    assert O.stream(g).min() >= 0.0


# ------------------------------------------------------------------ walls


def test_wall_density_balances_equal_temperature(oracle_mod):
    """Sec. 5.1: gas at rest at the wall temperature is re-emitted unchanged,
    n_W = n, on every wall (the discrete half-range sums mirror each other)."""
    cfg = prob(kind="cavity", nx=3, ny=2, nv=(12, 12, 6), vlo=(-5,) * 3, vhi=(5,) * 3, t_wall=1.7)
    O = oracle_mod.Oracle(cfg)
    f = np.tile(gauss(O, 1.3, (0, 0, 0), 1.7), (O.ncell, 1))
    nw = O.wall_density(f)
    np.testing.assert_allclose(nw[:2, :2], 1.3, rtol=1e-14)
    np.testing.assert_allclose(nw[2:, :3], 1.3, rtol=1e-14)


def test_wall_density_closed_form_limit(oracle_mod):
    """Sec. 5.1: for gas at rest (n, T) next to a wall at T_w the flux balance
    gives n_W = n sqrt(T / T_w) (half-range Gaussian fluxes (1/2) n sqrt(T/pi)
    and (1/2) n_W sqrt(T_w/pi)).  The discrete half-range sums carry the
    midpoint rule's O(dv^2) error at the kink v.n = 0, so the check is the
    limit: the error is small and falls fourfold when dv halves."""
    n, T, Tw = 1.3, 0.9, 1.7
    errs = []
    for nvx in (200, 400):
        cfg = prob(kind="cavity", nx=1, ny=1, nv=(nvx, 30, 30), vlo=(-9,) * 3, vhi=(9,) * 3, t_wall=Tw)
        O = oracle_mod.Oracle(cfg)
        f = np.tile(gauss(O, n, (0, 0, 0), T), (O.ncell, 1))
        errs.append(O.wall_density(f)[0, 0] / (n * math.sqrt(T / Tw)) - 1.0)
    assert abs(errs[0]) < 1e-3
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.02)


def test_rest_cavity_is_stationary_under_streaming(oracle_mod):
    """With U_W = 0 and T_w = T, the rest Maxwellian is reproduced by the
    walls (n_W = n by the grid's symmetry), so streaming leaves it alone."""
    cfg = prob(kind="cavity", nx=5, ny=4, nv=(8, 8, 4), vlo=(-4,) * 3, vhi=(4,) * 3, t_wall=1.0)
    O = oracle_mod.Oracle(cfg)
    f = O.initial_state()
    out = O.stream(f)
    assert np.max(np.abs(out - f)) <= 1e-14 * np.max(f)


def test_cavity_mirror_symmetry(oracle_mod):
    """x -> 1 - x, v_x -> -v_x, U_W -> -U_W maps solutions to solutions (P7)."""
    nx, ny, nv = 6, 5, (6, 4, 2)
    base = prob(kind="cavity", nx=nx, ny=ny, nv=nv, vlo=(-3,) * 3, vhi=(3,) * 3, kn=0.3, lid_mach=0.4)
    O1 = oracle_mod.Oracle(base)
    O2 = oracle_mod.Oracle(dict(base, lid_mach=-0.4))
    f = O1.initial_state() * (1 + 0.2 * inputs.uniform(O1.shape, seed=21, lo=-1, hi=1))

    def mirror(a):
        a5 = a.reshape(ny, nx, nv[2], nv[1], nv[0])
        return a5[:, ::-1, :, :, ::-1].reshape(a.shape)
    out1 = O1.step(f, 3)
    out2 = O2.step(mirror(f), 3)
    np.testing.assert_allclose(mirror(out1), out2, rtol=1e-13, atol=1e-15)


def test_cavity_transpose_symmetry_without_lid(oracle_mod):
    """With a resting lid all four walls are alike: swapping x <-> y together
    with v_x <-> v_y maps solutions to solutions (pins 2D indexing)."""
    n, nv = 5, (4, 4, 2)
    cfg = prob(kind="cavity", nx=n, ny=n, nv=nv, vlo=(-3,) * 3, vhi=(3,) * 3, kn=0.3, t_wall=1.4)
    O = oracle_mod.Oracle(cfg)
    f = O.initial_state() * (1 + 0.2 * inputs.uniform(O.shape, seed=23, lo=-1, hi=1))

    def tr(a):
        a5 = a.reshape(n, n, nv[2], nv[1], nv[0])
        return np.ascontiguousarray(a5.transpose(1, 0, 2, 4, 3)).reshape(a.shape)
    np.testing.assert_allclose(tr(O.step(f, 2)), O.step(tr(f), 2), rtol=1e-13, atol=1e-15)


def test_cavity_mass_conserved_over_steps(oracle_mod):
    """Walls pass no net mass (Sec. 5.1) and collisions conserve it up to the
    moment defect, so total mass is constant over many steps."""
    cfg = inputs.config("cavity_128_fp32", nx=6, ny=6)
    O = oracle_mod.Oracle(cfg)
    f = O.initial_state()
    m0 = O.totals(f)[0]
    f = O.step(f, 40)
    assert abs(O.totals(f)[0] - m0) <= 1e-11 * m0


def test_lid_shear_no_slip_and_limit(oracle_mod):
    """Lid shear (x-momentum flux through the lid face, Sec. 5.2's D before
    normalisation).  Gas drifting with the lid at the wall temperature carries
    no shear; otherwise the flux tends to (1/2) n sqrt(T/pi) (U - U_W) per unit
    lid length (half-range Gaussian flux times the slip), with the midpoint
    rule's O(dv^2) error at v_y = 0."""
    Tw, ma = 1.2, 0.3
    uw = ma * math.sqrt(GAMMA / 2)
    cfg = prob(kind="cavity", nx=4, ny=3, nv=(16, 16, 6), vlo=(-6,) * 3, vhi=(6,) * 3, t_wall=Tw, lid_mach=ma)
    O = oracle_mod.Oracle(cfg)
    f = np.tile(gauss(O, 1.1, (uw, 0, 0), Tw), (O.ncell, 1))
    assert abs(O.lid_shear(f)) < 1e-15
    n, U = 1.1, 0.05
    errs = []
    for nvy in (200, 400):
        cfg = prob(kind="cavity", nx=1, ny=1, nv=(40, nvy, 30), vlo=(-9,) * 3, vhi=(9,) * 3, t_wall=Tw,
                   lid_mach=ma)
        O = oracle_mod.Oracle(cfg)
        f = np.tile(gauss(O, n, (U, 0, 0), Tw), (O.ncell, 1))
        want = 0.5 * n * math.sqrt(Tw / math.pi) * (U - uw)
        errs.append(O.lid_shear(f) / want - 1.0)
    assert abs(errs[0]) < 1e-3
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.02)


# ------------------------------------------------------- shift streaming


def test_shift_streaming_integer_courant_is_translation(oracle_mod):
    """Sec. 2.1, Eq. (exact) and the text below it: with integer Courant
    numbers the shift form moves each v_x column by exactly C cells."""
    cfg = prob(kind="periodic1d", nx=11, x0=0.0, x1=11.0, nv=(4, 2, 2), vlo=(-2,) * 3, vhi=(2,) * 3,
               dt=2.0, limiter="shift")
    O = oracle_mod.Oracle(cfg)  # v_x = -1.5, -0.5, 0.5, 1.5; dx = 1 -> C = -3, -1, 1, 3
    g = inputs.uniform(O.shape, seed=71, lo=0.0, hi=1.0)
    out = O.stream(g, 2.0)
    vx, _, _ = O.velocity_nodes()
    want = np.empty_like(g)
    for j in range(O.nvel):
        want[:, j] = np.roll(g[:, j], int(round(vx[j] * 2.0)))
    np.testing.assert_array_equal(out, want)


def test_shift_streaming_below_unit_courant_is_eq_upwind(oracle_mod):
    """With |C| < 1 the integer part is zero and the shift form is Eq. (upwind)."""
    cfg = prob(kind="periodic1d", nx=9, nv=(6, 2, 2), vlo=(-3,) * 3, vhi=(3,) * 3, limiter="shift")
    O = oracle_mod.Oracle(cfg)
    Ou = oracle_mod.Oracle(dict(cfg, limiter="none"))
    g = inputs.uniform(O.shape, seed=72, lo=0.1, hi=1.0)
    np.testing.assert_allclose(O.stream(g, O.dt), Ou.stream(g, O.dt), rtol=1e-14, atol=1e-16)


def test_shift_streaming_large_courant(oracle_mod):
    """Large fractional Courant numbers on a periodic box: each column is a
    convex combination of two translated copies, so its sum is kept and the
    result matches interpolation of the exact translation of linear data."""
    cfg = prob(kind="periodic1d", nx=13, x0=0.0, x1=13.0, nv=(6, 2, 2), vlo=(-3,) * 3, vhi=(3,) * 3,
               dt=3.3, limiter="shift")
    O = oracle_mod.Oracle(cfg)  # C = v_x * 3.3: -8.25, -4.95, -1.65, 1.65, 4.95, 8.25
    g = inputs.uniform(O.shape, seed=73, lo=0.1, hi=1.0)
    out = O.stream(g, 3.3)
    np.testing.assert_allclose(out.sum(axis=0), g.sum(axis=0), rtol=1e-14)
    vx, _, _ = O.velocity_nodes()
    # exact translation of a periodic sampled profile, evaluated by linear
    # interpolation between the two neighbouring grid points
    for j in range(O.nvel):
        C = vx[j] * 3.3
        xs = (np.arange(13) - C) % 13
        lo = np.floor(xs).astype(int)
        w = xs - lo
        want = (1 - w) * g[lo % 13, j] + w * g[(lo + 1) % 13, j]
        np.testing.assert_allclose(out[:, j], want, rtol=1e-13)


def test_shift_streaming_far_field_inflow(oracle_mod):
    """Shock box, Courant numbers above the box width from the upstream side:
    every cell reached from outside takes the far-field Maxwellian (Eq. bc_shock)."""
    cfg = prob(kind="shock", nx=6, x0=-3.0, x1=3.0, nv=(4, 2, 2), vlo=(-2,) * 3, vhi=(10,) * 3,
               mach=1.5, dt=2.5, limiter="shift")
    O = oracle_mod.Oracle(cfg)  # v_x = -0.5, 2.5, 5.5, 8.5, dx = 1 -> C = -1.25, 6.25, 13.75, 21.25
    g = inputs.uniform(O.shape, seed=74, lo=0.1, hi=1.0)
    out = O.stream(g, 2.5)
    vx, _, _ = O.velocity_nodes()
    up = O.initial_state()[0]  # the upstream Maxwellian (cell 0 lies at x < 0)
    for j in range(O.nvel):
        C = vx[j] * 2.5
        if C >= 7.0:  # both sources of every cell lie left of the box
            np.testing.assert_allclose(out[:, j], up[j], rtol=1e-14)


# ------------------------------------------------------- cavity metrics
# D and G of the Table of Sec. 5.2: mean lid shear stress over p0 U_W and
# the main vortex's centre-line flow rate (the integral of V_x / U_W from the
# vortex centre up to the lid, over the height).


def metric_cfg(nx, ny, nv=(24, 16, 16)):
    return prob(kind="cavity", nx=nx, ny=ny, nv=nv, vlo=(-6,) * 3, vhi=(6,) * 3, lid_mach=0.05)


def shear_state(O, cfg, u_of_xy):
    """Cells hold Maxwellians n = T = 1 drifting with V_x = U_W u(x, y)."""
    uw = cfg["lid_mach"] * math.sqrt(GAMMA / 2)
    ny, nx = cfg["ny"], cfg["nx"]
    return np.array([gauss(O, 1.0, (uw * u_of_xy((c % nx + 0.5) / nx, (c // nx + 0.5) / ny), 0.0, 0.0), 1.0)
                     for c in range(nx * ny)])


def test_lid_shear_metric_free_molecular_limit(oracle_mod):
    """Gas at rest under the lid: the lid emits the incident mass flux
    1/(2 sqrt(pi)) with mean x-velocity U_W, so D = 1/sqrt(pi).  The
    half-range sums over v_y converge at second order in dv_y: the error
    falls fourfold per halving and Richardson's extrapolation hits the
    closed form."""
    D = []
    for nvy in (40, 80, 160):
        O = oracle_mod.Oracle(metric_cfg(3, 2, nv=(24, nvy, 16)))
        D.append(O.cavity_metrics(O.initial_state())[0])
    e = np.array(D) - 1 / math.sqrt(math.pi)
    assert 3.8 < e[0] / e[1] < 4.2 and 3.8 < e[1] / e[2] < 4.2
    assert abs((4 * D[2] - D[1]) / 3 - 1 / math.sqrt(math.pi)) < 5e-6


@pytest.mark.parametrize("nx", [6, 7])
def test_vortex_flow_rate_linear_profile(oracle_mod, nx):
    """u = s (y - a) + k (x - 1/2): on the centre line G = int_a^1 u dy =
    s (1 - a)^2 / 2, exact for the piecewise-linear rule; the x term vanishes
    only at x = 1/2 (even nx: mean of the middle columns, odd nx: the middle
    column), so a wrong column changes G."""
    cfg = metric_cfg(nx, 10)
    O = oracle_mod.Oracle(cfg)
    for s, a in [(0.8, 0.37), (1.3, 0.61)]:
        f = shear_state(O, cfg, lambda x, y: s * (y - a) + 0.4 * (x - 0.5))
        assert O.cavity_metrics(f)[1] == pytest.approx(s * (1 - a) ** 2 / 2, rel=1e-10)


def test_cavity_metrics_undefined_elsewhere(oracle_mod):
    """No lid motion or no cavity: D and G are NaN."""
    for cfg in (metric_cfg(4, 4) | dict(lid_mach=0.0), prob(kind="periodic2d", nx=4, ny=4, nv=(8, 8, 4))):
        O = oracle_mod.Oracle(cfg)
        assert np.all(np.isnan(O.cavity_metrics(O.initial_state())))


def test_vortex_flow_rate_takes_the_top_vortex(oracle_mod):
    """Two sign changes on the centre line: the integral starts at the upper
    zero (the main vortex's centre) and converges at second order in dy."""
    a, b = 0.3, 0.7

    def u(y):
        return (y - a) * (y - b)

    exact = (1 - b) ** 3 / 3 + (b - a) * (1 - b) ** 2 / 2
    err = []
    for ny in (20, 40):
        cfg = metric_cfg(4, ny)
        O = oracle_mod.Oracle(cfg)
        err.append(abs(O.cavity_metrics(shear_state(O, cfg, lambda x, y: u(y)))[1] - exact))
    assert err[1] < 0.3 * err[0] and err[1] < 2e-4


# ------------------------------------------------- reduced velocity space
# Two-dimensional problems with v_z integrated out (g = int f dv_z,
# h = int v_z^2 f dv_z), the projection the paper cites in Sec. 3 and Sec. 6.


def test_reduced_maxwellian_moments(oracle_mod):
    """The reduced Maxwellian pair has the moments of its parameters: n and V
    from g, T from g's (v_x, v_y) spread plus h (on a resolving grid)."""
    cfg = prob(kind="periodic2d", nx=2, ny=2, nv=(40, 40, 2), vlo=(-9, -9, -1), vhi=(9, 9, 1), reduced=True)
    O = oracle_mod.Oracle(cfg)
    for n, V, T in [(1.0, (0.0, 0.0), 1.0), (2.5, (0.7, -0.3), 1.7)]:
        phi = O.maxwellian(n, np.array([V[0], V[1], 0.0]), T)
        g, h = phi[:1600], phi[1600:]
        np.testing.assert_allclose(h, 0.5 * T * g, rtol=1e-15)
        m = O.moments(np.tile(phi, (O.ncell, 1)))[0]
        np.testing.assert_allclose(m, [n, V[0], V[1], 0.0, T], rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("kind", ["cavity", "periodic2d"])
@pytest.mark.parametrize("splitting", ["strang", "lie"])
def test_reduced_model_is_the_projection_of_the_full_one(oracle_mod, kind, splitting):
    """With the linear (first-order upwind) streaming every operation commutes
    with integrating over v_z: stepping the full model on a resolving v_z grid
    and projecting equals stepping the projected state in the reduced model.
    The initial state is even in v_z (V_z = 0) and varies with x, v_x, v_y."""
    common = dict(kind=kind, nx=5, ny=4, kn=0.4, lid_mach=0.3, t_wall=1.2, splitting=splitting, limiter="none")
    full = prob(nv=(6, 5, 24), vlo=(-3, -3, -6), vhi=(3, 3, 6), **common)
    red = prob(nv=(6, 5, 2), vlo=(-3, -3, -1), vhi=(3, 3, 1), reduced=True, **common)
    F, R = oracle_mod.Oracle(full), oracle_mod.Oracle(red)
    xi = inputs.uniform((F.ncell, 1, 5, 6), seed=61, lo=-1, hi=1)
    f0 = (F.initial_state().reshape(F.ncell, 24, 5, 6) * (1 + 0.3 * xi)).reshape(F.shape)
    vz = F.velocity_nodes()[2].reshape(24, 5, 6)[:, 0, 0]
    dvz = 0.5

    def project(f):
        f = f.reshape(-1, 24, 5, 6)
        g = f.sum(axis=1) * dvz
        h = (f * vz[None, :, None, None] ** 2).sum(axis=1) * dvz
        return np.concatenate([g.reshape(-1, 30), h.reshape(-1, 30)], axis=1)

    got = R.step(project(f0), 3)
    want = project(F.step(f0, 3))
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())
    np.testing.assert_allclose(R.moments(got), F.moments(F.step(f0, 3)), rtol=1e-11, atol=1e-13)


def test_reduced_effective_parameters_and_conservation(oracle_mod):
    """Conservative Maxwellian in the reduced space: the effective parameters
    of a sampled reduced Maxwellian's grid moments are its parameters, and a
    periodic run conserves mass, momentum and energy to rounding (the point
    form drifts)."""
    cfg = prob(kind="periodic2d", nx=3, ny=3, nv=(8, 8, 2), vlo=(-3, -3, -1), vhi=(3, 3, 1), kn=0.3,
               reduced=True, maxwellian="conservative")
    O, P = oracle_mod.Oracle(cfg), oracle_mod.Oracle(dict(cfg, maxwellian="point"))
    phi = O.maxwellian(1.3, np.array([0.3, -0.2, 0.0]), 0.8)
    m = O.moments(np.tile(phi, (O.ncell, 1)))[0]
    assert np.max(np.abs(m - [1.3, 0.3, -0.2, 0.0, 0.8])) > 1e-5
    q, it = O.effective_parameters(m[0], m[1:4], m[4])
    np.testing.assert_allclose(q, [1.3, 0.3, -0.2, 0.0, 0.8], rtol=0, atol=2e-14)
    assert it <= 6
    f = np.tile(O.maxwellian(1.0, np.array([0.2, 0.0, 0.0]), 1.0), (O.ncell, 1))
    f *= 1 + 0.4 * inputs.uniform(O.shape, seed=43, lo=-1, hi=1)
    t0 = O.totals(f)[:5]
    np.testing.assert_allclose(O.totals(O.step(f, 6))[:5], t0, rtol=1e-13, atol=1e-14)
    assert abs(P.totals(P.step(f, 6))[4] - t0[4]) > 1e-7 * abs(t0[4])


@pytest.mark.parametrize("kind,limiter,cfl", [("shock", "none", 0.5), ("periodic1d", "none", 0.5),
                                               ("shock", "shift", 3.3)])
@pytest.mark.parametrize("splitting", ["strang", "lie"])
def test_reduced_1d_model_is_the_projection_of_the_full_one(oracle_mod, kind, limiter, cfl, splitting):
    """One-dimensional problems with v_y and v_z integrated out (g = int f,
    h = int (v_y^2 + v_z^2) f over both): with linear streaming (first-order
    upwind or its translation form) stepping the full model on resolving
    (v_y, v_z) grids (32 nodes on [-8, 8]) and projecting equals stepping the
    projected state."""
    common = dict(kind=kind, nx=7, x0=-1.0 if kind == "shock" else 0.0, kn=0.4, mach=1.5, cfl=cfl,
                  splitting=splitting, limiter=limiter, omega=0.74)
    full = prob(nv=(8, 32, 32), vlo=(-4, -8, -8), vhi=(5, 8, 8), **common)
    red = prob(nv=(8, 1, 2), vlo=(-4, -1, -1), vhi=(5, 1, 1), reduced=True, **common)
    F, R = oracle_mod.Oracle(full), oracle_mod.Oracle(red)
    xi = inputs.uniform((F.ncell, 1, 1, 8), seed=62, lo=-1, hi=1)
    f0 = (F.initial_state().reshape(F.ncell, 32, 32, 8) * (1 + 0.3 * xi)).reshape(F.shape)
    _, vy, vz = (v.reshape(32, 32, 8)[:, :, 0] for v in F.velocity_nodes())
    dA = 0.5 * 0.5

    def project(f):
        f = f.reshape(-1, 32, 32, 8)
        g = f.sum(axis=(1, 2)) * dA
        h = (f * (vy ** 2 + vz ** 2)[None, :, :, None]).sum(axis=(1, 2)) * dA
        return np.concatenate([g, h], axis=1)

    got = R.step(project(f0), 3)
    want = project(F.step(f0, 3))
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


def test_reduced_1d_maxwellian_and_effective_parameters(oracle_mod):
    """The 1D reduced Maxwellian pair (h = T g) has the moments of its
    parameters on a resolving grid; on a coarse one the effective parameters
    of a sampled pair's moments are its parameters."""
    fine = prob(kind="periodic1d", nx=2, nv=(60, 1, 2), vlo=(-9, -1, -1), vhi=(9, 1, 1), reduced=True)
    O = oracle_mod.Oracle(fine)
    phi = O.maxwellian(1.7, np.array([0.6, 0.0, 0.0]), 1.3)
    np.testing.assert_allclose(phi[60:], 1.3 * phi[:60], rtol=1e-15)
    np.testing.assert_allclose(O.moments(np.tile(phi, (2, 1)))[0], [1.7, 0.6, 0, 0, 1.3], rtol=1e-11, atol=1e-13)
    coarse = prob(kind="periodic1d", nx=2, nv=(8, 1, 2), vlo=(-3, -1, -1), vhi=(3, 1, 1), reduced=True,
                  maxwellian="conservative")
    C = oracle_mod.Oracle(coarse)
    phi = C.maxwellian(1.1, np.array([0.4, 0.0, 0.0]), 0.9)
    m = C.moments(np.tile(phi, (2, 1)))[0]
    assert np.max(np.abs(m - [1.1, 0.4, 0, 0, 0.9])) > 1e-5
    q, it = C.effective_parameters(m[0], m[1:4], m[4])
    np.testing.assert_allclose(q, [1.1, 0.4, 0, 0, 0.9], rtol=0, atol=2e-14)
    assert it <= 6
    # quadratic convergence from defects near 1e-2 (6 nodes on [-2.5, 2.5]):
    # at most 5 steps with the exact Jacobian, 6 with a slipped T~ exponent
    V = oracle_mod.Oracle(dict(coarse, nv=(6, 1, 2), vlo=(-2.5, -1, -1), vhi=(2.5, 1, 1)))
    for v, T, most in [(0.5, 1.0, 5), (-0.7, 0.6, 4), (0.0, 1.5, 5)]:
        assert V.effective_parameters(1.0, np.array([v, 0.0, 0.0]), T)[1] <= most


# ------------------------------------------------------------------ twin


@pytest.mark.parametrize("kind", ["shock", "periodic1d", "periodic2d", "cavity"])
@pytest.mark.parametrize("splitting,limiter", [("strang", "minmod"), ("lie", "none"), ("strang", "none")])
def test_twin_agrees(oracle_mod, kind, splitting, limiter):
    """Brute force on tiny inputs: the C oracle and the separately written
    NumPy twin agree to rounding after three steps."""
    from oracle.twin import Twin
    cfg = prob(kind=kind, nx=5, ny=4, nv=(4, 4, 2), vlo=(-3, -3, -2), vhi=(3, 3, 2), kn=0.4,
               mach=1.5, x0=-1.0 if kind == "shock" else 0.0, lid_mach=0.25, t_wall=1.2,
               splitting=splitting, limiter=limiter)
    O, W = oracle_mod.Oracle(cfg), Twin(cfg)
    f = O.initial_state() * (1 + 0.3 * inputs.uniform(O.shape, seed=29, lo=-1, hi=1))
    assert W.dt == pytest.approx(O.dt, rel=1e-15)
    np.testing.assert_allclose(O.step(f, 3), W.step(f, 3), rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("kind", ["shock", "periodic1d"])
@pytest.mark.parametrize("cfl", [0.7, 3.6])
def test_twin_agrees_shift(oracle_mod, kind, cfl):
    """The C oracle's shift streaming and the twin's separately written one
    (index gathers) agree to rounding after three Lie steps, below and above
    unit Courant number."""
    from oracle.twin import Twin
    cfg = prob(kind=kind, nx=7, nv=(6, 3, 2), vlo=(-3, -3, -2), vhi=(4, 3, 2), kn=0.4, mach=1.5,
               x0=-1.0 if kind == "shock" else 0.0, cfl=cfl, splitting="lie", limiter="shift")
    O, W = oracle_mod.Oracle(cfg), Twin(cfg)
    f = O.initial_state() * (1 + 0.3 * inputs.uniform(O.shape, seed=75, lo=-1, hi=1))
    np.testing.assert_allclose(O.step(f, 3), W.step(f, 3), rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("kind", ["cavity", "periodic2d", "shock", "periodic1d"])
@pytest.mark.parametrize("maxwellian,limiter", [("point", "minmod"), ("conservative", "minmod"),
                                                ("point", "shift")])
def test_twin_agrees_reduced(oracle_mod, kind, maxwellian, limiter):
    """Reduced velocity space (v_z out for 2D kinds, v_y and v_z out for 1D
    kinds): the C oracle and the twin's separate whole-array code agree to
    rounding after three steps, also with the minmod limiter (which the
    projection pins cannot cover) and the effective Maxwellian (SciPy's root
    finder against the C Newton solve)."""
    from oracle.twin import Twin
    two = kind in ("cavity", "periodic2d")
    if limiter == "shift" and two:
        pytest.skip("translation-form streaming is one-dimensional")
    cfg = prob(kind=kind, nx=5, ny=4, nv=(6, 4, 2) if two else (6, 1, 2), vlo=(-3, -3, -1), vhi=(3, 3, 1),
               kn=0.4, mach=1.5, x0=-1.0 if kind == "shock" else 0.0, lid_mach=0.25, t_wall=1.2,
               maxwellian=maxwellian, limiter=limiter, cfl=2.6 if limiter == "shift" else 0.5,
               splitting="lie" if limiter == "shift" else "strang", reduced=True)
    O, W = oracle_mod.Oracle(cfg), Twin(cfg)
    f = O.initial_state() * (1 + 0.3 * inputs.uniform(O.shape, seed=57, lo=-1, hi=1))
    np.testing.assert_allclose(O.step(f, 3), W.step(f, 3), rtol=1e-12, atol=1e-15)


def test_time_step_rule(oracle_mod):
    """dt = CFL / max sum_d |v_d| / dx_d over velocity cell centres."""
    O = oracle_mod.Oracle(inputs.config("shock_m1.5_fp64"))
    assert O.dt == pytest.approx(0.5 * (40 / 256) / (6 - 6 / 32), rel=1e-15)
    O = oracle_mod.Oracle(inputs.config("cavity_128_fp32"))
    assert O.dt == pytest.approx(0.5 / (2 * 128 * (5 - 5 / 24)), rel=1e-15)


def test_steady_shock_connects_rankine_hugoniot_states(oracle_mod):
    """Sec. 4.1: the long-time solution is a steady shock joining the two
    far-field states of Eq. (RH).  Steadiness of the 1D BGK equation means the
    fluxes of mass, x-momentum and energy are the same at every x; they must
    equal the Rankine-Hugoniot fluxes (to the discretisation error of this
    coarse grid, which decays as the transient leaves)."""
    cfg = inputs.config("shock_m1.5_fp64", nx=64, nv=(16, 16, 16))
    O = oracle_mod.Oracle(cfg)
    f = O.step(O.initial_state(), 1200)  # t = 66.7 upstream collision times
    vx, vy, vz = O.velocity_nodes()
    dV = (12 / 16) ** 3
    up, dn = oracle_mod.Oracle.rankine_hugoniot(1.5)
    n, V, T = up
    fluxes = {
        "mass": ((f * vx).sum(1) * dV, n * V),
        "momentum": ((f * vx * vx).sum(1) * dV, n * V * V + n * T / 2),
        "energy": ((f * vx * (vx * vx + vy * vy + vz * vz)).sum(1) * dV, n * V * (V * V + 2.5 * T)),
    }
    for name, (prof, want) in fluxes.items():
        assert np.max(np.abs(prof / want - 1.0)) < 2.5e-3, name
    m = O.moments(f)
    np.testing.assert_allclose(m[0, [0, 1, 4]], up, rtol=2e-3)
    np.testing.assert_allclose(m[-1, [0, 1, 4]], dn, rtol=2e-3)


# ------------------------------------------------- three spatial dimensions
# The extension of Sec. 2.1 to three directions: a cube with six diffuse
# walls (lid at y = y1 moving along x) and a periodic box.


def cube(**kw):
    d = prob(kind="cavity3d", nx=4, ny=3, nz=4, z0=0.0, z1=1.0, nv=(8, 6, 8), vlo=(-4.0,) * 3,
             vhi=(4.0,) * 3, kn=0.3, lid_mach=0.3, t_wall=1.1, cfl=0.45)
    d.update(kw)
    return d


def as6(O, f):
    """f[cell][v] as f[iz][iy][ix][jz][jy][jx]."""
    nvx, nvy, nvz = O.nv
    return np.asarray(f).reshape(O.nz, O.ny, O.nx, nvz, nvy, nvx)


def swap_xz(O, f):
    """The state mirrored through the plane x = z: f'(x, y, z; v_x, v_y, v_z) =
    f(z, y, x; v_z, v_y, v_x) (needs nx = nz and equal x and z velocity axes)."""
    return np.ascontiguousarray(as6(O, f).transpose(2, 1, 0, 5, 4, 3)).reshape(O.shape)


def perturbed3(O, seed, amp=0.3):
    return O.initial_state() * (1 + amp * inputs.uniform(O.shape, seed=seed, lo=-1, hi=1))


def test_z_uniform_box_reduces_to_the_2d_step(oracle_mod):
    """A periodic box whose state does not depend on z: the z fluxes vanish
    term by term, so four steps equal the two-dimensional periodic steps bit
    for bit (same dt)."""
    c2 = prob(kind="periodic2d", nx=5, ny=4, nv=(8, 6, 6), vlo=(-4.0,) * 3, vhi=(4.0,) * 3, kn=0.3, dt=0.01)
    c3 = dict(c2, kind="periodic3d", nz=3, z0=0.0, z1=1.0)
    O2, O3 = oracle_mod.Oracle(c2), oracle_mod.Oracle(c3)
    f2 = perturbed3(O2, 201)
    f3 = np.tile(f2, (3, 1))
    got = O3.step(f3, 4).reshape(3, O2.ncell, O2.nvel)
    want = O2.step(f2, 4)
    for iz in range(3):
        assert np.array_equal(got[iz], want)


@pytest.mark.parametrize("limiter", ["minmod", "none"])
def test_periodic_cube_commutes_with_swapping_x_and_z(oracle_mod, limiter):
    """On a cubic periodic box with equal x and z velocity axes, stepping the
    state mirrored through x = z gives the mirrored step: the z stencil
    computes what the x stencil does (a dropped, mis-signed or mis-indexed z
    term fails this)."""
    cfg = prob(kind="periodic3d", nx=5, ny=3, nz=5, z0=0.0, z1=1.0, nv=(8, 6, 8), vlo=(-4.0,) * 3,
               vhi=(4.0,) * 3, kn=0.3, cfl=0.4, limiter=limiter)
    O = oracle_mod.Oracle(cfg)
    f = perturbed3(O, 202)
    a = O.step(swap_xz(O, f), 3)
    b = swap_xz(O, O.step(f, 3))
    assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(b))


def test_cube_with_resting_lid_commutes_with_swapping_x_and_z(oracle_mod):
    """All six walls at rest: the cube is symmetric under x <-> z, so the
    z walls (numbers 4, 5) must act as the x walls do."""
    cfg = cube(nz=4, lid_mach=0.0)
    O = oracle_mod.Oracle(cfg)
    f = perturbed3(O, 203)
    a = O.step(swap_xz(O, f), 3)
    b = swap_xz(O, O.step(f, 3))
    assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(b))


def test_driven_cube_mirror_in_z(oracle_mod):
    """The lid moves along x, so z -> z1 - z, v_z -> -v_z maps solutions to
    solutions on a symmetric v_z axis."""
    cfg = cube()
    O = oracle_mod.Oracle(cfg)
    f = perturbed3(O, 204)

    def mirror(x):
        return np.ascontiguousarray(as6(O, x)[::-1, :, :, ::-1, :, :]).reshape(O.shape)

    a = O.step(mirror(f), 3)
    b = mirror(O.step(f, 3))
    assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(b))


def test_cube_at_rest_is_stationary_under_streaming(oracle_mod):
    """A gas at rest at the wall temperature with the lid at rest: every wall
    density is 1 (equal incident and emitted fluxes of the same Maxwellian)
    and streaming leaves the state unchanged."""
    cfg = cube(lid_mach=0.0, t_wall=1.0)
    O = oracle_mod.Oracle(cfg)
    f = O.initial_state()
    g = O.stream(f)
    assert np.max(np.abs(g - f)) <= 1e-14 * np.max(f)


def test_cube_streaming_conserves_mass(oracle_mod):
    """Six diffuse walls with zero net mass flux each: one streaming pass of
    a perturbed state keeps the total mass to rounding, while momentum and
    energy change at the walls."""
    cfg = cube()
    O = oracle_mod.Oracle(cfg)
    f = perturbed3(O, 205)
    t0, t1 = O.totals(f), O.totals(O.stream(f))
    assert abs(t1[0] - t0[0]) <= 1e-14 * t0[0]
    assert abs(t1[4] - t0[4]) > 1e-9 * t0[4]


def test_cube_time_step_sums_three_courant_numbers(oracle_mod):
    cfg = cube(nx=4, ny=5, nz=2, nv=(8, 6, 10), vlo=(-4.0, -3.0, -5.0), vhi=(4.0, 3.0, 5.0), cfl=0.5)
    O = oracle_mod.Oracle(cfg)
    vx, vy, vz = 4.0 - 0.5, 3.0 - 0.5, 5.0 - 0.5
    assert O.dt == pytest.approx(0.5 / (vx * 4 + vy * 5 + vz * 2), rel=1e-15)
