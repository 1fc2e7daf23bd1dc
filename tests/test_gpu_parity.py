"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (written here, derived in the design notes):
  FP64 path: every f value within 1e-12 * max|f_ref|, moments within 1e-12;
  FP32 path: moments within 1e-5 (n and T relative, V over the problem's
  speed scale: the upstream speed for shocks, the lid speed for cavities).
"""
import math

import numpy as np
import pytest
import torch

from paper_0903_4044_amd import inputs

pytestmark = pytest.mark.gpu

GAMMA = 5.0 / 3.0


@pytest.fixture(scope="module")
def B():
    from paper_0903_4044_amd import binding
    binding.load()
    return binding


def small(kind, **kw):
    d = dict(kind=kind, nx=9, ny=7, x0=-2.0 if kind == "shock" else 0.0, x1=2.0 if kind == "shock" else 1.0,
             y0=0.0, y1=1.0, nv=(12, 10, 6), vlo=(-4.0, -4.0, -3.0), vhi=(4.0, 4.0, 3.0), kn=0.3, omega=0.5,
             cfl=0.5, dt=0.0, mach=1.5, lid_mach=0.2, t_wall=1.1, splitting="strang", limiter="minmod")
    d.update(kw)
    return d


def speed_scale(cfg):
    if cfg["kind"] == "shock":
        return cfg["mach"] * math.sqrt(GAMMA / 2)
    if cfg["kind"] in ("cavity", "cavity3d") and cfg.get("lid_mach", 0.0) != 0.0:
        return abs(cfg["lid_mach"]) * math.sqrt(GAMMA / 2)
    return 1.0


def moment_errors(got, ref, cfg):
    """(e_n, e_V, e_T): relative density / temperature, velocity over the speed scale."""
    got, ref = np.asarray(got), np.asarray(ref)
    e_n = np.max(np.abs(got[:, 0] - ref[:, 0]) / np.abs(ref[:, 0]))
    e_T = np.max(np.abs(got[:, 4] - ref[:, 4]) / np.abs(ref[:, 4]))
    e_V = np.max(np.abs(got[:, 1:4] - ref[:, 1:4])) / speed_scale(cfg)
    return e_n, e_V, e_T


def to_dev(x, dtype):
    return torch.tensor(np.ascontiguousarray(x).reshape(-1), dtype=dtype, device="cuda")


def perturbed_initial(O, seed, amp=0.2):
    return O.initial_state() * (1 + amp * inputs.uniform(O.shape, seed=seed, lo=-1, hi=1))


def check_fp64(y, ref, O, cfg, tol=1e-12):
    y = y.cpu().numpy().reshape(O.shape)
    assert np.max(np.abs(y - ref)) <= tol * np.max(np.abs(ref)), np.max(np.abs(y - ref)) / np.max(np.abs(ref))
    e = moment_errors(O.moments(y), O.moments(ref), cfg)
    assert max(e) <= tol, e


# --------------------------------------------------------------- small cases

CASES = [
    ("shock", {}), ("shock", dict(nx=1)), ("shock", dict(nx=2, mach=3.0)),
    ("shock", dict(splitting="lie", limiter="none")), ("shock", dict(limiter="none")),
    ("periodic1d", dict(nx=5)), ("periodic1d", dict(splitting="lie")),
    ("cavity", {}), ("cavity", dict(nx=1, ny=1)), ("cavity", dict(nx=2, ny=5, lid_mach=-0.3, t_wall=0.8)),
    ("cavity", dict(splitting="lie", limiter="none")),
    ("periodic2d", dict(nx=4, ny=3)),
    ("shock", dict(nv=(16, 16, 8))), ("cavity", dict(nv=(24, 24, 24), nx=3, ny=4)),
    ("shock", dict(nv=(128, 4, 2), nx=3, vlo=(-6, -3, -3), vhi=(6, 3, 3))),
]


@pytest.mark.parametrize("kind,over", CASES)
@pytest.mark.parametrize("nsteps", [1, 4, 7])
def test_fp64_small(B, oracle_mod, kind, over, nsteps):
    cfg = small(kind, **over)
    O = oracle_mod.Oracle(cfg)
    C = B.Context(cfg, "fp64")
    f0 = perturbed_initial(O, seed=100 + nsteps)
    ref = O.step(f0, nsteps)
    y = C.step(to_dev(f0, torch.float64), n=nsteps)
    torch.cuda.synchronize()
    assert C.dts[0] == pytest.approx(O.dt, rel=1e-14)
    check_fp64(y, ref, O, cfg)


@pytest.mark.parametrize("kind,over", [c for c in CASES if not c[1].get("nx") == 1])
def test_fp32_small(B, oracle_mod, kind, over):
    cfg = small(kind, **over)
    O = oracle_mod.Oracle(cfg)
    C = B.Context(cfg, "fp32")
    f0 = perturbed_initial(O, seed=7)
    ref = O.step(f0, 12)
    y = C.step(to_dev(f0, torch.float32), n=12)
    got = C.moments(y).cpu().numpy()
    e = moment_errors(got, O.moments(ref), cfg)
    assert max(e) <= 1e-5, e


def test_zero_steps_copies(B):
    cfg = small("shock")
    C = B.Context(cfg, "fp64")
    x = C.initial_state()
    y = C.step(x, n=0)
    assert torch.equal(x, y)


def test_initial_state_and_moments(B, oracle_mod):
    for name in ("shock_m1.5_fp64", "cavity_64_adjoint"):
        cfg = inputs.config(name)
        O = oracle_mod.Oracle(cfg)
        C = B.Context(cfg, "fp64")
        f = C.initial_state()
        ref = O.initial_state()
        np.testing.assert_allclose(f.cpu().numpy().reshape(O.shape), ref, rtol=1e-13, atol=1e-300)
        np.testing.assert_allclose(C.moments(f).cpu().numpy(), O.moments(ref), rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("nx", [9, 15])
def test_shock_initial_state_with_a_centre_on_zero(B, oracle_mod, nx):
    """An odd cell count on a symmetric box puts the middle centre on x = 0
    (rounded there without a fused multiply-add): it takes the downstream
    state on the GPU as in the oracle."""
    cfg = small("shock", nx=nx)
    O = oracle_mod.Oracle(cfg)
    for prec, tol in (("fp64", 1e-14), ("fp32", 1e-6)):
        C = B.Context(cfg, prec, tune="off")
        got = C.initial_state().double().cpu().numpy().reshape(O.shape)
        np.testing.assert_allclose(got, O.initial_state(), rtol=tol, atol=0)


def test_batched_matches_single_and_oracle(B, oracle_mod):
    """Uneven instances in one context: each equals its own oracle run and
    its own single-instance context bit for bit."""
    cfgs = [small("cavity", nx=n, ny=m, kn=k, lid_mach=u)
            for n, m, k, u in [(3, 3, 0.1, 0.1), (6, 5, 1.0, 0.3), (2, 7, 0.05, 0.05), (9, 9, 0.4, 0.2)]]
    C = B.Context(cfgs, "fp64")
    f0s = [perturbed_initial(oracle_mod.Oracle(c), seed=40 + i) for i, c in enumerate(cfgs)]
    x = torch.cat([to_dev(f, torch.float64) for f in f0s])
    y = C.step(x, n=5)
    for i, c in enumerate(cfgs):
        O = oracle_mod.Oracle(c)
        yi = C.instance_view(y, i)
        check_fp64(yi, O.step(f0s[i], 5), O, c)
        Ci = B.Context(c, "fp64")
        shape = {k: v for k, v in C.launch().items() if k != "tuned_us"}
        try:
            Ci.set_launch(**shape)
            same = True
        except B.BGKError:  # the shape's jz chunking is not available to the smaller context
            same = False
        yi1 = Ci.step(to_dev(f0s[i], torch.float64), n=5).view_as(yi)
        if same:
            assert torch.equal(yi1, yi)
        else:
            check_fp64(yi1, yi.cpu().numpy(), O, c)


# --------------------------------------------------------------- full size


def test_shock_m15_fp64_full_run(B, oracle_mod):
    """Mach 1.5 shock, 256 x 32^3, FP64, all 200 Strang steps."""
    cfg = inputs.config("shock_m1.5_fp64")
    O = oracle_mod.Oracle(cfg)
    C = B.Context(cfg, "fp64")
    f0 = O.initial_state()
    x = C.initial_state()
    np.testing.assert_allclose(x.cpu().numpy().reshape(O.shape), f0, rtol=1e-13, atol=1e-300)
    y = C.step(x, n=cfg["steps"])
    ref = O.step(f0, cfg["steps"])
    check_fp64(y, ref, O, cfg)


@pytest.mark.parametrize("name,precision,nsteps", [
    ("shock_m3_fp32", "fp32", 2), ("shock_m3_fp32", "fp64", 1),
    ("cavity_128_fp32", "fp32", 2), ("cavity_128_fp32", "fp64", 1),
    ("cube_48_fp32", "fp32", 2), ("cube_48_fp32", "fp64", 1)])
def test_full_size_few_steps(B, oracle_mod, name, precision, nsteps):
    """Full-size grids in the benchmark's launch configuration, a few steps."""
    cfg = inputs.config(name)
    O = oracle_mod.Oracle(cfg)
    C = B.Context(cfg, precision)
    x = C.initial_state()
    y = C.step(x, n=nsteps)
    ref = O.step(O.initial_state(), nsteps)
    if precision == "fp64":
        check_fp64(y, ref, O, cfg)
    else:
        e = moment_errors(C.moments(y).cpu().numpy(), O.moments(ref), cfg)
        assert max(e) <= 1e-5, e


def test_shock_m3_fp32_golden(B):
    """Mach 3 shock, 1024 x 48^3, FP32 f: moments against stored oracle runs
    (tests/golden/make_golden.py) up to the full 2000 steps."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "shock_m3_fp32_oracle.npz")
    if not os.path.exists(path):
        pytest.skip("golden file not generated")
    G = np.load(path)
    cfg = inputs.config("shock_m3_fp32")
    C = B.Context(cfg, "fp32")
    assert C.dts[0] == pytest.approx(float(G["dt"]), rel=1e-14)
    f = C.initial_state()
    done = 0
    for m in [int(s) for s in G["steps"]]:
        f = C.step(f, n=m - done)
        done = m
        e = moment_errors(C.moments(f).cpu().numpy(), G[f"moments_{m}"], cfg)
        assert max(e) <= 1e-5, (m, e)
    # stochastic rounding keeps the full run near 1e-7 (round-to-nearest
    # reached 1.6e-5 in T by step 2000)
    assert max(e) <= 1e-6, e


def test_rounding_seed_contract(B):
    """bgk_step(n) advances the rounding seed by n; the same seed repeats an
    FP32 run bit for bit, another seed changes the rounding (not the moments
    beyond rounding)."""
    cfg = small("cavity", nx=6, ny=5, nv=(16, 16, 8))
    C = B.Context(cfg, "fp32")
    x = C.initial_state()
    assert C.seed() == 0
    a = C.step(x, n=3)
    assert C.seed() == 3
    C.set_seed(0)
    b = C.step(x, n=3)
    assert torch.equal(a, b)
    C.set_seed(12345)
    c = C.step(x, n=3)
    assert not torch.equal(a, c)
    ma, mc = C.moments(a).cpu().numpy(), C.moments(c).cpu().numpy()
    assert np.max(np.abs(ma - mc) / np.maximum(np.abs(ma), 1.0)) < 1e-6


def test_fp32_tracks_slow_relaxation_drift(B, oracle_mod):
    """A uniform hot state (the Mach-3 downstream state on the 48^3 [-8, 8]
    grid) in a periodic box: streaming is the identity, and the FP64 dynamics
    drift slowly because the truncated grid's Maxwellian has a small moment
    defect.  The per-step change is far below half an ulp of f, so FP32 with
    round-to-nearest would freeze (off by ~1e-5 in T after 400 steps);
    unbiased stochastic rounding follows the drift."""
    cfg = inputs.config("shock_m3_fp32", kind="periodic1d", nx=2, x0=0.0, x1=1.0)
    O = oracle_mod.Oracle(cfg)
    up, dn = O.rankine_hugoniot(3.0)
    f0 = np.tile(O.maxwellian(dn[0], [dn[1], 0.0, 0.0], dn[2]), (O.ncell, 1))
    nsteps = 400
    ref = O.step(f0, nsteps)
    m0, mr = O.moments(f0), O.moments(ref)
    drift = abs(mr[0, 4] - m0[0, 4]) / m0[0, 4]
    assert drift > 2e-6  # the oracle does drift
    C = B.Context(cfg, "fp32")
    y = C.step(to_dev(f0, torch.float32), n=nsteps)
    e = moment_errors(C.moments(y).cpu().numpy(), mr, cfg)
    assert max(e) <= 5e-7, (e, drift)


@pytest.mark.parametrize("kind,nv,prec", [("periodic2d", (128, 128, 2), "fp64"), ("cavity", (128, 2, 128), "fp64"),
                                          ("shock", (128, 128, 4), "fp32"), ("cavity", (2, 128, 128), "fp32")])
def test_largest_velocity_axis(B, oracle_mod, kind, nv, prec):
    """128 points on a velocity axis (the largest the library takes): the
    table entries of a workgroup are largest, and the step still matches."""
    cfg = small(kind, nx=3, ny=2, nv=nv, vlo=(-6.0,) * 3, vhi=(6.0,) * 3)
    O = oracle_mod.Oracle(cfg)
    f0 = perturbed_initial(O, seed=70)
    ref = O.step(f0, 2)
    C = B.Context(cfg, prec, tune="off")
    y = C.step(to_dev(f0, C.dtype), n=2)
    if prec == "fp64":
        check_fp64(y, ref, O, cfg)
        lam = inputs.uniform(O.shape, seed=71, lo=-1, hi=1)
        lref, gref = O.step_adjoint(f0, lam)
        got, _ = C.step_adjoint(to_dev(f0, torch.float64), to_dev(lam, torch.float64))
        got = got.cpu().numpy().reshape(O.shape)
        assert np.max(np.abs(got - lref)) <= 1e-12 * np.max(np.abs(lref))
    else:
        e = moment_errors(C.moments(y).cpu().numpy(), O.moments(ref), cfg)
        assert max(e) <= 1e-5, e


def test_velocity_axis_above_limit_rejected(B):
    with pytest.raises(B.BGKError) as ei:
        B.Context(small("shock", nv=(130, 8, 8)), "fp64")
    assert ei.value.code == B.E_UNSUPPORTED


# --------------------------------------------------------------- errors


def test_alias_rejected(B):
    C = B.Context(small("shock"), "fp64")
    x = C.initial_state()
    with pytest.raises(B.BGKError) as ei:
        C.step(x, x, n=1)
    assert ei.value.code == B.E_ALIAS


def test_check_flags_nonfinite_and_negative(B):
    C = B.Context(small("cavity"), "fp32")
    x = C.initial_state()
    assert C.check(x) == B.OK
    y = x.clone()
    y[5 * C.nvel + 3] = float("nan")
    assert C.check(y) == B.E_NONFINITE
    z = x.clone()
    z[2 * C.nvel:3 * C.nvel] *= -1.0
    assert C.check(z) == B.E_NEGATIVE


# --------------------------------------------------------------- launch shapes


def test_autotune_keeps_parity(B, oracle_mod):
    cfg = small("cavity", nx=6, ny=5, nv=(16, 16, 8))
    O = oracle_mod.Oracle(cfg)
    C = B.Context(cfg, "fp64", tune="off")
    f0 = perturbed_initial(O, seed=61)
    x = to_dev(f0, torch.float64)
    shape = C.autotune(x)
    assert shape["tuned_us"] > 0
    check_fp64(C.step(x, n=5), O.step(f0, 5), O, cfg)


@pytest.mark.parametrize("kind", ["shock", "cavity"])
def test_every_shape_matches_oracle(B, oracle_mod, kind):
    """Each launch shape (vector width, pipeline mode, jz chunks, persistent
    grid) computes the same step to rounding."""
    cfg = small(kind, nv=(16, 16, 8), nx=7, ny=6)
    O = oracle_mod.Oracle(cfg)
    f0 = perturbed_initial(O, seed=62)
    ref = O.step(f0, 3)
    for prec, tol in (("fp64", 1e-12), ("fp32", None)):
        C = B.Context(cfg, prec, tune="off")
        x = to_dev(f0, C.dtype)
        for vec in (1, 2, 4):
            for unroll in (1, 2, 3, 4):
                for vsplit in (1, 3):
                    for persist in (0, 1):
                        try:
                            C.set_launch(vec, unroll, vsplit, persist)
                        except B.BGKError:
                            continue
                        y = C.step(x, n=3)
                        if tol:
                            check_fp64(y, ref, O, cfg, tol)
                        else:
                            e = moment_errors(C.moments(y).cpu().numpy(), O.moments(ref), cfg)
                            assert max(e) <= 1e-5, (vec, unroll, vsplit, persist, e)


@pytest.mark.parametrize("kind,nx", [("shock", 9), ("periodic1d", 7), ("cavity", 5)])
def test_pipeline_modes_match_bitwise(B, oracle_mod, kind, nx):
    """The jz-loop pipeline modes (two planes per stage; one plane with 1, 2
    or 3 planes in flight) compute the same step bit for bit, FP32 rounding
    bits included."""
    cfg = small(kind, nv=(16, 16, 8), nx=nx, ny=4)
    O = oracle_mod.Oracle(cfg)
    f0 = perturbed_initial(O, seed=63)
    ran = 0
    for prec in ("fp64", "fp32"):
        C = B.Context(cfg, prec, tune="off")
        x = to_dev(f0, C.dtype)
        for vec in (1, 2, 4):
            for vsplit in (1, 3):
                ref = None
                for unroll in (2, 1, 3, 4):
                    try:
                        C.set_launch(vec, unroll, vsplit, 0)
                    except B.BGKError:
                        break
                    C.set_seed(7)
                    y = C.step(x, n=3)
                    if ref is None:
                        ref = y.clone()
                    else:
                        assert torch.equal(y, ref), (prec, vec, vsplit, unroll)
                        ran += 1
    assert ran >= 12


def test_graph_replay_matches_eager(B):
    """Graph replay of the steady two-step sequence gives the eager result bit
    for bit, on repeated calls with eager work and syncs in between."""
    cfg = small("cavity", nx=8, ny=6, nv=(16, 16, 8))
    C = B.Context(cfg, "fp32")
    x = C.initial_state()
    torch.cuda.synchronize()
    ref = {}
    for n in (5, 6, 9):
        C.set_seed(100 + n)
        ref[n] = C.step(x, n=n).clone()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        C.set_graph(True)
        out = torch.empty_like(x)
        for rep in range(3):
            for n in (5, 6, 9):
                C.set_seed(100 + n)
                C.step(x, out, n=n)
                side.synchronize()
                assert torch.equal(out, ref[n]), (rep, n)
                C.moments(out)  # eager work between replays
        C.set_graph(False)
    torch.cuda.synchronize()


def test_workspace_is_the_callers(B):
    """bgk_sizes reports the workspaces (one f for bgk_step; two and a byte
    per element, rounded up to 256, for the reverse sweep); bgk_step needs
    one for n >= 2 and rejects one that overlaps f_in or f_out; the output
    matches a run with the binding's own workspace."""
    cfg = small("cavity", nx=5, ny=4, nv=(12, 12, 8))
    C = B.Context(cfg, "fp32")
    fb = C.f_elems * 4
    assert C.ws_step_bytes == fb and C.ws_adjoint_bytes == 2 * fb + (C.f_elems + 255) // 256 * 256
    L = B.load()
    s = torch.cuda.current_stream().cuda_stream
    x = C.initial_state()
    y = torch.full_like(x, float("nan"))
    C.set_seed(3)
    assert L.bgk_step(C.h, x.data_ptr(), y.data_ptr(), 2, None, s) == B.E_INVALID
    big = torch.empty(3 * C.f_elems, dtype=torch.float32, device="cuda")
    assert L.bgk_step(C.h, x.data_ptr(), big.data_ptr(), 2, big[C.f_elems // 2:].data_ptr(), s) == B.E_ALIAS
    assert L.bgk_step(C.h, big.data_ptr(), big[C.f_elems // 2:].data_ptr(), 1, None, s) == B.E_ALIAS
    ws = torch.empty(fb, dtype=torch.uint8, device="cuda")
    assert L.bgk_step(C.h, x.data_ptr(), y.data_ptr(), 3, ws.data_ptr(), s) == B.OK
    C.set_seed(3)
    z = C.step(x, n=3)
    torch.cuda.synchronize()
    assert torch.equal(y, z)
    assert L.bgk_step(C.h, x.data_ptr(), y.data_ptr(), 1, None, s) == B.OK  # one step needs no workspace
    g = torch.zeros(2, dtype=torch.float64, device="cuda")
    lam = torch.ones_like(x)
    assert L.bgk_step_adjoint(C.h, x.data_ptr(), lam.data_ptr(), y.data_ptr(), g.data_ptr(), None, s) == B.E_INVALID
    torch.cuda.synchronize()


def _golden(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    return np.load(path) if os.path.exists(path) else None


def test_cavity_128_fp32_golden(B):
    """128^2 cavity, 24^3 velocities, FP32 f, lid Mach 0.1, Kn 0.1: moments
    against the stored oracle run (tests/golden/make_golden.py) at every
    stored step count, up to the workload's 5000 steps, within 1e-5."""
    G = _golden("cavity_128_fp32_oracle.npz")
    if G is None:
        pytest.skip("golden file not generated")
    cfg = inputs.config("cavity_128_fp32")
    C = B.Context(cfg, "fp32")
    assert C.dts[0] == pytest.approx(float(G["dt"]), rel=1e-14)
    f = C.initial_state()
    done, worst = 0, {}
    for m in [int(s) for s in G["steps"]]:
        f = C.step(f, n=m - done)
        done = m
        e = moment_errors(C.moments(f).cpu().numpy(), G[f"moments_{m}"], cfg)
        worst[m] = e
        assert max(e) <= 1e-5, (m, e)
    print("cavity_128_fp32 moment errors by step:", {m: tuple(f"{x:.2e}" for x in e) for m, e in worst.items()})


def test_batch_64_cavities_golden(B):
    """The seeded batch of 64 uneven cavities in one FP32 context, on a
    persistent grid (2 workgroups per compute unit walking all 425 472 work
    items) with graph replay on a side stream: the instances whose oracle
    runs are stored (tests/golden/make_batch_golden.py) match them within
    1e-5 after 1, 10, 100 and 1000 steps.  Steps 100 to 1000 are nine
    100-step calls ping-ponging between two buffers, so each of the two
    captured graphs is replayed."""
    import glob
    import os
    files = sorted(glob.glob(os.path.join(os.path.dirname(__file__), "golden", "batch_cavity_*_oracle.npz")))
    if not files:
        pytest.skip("golden files not generated")
    gold = [np.load(p) for p in files]
    probs = inputs.batch_cavities()
    C = B.Context(probs, "fp32")
    shape = C.launch()
    C.set_launch(shape["vec"], shape["unroll"], shape["vsplit"], 2)
    for G in gold:
        i = int(G["index"])
        assert probs[i]["nx"] == int(G["side"]) and probs[i]["kn"] == pytest.approx(float(G["kn"]), rel=1e-15)
        assert C.dts[i] == pytest.approx(float(G["dt"]), rel=1e-14)
    side = torch.cuda.Stream()
    seen = {}

    def check(f, m):
        mom = C.moments(f).cpu().numpy()
        for G in gold:
            if f"moments_{m}" not in G.files:
                continue
            i = int(G["index"])
            c0 = C.cell_offsets[i]
            ref = G[f"moments_{m}"]
            e = moment_errors(mom[c0:c0 + ref.shape[0]], ref, probs[i])
            seen[(i, m)] = e
            assert max(e) <= 1e-5, (i, m, e)

    with torch.cuda.stream(side):
        C.set_graph(True)
        x = C.initial_state()
        a = C.empty()
        b = C.empty()
        C.step(x, a, n=1)
        check(a, 1)
        C.step(a, b, n=9)
        check(b, 10)
        C.step(b, a, n=90)
        check(a, 100)
        del x
        src, dst = a, b
        for _ in range(9):
            C.step(src, dst, n=100)
            src, dst = dst, src
        check(src, 1000)
        C.set_graph(False)
    torch.cuda.synchronize()
    assert any(m == 1000 for _, m in seen), "no stored instance reached 1000 steps"
    print("batch moment errors:", {k: tuple(f"{x:.2e}" for x in e) for k, e in sorted(seen.items())})


@pytest.mark.parametrize("name", ["shock_m3_fp32", "cavity_128_fp32"])
def test_every_shape_full_size(B, oracle_mod, name):
    """Every launch shape on the full Mach-3 shock (1024 x 48^3) and the full
    128^2 x 24^3 cavity, FP32, two steps from the initial state: every element
    written (the step's output starts as NaN) and the moments within 1e-5 of
    the oracle.  The register-heaviest kernels (four jx per lane, deep jz
    pipelines) exist only at such sizes in the tuned shapes."""
    cfg = inputs.config(name)
    O = oracle_mod.Oracle(cfg)
    ref = O.moments(O.step(O.initial_state(), 2))
    C = B.Context(cfg, "fp32", tune="off")
    x = C.initial_state()
    ran = 0
    for vec in (1, 2, 4):
        for unroll in (1, 2, 3, 4):
            for vsplit in (1, 2):
                for persist in (0, 2):
                    try:
                        C.set_launch(vec, unroll, vsplit, persist)
                    except B.BGKError:
                        continue
                    y = C.step(x, n=2)
                    e = moment_errors(C.moments(y).cpu().numpy(), ref, cfg)
                    assert max(e) <= 1e-5, (vec, unroll, vsplit, persist, e)
                    ran += 1
    assert ran >= 16
