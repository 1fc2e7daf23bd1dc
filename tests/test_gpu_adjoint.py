"""Reverse sweep on the GPU (bgk_step_adjoint, bgk_lid_shear[_grad], the
checkpointed autograd rollout) against the oracle's FP64 reverse sweep and
against central finite differences of the GPU forward map.

Tolerances: FP64 path 1e-12 relative to the largest adjoint entry (and to
each parameter gradient); FP32 path 1e-4 relative on the gradients of the
full rollout (FP32 storage of f and of the adjoint, and minmod branch
decisions taken on FP32 values).
"""
import os

import numpy as np
import pytest
import torch

from paper_0903_4044_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_0903_4044_amd import binding
    binding.load()
    return binding


def small(kind, **kw):
    d = dict(kind=kind, nx=7, ny=5, x0=-2.0 if kind == "shock" else 0.0, x1=2.0 if kind == "shock" else 1.0,
             y0=0.0, y1=1.0, nv=(8, 6, 4), vlo=(-4.0, -4.0, -3.0), vhi=(4.0, 4.0, 3.0), kn=0.3, omega=0.5,
             cfl=0.5, dt=0.0, mach=1.5, lid_mach=0.25, t_wall=1.1, splitting="strang", limiter="minmod")
    d.update(kw)
    return d


def dev(x, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(x).reshape(-1), dtype=dtype, device="cuda")


def host(t, shape):
    return t.detach().cpu().numpy().astype(np.float64).reshape(shape)


CASES = [("shock", {}), ("shock", dict(nx=2)), ("periodic1d", {}), ("periodic2d", dict(nx=4, ny=3)),
         ("cavity", {}), ("cavity", dict(nx=1, ny=1)), ("cavity", dict(nx=2, ny=5, lid_mach=-0.3)),
         ("cavity", dict(splitting="lie")), ("cavity", dict(limiter="none")), ("shock", dict(splitting="lie")),
         ("cavity", dict(nv=(16, 16, 8), nx=5, ny=4))]


@pytest.mark.parametrize("kind,over", CASES)
def test_step_adjoint_matches_oracle_fp64(B, oracle_mod, kind, over):
    cfg = small(kind, **over)
    O = oracle_mod.Oracle(cfg)
    C = B.Context(cfg, "fp64")
    f = O.initial_state() * (1 + 0.2 * inputs.uniform(O.shape, seed=31, lo=-1, hi=1))
    lam = inputs.uniform(O.shape, seed=32, lo=-1, hi=1)
    ref, gref = O.step_adjoint(f, lam)
    got, grad = C.step_adjoint(dev(f), dev(lam))
    got = host(got, O.shape)
    grad = grad.cpu().numpy()[0]
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref)), np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    for i in range(2):
        assert abs(grad[i] - gref[i]) <= 1e-12 * max(abs(gref[i]), 1e-300) or (gref[i] == 0 and abs(grad[i]) < 1e-18)


def test_step_adjoint_fp32(B, oracle_mod):
    cfg = small("cavity", nv=(16, 16, 8), nx=6, ny=5)
    O = oracle_mod.Oracle(cfg)
    C = B.Context(cfg, "fp32")
    f = O.initial_state() * (1 + 0.2 * inputs.uniform(O.shape, seed=33, lo=-1, hi=1))
    lam = inputs.uniform(O.shape, seed=34, lo=-1, hi=1)
    ref, gref = O.step_adjoint(f, lam)
    got, grad = C.step_adjoint(dev(f, torch.float32), dev(lam, torch.float32))
    got = host(got, O.shape)
    err = np.abs(got - ref) / np.max(np.abs(ref))
    assert np.percentile(err, 99.9) <= 1e-5 and np.max(err) <= 1e-3, (np.percentile(err, 99.9), err.max())
    np.testing.assert_allclose(grad.cpu().numpy()[0], gref, rtol=1e-4)


def test_lid_shear_and_seed(B, oracle_mod):
    cfg = small("cavity", nv=(16, 16, 8))
    O = oracle_mod.Oracle(cfg)
    C = B.Context(cfg, "fp64")
    f = O.initial_state() * (1 + 0.2 * inputs.uniform(O.shape, seed=35, lo=-1, hi=1))
    x = dev(f)
    L = C.lid_shear(x).cpu().numpy()[0]
    assert L == pytest.approx(O.lid_shear(f), rel=1e-13)
    lam, grad = C.lid_shear_grad(x)
    lref, gref = O.lid_shear_grad(f)
    np.testing.assert_allclose(host(lam, O.shape), lref, rtol=1e-13, atol=1e-17)
    assert grad.cpu().numpy()[0, 1] == pytest.approx(gref[1], rel=1e-12)


def test_rollout_autograd_matches_oracle(B, oracle_mod):
    """Checkpointed rollout (every 2 steps) through torch.autograd."""
    from paper_0903_4044_amd import solver
    cfg = small("cavity", nx=6, ny=5, nv=(8, 8, 4), kn=0.1, lid_mach=0.1, t_wall=1.0)
    O = oracle_mod.Oracle(cfg)
    C = B.Context(cfg, "fp64")
    f0 = O.initial_state() * (1 + 1e-3 * inputs.noise(O.shape, seed=36))
    Lr, lam0, gkn, gtw = O.rollout_gradient(f0, 7)
    x = dev(f0).requires_grad_(True)
    kn = torch.tensor(cfg["kn"], dtype=torch.float64, requires_grad=True)
    tw = torch.tensor(cfg["t_wall"], dtype=torch.float64, requires_grad=True)
    fN = solver.rollout(x, kn, tw, C, 7, every=2)
    L = solver.lid_shear(fN, tw, C)
    L.backward()
    assert float(L.detach()) == pytest.approx(Lr, rel=1e-12)
    g0 = host(x.grad, O.shape)
    assert np.max(np.abs(g0 - lam0)) <= 1e-11 * np.max(np.abs(lam0))
    assert float(kn.grad) == pytest.approx(gkn, rel=1e-11)
    assert float(tw.grad) == pytest.approx(gtw, rel=1e-11)


@pytest.mark.parametrize("kind", ["shock", "cavity"])
def test_branch_record_fully_written(B, kind):
    """The recording streaming pass of a reverse step writes a branch byte for
    every element over the workspace's 0xFF poison: each 2-bit code is 0, 1
    or 2, and a one-dimensional kind leaves the y half zero."""
    cfg = small(kind)
    C = B.Context(cfg, "fp64")
    f = C.initial_state()
    xi = dev(inputs.noise((C.f_elems,), seed=43), C.dtype)
    f = f * (1 + 0.05 * xi)
    lam = dev(inputs.noise((C.f_elems,), seed=44), C.dtype)
    C.step_adjoint(f, lam)
    torch.cuda.synchronize()
    fb = C.f_elems * 8
    rec = C.workspace("adjoint")[2 * fb:2 * fb + C.f_elems].to(torch.int32)
    for shift in (0, 2, 4, 6):
        assert int(((rec >> shift) & 3).max()) <= 2, shift
    if kind == "shock":
        assert int((rec >> 4).max()) == 0
    # the limiter takes each branch somewhere on a perturbed state
    for code in (0, 1, 2):
        assert bool(((rec & 3) == code).any()), code


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_rollout_keeping_every_state_equals_checkpointed(B, prec):
    """Checkpoints with every = None keep every state when the trajectory
    fits the free memory (no segment recomputation).  The trajectory is the checkpointed rollout's
    bit for bit, and so are the FP64 gradients.  In FP32 a reverse step
    rounds its recomputed intermediate h stochastically with bits keyed by
    the context's rounding counter, which the recomputation of the
    checkpointed rollout advances differently, so there the gradients agree
    to rounding (1e-5)."""
    from paper_0903_4044_amd import solver
    cfg = small("cavity", nx=6, ny=5, kn=0.1, lid_mach=0.1, t_wall=1.0)
    C = B.Context(cfg, prec)
    f0 = C.initial_state()
    xi = dev(inputs.noise((C.f_elems,), seed=41), C.dtype)
    f0 = f0 * (1 + 1e-3 * xi)
    out = []
    for every in (3, None):
        C.set_seed(77)
        x = f0.clone().requires_grad_(True)
        kn = torch.tensor(cfg["kn"], dtype=torch.float64, requires_grad=True)
        tw = torch.tensor(cfg["t_wall"], dtype=torch.float64, requires_grad=True)
        L = solver.lid_shear(solver.rollout(x, kn, tw, C, 8, every=every, mode="checkpoint"), tw, C)
        L.backward()
        out.append((C.last_rollout["every"], float(L.detach()), x.grad.clone(), float(kn.grad), float(tw.grad)))
    (e3, L3, g3, k3, t3), (e1, L1, g1, k1, t1) = out
    assert e3 == 3 and e1 == 1
    assert L1 == L3
    if prec == "fp64":
        assert k1 == k3 and t1 == t3
        assert torch.equal(g1, g3)
    else:
        assert k1 == pytest.approx(k3, rel=1e-5) and t1 == pytest.approx(t3, rel=1e-5)
        assert float((g1 - g3).abs().max()) <= 1e-5 * float(g3.abs().max())


@pytest.mark.parametrize("kind", ["shock", "cavity"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_step_record_matches_step_and_adjoint(B, kind, prec):
    """bgk_step_record advances f as a one-step bgk_step (the same rounding
    counter; moment sums may be added in another order), and the reverse step
    from its record equals bgk_step_adjoint's recomputation: FP64 to 1e-12.
    In FP32 the recomputed intermediate h is rounded with the counter of the
    reverse call, the recorded one with the forward's, so there 1e-4 of the
    largest entry."""
    cfg = small(kind)
    C = B.Context(cfg, prec)
    f = C.initial_state()
    f = f * (1 + 0.05 * dev(inputs.noise((C.f_elems,), seed=45), C.dtype))
    C.set_seed(11)
    y1 = C.step(f, n=1)
    s1 = C.seed()
    C.set_seed(11)
    y2, rec = C.step_record(f)
    assert C.seed() == s1
    tol = 1e-13 if prec == "fp64" else 1e-6
    assert float((y1 - y2).abs().max()) <= tol * float(y1.abs().max())
    lam = dev(inputs.noise((C.f_elems,), seed=46), C.dtype)
    l1, g1 = C.step_adjoint(f, lam)
    l2, g2 = C.step_adjoint_record(f, rec, lam)
    torch.cuda.synchronize()
    tol = 1e-12 if prec == "fp64" else 1e-4
    assert float((l1 - l2).abs().max()) <= tol * float(l1.abs().max())
    assert torch.allclose(g1, g2, rtol=tol, atol=tol * float(g1.abs().max()))


@pytest.mark.parametrize("kind", ["shock", "cavity"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_adjoint_sweep_matches_per_step(B, kind, prec):
    """bgk_adjoint_sweep_record over 5 recorded steps (the close pass of each
    step forming the sums of the step before) against 5 calls of
    bgk_step_adjoint_record: lambda^0 to 1e-12 of its largest entry in FP64
    and 1e-6 in FP32, the parameter gradients to 1e-12 relative (summed in
    another order); no steps gives lambda^0 = lambda^N."""
    cfg = small(kind)
    C = B.Context(cfg, prec)
    f = C.initial_state()
    f = f * (1 + 0.05 * dev(inputs.noise((C.f_elems,), seed=48), C.dtype))
    states, recs = [], []
    for _ in range(5):
        states.append(f)
        f, rec = C.step_record(f)
        recs.append(rec)
    lamN = dev(inputs.noise((C.f_elems,), seed=49), C.dtype)
    lam, g1 = lamN.clone(), C.grad_buffer()
    for i in range(4, -1, -1):
        lam, _ = C.step_adjoint_record(states[i], recs[i], lam, None, g1)
    l2, g2 = C.adjoint_sweep_record(states, recs, lamN)
    torch.cuda.synchronize()
    tol = 1e-12 if prec == "fp64" else 1e-6
    assert float((lam - l2).abs().max()) <= tol * float(lam.abs().max())
    assert torch.allclose(g1, g2, rtol=1e-12, atol=1e-12 * float(g1.abs().max()))
    l0, _ = C.adjoint_sweep_record([], [], lamN)
    torch.cuda.synchronize()
    assert torch.equal(l0, lamN)


def test_step_record_rules(B):
    """Record entry points: the record must not overlap f_in or f_out, lam_n
    not the record; 3D contexts have no reverse sweep (BGK_E_UNSUPPORTED)."""
    L = B.load()
    C = B.Context(small("cavity"), "fp64")
    f = C.initial_state()
    s = torch.cuda.current_stream().cuda_stream
    big = torch.empty(C.record_bytes + 16 * C.f_elems, dtype=torch.uint8, device="cuda")
    out = torch.empty_like(f)
    assert L.bgk_step_record(C.h, f.data_ptr(), out.data_ptr(), f.data_ptr(), s) == B.E_ALIAS
    assert L.bgk_step_record(C.h, f.data_ptr(), big.data_ptr(), big.data_ptr(), s) == B.E_ALIAS
    assert L.bgk_step_record(C.h, f.data_ptr(), out.data_ptr(), None, s) == B.E_INVALID
    rec = torch.empty(C.record_bytes, dtype=torch.uint8, device="cuda")
    out, rec = C.step_record(f, out, rec)
    grad = C.grad_buffer()
    ws = C.workspace("adjoint")
    assert L.bgk_step_adjoint_record(C.h, f.data_ptr(), rec.data_ptr(), f.data_ptr(), rec.data_ptr(),
                                     grad.data_ptr(), ws.data_ptr(), s) == B.E_ALIAS
    import ctypes
    arr = (ctypes.c_void_p * 1)(f.data_ptr())
    rarr = (ctypes.c_void_p * 1)(rec.data_ptr())
    lam = torch.zeros_like(f)
    assert L.bgk_adjoint_sweep_record(C.h, 1, None, rarr, lam.data_ptr(), out.data_ptr(), grad.data_ptr(),
                                      ws.data_ptr(), s) == B.E_INVALID
    assert L.bgk_adjoint_sweep_record(C.h, 1, arr, rarr, lam.data_ptr(), f.data_ptr(), grad.data_ptr(),
                                      ws.data_ptr(), s) == B.E_ALIAS
    assert L.bgk_adjoint_sweep_record(C.h, -1, arr, rarr, lam.data_ptr(), out.data_ptr(), grad.data_ptr(),
                                      ws.data_ptr(), s) == B.E_INVALID
    cube = small("cavity3d", nx=4, ny=3, nz=4, z0=0.0, z1=1.0, nv=(8, 6, 8), vlo=(-4.0, -3.0, -4.0),
                 vhi=(4.0, 3.0, 4.0), lid_mach=0.2)
    C3 = B.Context(cube, "fp64")
    with pytest.raises(B.BGKError) as e:
        C3.step_record(C3.initial_state())
    assert e.value.code == B.E_UNSUPPORTED


def test_rollout_record_mode_matches_oracle(B, oracle_mod):
    """The rollout with step records (mode "record") through torch.autograd
    against the oracle's reverse sweep, as the checkpointed rollout."""
    from paper_0903_4044_amd import solver
    cfg = small("cavity", nx=6, ny=5, nv=(8, 8, 4), kn=0.1, lid_mach=0.1, t_wall=1.0)
    O = oracle_mod.Oracle(cfg)
    C = B.Context(cfg, "fp64")
    f0 = O.initial_state() * (1 + 1e-3 * inputs.noise(O.shape, seed=36))
    Lr, lam0, gkn, gtw = O.rollout_gradient(f0, 7)
    x = dev(f0).requires_grad_(True)
    kn = torch.tensor(cfg["kn"], dtype=torch.float64, requires_grad=True)
    tw = torch.tensor(cfg["t_wall"], dtype=torch.float64, requires_grad=True)
    C.set_seed(5)
    L = solver.lid_shear(solver.rollout(x, kn, tw, C, 7, mode="record"), tw, C)
    s_after_forward = C.seed()
    L.backward()
    assert C.last_rollout == {"mode": "record", "every": 1}
    assert C.seed() == s_after_forward
    assert float(L.detach()) == pytest.approx(Lr, rel=1e-12)
    g0 = host(x.grad, O.shape)
    assert np.max(np.abs(g0 - lam0)) <= 1e-11 * np.max(np.abs(lam0))
    assert float(kn.grad) == pytest.approx(gkn, rel=1e-11)
    assert float(tw.grad) == pytest.approx(gtw, rel=1e-11)


def _loss(B, cfg, prec, f0, nsteps):
    C = B.Context(cfg, prec)
    return float(C.lid_shear(C.step(f0, n=nsteps))[0])


@pytest.mark.parametrize("mode", ["checkpoint", "record"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_full_adjoint_workload(B, prec, mode):
    """64^2 cavity, 24^3 velocities, 200 steps, checkpoints every 20 or step
    records of every step (nothing recomputed in the reverse sweep): the GPU
    gradients against the stored FP64 oracle reverse sweep (loss, dL/dKn,
    dL/dT_w, three seeded projections of dL/df0 and lambda^0 on four cells),
    and, in FP64, against central differences of the GPU forward map.  FP32
    gradients are 1e-4 relative; a projection's error is bounded by 1e-4 of
    the sum of its terms' magnitudes (a signed sum cancels).  The
    difference quotient crosses minmod kinks: at a relative step of 1e-6 it
    is off by 1.2e-5 in dL/dT_w, so the step is 1e-7 and the bound 1e-5."""
    from paper_0903_4044_amd import solver
    path = os.path.join(os.path.dirname(__file__), "golden", "cavity_64_adjoint_oracle.npz")
    cfg = inputs.config("cavity_64_adjoint")
    C = B.Context(cfg, prec)
    nsteps = cfg["steps"]
    f0 = C.initial_state()
    xi = dev(inputs.noise((C.f_elems,)), C.dtype)
    f0 = (f0 * (1 + 1e-3 * xi)).requires_grad_(True)
    kn = torch.tensor(cfg["kn"], dtype=torch.float64, requires_grad=True)
    tw = torch.tensor(cfg["t_wall"], dtype=torch.float64, requires_grad=True)
    every = 20 if mode == "checkpoint" else None
    L = solver.lid_shear(solver.rollout(f0, kn, tw, C, nsteps, every=every, mode=mode), tw, C)
    L.backward()
    assert C.last_rollout["mode"] == mode
    tol = 1e-10 if prec == "fp64" else 1e-4
    G = np.load(path)
    print(f"{prec}: L {float(L.detach())!r} dKn {float(kn.grad)!r} dTw {float(tw.grad)!r}")
    assert float(L.detach()) == pytest.approx(float(G["L"]), rel=1e-12 if prec == "fp64" else 1e-5)
    assert float(kn.grad) == pytest.approx(float(G["grad"][0]), rel=tol)
    assert float(tw.grad) == pytest.approx(float(G["grad"][1]), rel=tol)
    base = f0.detach()
    for s, want in zip(G["dirs"], G["proj"]):
        d = dev(inputs.noise((C.f_elems,), seed=int(s)), C.dtype) * base
        prod = f0.grad.double() * d.double()
        got, scale = float(torch.sum(prod)), float(torch.sum(torch.abs(prod)))
        # FP32: the projection is a sum of terms of both signs, so its error is
        # bounded relative to the sum of their magnitudes
        bound = tol * abs(float(want)) if prec == "fp64" else tol * scale
        assert abs(got - float(want)) <= bound, (int(s), got, float(want), scale)
    lam = f0.grad.double().reshape(inputs.ncells(cfg), inputs.nvel(cfg))[torch.as_tensor(G["cells"])].cpu().numpy()
    ref = G["lam0_cells"]
    err = np.abs(lam - ref) / np.max(np.abs(ref))
    if prec == "fp64":
        assert err.max() <= 1e-10, err.max()
    else:
        # The adjoint is piecewise constant in the state (minmod branches).
        # FP32 rounding of f moves near-ties to the other branch, which changes
        # the entry by C k mu (k = (1 - C)/2) there and spreads from it, so
        # the FP32 bound is on the bulk of the entries, with a looser one on
        # every entry.  Measured with the recomputed trajectory equal to the
        # forward one: p99 4.1e-4, max 8.8e-3 of max |lambda^0|.
        print(f"fp32 lambda0 on sampled cells: p99 {np.percentile(err, 99):.3e} max {err.max():.3e}")
        assert np.percentile(err, 99) <= 2e-3 and err.max() <= 3e-2, (np.percentile(err, 99), err.max())
    if prec == "fp64":
        x = f0.detach()
        for key, got in (("kn", float(kn.grad)), ("t_wall", float(tw.grad))):
            h = 1e-7 * cfg[key]
            fd = (_loss(B, dict(cfg, **{key: cfg[key] + h}), prec, x, nsteps) -
                  _loss(B, dict(cfg, **{key: cfg[key] - h}), prec, x, nsteps)) / (2 * h)
            assert got == pytest.approx(fd, rel=1e-5), key


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_checkpoint_recompute_reproduces_forward(B, oracle_mod, prec):
    """The backward pass recomputes each checkpoint segment from its stored
    state and rounding seed; the recomputed states are the forward pass's,
    bit for bit (FP32 included: the same rounding counters), so the reverse
    sweep differentiates the trajectory the loss was computed on.  The
    caller's rounding seed is restored after the backward pass."""
    from paper_0903_4044_amd import solver
    cfg = small("cavity", nx=6, ny=5)
    O = oracle_mod.Oracle(cfg)
    C = B.Context(cfg, prec)
    f0 = dev(O.initial_state() * (1 + 0.2 * inputs.uniform(O.shape, seed=37, lo=-1, hi=1)), C.dtype)
    nsteps, every = 11, 4
    C.set_seed(500)
    fN, ckpt, seeds = solver.forward_checkpoints(C, f0, nsteps, every)
    assert len(ckpt) == 3 and seeds[0] == 500
    ends = ckpt[1:] + [fN]
    for seg in range(len(ckpt)):
        k = min(every, nsteps - seg * every)
        states = solver.recompute_segment(C, ckpt[seg], seeds[seg], k)
        last = C.step(states[-1], n=1)
        assert torch.equal(last, ends[seg]), seg
    # through autograd: the seed after backward is the caller's
    C.set_seed(900)
    x = f0.clone().requires_grad_(True)
    kn = torch.tensor(cfg["kn"], dtype=torch.float64, requires_grad=True)
    tw = torch.tensor(cfg["t_wall"], dtype=torch.float64, requires_grad=True)
    L = solver.lid_shear(solver.rollout(x, kn, tw, C, nsteps, every=every), tw, C)
    s_after_forward = C.seed()
    L.backward()
    assert C.seed() == s_after_forward
    assert torch.isfinite(x.grad).all()
