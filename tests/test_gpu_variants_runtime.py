"""The runtime paths (graph replay, autotuning) with the next-row variants:
translation-form streaming, the conservative Maxwellian and the reduced
velocity space."""
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


VARIANTS = {
    "conservative_cavity": dict(kind="cavity", nx=8, ny=6, nv=(16, 16, 8), vlo=(-4.0,) * 3, vhi=(4.0,) * 3,
                                maxwellian="conservative"),
    "reduced_cavity": dict(kind="cavity", nx=8, ny=6, nv=(16, 16, 2), vlo=(-4.0, -4.0, -1.0),
                           vhi=(4.0, 4.0, 1.0), reduced=True),
    "reduced_shift_shock": dict(kind="shock", nx=40, x0=-2.0, x1=2.0, nv=(24, 1, 2), vlo=(-4.0, -1.0, -1.0),
                                vhi=(5.0, 1.0, 1.0), limiter="shift", splitting="lie", cfl=3.3, reduced=True),
    "shift_shock": dict(kind="shock", nx=40, x0=-2.0, x1=2.0, nv=(12, 6, 4), vlo=(-4.0, -3.0, -3.0),
                        vhi=(5.0, 3.0, 3.0), limiter="shift", splitting="lie", cfl=3.3),
}


def config(name):
    d = dict(ny=1, x0=0.0, x1=1.0, y0=0.0, y1=1.0, kn=0.3, omega=0.5, cfl=0.5, dt=0.0, mach=1.5, lid_mach=0.2,
             t_wall=1.1, splitting="strang", limiter="minmod", maxwellian="point")
    d.update(VARIANTS[name])
    return d


@pytest.mark.parametrize("name", list(VARIANTS))
def test_graph_replay_matches_eager(B, name):
    """Graph replay gives the eager result bit for bit, replayed repeatedly
    with eager work and synchronisations in between."""
    C = B.Context(config(name), "fp32", tune="off")
    x = C.initial_state()
    torch.cuda.synchronize()
    ref = {}
    for n in (4, 7):
        C.set_seed(200 + n)
        ref[n] = C.step(x, n=n).clone()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        C.set_graph(True)
        out = torch.empty_like(x)
        for rep in range(3):
            for n in (4, 7):
                C.set_seed(200 + n)
                C.step(x, out, n=n)
                side.synchronize()
                assert torch.equal(out, ref[n]), (rep, n)
                C.moments(out)
        C.set_graph(False)
    torch.cuda.synchronize()


@pytest.mark.parametrize("name", list(VARIANTS))
def test_autotune_keeps_parity(B, oracle_mod, name):
    """Whatever shape the autotuner picks, FP64 steps match the oracle."""
    cfg = config(name)
    O = oracle_mod.Oracle(cfg)
    f0 = O.initial_state() * (1 + 0.2 * inputs.uniform(O.shape, seed=107, lo=-1, hi=1))
    C = B.Context(cfg, "fp64", tune="off")
    x = torch.tensor(f0.reshape(-1), dtype=torch.float64, device="cuda")
    assert C.autotune(x)["tuned_us"] > 0
    ref = O.step(f0, 4)
    y = C.step(x, n=4).cpu().numpy().reshape(O.shape)
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def run_batch(B, oracle_mod, probs, nsteps, seed):
    C = B.Context(probs, "fp64", tune="off")
    f = C.empty()
    refs = []
    for i, p in enumerate(probs):
        O = oracle_mod.Oracle(p)
        f0 = O.initial_state() * (1 + 0.2 * inputs.uniform(O.shape, seed=seed + i, lo=-1, hi=1))
        C.instance_view(f, i).copy_(torch.from_numpy(f0))
        refs.append(O.step(f0, nsteps))
    y = C.step(f, n=nsteps)
    for i, ref in enumerate(refs):
        got = C.instance_view(y, i).cpu().numpy()
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max(), err_msg=str(i))


def test_batch_mixes_maxwellian_forms(B, oracle_mod):
    """The Maxwellian form is per instance: a conservative and a point-value
    cavity of different sizes in one context each match their own oracle."""
    a = config("conservative_cavity")
    b = dict(a, nx=5, ny=9, maxwellian="point", kn=0.8)
    run_batch(B, oracle_mod, [a, b], 4, 300)


def test_batch_of_translation_form_shocks(B, oracle_mod):
    """Shocks of uneven length and Mach number streamed in the translation
    form in one context (each with its own Courant numbers)."""
    a = config("shift_shock")
    b = dict(a, nx=23, mach=2.2, x0=-3.0, x1=1.5)
    run_batch(B, oracle_mod, [a, b], 5, 310)
