"""GPU tests of the steady-state drivers: batched and plain runs to residual
< 1e-8 (FP64 storage) agree; FP32 runs stop at their rounding floor."""
import sys

import numpy as np
import pytest

from workloads import SplitMix64, cavity_sides, channel_sides, random_obstacles

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mods():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_10251_amd import lbm as L
    from paper_1806_10251_amd import steady
    L.load()
    return L, steady


def cases():
    rng = SplitMix64(77)
    return [
        dict(nx=48, ny=48, sides=cavity_sides(), solid=random_obstacles(rng, 48, 48, "cavity"),
             kw=dict(nu=0.1 * 48 / 100, gamma=0.5, u_lid=0.1)),
        dict(nx=128, ny=32, sides=channel_sides(), solid=random_obstacles(rng, 128, 32, "channel"),
             kw=dict(nu=0.05 * 32 / 40, gamma=0.5, u_in_max=0.05)),
        dict(nx=40, ny=40, sides=cavity_sides(), solid=None,
             kw=dict(nu=0.1 * 40 / 50, gamma=1.0, u_lid=0.1)),
    ]


def test_batch_and_plain_reach_the_same_steady_state(mods):
    L, steady = mods
    cs = cases()
    grids = [L.make_grid(c["nx"], c["ny"], c["sides"]) for c in cs]
    params = [L.make_params(storage="f64", check_every=100, **c["kw"]) for c in cs]
    b = L.Batch(grids, [c["solid"] for c in cs], params)
    steps, st, sec = steady.run_batch(b, tol=1e-8, max_steps=400000)
    _say("batch", list(steps), list(st), round(sec, 2))
    assert all(st == 1), st
    for i, c in enumerate(cs):
        lat = L.Lattice(c["nx"], c["ny"], c["sides"], solid=c["solid"], storage="f64",
                        check_every=100, **c["kw"])
        res = steady.run_single(lat, tol=1e-8, max_steps=400000)
        _say("plain", i, res.steps, res.status)
        assert res.status == "converged"
        assert res.residual < 1e-8
        assert res.steps == steps[i]
        _, uxb, uyb = b.fields(i, c["ny"], c["nx"])
        _, uxs, uys = lat.fields()
        assert np.abs(uxb - uxs).max() < 1e-13
        assert np.abs(uyb - uys).max() < 1e-13
        lat.close()


def test_fp32_stops_at_its_floor(mods):
    """FP32 storage: the plateau rule ends the run; the floor is above 1e-8
    but the field agrees with the FP64 steady state to FP32 accuracy."""
    L, steady = mods
    c = cases()[0]
    a = L.Lattice(c["nx"], c["ny"], c["sides"], solid=c["solid"], storage="f32", check_every=100,
                  **c["kw"])
    ra = steady.run_single(a, tol=1e-8, max_steps=400000, plateau_checks=10)
    f = L.Lattice(c["nx"], c["ny"], c["sides"], solid=c["solid"], storage="f64", check_every=100,
                  **c["kw"])
    rf = steady.run_single(f, tol=1e-8, max_steps=400000)
    _say("fp32", ra.status, ra.steps, ra.residual, "fp64", rf.status, rf.steps)
    assert ra.status in ("plateau", "converged") and rf.status == "converged"
    _, uxa, uya = a.fields()
    _, uxf, uyf = f.fields()
    U = c["kw"]["u_lid"]
    assert max(np.abs(uxa - uxf).max(), np.abs(uya - uyf).max()) / U < 1e-4


def _oracle_steps_to(n, re, u, gamma, tol, check=100, max_steps=200000):
    """Steps until the one-step residual first falls below tol at a check
    step (every `check` steps, from step 2 * check on), by the FP64 oracle:
    the same stopping rule as the GPU driver."""
    import oracle
    o = oracle.Oracle(n, n, cavity_sides(), nu=u * n / re, gamma=gamma, u_lid=u)
    s = 0
    while s < max_steps:
        o.step(check)
        s += check
        if s >= 2 * check and o.residual < tol:
            return s
    return None


def test_preconditioning_accelerates_convergence(mods):
    """Sec. 6: steps to steady state fall with gamma (the momentum equation
    of eq. 1 runs 1/gamma times faster while its steady state is unchanged).
    64^2 cavity, Re 100, U 0.05, FP64, residual 1e-6: gamma 0.5 and 0.25
    against gamma 1.  The step counts are those of the FP64 oracle run with
    the same stopping rule (within one check interval); the gain flattens
    below 0.5 at this Mach number."""
    L, steady = mods
    _say("gamma sweep cavity 64x64 Re 100 U 0.05 f64 gammas 1, 0.5, 0.25")
    gammas = [1.0, 0.5, 0.25]
    rows = steady.gamma_sweep("cavity", 64, 100.0, 0.05, gammas, tols=(1e-6,),
                              max_steps=200000)
    steps = {r["gamma"]: r["steps_to"]["1e-06"] for r in rows}
    _say("steps to 1e-6:", steps)
    ref = {g: _oracle_steps_to(64, 100.0, 0.05, g, 1e-6) for g in gammas}
    _say("oracle steps to 1e-6:", ref)
    assert all(r["status"] == "converged" for r in rows)
    for g in gammas:
        assert ref[g] is not None and abs(steps[g] - ref[g]) <= 100, (g, steps[g], ref[g])
    assert steps[0.5] < 0.6 * steps[1.0]
    assert steps[0.25] < min(0.45 * steps[1.0], steps[0.5])
