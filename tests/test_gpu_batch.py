"""GPU tests of the batched persistent solver (through the C ABI)."""
import sys

import numpy as np
import pytest

import oracle
from workloads import SplitMix64, cavity_sides, channel_sides, random_obstacles

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_10251_amd import lbm as L
    L.load()
    return L


def small_cases():
    """Cavities and channels of uneven size, Re and gamma, with obstacles."""
    rng = SplitMix64(2024)
    cases = []
    m1 = random_obstacles(rng, 40, 40, "cavity")
    m2 = random_obstacles(rng, 96, 24, "channel")
    cases.append(dict(nx=48, ny=48, sides=cavity_sides(), solid=None,
                      kw=dict(nu=0.1 * 48 / 100, gamma=0.5, u_lid=0.1)))
    cases.append(dict(nx=40, ny=40, sides=cavity_sides(), solid=m1,
                      kw=dict(nu=0.1 * 40 / 200, gamma=0.8, u_lid=0.1)))
    cases.append(dict(nx=96, ny=24, sides=channel_sides(), solid=m2,
                      kw=dict(nu=0.05 * 24 / 20, gamma=0.3, u_in_max=0.05)))
    cases.append(dict(nx=64, ny=16, sides=channel_sides(), solid=None,
                      kw=dict(nu=0.05 * 16 / 30, gamma=1.0, u_in_max=0.05)))
    cases.append(dict(nx=70, ny=66, sides=cavity_sides(), solid=None,
                      kw=dict(nu=0.1 * 70 / 400, gamma=1.0, u_lid=0.1)))
    return cases


def make_batch(L, cases, K=100):
    grids = [L.make_grid(c["nx"], c["ny"], c["sides"]) for c in cases]
    params = [L.make_params(storage="f32", check_every=K, **c["kw"]) for c in cases]
    masks = [c["solid"] for c in cases]
    return L.Batch(grids, masks, params)


@pytest.mark.parametrize("by,sched", [(4, 0), (8, 0), (16, 0), (4, 2)])
def test_batch_matches_single_lattice_runs(lbm, by, sched):
    """Each case retired by the batch equals a single-lattice run of the same
    number of steps (same arithmetic, bit for bit up to rounding order)."""
    cases = small_cases()
    _say("batch vs single, block height", by, "schedule", sched)
    b = make_batch(lbm, cases)
    b.set_launch(by, sched)
    steps = b.run(1e-6, 30000)
    _say("steps per case", list(steps))
    assert all(s > 0 for s in steps)
    assert all(s % 100 == 0 for s in steps)
    for i, c in enumerate(cases):
        rb, uxb, uyb = b.fields(i, c["ny"], c["nx"])
        assert b.residual(i) < 1e-6 or steps[i] == 30000
        g = lbm.Lattice(c["nx"], c["ny"], c["sides"], solid=c["solid"], storage="f32",
                        check_every=100, **c["kw"])
        g.step(int(steps[i]))
        rs, uxs, uys = g.fields()
        assert np.abs(uxb - uxs).max() < 1e-7, i
        assert np.abs(uyb - uys).max() < 1e-7, i
        assert np.abs(rb - rs).max() < 1e-6, i
        g.close()
    b.close()


def test_batch_per_class_launches_match_single_lattice_runs(lbm):
    """With 2048 or more active items the graph schedule launches one kernel
    per item class and step (interior tiles, closed-lattice boundary tiles,
    outlet boundary tiles); with fewer, one kernel for all.  The small
    batches above take the single launch; this one (2304 tiles of 64 x 4)
    takes the per-class launches, and each case equals its single-lattice
    run after the same 300 steps."""
    rng = SplitMix64(77)
    cases = []
    for k in range(6):
        cases.append(dict(nx=256, ny=256, sides=cavity_sides(),
                          solid=random_obstacles(rng, 256, 256, "cavity") if k % 2 else None,
                          kw=dict(nu=0.1 * 256 / (100 + 150 * k), gamma=0.3 + 0.1 * k,
                                  u_lid=0.1)))
        cases.append(dict(nx=512, ny=64, sides=channel_sides(),
                          solid=random_obstacles(rng, 512, 64, "channel") if k % 2 else None,
                          kw=dict(nu=0.05 * 64 / (20 + 10 * k), gamma=0.4 + 0.1 * k,
                                  u_in_max=0.05)))
    tiles = sum(-(-c["nx"] // 64) * -(-c["ny"] // 4) for c in cases)
    assert tiles >= 2048
    _say("per-class launches:", len(cases), "cases,", tiles, "tiles")
    b = make_batch(lbm, cases)
    b.set_launch(4, 0)
    b.run(0.0, 300)
    for i in (0, 1, 2, 3):
        c = cases[i]
        rb, uxb, uyb = b.fields(i, c["ny"], c["nx"])
        g = lbm.Lattice(c["nx"], c["ny"], c["sides"], solid=c["solid"], storage="f32",
                        check_every=100, **c["kw"])
        g.step(300)
        rs, uxs, uys = g.fields()
        assert np.abs(uxb - uxs).max() < 1e-7, i
        assert np.abs(uyb - uys).max() < 1e-7, i
        assert np.abs(rb - rs).max() < 1e-6, i
        g.close()
    b.close()


@pytest.mark.parametrize("sched,chunks", [(1, (300,)), (2, (300,)), (0, (130, 70, 100)),
                                          (2, (1, 149, 150))])
def test_batch_schedules_and_partial_windows(lbm, sched, chunks):
    """Interleaved and dataflow schedules, and runs that stop between check
    steps (partial windows), give the single-lattice result."""
    cases = small_cases()[:3]
    _say("schedule", sched, "chunks", chunks)
    b = make_batch(lbm, cases)
    b.set_launch(4, sched)
    total = np.zeros(len(cases), dtype=np.int64)
    for n in chunks:
        total += b.run(0.0, n)
    assert all(s == 300 for s in total)
    for i, c in enumerate(cases):
        g = lbm.Lattice(c["nx"], c["ny"], c["sides"], solid=c["solid"], storage="f32",
                        check_every=100, **c["kw"])
        g.step(300)
        np.testing.assert_allclose(b.fields(i, c["ny"], c["nx"])[1], g.fields()[1], atol=1e-7)
        g.close()
    b.close()


def test_batch_rejects_bad_launch(lbm):
    b = make_batch(lbm, small_cases()[:1])
    with pytest.raises(lbm.LbmError):
        b.set_launch(5, 0)
    with pytest.raises(lbm.LbmError):
        b.set_launch(4, 3)


def test_batch_against_oracle(lbm):
    cases = small_cases()
    _say("batch vs oracle 400 steps")
    b = make_batch(lbm, cases)
    steps = b.run(0.0, 400)
    assert all(s == 400 for s in steps)
    for i, c in enumerate(cases):
        o = oracle.Oracle(c["nx"], c["ny"], c["sides"], solid=c["solid"], **c["kw"])
        o.step(400)
        _, uxo, uyo = o.fields()
        _, uxb, uyb = b.fields(i, c["ny"], c["nx"])
        U = c["kw"].get("u_lid", 0) or c["kw"].get("u_in_max")
        err = max(np.abs(uxb - uxo).max(), np.abs(uyb - uyo).max()) / U
        assert err < 1e-5, (i, err)


def test_batch_reports_diverging_case(lbm):
    cases = small_cases()[:2]
    cases.append(dict(nx=32, ny=32, sides=cavity_sides(), solid=None,
                      kw=dict(nu=0.0032, gamma=0.05, u_lid=0.1)))
    _say("batch with an unstable case")
    b = make_batch(lbm, cases)
    steps = b.run(1e-6, 30000)
    _say("steps", list(steps))
    assert b.diverged
    assert steps[2] < 0
    assert steps[0] > 0 and steps[1] > 0 and steps[0] < 30000 and steps[1] < 30000
