"""GPU parity of the kernel variants against the FP64 oracle: strain_fd = 1
(the strain rates d_x u_x, d_y u_y of the GI corrections from the velocity
at the same time level instead of eqs. 51-55), mrt = 1 (the raw-moment MRT
form of the collision, eq. 7) and both together.

Each case prints its name, shape and parameters before the GPU work starts.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from workloads import (SplitMix64, cavity_sides, channel_sides, four_roll_mill_force,
                       periodic_sides, random_obstacles)

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


def _max_du(o, g, U):
    _, uo, vo = o.fields()
    _, ug, vg = g.fields()
    return max(np.abs(ug - uo).max(), np.abs(vg - vo).max()) / U


VARIANTS = [dict(strain_fd=1), dict(mrt=1), dict(mrt=1, strain_fd=1)]
VIDS = ["fd-strain", "mrt", "mrt+fd-strain"]


@pytest.mark.parametrize("var", VARIANTS, ids=VIDS)
@pytest.mark.parametrize("storage,tol", [("f64", 1e-11), ("f32", 1e-5)])
def test_ragged_cavity_with_obstacles_every_launch_shape(lbm, storage, tol, var):
    """150 x 77 cavity with seeded obstacles (several tiles, ragged tails),
    gamma 0.4, 150 steps, every launch shape."""
    nx, ny, U = 150, 77, 0.08
    m = random_obstacles(SplitMix64(5), nx, ny, "cavity")
    kw = dict(nu=0.05, gamma=0.4, u_lid=U, **var)
    o = oracle.Oracle(nx, ny, cavity_sides(), solid=m, **kw)
    o.step(150)
    for shape in lbm.launch_shapes():
        _say("variant", var, "ragged cavity", storage, shape)
        g = lbm.Lattice(nx, ny, cavity_sides(), solid=m, storage=storage, **kw)
        g.set_launch(*shape)
        g.step(150)
        err = _max_du(o, g, U)
        assert err < tol, (shape, err)
        g.close()


@pytest.mark.parametrize("var", VARIANTS, ids=VIDS)
@pytest.mark.parametrize("stencil", [0, 1])
def test_channel_with_obstacle_and_outlet(lbm, stencil, var):
    nx, ny, U = 200, 40, 0.04
    m = np.zeros((ny, nx), np.uint8)
    m[15:25, 60:70] = 1
    _say("variant", var, "channel obstacle", nx, ny, "stencil", stencil)
    kw = dict(nu=0.05, gamma=0.3, u_in_max=U, drho_stencil=stencil, **var)
    o = oracle.Oracle(nx, ny, channel_sides(), solid=m, **kw)
    g = lbm.Lattice(nx, ny, channel_sides(), solid=m, storage="f64", **kw)
    o.step(300)
    g.step(300)
    assert _max_du(o, g, U) < 1e-11


@pytest.mark.parametrize("var", VARIANTS + [dict(mrt=1, gi_correct=0)],
                         ids=VIDS + ["mrt-uncorrected"])
def test_four_roll_mill_with_force_field(lbm, var):
    """A per-node force with each variant (the velocity in the finite
    differences carries the per-node F/(2 gamma) shift): four-rolls mill
    80 x 80, gamma 0.3, 400 steps."""
    n, u0, gamma = 80, 0.045, 0.3
    nu = u0 * n / 20.0
    _say("variant", var, "four-roll mill", n, "gamma", gamma)
    fx, fy = four_roll_mill_force(n, u0, nu)
    k = 2 * math.pi / n
    x = (np.arange(n) + 0.5) * k
    X, Y = np.meshgrid(x, x)
    init = (None, u0 * np.sin(X) * np.sin(Y), u0 * np.cos(X) * np.cos(Y))
    kw = dict(nu=nu, gamma=gamma, **var)
    o = oracle.Oracle(n, n, periodic_sides(), **kw)
    g = lbm.Lattice(n, n, periodic_sides(), storage="f64", **kw)
    for lat in (o, g):
        lat.set_force_field(fx, fy)
        lat.init_fields(*init)
        lat.step(400)
    assert _max_du(o, g, u0) < 1e-11


@pytest.mark.parametrize("var", VARIANTS, ids=VIDS)
def test_batch_rejects_variants(lbm, var):
    _say("batch rejects", var)
    grid = lbm.make_grid(32, 32, cavity_sides())
    params = lbm.make_params(nu=0.02, gamma=0.5, u_lid=0.1, storage="f32", check_every=100,
                             **var)
    with pytest.raises(lbm.LbmError):
        lbm.Batch([grid], [None], [params])
