"""GPU parity of the singular-system guard of the strain solve (eqs. 51-55;
the paper does not treat a singular 2x2 system, reading R5 replaces it by
its gamma-free form and counts the nodes).

A decaying Taylor-Green vortex at gamma = 0.2 whose peak speed (0.12) lies
beyond the threshold where the system degenerates: the guard fires at up to
192 nodes in the first steps and at none once viscosity has slowed the flow
(the oracle counts 192, 128, 112, 48, 32 at steps 10 ... 50 with these
parameters).  The run stays smooth and finite.  FP64 on both sides: guard
decisions are taken in the same precision, so the counts must be equal at
every check step, and the fields agree to rounding-order differences.
"""
import sys

import numpy as np
import pytest

import oracle
from workloads import periodic_sides

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


@pytest.mark.parametrize("n,launch", [(32, None), (96, (4, 2))])
def test_guard_counts_and_fields_match_oracle(lbm, n, launch):
    U0, gamma, nu = 0.12, 0.2, 0.01
    _say(f"guard Taylor-Green {n}x{n} f64 U0 {U0} gamma {gamma} nu {nu} launch {launch}")
    x = (np.arange(n) + 0.5) * 2 * np.pi / n
    X, Y = np.meshgrid(x, x)
    # the 32^2 vortex's shape on a larger lattice: four periods across
    m = n // 32
    init = (np.ones((n, n)), U0 * np.sin(m * X) * np.cos(m * Y),
            -U0 * np.cos(m * X) * np.sin(m * Y))
    o = oracle.Oracle(n, n, periodic_sides(), nu=nu, gamma=gamma)
    g = lbm.Lattice(n, n, periodic_sides(), storage="f64", check_every=10, nu=nu, gamma=gamma)
    if launch:
        g.set_launch(*launch)
    o.init_fields(*init)
    g.init_fields(*init)
    counts_o, counts_g = [], []
    for _ in range(8):
        o.step(10)
        g.step(10)
        counts_o.append(o.guard_count)
        counts_g.append(g.guard_count)
    _say("guard counts oracle", counts_o, "gpu", counts_g)
    assert counts_o[0] > 0 and counts_o[-1] == 0
    assert counts_g == counts_o
    _, uxo, uyo = o.fields()
    _, uxg, uyg = g.fields()
    err = max(np.abs(uxg - uxo).max(), np.abs(uyg - uyo).max()) / U0
    _say("max|du|/U0 =", err)
    assert err < 1e-11
    fo, fg = o.get_f(), g.populations()
    assert np.abs(fo - fg).max() < 1e-11
