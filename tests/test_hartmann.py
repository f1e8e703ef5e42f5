"""Hartmann flow (Sec. 6) on the oracle: a spatially varying body force.

The effective force F_x(z) = F_b + B0 dB_x/dz = F_b Ha cosh(Ha z/L) / sinh(Ha)
across a channel of half width L drives the closed-form profile
u(z) = F_b L^2 / (Ha nu) coth(Ha) [1 - cosh(Ha z/L) / cosh(Ha)]
(the paper's sqrt(eta/nu) form with eta = B0^2 L^2 / (Ha^2 nu)).  The closed
form is pinned to the ODE nu u'' + F_x = 0 with u(+-L) = 0 and to the
Poiseuille parabola as Ha -> 0; the oracle is pinned to the closed form with
second-order convergence under grid refinement (half-way bounce-back walls).
"""
import math

import numpy as np
import pytest

import oracle
from workloads import hartmann_force, poiseuille_sides


def hartmann_profile(z, L, f_b, ha, nu):
    return f_b * L * L / (ha * nu) / math.tanh(ha) * (1 - np.cosh(ha * z / L) / math.cosh(ha))


def test_closed_form_solves_the_momentum_balance():
    L, f_b, ha, nu = 1.0, 2e-3, 6.0, 0.05
    z = np.linspace(-L, L, 4001)
    h = z[1] - z[0]
    u = hartmann_profile(z, L, f_b, ha, nu)
    upp = (u[2:] - 2 * u[1:-1] + u[:-2]) / (h * h)
    force = f_b * ha * np.cosh(ha * z[1:-1] / L) / math.sinh(ha)
    assert np.abs(nu * upp + force).max() < 1e-5 * force.max()
    assert abs(u[0]) < 1e-15 and abs(u[-1]) < 1e-15


def test_closed_form_tends_to_poiseuille():
    L, f_b, nu = 3.0, 1e-3, 0.1
    z = np.linspace(-L, L, 101)
    u = hartmann_profile(z, L, f_b, 1e-4, nu)
    parabola = f_b * (L * L - z * z) / (2 * nu)
    assert np.abs(u - parabola).max() < 1e-7 * parabola.max()
    fx, _ = hartmann_force(4, 16, f_b, 1e-6)
    assert np.allclose(fx, f_b, rtol=1e-9)


def _steady(ny, ha, gamma=0.1, nu=0.02, umax=0.0115):
    L = ny / 2.0
    # F_b from the requested centre-line speed
    f_b = umax * ha * nu * math.tanh(ha) / (L * L * (1 - 1 / math.cosh(ha)))
    fx, fy = hartmann_force(4, ny, f_b, ha)
    o = oracle.Oracle(4, ny, poiseuille_sides(), nu=nu, gamma=gamma)
    o.set_force_field(fx, fy)
    while o.steps < 400000:
        o.step(1000)
        if o.residual < 1e-13:
            break
    else:
        raise RuntimeError("no steady state")
    z = np.arange(ny) + 0.5 - L
    ua = hartmann_profile(z, L, f_b, ha, nu)
    u = o.fields()[1][:, 1]
    return math.sqrt(((u - ua) ** 2).sum() / (ua ** 2).sum())


@pytest.mark.parametrize("ha,bound", [(2.0, 1e-3), (10.0, 1e-2)])
def test_oracle_hartmann_second_order(ha, bound):
    """gamma = 0.1 and a centre-line speed of Mach 0.02 (in units of the
    lattice sound speed), as in the paper's Hartmann runs."""
    e32, e64 = _steady(32, ha), _steady(64, ha)
    assert e64 < bound
    assert 3.5 < e32 / e64 < 4.5
