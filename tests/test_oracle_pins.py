"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

None of these tests compares the oracle with itself.  Each one checks the
oracle's output against an independent statement: a printed equation of the
paper evaluated separately, a closed-form solution, a conservation law, or a
brute-force construction (a 9x9 central-moment matrix inverted numerically).
"""
import math

import numpy as np
import pytest

import oracle
from workloads import (SplitMix64, cavity_sides, channel_sides, diagonal_shear_wave,
                       periodic_sides, poiseuille_sides, axis_shear_wave)

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
# exponents (m, n) of the nine moments ex^m ey^n, in the order of eq. 5
BASIS = [(0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1), (2, 1), (1, 2), (2, 2)]


def raw_matrix():
    return np.array([[EX[a] ** m * EY[a] ** n for a in range(9)] for (m, n) in BASIS])


def central_matrix(ux, uy):
    return np.array([[(EX[a] - ux) ** m * (EY[a] - uy) ** n for a in range(9)]
                     for (m, n) in BASIS])


def printed_raw_equilibrium(rho, ux, uy, gamma):
    """Preconditioned raw moment equilibria as printed in Sec. 3 (orders <= 3;
    the fourth order is filled from the printed expression too, it does not
    enter any central moment of order <= 3)."""
    return np.array([
        rho, rho * ux, rho * uy,
        rho / 3 + rho * ux ** 2 / gamma,
        rho / 3 + rho * uy ** 2 / gamma,
        rho * ux * uy / gamma,
        rho * uy / 3 + rho * ux ** 2 * uy / gamma ** 2,
        rho * ux / 3 + rho * ux * uy ** 2 / gamma ** 2,
        rho / 9 + rho * (ux ** 2 + uy ** 2) / 3 + rho * ux ** 2 * uy ** 2,
    ])


def printed_source_moments(fx, fy, ux, uy, gamma):
    """Source raw moments sigma' as printed in Sec. 3."""
    return np.array([
        0.0, fx / gamma, fy / gamma,
        2 * fx * ux / gamma ** 2, 2 * fy * uy / gamma ** 2, (fx * uy + fy * ux) / gamma ** 2,
        fy * ux ** 2 + 2 * fx * ux * uy, fx * uy ** 2 + 2 * fy * uy * ux,
        2 * (fx * ux * uy ** 2 + fy * uy * ux ** 2),
    ])


def defect_terms(rho, ux, uy, dxux, dyuy, drx, dry, w3, w4, w5, gamma):
    """Non-GI defect terms E_grho^j + E_gu^j, eqs. 26-28, as printed."""
    A = 4 / gamma ** 2 - 1 / gamma
    B = 1 / gamma ** 2 - 1 / gamma
    C = 1 / gamma - 1
    E3 = (2 / (3 * w3)) * C * (ux * drx + uy * dry) + \
        (rho / w3) * ((A * ux ** 2 + B * uy ** 2) * dxux + (A * uy ** 2 + B * ux ** 2) * dyuy)
    E4 = (2 / (3 * w4)) * C * (ux * drx - uy * dry) + \
        (rho / w4) * ((A * ux ** 2 - B * uy ** 2) * dxux + (-A * uy ** 2 + B * ux ** 2) * dyuy)
    E5 = (1 / (3 * w5)) * C * (ux * dry + uy * drx) + \
        (rho / w5) * B * ux * uy * (dxux + dyuy)
    return E3, E4, E5


def random_state(rng, amp=0.05, u=(0.04, -0.03)):
    """Populations near a moving equilibrium with random non-equilibrium parts."""
    rho = 1.0 + 0.02 * (rng.uniform() - 0.5)
    feq = oracle.equilibrium(rho, u[0], u[1], 1.0)
    return feq * (1.0 + amp * (rng.uniform_array(9) - 0.5))


# ---------------------------------------------------------------------------
# Lattice algebra
# ---------------------------------------------------------------------------

def test_moment_map_is_inverse_of_raw_moments(oracle_lib):
    rng = SplitMix64(1)
    T = raw_matrix()
    for _ in range(20):
        f = rng.uniform_array(9, -1, 1)
        m = oracle.raw_moments(f)
        np.testing.assert_allclose(m, T @ f, atol=1e-14)
        np.testing.assert_allclose(oracle.moments_to_pop(m), f, atol=1e-14)
        m2 = rng.uniform_array(9, -1, 1)
        np.testing.assert_allclose(T @ oracle.moments_to_pop(m2), m2, atol=1e-14)


@pytest.mark.parametrize("gamma", [1.0, 0.5, 0.2, 0.05])
def test_equilibrium_matches_printed_raw_equilibria(oracle_lib, gamma):
    """Orders <= 3 equal the printed raw equilibria (incl. the gamma^2 boxed
    cubic terms); the central fourth-order moment is rho/9 (Sec. 5 kernel)."""
    rho, ux, uy = 1.013, 0.031, -0.022
    f = oracle.equilibrium(rho, ux, uy, gamma)
    m = raw_matrix() @ f
    np.testing.assert_allclose(m[:8], printed_raw_equilibrium(rho, ux, uy, gamma)[:8],
                               rtol=1e-13, atol=1e-16)
    c = central_matrix(ux, uy) @ f
    assert abs(c[8] - rho / 9) < 1e-15
    # rest state is w * rho
    np.testing.assert_allclose(oracle.equilibrium(1.0, 0, 0, gamma), W, atol=1e-16)


# ---------------------------------------------------------------------------
# Collision
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("gamma,force", [(1.0, False), (0.5, False), (0.2, True), (0.7, True)])
def test_collision_conserves_mass_and_momentum(oracle_lib, gamma, force):
    rng = SplitMix64(7)
    fx, fy = (1e-4, -2e-4) if force else (0.0, 0.0)
    for _ in range(10):
        fb = random_state(rng)
        fo, d = oracle.collide(fb, 0.003, -0.002, nu=0.05, gamma=gamma, fx=fx, fy=fy,
                               omega3=1.3, omega6=0.9, omega7=1.1, omega8=1.2)
        assert abs(fo.sum() - fb.sum()) < 1e-15
        # momentum changes by the source's first moment F/gamma only
        assert abs((EX * fo).sum() - (EX * fb).sum() - fx / gamma) < 1e-15
        assert abs((EY * fo).sum() - (EY * fb).sum() - fy / gamma) < 1e-15


@pytest.mark.parametrize("gi", [0, 1])
@pytest.mark.parametrize("gamma,force", [(1.0, False), (0.5, False), (0.3, True), (0.1, False)])
def test_collision_is_central_moment_relaxation(oracle_lib, gi, gamma, force):
    """Brute force: relax the central moments of f = fbar + S/2 about u toward
    their equilibria (+ the extended-equilibrium corrections when GI is on),
    invert the 9x9 central-moment matrix numerically, add S/2, and compare
    with the cascaded kernel.  Central equilibria of orders <= 3 come from the
    printed raw equilibria (GI kernel) or are zero at third order (eq. 4);
    the fourth-order target is rho/9."""
    rng = SplitMix64(11 + gi)
    w3, w6, w7, w8 = 1.3, 0.9, 1.1, 1.2
    nu = 0.04
    w4 = w5 = oracle.omega_from_nu(nu, gamma)
    fx, fy = (2e-5, -1e-5) if force else (0.0, 0.0)
    for _ in range(8):
        fb = random_state(rng, amp=0.03)
        drx, dry = 2e-3 * (rng.uniform() - 0.5), 2e-3 * (rng.uniform() - 0.5)
        fo, d = oracle.collide(fb, drx, dry, nu=nu, gamma=gamma, fx=fx, fy=fy, omega3=w3,
                               omega6=w6, omega7=w7, omega8=w8, gi_correct=gi)
        assert d["guarded"] == 0
        T = raw_matrix()
        rho = fb.sum()
        ux = ((EX * fb).sum() + fx / (2 * gamma)) / rho
        uy = ((EY * fb).sum() + fy / (2 * gamma)) / rho
        S = np.linalg.solve(T, printed_source_moments(fx, fy, ux, uy, gamma))
        f = fb + 0.5 * S
        M = central_matrix(ux, uy)
        c = M @ f
        assert abs(c[1]) < 1e-14 and abs(c[2]) < 1e-14
        ceq = M @ np.linalg.solve(T, printed_raw_equilibrium(rho, ux, uy, gamma))
        if not gi:
            ceq[6] = ceq[7] = 0.0
        ceq[8] = rho / 9
        if gi:
            E3, E4, E5 = defect_terms(rho, ux, uy, d["dxux"], d["dyuy"], drx, dry, w3, w4, w5,
                                      gamma)
            # constraint eq. 44: m^eq(1) = -(1 - w/2) (E_grho + E_gu)
            D3, D4, D5 = -(1 - w3 / 2) * E3, -(1 - w4 / 2) * E4, -(1 - w5 / 2) * E5
        else:
            D3 = D4 = D5 = 0.0
        s_c, d_c = c[3] + c[4], c[3] - c[4]
        s_e, d_e = ceq[3] + ceq[4], ceq[3] - ceq[4]
        s_n = s_c + w3 * (s_e + D3 - s_c)
        d_n = d_c + w4 * (d_e + D4 - d_c)
        cn = c.copy()
        cn[3], cn[4] = 0.5 * (s_n + d_n), 0.5 * (s_n - d_n)
        cn[5] = c[5] + w5 * (ceq[5] + D5 - c[5])
        cn[6] = c[6] + w6 * (ceq[6] - c[6])
        cn[7] = c[7] + w7 * (ceq[7] - c[7])
        cn[8] = c[8] + w8 * (ceq[8] - c[8])
        expect = np.linalg.solve(M, cn) + 0.5 * S
        np.testing.assert_allclose(fo, expect, rtol=0, atol=2e-15)


@pytest.mark.parametrize("gamma", [1.0, 0.5, 0.2])
def test_equilibrium_is_fixed_point(oracle_lib, gamma):
    for (rho, ux, uy) in [(1.0, 0.0, 0.0), (1.02, 0.05, -0.03), (0.97, -0.02, 0.04)]:
        feq = oracle.equilibrium(rho, ux, uy, gamma)
        fo, d = oracle.collide(feq, 0.0, 0.0, nu=0.03, gamma=gamma, omega3=1.4)
        np.testing.assert_allclose(fo, feq, atol=2e-16)
        assert abs(d["dxux"]) < 1e-14 and abs(d["dyuy"]) < 1e-14


def _raw_basis():
    """Rows of the non-orthogonal moment basis of eq. 5."""
    return np.array([np.ones(9), EX, EY, EX ** 2 + EY ** 2, EX ** 2 - EY ** 2, EX * EY,
                     EX ** 2 * EY, EX * EY ** 2, EX ** 2 * EY ** 2], dtype=np.float64)


@pytest.mark.parametrize("gamma,force", [(1.0, False), (0.5, True), (0.2, False)])
def test_mrt_form_is_raw_moment_relaxation(oracle_lib, gamma, force):
    """Brute force for the raw-moment MRT form (eq. 7, uncorrected so that no
    correction is retyped here): raw moments of f = fbar + S/2 in the basis
    of eq. 5 relax towards the printed raw equilibria of Sec. 3 with the
    rates (0, 0, 0, w3, w4, w5, w6, w7, w8); the populations follow by a
    numerical inverse of the basis, plus the source S."""
    T = _raw_basis()
    Ti = np.linalg.inv(T)
    rng = SplitMix64(21)
    fx, fy = (2e-4, -1e-4) if force else (0.0, 0.0)
    nu, w3, w6, w7, w8 = 0.04, 1.3, 0.9, 1.1, 1.2
    w4 = oracle.omega_from_nu(nu, gamma)
    for _ in range(8):
        fb = random_state(rng)
        fo, d = oracle.collide(fb, 0.0, 0.0, nu=nu, gamma=gamma, fx=fx, fy=fy, omega3=w3,
                               omega6=w6, omega7=w7, omega8=w8, gi_correct=0, mrt=1)
        rho = fb.sum()
        ux = ((EX * fb).sum() + 0.5 * fx / gamma) / rho
        uy = ((EY * fb).sum() + 0.5 * fy / gamma) / rho
        # source: raw moments of S listed in Sec. 3, mapped by the numerical inverse
        sk = np.array([0.0, fx / gamma, fy / gamma,
                       (2 * fx * ux + 2 * fy * uy) / gamma ** 2,
                       (2 * fx * ux - 2 * fy * uy) / gamma ** 2, (fx * uy + fy * ux) / gamma ** 2,
                       fy * ux * ux + 2 * fx * ux * uy, fx * uy * uy + 2 * fy * uy * ux,
                       2 * (fx * ux * uy * uy + fy * uy * ux * ux)])
        S = Ti @ sk
        m = T @ (fb + 0.5 * S)
        eq = np.array([rho, rho * ux, rho * uy,
                       2 * rho / 3 + rho * (ux * ux + uy * uy) / gamma,
                       rho * (ux * ux - uy * uy) / gamma, rho * ux * uy / gamma,
                       rho * uy / 3 + rho * ux * ux * uy / gamma ** 2,
                       rho * ux / 3 + rho * ux * uy * uy / gamma ** 2,
                       rho / 9 + rho * (ux * ux + uy * uy) / 3 + rho * ux * ux * uy * uy])
        lam = np.array([0, 0, 0, w3, w4, w4, w6, w7, w8])
        ref = fb + Ti @ (-lam * (m - eq)) + S
        np.testing.assert_allclose(fo, ref, rtol=0, atol=2e-15)


@pytest.mark.parametrize("gamma", [1.0, 0.4])
def test_mrt_form_conserves_and_keeps_printed_equilibrium(oracle_lib, gamma):
    T = _raw_basis()
    rng = SplitMix64(8)
    for _ in range(6):
        fb = random_state(rng)
        fo, _ = oracle.collide(fb, 0.002, -0.001, nu=0.05, gamma=gamma, fx=1e-4, fy=2e-4,
                               mrt=1)
        assert abs(fo.sum() - fb.sum()) < 1e-15
        assert abs((EX * fo).sum() - (EX * fb).sum() - 1e-4 / gamma) < 1e-15
        assert abs((EY * fo).sum() - (EY * fb).sum() - 2e-4 / gamma) < 1e-15
    for (rho, ux, uy) in [(1.0, 0.0, 0.0), (1.03, 0.04, -0.02)]:
        eq = np.array([rho, rho * ux, rho * uy,
                       2 * rho / 3 + rho * (ux * ux + uy * uy) / gamma,
                       rho * (ux * ux - uy * uy) / gamma, rho * ux * uy / gamma,
                       rho * uy / 3 + rho * ux * ux * uy / gamma ** 2,
                       rho * ux / 3 + rho * ux * uy * uy / gamma ** 2,
                       rho / 9 + rho * (ux * ux + uy * uy) / 3 + rho * ux * ux * uy * uy])
        feq = np.linalg.solve(T, eq)
        fo, d = oracle.collide(feq, 0.0, 0.0, nu=0.03, gamma=gamma, omega3=1.4, mrt=1)
        np.testing.assert_allclose(fo, feq, atol=3e-16)


def test_shear_wave_decay_is_galilean_invariant_mrt(oracle_lib):
    """The GI property for the raw-moment MRT form with the same extended
    equilibria (Sec. 5 notes that such a scheme follows from the analysis)."""
    n, m, steps, gamma = 64, 1, 2000, 0.5
    rc = [_diag_wave_rate(n, m, steps, gamma, u, 1, mrt=1) for u in (0.0, 0.05, 0.1)]
    ru = [_diag_wave_rate(n, m, steps, gamma, u, 0, mrt=1) for u in (0.0, 0.1)]
    exact = rc[0][1]
    corr = [r for r, _ in rc]
    spread_c = (max(corr) - min(corr)) / exact
    spread_u = abs(ru[1][0] - ru[0][0]) / exact
    assert abs(corr[0] - exact) / exact < 2e-3
    assert spread_c < 1e-3
    assert spread_u > 0.05


@pytest.mark.parametrize("gamma", [1.0, 0.3])
def test_uniform_flow_stays_uniform(oracle_lib, gamma):
    o = oracle.Oracle(12, 10, periodic_sides(), nu=0.05, gamma=gamma)
    o.init_fields(np.full((10, 12), 1.01), np.full((10, 12), 0.04), np.full((10, 12), -0.02))
    f0 = o.get_f()
    o.step(25)
    np.testing.assert_allclose(o.get_f(), f0, atol=1e-15)
    r, ux, uy = o.fields()
    assert np.abs(ux - 0.04).max() < 1e-14 and np.abs(uy + 0.02).max() < 1e-14


# ---------------------------------------------------------------------------
# GI corrections and the strain-rate estimator
# ---------------------------------------------------------------------------

def test_gamma_one_reduces_to_standard_gi_form(oracle_lib):
    """At gamma = 1: Delta3 = -3 h3 rho (ux^2 dxux + uy^2 dyuy), Delta4 =
    -3 h4 rho (ux^2 dxux - uy^2 dyuy), Delta5 = 0 (the gamma = 1 limit stated
    after eq. 47); with the corrections removed the kernel is eq. 4."""
    rng = SplitMix64(3)
    w3, nu = 1.2, 0.03
    w4 = oracle.omega_from_nu(nu, 1.0)
    h3, h4 = 1 / w3 - 0.5, 1 / w4 - 0.5
    for _ in range(5):
        fb = random_state(rng)
        fo, d = oracle.collide(fb, 1e-3, 2e-3, nu=nu, gamma=1.0, omega3=w3)
        f0, d0 = oracle.collide(fb, 1e-3, 2e-3, nu=nu, gamma=1.0, omega3=w3, gi_correct=0)
        rho, ux, uy, X, Y = d["rho"], d["ux"], d["uy"], d["dxux"], d["dyuy"]
        D3 = -3 * h3 * rho * (ux ** 2 * X + uy ** 2 * Y)
        D4 = -3 * h4 * rho * (ux ** 2 * X - uy ** 2 * Y)
        # the difference of the two kernels is K3 g3 + K4 g4 + cascade terms; compare
        # the post-collision second-order raw moments, which see only w*Delta
        T = raw_matrix()
        mo, m0 = T @ fo, T @ f0
        assert abs((mo[3] + mo[4]) - (m0[3] + m0[4]) - w3 * D3) < 1e-15
        assert abs((mo[3] - mo[4]) - (m0[3] - m0[4]) - w4 * D4) < 1e-15
        assert abs(mo[5] - m0[5]) < 1e-16


@pytest.mark.parametrize("gamma", [1.0, 0.5, 0.2])
def test_strain_estimator_satisfies_chapman_enskog_relations(oracle_lib, gamma):
    """The estimated strains must satisfy eq. 39 and eq. 40 with the
    constraint eq. 44: m3 = -2rho/(3w3)(X+Y) + (w3/2)(E_grho^3+E_gu^3) and
    m4 = -2rho/(3w4)(X-Y) + (w4/2)(E_grho^4+E_gu^4), with E from eqs. 26-27
    (this is what the printed eq. 55b fails: it flips the sign of Y at u=0)."""
    rng = SplitMix64(5)
    w3 = 1.1
    w4 = oracle.omega_from_nu(0.03, gamma)
    for _ in range(10):
        rho = 1 + 0.01 * rng.uniform()
        ux, uy = 0.03 * rng.uniform(-1, 1), 0.03 * rng.uniform(-1, 1)
        m3, m4 = 1e-3 * rng.uniform(-1, 1), 1e-3 * rng.uniform(-1, 1)
        drx, dry = 1e-3 * rng.uniform(-1, 1), 1e-3 * rng.uniform(-1, 1)
        X, Y, g = oracle.strain(rho, ux, uy, m3, m4, drx, dry, w3, w4, gamma)
        assert not g
        E3, E4, _ = defect_terms(rho, ux, uy, X, Y, drx, dry, w3, w4, w4, gamma)
        assert abs(m3 - (-2 * rho / (3 * w3) * (X + Y) + 0.5 * w3 * E3)) < 1e-16
        assert abs(m4 - (-2 * rho / (3 * w4) * (X - Y) + 0.5 * w4 * E4)) < 1e-16


def test_strain_estimator_zero_velocity_limit(oracle_lib):
    w3, w4 = 1.3, 0.8
    for (m3, m4) in [(1e-3, 0.0), (0.0, 1e-3), (2e-3, -5e-4)]:
        X, Y, _ = oracle.strain(1.0, 0.0, 0.0, m3, m4, 0.0, 0.0, w3, w4, 1.0)
        assert abs(X - (-0.75 * (w3 * m3 + w4 * m4))) < 1e-17
        assert abs(Y - (-0.75 * (w3 * m3 - w4 * m4))) < 1e-17


def test_strain_guard_on_singular_system(oracle_lib):
    # gamma = 0.05: A = 380; |u| = 0.04 makes c1 change sign for w3 = 1
    X, Y, g = oracle.strain(1.0, 0.04, 0.0, 1e-4, 1e-4, 0.0, 0.0, 1.0, 0.5, 0.05)
    assert g
    Xr, Yr, _ = oracle.strain(1.0, 0.0, 0.0, 1e-4, 1e-4, 0.0, 0.0, 1.0, 0.5, 1.0)
    assert abs(X - Xr) < 1e-16 and abs(Y - Yr) < 1e-16


@pytest.mark.parametrize("gamma", [1.0, 0.5])
def test_strain_estimator_matches_finite_differences(oracle_lib, gamma):
    """In a decaying Taylor-Green flow on a background velocity, the locally
    estimated dxux, dyuy agree with central differences of u to a few %."""
    n = 64
    U0, Ub = 0.01, 0.03
    x = (np.arange(n) + 0.5) * 2 * np.pi / n
    X, Y = np.meshgrid(x, x)
    ux = Ub + U0 * np.sin(X) * np.cos(Y)
    uy = -U0 * np.cos(X) * np.sin(Y)
    nu = 0.02 * gamma
    o = oracle.Oracle(n, n, periodic_sides(), nu=nu, gamma=gamma)
    o.init_fields(np.ones((n, n)), ux, uy)
    o.step(200)
    f = o.get_f()
    fb = np.stack([np.roll(np.roll(f[a], int(EY[a]), axis=0), int(EX[a]), axis=1)
                   for a in range(9)])
    rho = fb.sum(0)
    u = (EX[:, None, None] * fb).sum(0) / rho
    v = (EY[:, None, None] * fb).sum(0) / rho
    dudx = (np.roll(u, -1, 1) - np.roll(u, 1, 1)) / 2
    dvdy = (np.roll(v, -1, 0) - np.roll(v, 1, 0)) / 2
    errs = []
    scale = np.abs(dudx).max()
    for (j, i) in [(5, 7), (20, 40), (33, 12), (50, 50), (10, 60)]:
        gx = 3 * sum(W[a] * EX[a] * rho[(j + int(EY[a])) % n, (i + int(EX[a])) % n]
                      for a in range(1, 9))
        gy = 3 * sum(W[a] * EY[a] * rho[(j + int(EY[a])) % n, (i + int(EX[a])) % n]
                      for a in range(1, 9))
        _, d = oracle.collide(fb[:, j, i], gx, gy, nu=nu, gamma=gamma)
        errs.append(abs(d["dxux"] - dudx[j, i]) / scale)
        errs.append(abs(d["dyuy"] - dvdy[j, i]) / scale)
    assert max(errs) < 0.03, errs


# ---------------------------------------------------------------------------
# The GI property: shear-wave decay independent of the background velocity
# ---------------------------------------------------------------------------

def _diag_wave_rate(n, m, steps, gamma, ux0, gi, strain_fd=0, mrt=0):
    nu_ratio = 0.05       # nu/gamma = (1/w - 1/2)/3
    o = oracle.Oracle(n, n, periodic_sides(), nu=nu_ratio * gamma, gamma=gamma,
                      gi_correct=gi, strain_fd=strain_fd, mrt=mrt)
    o.init_fields(*diagonal_shear_wave(n, 1e-3, m, ux0))
    k = 2 * math.pi * m / n
    x = np.arange(n) + 0.5
    Xg, Yg = np.meshgrid(x, x)
    ph = np.exp(-1j * k * (Xg + Yg))
    ts, la = [], []
    for _ in range(steps // 50):
        o.step(50)
        _, ux, uy = o.fields()
        ts.append(o.steps)
        la.append(math.log(abs((((ux - uy) / math.sqrt(2)) * ph).mean())))
    ts, la = np.array(ts), np.array(la)
    sel = ts >= 200
    rate = -np.polyfit(ts[sel], la[sel], 1)[0]
    return rate, nu_ratio * 2 * k * k


@pytest.mark.parametrize("gamma", [1.0, 0.5])
def test_shear_wave_decay_is_galilean_invariant(oracle_lib, gamma):
    """Diagonal shear wave (dxux = -dyuy != 0) on a background Ux: the decay
    rate of the corrected scheme does not depend on Ux and equals
    (nu/gamma) |k|^2 (eqs. 48-49); the uncorrected eq. 4 scheme shifts by
    O(Ux^2/gamma^2) (defects of eqs. 26-27)."""
    n, m, steps = 64, 1, 2000
    rc = [_diag_wave_rate(n, m, steps, gamma, u, 1) for u in (0.0, 0.05, 0.1)]
    ru = [_diag_wave_rate(n, m, steps, gamma, u, 0) for u in (0.0, 0.05, 0.1)]
    exact = rc[0][1]
    corr = [r for r, _ in rc]
    unc = [r for r, _ in ru]
    spread_c = (max(corr) - min(corr)) / exact
    spread_u = (max(unc) - min(unc)) / exact
    assert abs(corr[0] - exact) / exact < 2e-3
    assert spread_c < 2e-3
    assert spread_u > 10 * spread_c
    assert spread_u > (0.02 if gamma == 1.0 else 0.05)


def test_shear_wave_decay_is_galilean_invariant_with_fd_strain(oracle_lib):
    """The same GI property with the strain rates of the corrections taken
    from finite differences of the velocity (the alternative of Sec. 5)."""
    n, m, steps, gamma = 64, 1, 2000, 0.5
    rc = [_diag_wave_rate(n, m, steps, gamma, u, 1, strain_fd=1) for u in (0.0, 0.05, 0.1)]
    ru = [_diag_wave_rate(n, m, steps, gamma, u, 0) for u in (0.0, 0.1)]
    exact = rc[0][1]
    corr = [r for r, _ in rc]
    spread_c = (max(corr) - min(corr)) / exact
    spread_u = abs(ru[1][0] - ru[0][0]) / exact
    assert abs(corr[0] - exact) / exact < 2e-3
    assert spread_c < 3e-3
    assert spread_u > 10 * spread_c


def test_residual_is_the_one_step_relative_change(oracle_lib):
    """The steady-state residual r = ||u^{n+1} - u^n|| / ||u^n|| (the paper
    plots it without a definition): for a single decaying shear mode at rest,
    u^n = a^n u^0 after the transient, so r = 1 - a with a the per-step decay
    factor, measured here from the fields 200 steps apart."""
    n, gamma = 32, 0.5
    o = oracle.Oracle(n, n, periodic_sides(), nu=0.05 * gamma, gamma=gamma)
    o.init_fields(*axis_shear_wave(n, 1e-3, 1, 0.0))
    o.step(400)
    u0 = o.fields()[2]
    o.step(200)
    u1 = o.fields()[2]
    a = (math.sqrt((u1 ** 2).sum() / (u0 ** 2).sum())) ** (1.0 / 200)
    assert abs(o.residual - (1.0 - a)) < 1e-6 * (1.0 - a)


def test_axis_shear_wave_control(oracle_lib):
    """Axis-aligned wave (no diagonal strain): both schemes decay at
    (nu/gamma) k^2 regardless of Ux."""
    n, gamma = 64, 0.5
    k = 2 * math.pi / n
    for gi in (0, 1):
        rates = []
        for ux0 in (0.0, 0.1):
            o = oracle.Oracle(n, n, periodic_sides(), nu=0.05 * gamma, gamma=gamma, gi_correct=gi)
            o.init_fields(*axis_shear_wave(n, 1e-3, 1, ux0))
            x = np.arange(n) + 0.5
            ph = np.exp(-1j * k * x)[None, :]
            ts, la = [], []
            for _ in range(30):
                o.step(50)
                ts.append(o.steps)
                la.append(math.log(abs((o.fields()[2] * ph).mean())))
            ts, la = np.array(ts), np.array(la)
            rates.append(-np.polyfit(ts[4:], la[4:], 1)[0])
        assert abs(rates[0] - 0.05 * k * k) / (0.05 * k * k) < 3e-3
        assert abs(rates[1] - rates[0]) / rates[0] < 5e-3


# ---------------------------------------------------------------------------
# Boundaries and macroscopic closed forms
# ---------------------------------------------------------------------------

def _poiseuille(H, gamma, nu=0.1, fx=1e-6, steps=None):
    o = oracle.Oracle(4, H, poiseuille_sides(), nu=nu, gamma=gamma, fx=fx)
    steps = steps or int(8 * H * H / nu)
    o.step(steps)
    _, ux, _ = o.fields()
    y = np.arange(H) + 0.5
    exact = fx * y * (H - y) / (2 * nu)
    return ux[:, 2], exact


def test_poiseuille_closed_form_and_second_order(oracle_lib):
    errs = []
    for H in (8, 16, 32):
        u, ex = _poiseuille(H, 0.5)
        errs.append(np.abs(u - ex).max() / ex.max())
    assert errs[-1] < 5e-3
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


def test_poiseuille_independent_of_gamma(oracle_lib):
    u1, ex = _poiseuille(16, 1.0)
    u2, _ = _poiseuille(16, 0.3)
    assert np.abs(u1 - u2).max() / ex.max() < 2e-2
    assert np.abs(u2 - ex).max() / ex.max() < 2e-2


def test_cavity_conserves_mass(oracle_lib):
    o = oracle.Oracle(24, 20, cavity_sides(), nu=0.02, gamma=0.5, u_lid=0.1)
    o.step(1)
    m1 = o.mass
    o.step(500)
    assert abs(o.mass - 24 * 20) < 1e-10
    assert abs(o.mass - m1) < 1e-10


def test_lid_momentum_sign(oracle_lib):
    """The lid drags the fluid below it in +x."""
    o = oracle.Oracle(16, 16, cavity_sides(), nu=0.05, gamma=1.0, u_lid=0.1)
    o.step(300)
    _, ux, _ = o.fields()
    assert ux[-1, 8] > 0.03 and ux[-1, 8] < 0.1


def test_inlet_outlet_channel_keeps_parabola(oracle_lib):
    """Obstacle-free channel with a parabolic inlet and convective outlet
    settles to the inflow parabola everywhere (up to the wall slip error)."""
    nx, ny, U = 48, 12, 0.05
    o = oracle.Oracle(nx, ny, channel_sides(), nu=0.1, gamma=1.0, u_in_max=U)
    o.step(8000)
    assert o.residual < 1e-11          # converges: the outlet pins the density level
    rho, ux, uy = o.fields()
    y = np.arange(ny) + 0.5
    ex = 4 * U * y * (ny - y) / ny ** 2
    j = rho * ux
    for i in (nx // 4, nx // 2, nx - 2, nx - 1):
        # away from the inlet corners the mass flux rho*u carries the inflow
        # parabola (u itself varies with the density along the pressure drop)
        assert np.abs(j[:, i] - ex).max() / U < 1e-2
    flux = j.sum(axis=0)
    assert np.abs(flux - flux.mean()).max() / flux.mean() < 1e-9   # steady mass balance
    assert np.abs(uy[:, nx // 4:]).max() / U < 5e-3
    assert abs(rho[:, -1].mean() - 1.0) < 0.01    # outlet density held at rho0


def test_unstable_case_is_reported(oracle_lib):
    """U/gamma well above the lattice speed: the run diverges and the oracle
    reports it instead of returning garbage."""
    o = oracle.Oracle(32, 32, cavity_sides(), nu=0.0032, gamma=0.05, u_lid=0.1)
    with pytest.raises(FloatingPointError):
        for _ in range(50):
            o.step(100)


def test_rejects_invalid_configuration(oracle_lib):
    with pytest.raises(ValueError):
        oracle.Oracle(8, 8, (0, 1, 1, 1), nu=0.1, gamma=1.0)   # W periodic, E wall
    with pytest.raises(ValueError):
        oracle.Oracle(8, 8, cavity_sides(), nu=-0.1, gamma=1.0)
    m = np.zeros((8, 8), dtype=np.uint8)
    m[4, 7] = 1
    with pytest.raises(ValueError):
        oracle.Oracle(8, 8, channel_sides(), solid=m, nu=0.1, gamma=1.0)  # solid at outlet
    with pytest.raises(ValueError):
        oracle.Oracle(8, 8, cavity_sides(), solid=np.ones((8, 8), np.uint8), nu=0.1, gamma=1.0)
