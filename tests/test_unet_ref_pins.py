"""Pins of the NumPy FP64 U-Net reference against library routines,
adjoint identities and finite differences (CPU only)."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import unet_ref as U
from workloads import SplitMix64


def rnd(rng, *shape):
    return rng.standard_normal(shape)


def test_bf16_rounding_ties_to_even():
    one = 1.0
    assert U.bf16(np.array([one]))[0] == 1.0
    assert U.bf16(np.array([1 + 2 ** -8]))[0] == 1.0                 # tie -> even
    assert U.bf16(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6      # tie -> even (up)
    assert U.bf16(np.array([1 + 2 ** -8 + 2 ** -12]))[0] == 1 + 2 ** -7
    assert U.bf16(np.array([-2.5]))[0] == -2.5


def test_conv_matches_library_correlation():
    """Single channel pair: the 3x3 'same' cross-correlation of SciPy."""
    rng = np.random.default_rng(1)
    x = rnd(rng, 1, 9, 7, 1)
    w = rnd(rng, 1, 9, 1)
    k = w[0, :, 0].reshape(3, 3)
    ref = correlate2d(x[0, :, :, 0], k, mode="same", boundary="fill")
    np.testing.assert_allclose(U.conv3x3(x, w)[0, :, :, 0], ref, rtol=1e-13, atol=1e-13)


def test_conv_channel_sum_and_bias():
    """Many channels = sum over channel pairs of single-channel correlations."""
    rng = np.random.default_rng(2)
    x = rnd(rng, 2, 6, 5, 3)
    w = rnd(rng, 4, 9, 3)
    b = rnd(rng, 4)
    y = U.conv3x3(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate2d(x[n, :, :, c], w[o, :, c].reshape(3, 3), mode="same")
                             for c in range(3))
            np.testing.assert_allclose(y[n, :, :, o], ref, rtol=1e-12, atol=1e-12)


def test_conv_gradients_are_adjoints():
    rng = np.random.default_rng(3)
    x, w, dy = rnd(rng, 2, 5, 6, 4), rnd(rng, 3, 9, 4), rnd(rng, 2, 5, 6, 3)
    lhs = (U.conv3x3(x, w) * dy).sum()
    assert abs(lhs - (x * U.conv3x3_bwd_data(dy, w)).sum()) < 1e-10 * abs(lhs)
    dw, db = U.conv3x3_bwd_weight(dy, x)
    assert abs(lhs - (w * dw).sum()) < 1e-10 * abs(lhs)
    b = rnd(rng, 3)
    assert abs(((U.conv3x3(x, w, b) - U.conv3x3(x, w)) * dy).sum() - (b * db).sum()) < 1e-10


def test_pool_and_upsample_adjoints_and_identities():
    rng = np.random.default_rng(4)
    x, y = rnd(rng, 2, 8, 6, 3), rnd(rng, 2, 4, 3, 3)
    assert abs((U.pool2(x) * y).sum() - (x * U.pool2_bwd(y)).sum()) < 1e-12
    assert abs((U.up2(y) * x).sum() - (y * U.up2_bwd(x)).sum()) < 1e-12
    np.testing.assert_allclose(U.pool2(U.up2(y)), y, atol=1e-15)
    np.testing.assert_allclose(U.pool2(np.full((1, 4, 4, 2), 3.0)), 3.0)


def test_loss_gradient_by_finite_differences():
    rng = np.random.default_rng(5)
    out, t = rnd(rng, 1, 4, 4, 8), rnd(rng, 1, 4, 4, 3)
    fluid = rng.random((1, 4, 4)) > 0.3
    _, g = U.mse_loss(out, t, fluid)
    h = 1e-6
    for idx in [(0, 1, 2, 0), (0, 3, 3, 2), (0, 0, 0, 5)]:
        e = np.zeros_like(out)
        e[idx] = h
        fd = (U.mse_loss(out + e, t, fluid)[0] - U.mse_loss(out - e, t, fluid)[0]) / (2 * h)
        assert abs(fd - g[idx]) < 1e-7


def test_adam_first_step_closed_form():
    p, g = np.array([1.0, -2.0, 0.5]), np.array([0.3, -4.0, 1e-3])
    p1, m, v = U.adam(p, np.zeros(3), np.zeros(3), g, t=1, lr=0.01)
    np.testing.assert_allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_network_gradient_by_finite_differences():
    """Whole network at 8 x 8: backward equals central differences of the
    FP64 loss on sampled parameters of every layer."""
    rng = np.random.default_rng(6)
    lay, n = U.param_layout()
    params = np.zeros(n)
    for w_off, b_off, ci, co in lay:
        params[w_off:w_off + 9 * ci * co] = rng.standard_normal(9 * ci * co) * np.sqrt(2 / (9 * ci))
        params[b_off:b_off + co] = 0.05 * rng.standard_normal(co)
    x0 = rng.standard_normal((1, 8, 8, U.IN_CHANNELS))
    t = rng.standard_normal((1, 8, 8, 3))
    fluid = rng.random((1, 8, 8)) > 0.2
    loss, g = U.backward(params, x0, t, fluid)
    h = 1e-5
    picks = []
    for w_off, b_off, ci, co in lay:
        picks += [w_off + int(rng.integers(9 * ci * co)), b_off + int(rng.integers(co))]
    for i in picks:
        e = np.zeros(n)
        e[i] = h
        lp = U.mse_loss(U.forward(params + e, x0)[0], t, fluid)[0]
        lm = U.mse_loss(U.forward(params - e, x0)[0], t, fluid)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_make_input_layout():
    solid = np.zeros((1, 16, 16), np.uint8)
    solid[0, 0:4, 0:2] = 1
    x = U.make_input(solid, [[250.0, 0.5, 0.05]], 8)
    assert x.shape == (1, 8, 8, U.IN_CHANNELS)
    assert x[0, 0, 0, 0] == 1.0 and x[0, 1, 0, 0] == 1.0 and x[0, 0, 1, 0] == 0.0
    assert x[0, 3, 3, 1] == 0.5 and x[0, 3, 3, 2] == 0.5 and x[0, 3, 3, 3] == 0.5
    assert x[0, 7, 2, 6] == 1.0 and x[0, 6, 2, 6] == 0.0
    assert np.all(x[..., 8:] == 0)


def test_make_input_fraction_on_uneven_grids():
    """Solid fraction = mean of the mask over the nodes of each coarse cell;
    total solid area is kept when res divides fine, and every coarse cell
    sees at least one node when res > fine."""
    rng = np.random.default_rng(7)
    solid = (rng.random((1, 20, 20)) > 0.6).astype(np.uint8)
    x = U.make_input(solid, [[100.0, 0.5, 0.1]], 10)
    np.testing.assert_allclose(x[0, :, :, 0].mean(), solid.mean())
    y = U.make_input(solid, [[100.0, 0.5, 0.1]], 40)
    assert set(np.unique(y[0, :, :, 0])) <= {0.0, 1.0}
    np.testing.assert_allclose(y[0, ::2, ::2, 0], solid[0])


def test_channel_input_marks_the_inlet_and_keeps_the_solid_area():
    """A 4:1 channel maps onto the square input with four fine columns per
    coarse cell: the solid fraction keeps the solid area, and channel 6
    marks the inlet column (left), not the top row."""
    rng = np.random.default_rng(8)
    solid = (rng.random((1, 16, 64)) > 0.7).astype(np.uint8)
    x = U.make_input(solid, [[100.0, 0.5, 0.03, U.KIND_CHANNEL]], 16)
    np.testing.assert_allclose(x[0, :, :, 0].mean(), solid.mean())
    np.testing.assert_allclose(x[0, 2, 3, 0], solid[0, 2, 12:16].mean())
    assert np.all(x[0, :, 0, 6] == 1.0) and np.all(x[0, :, 1:, 6] == 0.0)
    c = U.make_input(solid[:, :, :16], [[100.0, 0.5, 0.03, U.KIND_CAVITY]], 16)
    assert np.all(c[0, 15, :, 6] == 1.0) and np.all(c[0, :15, :, 6] == 0.0)


def test_channel_fields_keep_the_prediction():
    """Uniform output (0, 1, 0): a channel gets rho = 1 and u = (U, 0) at
    every fluid node (interpolating a constant, no correction); a cavity of
    the same output gets its staggered x-momentum removed (a uniform u_x
    has a nonzero staggered sum on an odd number of fluid columns)."""
    out = np.zeros((1, 8, 8, 3))
    out[..., 1] = 1.0
    solid = np.zeros((1, 6, 24), bool)
    solid[0, 2:4, 10:13] = True
    r, a, b = U.fields_from_output(out, [[100.0, 0.5, 0.04, U.KIND_CHANNEL]], solid)
    fl = ~solid[0]
    assert np.all(r[0][fl] == 1.0) and np.allclose(a[0][fl], 0.04) and np.all(b[0] == 0.0)
    assert np.all(a[0][solid[0]] == 0.0)
    sq = np.zeros((1, 9, 9), bool)
    r, a, b = U.fields_from_output(out, [[100.0, 0.5, 0.04, U.KIND_CAVITY]], sq)
    sx = np.where(np.arange(9) % 2 == 0, 1.0, -1.0)[None, :]
    assert abs((sx * r[0] * a[0]).sum()) < 1e-15
    assert not np.allclose(a[0], 0.04)
