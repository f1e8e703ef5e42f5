"""Host logic of the warm-start driver (no GPU): training targets of the
network at its own resolution, case parameters and which cases a set of
weights covers."""
import numpy as np
import pytest

from workloads import Case


def _case(kind, nx, ny, mask=None, u=0.04):
    if mask is None:
        mask = np.zeros((ny, nx), np.uint8)
    return Case(kind, nx, ny, 100.0, 0.5, u, mask)


def test_targets_on_the_network_grid_are_cell_means_over_fluid_nodes():
    """A 4:1 channel on an 8 x 8 grid: each cell covers 4 x 1 nodes; its
    target is the mean over its fluid nodes, a cell without fluid is not
    fluid, and a channel's density target is zero."""
    from paper_1806_10251_amd import surrogate as S
    nx, ny, res = 32, 8, 8
    mask = np.zeros((ny, nx), np.uint8)
    mask[2, 4:8] = 1          # cell (J=2, I=1) all solid
    mask[5, 12] = 1           # cell (J=5, I=3): one of four nodes solid
    k = _case("channel", nx, ny, mask)
    X = np.arange(nx)[None, :] * np.ones((ny, 1))
    ux = 0.04 * (1.0 + X / nx)
    uy = 0.04 * 0.01 * np.arange(ny)[:, None] * np.ones((1, nx))
    rho = 1.0 + 0.001 * X
    t, fluid = S.targets([k], rho[None], ux[None], uy[None], res)
    assert t.shape == (1, res, res, 3) and fluid.shape == (1, res, res)
    assert fluid[0, 2, 1] == 0 and fluid.sum() == res * res - 1
    np.testing.assert_allclose(t[0, 0, 0, 1], np.mean(1.0 + np.arange(4) / nx), rtol=1e-6)
    np.testing.assert_allclose(t[0, 5, 3, 1], np.mean(1.0 + np.array([13, 14, 15]) / nx),
                               rtol=1e-6)
    np.testing.assert_allclose(t[0, 6, 2, 2], 0.06, rtol=1e-6)
    assert np.all(t[..., 0] == 0.0)
    assert np.all(t[0, 2, 1] == 0.0)


def test_targets_of_a_cavity_at_the_network_size_are_per_node():
    from paper_1806_10251_amd import surrogate as S
    n = 8
    mask = np.zeros((n, n), np.uint8)
    mask[3, 3] = 1
    k = _case("cavity", n, n, mask, u=0.1)
    rng = np.random.default_rng(3)
    rho = 1.0 + 1e-3 * rng.standard_normal((1, n, n))
    ux, uy = 0.1 * rng.standard_normal((2, 1, n, n))
    t, fluid = S.targets([k], rho, ux, uy, n)
    fl = mask == 0
    np.testing.assert_allclose(t[0, ..., 0][fl], ((rho[0] - 1) / 0.03)[fl], rtol=1e-5)
    np.testing.assert_allclose(t[0, ..., 1][fl], (ux[0] / 0.1)[fl], rtol=1e-5)
    assert np.all(t[0, 3, 3] == 0.0) and fluid[0, 3, 3] == 0


def test_case_params_and_coverage():
    from paper_1806_10251_amd import surrogate as S
    from paper_1806_10251_amd import unet as U
    cav, ch, rect = _case("cavity", 16, 16), _case("channel", 64, 16), _case("cavity", 32, 16)
    cp = S.case_params([cav, ch])
    assert cp.shape == (2, 4) and cp[0, 3] == U.KIND_CAVITY and cp[1, 3] == U.KIND_CHANNEL

    class Net:
        pass
    net = Net()
    assert S.covers(cav, net) and not S.covers(ch, net)       # no kinds record: cavities
    net.kinds = ("cavity", "channel")
    assert S.covers(cav, net) and S.covers(ch, net) and not S.covers(rect, net)
    net.kinds = ("channel",)
    assert not S.covers(cav, net) and S.covers(ch, net)


def test_weights_record_the_kinds_they_cover(tmp_path):
    from paper_1806_10251_amd import surrogate as S

    class Net:
        def __init__(self):
            self.p = np.arange(5, dtype=np.float32)

        def params(self):
            return self.p

        def set_params(self, p):
            self.p = np.array(p)
    a, b = Net(), Net()
    path = str(tmp_path / "w.npy")
    S.save(a, path, kinds=("cavity", "channel"))
    S.load_into(b, path)
    assert b.kinds == ("cavity", "channel") and np.array_equal(b.p, a.p)
    np.save(str(tmp_path / "old.npy"), a.p)
    S.load_into(b, str(tmp_path / "old.npy"))
    assert b.kinds == ("cavity",)
