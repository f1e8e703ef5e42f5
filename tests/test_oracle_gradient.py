"""Pins of the oracle's density-gradient step (Sec. 5: an isotropic finite
difference of rho at the same time level; central differences as the
alternative) and of its neighbour rule at walls, lids, solid nodes and
periodic sides (reading R7: a neighbour beyond a non-periodic side takes
the value of its mirror image across the half-way wall; a solid neighbour
contributes the node's own value; periodic sides wrap).

Every expected value below comes from mathematics the stencil must satisfy
(exactness on quadratic fields, the closed-form response to a sampled sine)
or is worked out by hand in the comment next to it; none re-evaluates the
oracle's formula.
"""
import math

import numpy as np
import pytest

import oracle
from workloads import cavity_sides, periodic_sides

WALL, LID, PER = oracle.WALL, oracle.LID, oracle.PERIODIC


def _lattice(nx, ny, sides, stencil, solid=None):
    return oracle.Oracle(nx, ny, sides, solid=solid, nu=0.1, gamma=0.5, drho_stencil=stencil)


@pytest.mark.parametrize("stencil", [0, 1])
def test_gradient_exact_for_quadratic_fields_in_the_interior(oracle_lib, stencil):
    """Both stencils differentiate every quadratic exactly: the isotropic one
    because sum_a w_a e_a e_a = I/3 and every odd moment of the weights
    vanishes, the central one by Taylor's theorem."""
    nx, ny = 11, 9
    x = np.arange(nx) + 0.5
    y = np.arange(ny) + 0.5
    X, Y = np.meshgrid(x, y)
    c = dict(a=0.7, b=-0.3, c=0.25, d=0.11, e=-0.07, f=0.05)
    q = (c["a"] + c["b"] * X + c["c"] * Y + c["d"] * X ** 2 + c["e"] * X * Y +
         c["f"] * Y ** 2)
    ex_gx = c["b"] + 2 * c["d"] * X + c["e"] * Y
    ex_gy = c["c"] + c["e"] * X + 2 * c["f"] * Y
    o = _lattice(nx, ny, cavity_sides(), stencil)
    gx, gy = o.fd_gradient(q)
    inner = (slice(1, ny - 1), slice(1, nx - 1))
    assert np.abs(gx[inner] - ex_gx[inner]).max() < 1e-13
    assert np.abs(gy[inner] - ex_gy[inner]).max() < 1e-13
    # a cubic is not differentiated exactly by the isotropic stencil: its
    # error is q_xxx/6 * 3 sum_a w_a ex^4 + q_xyy/2 * 3 sum_a w_a ex^2 ey^2
    # = q_xxx/6 + q_xyy/6 (sum_a w_a ex^4 = 1/3, sum_a w_a ex^2 ey^2 = 1/9);
    # for q = x^3 that is exactly 1 (central differences: q_xxx/6 = 1 too)
    gx3, _ = o.fd_gradient(X ** 3)
    assert np.abs(gx3[inner] - 3 * X[inner] ** 2 - 1.0).max() < 1e-10


@pytest.mark.parametrize("stencil", [0, 1])
def test_gradient_wraps_periodic_sides(oracle_lib, stencil):
    """On a periodic lattice a sampled sine q_i = sin(k (i + 1/2)) that does
    not depend on y has, with either stencil, the exact discrete derivative
    (q_{i+1} - q_{i-1})/2 = sin(k) cos(k (i + 1/2)) at every node, including
    the nodes whose stencil wraps across the side (i = 0 and i = n-1)."""
    n, m = 12, 5
    k = 2 * math.pi * 2 / n
    x = np.arange(n) + 0.5
    q = np.tile(np.sin(k * x), (m, 1))
    o = _lattice(n, m, periodic_sides(), stencil)
    gx, gy = o.fd_gradient(q)
    assert np.abs(gx - np.sin(k) * np.cos(k * x)[None, :]).max() < 1e-14
    assert np.abs(gy).max() < 1e-14
    # the same along y
    gx, gy = o.fd_gradient(np.tile(np.sin(2 * math.pi * (np.arange(m) + 0.5) / m)[:, None], (1, n)))
    ky = 2 * math.pi / m
    assert np.abs(gy - (np.sin(ky) * np.cos(ky * (np.arange(m) + 0.5)))[:, None]).max() < 1e-14
    assert np.abs(gx).max() < 1e-14


@pytest.mark.parametrize("sides", [cavity_sides(), [WALL, LID, LID, WALL]])
def test_gradient_at_walls_and_lids_hand_values(oracle_lib, sides):
    """R7 at non-periodic sides, whatever their kind (wall or lid): the walls
    lie half-way, so a neighbour beyond a side takes the value of its mirror
    image across the wall, the node on the lattice edge.  For the linear
    field q = i + 2 j on a 4 x 3 lattice:

    isotropic, interior node (1, 1): exact, (1, 2).
    isotropic, corner (0, 0), q = 0: E, N, NE are inside (q = 1, 2, 3); the
      mirrors give W -> (0, 0) = 0, S -> (0, 0) = 0, SW -> (0, 0) = 0,
      NW -> (0, 1) = 2, SE -> (1, 0) = 1, so
      gx = (1 - 0)/3 + ((3 - 2) + (1 - 0))/12 = 1/3 + 1/6 = 1/2,
      gy = (2 - 0)/3 + ((3 - 1) + (2 - 0))/12 = 2/3 + 1/3 = 1.
    isotropic, top edge (1, 2), q = 5: the mirrors give N -> (1, 2) = 5,
      NE -> (2, 2) = 6, NW -> (0, 2) = 4; E = 6, W = 4, S = 3, SE = 4, SW = 2:
      gx = (6 - 4)/3 + ((6 - 4) + (4 - 2))/12 = 2/3 + 1/3 = 1,
      gy = (5 - 3)/3 + ((6 - 4) + (4 - 2))/12 = 2/3 + 1/3 = 1.
    The derivative along a wall stays exact; across it, half the slope.
    central, corner (0, 0): gx = (1 - 0)/2 = 1/2, gy = (2 - 0)/2 = 1.
    central, top edge (1, 2): gx = (6 - 4)/2 = 1, gy = (5 - 3)/2 = 1.
    """
    nx, ny = 4, 3
    J, I = np.mgrid[0:ny, 0:nx]
    q = (I + 2 * J).astype(float)
    o = _lattice(nx, ny, sides, 0)
    gx, gy = o.fd_gradient(q)
    assert gx[1, 1] == pytest.approx(1.0, abs=1e-15) and gy[1, 1] == pytest.approx(2.0, abs=1e-15)
    assert gx[0, 0] == pytest.approx(0.5, abs=1e-15)
    assert gy[0, 0] == pytest.approx(1.0, abs=1e-15)
    assert gx[2, 1] == pytest.approx(1.0, abs=1e-15)
    assert gy[2, 1] == pytest.approx(1.0, abs=1e-15)
    o = _lattice(nx, ny, sides, 1)
    gx, gy = o.fd_gradient(q)
    assert gx[0, 0] == pytest.approx(0.5, abs=1e-15) and gy[0, 0] == pytest.approx(1.0, abs=1e-15)
    assert gx[2, 1] == pytest.approx(1.0, abs=1e-15) and gy[2, 1] == pytest.approx(1.0, abs=1e-15)


def test_gradient_mirror_next_to_a_solid_edge_node(oracle_lib):
    """A mirror image that is itself solid falls back to the node's own value:
    on a 4 x 3 cavity with the edge node (0, 2) solid and q = i + 2 j, node
    (1, 2) sees W = (0, 2) solid -> own 5, NW beyond the N wall -> mirror
    (0, 2), solid -> own 5, N -> mirror (1, 2) = 5, NE -> mirror (2, 2) = 6,
    E = 6, S = 3, SE = 4, SW = 2:
      gx = (6 - 5)/3 + ((6 - 5) + (4 - 2))/12 = 1/3 + 1/4 = 7/12,
      gy = (5 - 3)/3 + ((6 - 4) + (5 - 2))/12 = 2/3 + 5/12 = 13/12."""
    nx, ny = 4, 3
    J, I = np.mgrid[0:ny, 0:nx]
    q = (I + 2 * J).astype(float)
    solid = np.zeros((ny, nx), np.uint8)
    solid[2, 0] = 1
    o = _lattice(nx, ny, cavity_sides(), 0, solid=solid)
    gx, gy = o.fd_gradient(q)
    assert gx[2, 1] == pytest.approx(7 / 12, abs=1e-15)
    assert gy[2, 1] == pytest.approx(13 / 12, abs=1e-15)


def test_gradient_next_to_a_solid_node_hand_values(oracle_lib):
    """R7 at an obstacle: on a periodic 6 x 5 lattice with one solid node at
    (3, 2) and q = i, the node west of it, (2, 2), sees the solid east
    neighbour as its own value 2:
      isotropic gx = (2 - 1)/3 + ((3 - 1) + (3 - 1))/12 = 1/3 + 1/3 = 2/3,
      isotropic gy = (2 - 2)/3 + ((3 - 3) + (1 - 1))/12 = 0;
    the node north-east of it, (4, 3), has the solid node as its SW
    neighbour, read as 4:
      gx = (5 - 3)/3 + ((5 - 3) + (5 - 4))/12 = 2/3 + 1/4 = 11/12.
    Solid nodes themselves get 0."""
    nx, ny = 6, 5
    solid = np.zeros((ny, nx), np.uint8)
    solid[2, 3] = 1
    q = np.tile(np.arange(nx, dtype=float), (ny, 1))
    o = _lattice(nx, ny, periodic_sides(), 0, solid=solid)
    gx, gy = o.fd_gradient(q)
    assert gx[2, 2] == pytest.approx(2 / 3, abs=1e-15) and gy[2, 2] == pytest.approx(0.0, abs=1e-15)
    assert gx[3, 4] == pytest.approx(11 / 12, abs=1e-15)
    assert gx[2, 3] == 0.0 and gy[2, 3] == 0.0
    # away from the obstacle and the wrap the slope is exact
    assert gx[0, 1] == pytest.approx(1.0, abs=1e-15)
