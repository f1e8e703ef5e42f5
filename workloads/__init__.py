"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module holds geometry, case lists and initial fields only: none of the
lattice Boltzmann arithmetic.  Every generator is driven by SplitMix64
(Steele, Lea & Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014), written out here from its published definition so that a case
list is reproducible from its seed alone.

Conventions: arrays are row-major ``[ny][nx]``; node (i, j) sits at
x = i + 1/2, y = j + 1/2; side order is (W, E, S, N).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

PERIODIC, WALL, LID, INLET, OUTLET = 0, 1, 2, 3, 4
MASK64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 generator (64-bit state, golden-gamma increment)."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self, lo: float = 0.0, hi: float = 1.0) -> float:
        return lo + (hi - lo) * ((self.next_u64() >> 11) * (1.0 / (1 << 53)))

    def randint(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi] (inclusive)."""
        return lo + int(self.uniform() * (hi - lo + 1)) if hi > lo else lo

    def normal_array(self, n: int) -> np.ndarray:
        """Box-Muller normals (for seeded random populations in tests)."""
        out = np.empty(n)
        for k in range(0, n, 2):
            u1 = max(self.uniform(), 1e-300)
            u2 = self.uniform()
            r = math.sqrt(-2.0 * math.log(u1))
            out[k] = r * math.cos(2 * math.pi * u2)
            if k + 1 < n:
                out[k + 1] = r * math.sin(2 * math.pi * u2)
        return out

    def uniform_array(self, n: int, lo=0.0, hi=1.0) -> np.ndarray:
        return np.array([self.uniform(lo, hi) for _ in range(n)])


# --------------------------------------------------------------------------
# Geometries
# --------------------------------------------------------------------------

def cavity_sides():
    """Lid-driven cavity: stationary W/E/S walls, lid on N moving in +x."""
    return (WALL, WALL, WALL, LID)


def channel_sides():
    """Channel: parabolic inlet on W, convective outlet on E, walls S/N."""
    return (INLET, OUTLET, WALL, WALL)


def periodic_sides():
    return (PERIODIC, PERIODIC, PERIODIC, PERIODIC)


def poiseuille_sides():
    """Body-force channel: periodic in x, walls at y = 0 and y = ny."""
    return (PERIODIC, PERIODIC, WALL, WALL)


def centred_square_mask(nx: int, ny: int, side: int) -> np.ndarray:
    m = np.zeros((ny, nx), dtype=np.uint8)
    x0 = nx // 2 - side // 2
    y0 = ny // 2 - side // 2
    m[y0:y0 + side, x0:x0 + side] = 1
    return m


def _fluid_connected(mask: np.ndarray) -> bool:
    """Flood fill (4-connected) from the first fluid node."""
    ny, nx = mask.shape
    fluid = mask == 0
    total = int(fluid.sum())
    if total == 0:
        return False
    seen = np.zeros_like(fluid)
    start = np.argwhere(fluid)[0]
    stack = [tuple(start)]
    seen[start[0], start[1]] = True
    count = 0
    while stack:
        j, i = stack.pop()
        count += 1
        for dj, di in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            a, b = j + dj, i + di
            if 0 <= a < ny and 0 <= b < nx and fluid[a, b] and not seen[a, b]:
                seen[a, b] = True
                stack.append((a, b))
    return count == total


def random_obstacles(rng: SplitMix64, nx: int, ny: int, kind: str,
                     cover_lo=0.05, cover_hi=0.20, max_tries=200) -> np.ndarray:
    """1-4 axis-aligned rectangles covering cover_lo..cover_hi of the area.

    Rectangles keep a margin of 2 nodes from every side (3 from the lid row
    of a cavity, and 4 from the inlet/outlet columns of a channel) and are
    redrawn when the fluid would be split into disconnected parts, or when a
    channel cross-section would be more than half blocked (a velocity inlet
    then needs a pressure rise the weakly compressible scheme cannot hold).
    """
    area = nx * ny
    for _ in range(max_tries):
        k = rng.randint(1, 4)
        target = rng.uniform(cover_lo, cover_hi) * area
        m = np.zeros((ny, nx), dtype=np.uint8)
        mx0, mx1, my0, my1 = 2, nx - 2, 2, ny - 2
        if kind == "cavity":
            my1 = ny - 3
        else:
            mx0, mx1 = 4, nx - 4
        ok = True
        for _r in range(k):
            a = target / k
            ar = math.exp(rng.uniform(math.log(0.5), math.log(2.0)))
            w = max(1, int(round(math.sqrt(a * ar))))
            h = max(1, int(round(a / max(w, 1))))
            w = min(w, mx1 - mx0 - 1)
            h = min(h, my1 - my0 - 1)
            if w < 1 or h < 1:
                ok = False
                break
            x0 = rng.randint(mx0, mx1 - w)
            y0 = rng.randint(my0, my1 - h)
            m[y0:y0 + h, x0:x0 + w] = 1
        if not ok:
            continue
        cover = m.sum() / area
        if cover < cover_lo or cover > cover_hi:
            continue
        if kind == "channel" and m.sum(axis=0).max() > ny // 2:
            continue      # keep at least half of every cross-section open
        if kind == "cavity" and (m.sum(axis=0).max() > ny - 6 or m.sum(axis=1).max() > nx - 6):
            continue
        if not _fluid_connected(m):
            continue
        return m
    raise RuntimeError("could not draw an obstacle set")


@dataclass
class Case:
    """One steady case of the batched workload."""
    kind: str            # "cavity" or "channel"
    nx: int
    ny: int
    re: float
    gamma: float
    u_ref: float         # lid speed (cavity) or inlet peak (channel)
    mask: np.ndarray = field(repr=False)

    @property
    def sides(self):
        return cavity_sides() if self.kind == "cavity" else channel_sides()

    @property
    def length(self):
        """Reynolds length: the long side of the domain (cavity side, channel
        length)."""
        return self.nx

    @property
    def nu(self):
        return self.u_ref * self.length / self.re


def draw_cases(n: int, seed: int, side_lo=64, side_hi=512, re_lo=50.0, re_hi=1000.0,
               gamma_lo=0.05, gamma_hi=1.0, u_cavity=0.1, u_channel=0.05, channel_frac=0.5,
               ma_cavity=0.3, ma_channel=0.1, gi_max=0.2):
    """Seeded mix of cavities (s x s) and channels (4s x s) with obstacles.

    Reference speeds: lid speed ``u_cavity`` and inlet peak ``u_channel``,
    each lowered where needed so that
      * the preconditioned Mach number U / sqrt(gamma / 3) stays at or below
        ``ma_cavity`` / ``ma_channel`` (the channel bound is lower because
        flow through the gaps between obstacles runs about three times
        faster than the inlet peak), and
      * the size of the third-order GI correction coefficients at the
        fastest node, (1/omega - 1/2)(4/gamma^2 - 1/gamma) u_max^2 with
        1/omega - 1/2 = 3 nu / gamma, stays at or below ``gi_max`` (these
        grow like nu u^2 / gamma^3 and destabilise viscous, strongly
        preconditioned cases; u_max = U for a cavity, 3U for a channel).
    With nu = U L / Re the second bound is a cube-root cap on U.
    """
    rng = SplitMix64(seed)
    cases = []
    for _ in range(n):
        kind = "channel" if rng.uniform() < channel_frac else "cavity"
        s = rng.randint(side_lo, side_hi)
        re = rng.uniform(re_lo, re_hi)
        gamma = math.exp(rng.uniform(math.log(gamma_lo), math.log(gamma_hi)))
        nx, ny = (s, s) if kind == "cavity" else (4 * s, s)
        mask = random_obstacles(rng, nx, ny, kind)
        cs_g = math.sqrt(gamma / 3.0)
        accel = 1.0 if kind == "cavity" else 3.0
        gi_cap = (gi_max * re * gamma /
                  (3.0 * nx * (4.0 / gamma ** 2 - 1.0 / gamma) * accel ** 2)) ** (1.0 / 3.0)
        if kind == "cavity":
            u = min(u_cavity, ma_cavity * cs_g, gi_cap)
        else:
            u = min(u_channel, ma_channel * cs_g, gi_cap)
        cases.append(Case(kind, nx, ny, re, gamma, u, mask))
    return cases


# --------------------------------------------------------------------------
# Initial fields
# --------------------------------------------------------------------------

def diagonal_shear_wave(n: int, amp: float, mode: int, ux0: float):
    """u' = amp sin(k (x + y)) (1, -1)/sqrt(2) on a background (ux0, 0).

    k = 2 pi mode / n; x, y at node centres.  Returns (rho, ux, uy) with
    rho = 1.
    """
    x = np.arange(n) + 0.5
    X, Y = np.meshgrid(x, x)
    k = 2.0 * math.pi * mode / n
    s = amp * np.sin(k * (X + Y)) / math.sqrt(2.0)
    return np.ones((n, n)), ux0 + s, -s


def axis_shear_wave(n: int, amp: float, mode: int, ux0: float):
    """u_y = amp sin(k x) on a background (ux0, 0)."""
    x = np.arange(n) + 0.5
    X, _ = np.meshgrid(x, x)
    k = 2.0 * math.pi * mode / n
    return np.ones((n, n)), np.full((n, n), ux0), amp * np.sin(k * X)


def random_populations(rng: SplitMix64, shape, lo=0.8, hi=1.2):
    """Positive random numbers for 'arbitrary population' tests."""
    n = int(np.prod(shape))
    return rng.uniform_array(n, lo, hi).reshape(shape)


def four_roll_mill_force(n: int, u0: float, nu: float):
    """Body force of the four-rolls mill flow (Sec. 6) on an n x n periodic
    lattice, node centres at (i + 1/2) 2 pi / n: F = 2 nu k^2 u0 (sin kx sin ky,
    cos kx cos ky), k = 2 pi / n.  Returns fx, fy as [n][n] arrays."""
    k = 2 * math.pi / n
    x = (np.arange(n) + 0.5) * k
    X, Y = np.meshgrid(x, x)
    c = 2 * nu * k * k * u0
    return c * np.sin(X) * np.sin(Y), c * np.cos(X) * np.cos(Y)


def hartmann_force(nx: int, ny: int, f_b: float, ha: float):
    """Effective body force of the Hartmann flow (Sec. 6): the driving force
    F_b plus the Lorentz force B0 dB_x/dz of the induced field, which
    simplifies to F_b Ha cosh(Ha z / L) / sinh(Ha) across a channel of half
    width L = ny / 2 (z = y + 1/2 - L at node centres; walls half-way).
    Returns fx, fy as [ny][nx] arrays (fy = 0)."""
    L = ny / 2.0
    z = np.arange(ny) + 0.5 - L
    col = f_b * ha * np.cosh(ha * z / L) / math.sinh(ha) if ha > 0 else np.full(ny, f_b)
    fx = np.repeat(col[:, None], nx, axis=1)
    return fx, np.zeros_like(fx)
