"""Plain FP64 CPU oracle of the GI-corrected preconditioned cascaded D2Q9 LBM.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``.  The product path never imports
it, and it shares no code with the HIP library.

The arithmetic lives in ``lbm_oracle.c`` (plain C, double precision; see the
paper map at the top of that file).  This module only marshals arguments to it
through ctypes.  Build it with ``build()`` (gcc, no GPU needed).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

PERIODIC, WALL, LID, INLET, OUTLET = 0, 1, 2, 3, 4


class OracleParams(ctypes.Structure):
    _fields_ = [
        ("nu", ctypes.c_double),
        ("omega3", ctypes.c_double),
        ("omega6", ctypes.c_double),
        ("omega7", ctypes.c_double),
        ("omega8", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("u_lid", ctypes.c_double),
        ("u_in_max", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("fx", ctypes.c_double),
        ("fy", ctypes.c_double),
        ("gi_correct", ctypes.c_int32),
        ("drho_stencil", ctypes.c_int32),
        ("strain_fd", ctypes.c_int32),
        ("mrt", ctypes.c_int32),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int32),
                                 ctypes.c_void_p, ctypes.POINTER(OracleParams)]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = None
        L.orc_init_fields.argtypes = [ctypes.c_void_p, dp, dp, dp]
        L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        L.orc_step.restype = ctypes.c_int
        for name in ("orc_residual", "orc_mass", "orc_omega4"):
            getattr(L, name).argtypes = [ctypes.c_void_p]
            getattr(L, name).restype = ctypes.c_double
        for name in ("orc_steps", "orc_guard_count"):
            getattr(L, name).argtypes = [ctypes.c_void_p]
            getattr(L, name).restype = ctypes.c_int64
        L.orc_fields.argtypes = [ctypes.c_void_p, dp, dp, dp]
        L.orc_get_f.argtypes = [ctypes.c_void_p, dp]
        L.orc_set_f.argtypes = [ctypes.c_void_p, dp]
        L.orc_set_force_field.argtypes = [ctypes.c_void_p, dp, dp]
        L.orc_set_force_field.restype = ctypes.c_int
        L.orc_raw_moments.argtypes = [dp, dp]
        L.orc_moments_to_pop.argtypes = [dp, dp]
        L.orc_equilibrium.argtypes = [ctypes.c_double] * 4 + [dp]
        L.orc_strain.argtypes = [ctypes.c_double] * 10 + [dp, dp]
        L.orc_strain.restype = ctypes.c_int
        L.orc_collide.argtypes = [dp, ctypes.c_double, ctypes.c_double,
                                  ctypes.POINTER(OracleParams), ctypes.c_double,
                                  ctypes.c_double, dp, dp]
        L.orc_fd_gradient.argtypes = [ctypes.c_void_p, dp, dp, dp]
        L.orc_fd_gradient.restype = None
        L.orc_omega_from_nu.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_omega_from_nu.restype = ctypes.c_double
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(nu, gamma, omega3=1.0, omega6=1.0, omega7=1.0, omega8=1.0, u_lid=0.0,
                u_in_max=0.0, rho0=1.0, fx=0.0, fy=0.0, gi_correct=1, drho_stencil=0,
                strain_fd=0, mrt=0):
    return OracleParams(nu, omega3, omega6, omega7, omega8, gamma, u_lid, u_in_max, rho0,
                        fx, fy, gi_correct, drho_stencil, strain_fd, mrt)


def set_threads(n):
    """OpenMP threads of the oracle's loops in this process (timing only)."""
    lib().orc_set_threads(int(n))


def omega_from_nu(nu, gamma):
    """w4 = w5 = 1 / (3 nu / gamma + 1/2)  (nu = gamma/3 (1/w - 1/2), eq. 49)."""
    return lib().orc_omega_from_nu(nu, gamma)


class Oracle:
    """One lattice, stepped by the C oracle.  Arrays are row-major [ny][nx]."""

    def __init__(self, nx, ny, sides, solid=None, **params):
        self.nx, self.ny = int(nx), int(ny)
        self.params = make_params(**params)
        sd = (ctypes.c_int32 * 4)(*[int(s) for s in sides])
        self._solid = None
        ptr = None
        if solid is not None:
            self._solid = np.ascontiguousarray(solid, dtype=np.uint8).reshape(self.ny, self.nx)
            ptr = self._solid.ctypes.data_as(ctypes.c_void_p)
        h = lib().orc_create(self.nx, self.ny, sd, ptr, ctypes.byref(self.params))
        if not h:
            raise ValueError("oracle rejected the configuration")
        self._h = ctypes.c_void_p(h)
        self.init_fields()

    def close(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def init_fields(self, rho=None, ux=None, uy=None):
        arrs = []
        for a in (rho, ux, uy):
            if a is None:
                arrs.append(None)
            else:
                arrs.append(np.ascontiguousarray(a, dtype=np.float64).reshape(self.ny, self.nx))
        lib().orc_init_fields(self._h, *[(_dp(a) if a is not None else None) for a in arrs])

    def step(self, n=1):
        rc = lib().orc_step(self._h, int(n))
        if rc != 0:
            raise FloatingPointError("oracle run became unstable (non-finite fields)")

    @property
    def residual(self):
        return lib().orc_residual(self._h)

    @property
    def mass(self):
        return lib().orc_mass(self._h)

    @property
    def steps(self):
        return lib().orc_steps(self._h)

    @property
    def guard_count(self):
        return lib().orc_guard_count(self._h)

    @property
    def omega4(self):
        return lib().orc_omega4(self._h)

    def fields(self):
        r = np.zeros((self.ny, self.nx))
        ux = np.zeros_like(r)
        uy = np.zeros_like(r)
        lib().orc_fields(self._h, _dp(r), _dp(ux), _dp(uy))
        return r, ux, uy

    def get_f(self):
        f = np.zeros((9, self.ny, self.nx))
        lib().orc_get_f(self._h, _dp(f))
        return f

    def set_f(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == (9, self.ny, self.nx)
        lib().orc_set_f(self._h, _dp(f))

    def fd_gradient(self, q):
        """Finite-difference gradient (gx, gy) of a node field q [ny][nx] with
        this lattice's stencil, sides and solid mask (the density-gradient
        step; solid nodes get 0)."""
        q = np.ascontiguousarray(q, dtype=np.float64).reshape(self.ny, self.nx)
        gx = np.zeros_like(q)
        gy = np.zeros_like(q)
        lib().orc_fd_gradient(self._h, _dp(q), _dp(gx), _dp(gy))
        return gx, gy

    def set_force_field(self, fx, fy):
        """Per-node body force [ny][nx] (None, None: the uniform force)."""
        if fx is None and fy is None:
            rc = lib().orc_set_force_field(self._h, None, None)
        else:
            self._ffx = np.ascontiguousarray(fx, dtype=np.float64).reshape(self.ny, self.nx)
            self._ffy = np.ascontiguousarray(fy, dtype=np.float64).reshape(self.ny, self.nx)
            rc = lib().orc_set_force_field(self._h, _dp(self._ffx), _dp(self._ffy))
        if rc:
            raise ValueError("bad force field")


# --- single-node entry points (unit-level pins) -----------------------------

def raw_moments(f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    m = np.zeros(9)
    lib().orc_raw_moments(_dp(f), _dp(m))
    return m


def moments_to_pop(m):
    m = np.ascontiguousarray(m, dtype=np.float64)
    f = np.zeros(9)
    lib().orc_moments_to_pop(_dp(m), _dp(f))
    return f


def equilibrium(rho, ux, uy, gamma):
    f = np.zeros(9)
    lib().orc_equilibrium(rho, ux, uy, gamma, _dp(f))
    return f


def strain(rho, ux, uy, m3, m4, drx, dry, omega3, omega4, gamma):
    a = np.zeros(1)
    b = np.zeros(1)
    g = lib().orc_strain(rho, ux, uy, m3, m4, drx, dry, omega3, omega4, gamma, _dp(a), _dp(b))
    return a[0], b[0], bool(g)


def collide(fbar, drx, dry, nu, gamma, **kw):
    """One node's collision; returns (f_out[9], diag dict)."""
    p = make_params(nu=nu, gamma=gamma, **kw)
    w = omega_from_nu(nu, gamma)
    fb = np.ascontiguousarray(fbar, dtype=np.float64)
    fo = np.zeros(9)
    dg = np.zeros(8)
    lib().orc_collide(_dp(fb), drx, dry, ctypes.byref(p), w, w, _dp(fo), _dp(dg))
    keys = ("rho", "ux", "uy", "dxux", "dyuy", "guarded", "m3", "m4")
    return fo, dict(zip(keys, dg))
