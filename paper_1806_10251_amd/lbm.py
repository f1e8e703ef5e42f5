"""ctypes binding of the C ABI in include/lbm.h (argument marshalling only).

Every step of the method runs in the HIP library ``liblbm.so``; this module
converts numpy arrays and torch tensors to pointers and status codes to
exceptions.  Importing it does not touch the GPU.  ``load()`` raises if the
library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EUNSTABLE, LBM_ESTATE = 0, -1, -2, -3, -4, -5
PERIODIC, WALL, LID, INLET, OUTLET = 0, 1, 2, 3, 4
STORE_F64, STORE_F32, STORE_BF16, STORE_F16 = 0, 1, 2, 3
STORAGE_NAMES = {"f64": STORE_F64, "f32": STORE_F32, "bf16": STORE_BF16, "f16": STORE_F16}

# Symbols the library exports (all declared in include/lbm.h).
EXPORTS = (
    "lbm_create", "lbm_init_fields", "lbm_init_fields_device", "lbm_set_stream", "lbm_step",
    "lbm_residual", "lbm_mass", "lbm_guard_count", "lbm_steps", "lbm_fields",
    "lbm_fields_device", "lbm_populations", "lbm_save", "lbm_load", "lbm_set_launch",
    "lbm_get_launch", "lbm_launch_shapes", "lbm_set_timing", "lbm_last_step_ms", "lbm_destroy",
    "lbm_last_error", "lbm_batch_create", "lbm_batch_init_fields",
    "lbm_batch_init_fields_device", "lbm_batch_set_stream", "lbm_batch_run",
    "lbm_batch_residual", "lbm_batch_fields", "lbm_batch_set_launch", "lbm_batch_destroy",
    "lbm_set_storage", "lbm_batch_set_plateau", "lbm_batch_status", "lbm_batch_set_enabled",
    "lbm_batch_set_storage", "lbm_average_last_two", "lbm_batch_average_last_two",
    "lbm_set_force_field", "lbm_fields_noalloc",
)


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class UnstableError(LbmError):
    pass


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("side", ctypes.c_int32 * 4)]


class Params(ctypes.Structure):
    _fields_ = [
        ("nu", ctypes.c_double), ("omega3", ctypes.c_double), ("omega6", ctypes.c_double),
        ("omega7", ctypes.c_double), ("omega8", ctypes.c_double), ("gamma", ctypes.c_double),
        ("u_lid", ctypes.c_double), ("u_in_max", ctypes.c_double), ("rho0", ctypes.c_double),
        ("fx", ctypes.c_double), ("fy", ctypes.c_double), ("storage_scale", ctypes.c_double),
        ("storage", ctypes.c_int32), ("gi_correct", ctypes.c_int32),
        ("drho_stencil", ctypes.c_int32), ("check_every", ctypes.c_int32),
        ("strain_fd", ctypes.c_int32), ("mrt", ctypes.c_int32),
    ]


_lib = None


def load():
    """Load liblbm.so (raises when it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python -m paper_1806_10251_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "lbm_create": [P(Grid), vp, P(Params), P(vp)],
        "lbm_init_fields": [vp, vp, vp, vp],
        "lbm_init_fields_device": [vp, vp, vp, vp],
        "lbm_set_stream": [vp, vp],
        "lbm_step": [vp, i64],
        "lbm_residual": [vp, P(dbl)],
        "lbm_mass": [vp, P(dbl)],
        "lbm_guard_count": [vp, P(i64)],
        "lbm_steps": [vp, P(i64)],
        "lbm_fields": [vp, vp, vp, vp],
        "lbm_fields_noalloc": [vp, vp, vp, vp],
        "lbm_fields_device": [vp, vp, vp, vp],
        "lbm_populations": [vp, vp],
        "lbm_save": [vp, ctypes.c_char_p],
        "lbm_load": [vp, ctypes.c_char_p],
        "lbm_set_launch": [vp, i32, i32],
        "lbm_average_last_two": [vp],
        "lbm_batch_average_last_two": [vp],
        "lbm_get_launch": [vp, P(i32), P(i32)],
        "lbm_launch_shapes": [P(i32), i32],
        "lbm_set_timing": [vp, i32],
        "lbm_last_step_ms": [vp, P(dbl)],
        "lbm_batch_create": [i32, P(Grid), P(vp), P(Params), P(vp)],
        "lbm_batch_init_fields": [vp, i32, vp, vp, vp],
        "lbm_batch_init_fields_device": [vp, i32, vp, vp, vp],
        "lbm_batch_set_stream": [vp, vp],
        "lbm_batch_run": [vp, dbl, i64, vp],
        "lbm_batch_residual": [vp, i32, P(dbl)],
        "lbm_batch_fields": [vp, i32, vp, vp, vp],
        "lbm_batch_set_launch": [vp, i32, i32],
        "lbm_set_storage": [vp, i32, dbl],
        "lbm_set_force_field": [vp, vp, vp],
        "lbm_batch_set_plateau": [vp, i32, dbl],
        "lbm_batch_status": [vp, vp],
        "lbm_batch_set_enabled": [vp, vp],
        "lbm_batch_set_storage": [vp, i32],
    }
    for name, args in sig.items():
        if not hasattr(L, name):
            continue
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.lbm_destroy.argtypes = [vp]
    L.lbm_destroy.restype = None
    if hasattr(L, "lbm_batch_destroy"):
        L.lbm_batch_destroy.argtypes = [vp]
        L.lbm_batch_destroy.restype = None
    L.lbm_last_error.argtypes = []
    L.lbm_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(rc):
    if rc != LBM_OK:
        msg = load().lbm_last_error().decode(errors="replace")
        if rc == LBM_EUNSTABLE:
            raise UnstableError(rc, msg)
        raise LbmError(rc, msg)


def _host_ptr(a, dtype):
    if a is None:
        return None, None
    arr = np.ascontiguousarray(a, dtype=dtype)
    return arr, arr.ctypes.data_as(ctypes.c_void_p)


def _dev_ptr(t):
    """Device pointer of a contiguous torch CUDA/HIP tensor (or None)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("device tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def make_grid(nx, ny, sides):
    return Grid(int(nx), int(ny), (ctypes.c_int32 * 4)(*[int(s) for s in sides]))


def make_params(nu, gamma, storage="f32", omega3=1.0, omega6=1.0, omega7=1.0, omega8=1.0,
                u_lid=0.0, u_in_max=0.0, rho0=1.0, fx=0.0, fy=0.0, storage_scale=0.0,
                gi_correct=1, drho_stencil=0, check_every=1, strain_fd=0, mrt=0):
    st = STORAGE_NAMES[storage] if isinstance(storage, str) else int(storage)
    return Params(nu, omega3, omega6, omega7, omega8, gamma, u_lid, u_in_max, rho0, fx, fy,
                  storage_scale, st, gi_correct, drho_stencil, check_every, strain_fd, mrt)


def launch_shapes():
    L = load()
    buf = (ctypes.c_int32 * 64)()
    n = L.lbm_launch_shapes(buf, 32)
    return [(buf[2 * i], buf[2 * i + 1]) for i in range(n)]


def _ready(*tensors):
    """Wait for the current torch stream when device tensors are passed:
    they may still be being written there."""
    if any(t is not None and hasattr(t, "data_ptr") for t in tensors):
        import torch
        torch.cuda.current_stream().synchronize()


class Lattice:
    """One lattice on the current HIP device (wraps lbm_ctx)."""

    def __init__(self, nx, ny, sides, solid=None, **params):
        L = load()
        self.nx, self.ny = int(nx), int(ny)
        self._grid = make_grid(nx, ny, sides)
        self._params = make_params(**params)
        self._mask, mp = _host_ptr(None if solid is None else np.asarray(solid).reshape(ny, nx),
                                   np.uint8)
        h = ctypes.c_void_p()
        _check(L.lbm_create(ctypes.byref(self._grid), mp, ctypes.byref(self._params),
                            ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # --- state -----------------------------------------------------------
    def init_fields(self, rho=None, ux=None, uy=None):
        arrs = [_host_ptr(a, np.float64) for a in (rho, ux, uy)]
        _check(load().lbm_init_fields(self._h, *[p for _, p in arrs]))

    def init_fields_device(self, rho=None, ux=None, uy=None):
        """Device float32 tensors; the library reads them on its own stream,
        so the producing (current torch) stream is synchronised first."""
        _ready(rho, ux, uy)
        _check(load().lbm_init_fields_device(self._h, _dev_ptr(rho), _dev_ptr(ux), _dev_ptr(uy)))

    def set_stream(self, stream):
        """stream: a torch.cuda.Stream, a raw hipStream_t int, or None."""
        raw = getattr(stream, "cuda_stream", stream)
        _check(load().lbm_set_stream(self._h, ctypes.c_void_p(raw) if raw else None))

    def step(self, n=1):
        _check(load().lbm_step(self._h, int(n)))

    @property
    def residual(self):
        r = ctypes.c_double()
        _check(load().lbm_residual(self._h, ctypes.byref(r)))
        return r.value

    @property
    def mass(self):
        r = ctypes.c_double()
        _check(load().lbm_mass(self._h, ctypes.byref(r)))
        return r.value

    @property
    def guard_count(self):
        r = ctypes.c_int64()
        _check(load().lbm_guard_count(self._h, ctypes.byref(r)))
        return r.value

    @property
    def steps(self):
        r = ctypes.c_int64()
        _check(load().lbm_steps(self._h, ctypes.byref(r)))
        return r.value

    def fields(self):
        out = [np.zeros((self.ny, self.nx)) for _ in range(3)]
        _check(load().lbm_fields(self._h, *[o.ctypes.data_as(ctypes.c_void_p) for o in out]))
        return tuple(out)

    def fields_noalloc(self, rho=True, ux=True, uy=True):
        """fields() through the entry point that allocates no device memory
        (a fixed per-GPU staging array; concurrent calls on one GPU race).
        Unrequested fields come back as None."""
        out = [np.zeros((self.ny, self.nx)) if w else None for w in (rho, ux, uy)]
        ptr = [o.ctypes.data_as(ctypes.c_void_p) if o is not None else None for o in out]
        _check(load().lbm_fields_noalloc(self._h, *ptr))
        return tuple(out)

    def fields_device(self, rho=None, ux=None, uy=None):
        """Write the fields into device float32 tensors (synchronises)."""
        _check(load().lbm_fields_device(self._h, _dev_ptr(rho), _dev_ptr(ux), _dev_ptr(uy)))

    def populations(self):
        f = np.zeros((9, self.ny, self.nx))
        _check(load().lbm_populations(self._h, f.ctypes.data_as(ctypes.c_void_p)))
        return f

    def set_storage(self, storage, storage_scale=0.0):
        st = STORAGE_NAMES[storage] if isinstance(storage, str) else int(storage)
        _check(load().lbm_set_storage(self._h, st, float(storage_scale)))

    def set_force_field(self, fx, fy):
        """Per-node body force (host arrays [ny][nx]); None, None: uniform force."""
        arrs = [None if a is None else
                np.ascontiguousarray(a, dtype=np.float64).reshape(self.ny, self.nx)
                for a in (fx, fy)]
        ptrs = [None if a is None else a.ctypes.data_as(ctypes.c_void_p) for a in arrs]
        _check(load().lbm_set_force_field(self._h, *ptrs))

    def save(self, path):
        _check(load().lbm_save(self._h, str(path).encode()))

    def load_checkpoint(self, path):
        _check(load().lbm_load(self._h, str(path).encode()))

    def average_last_two(self):
        """Replace the state by the mean of the last two steps' states."""
        _check(load().lbm_average_last_two(self._h))

    # --- launch shape / timing ----------------------------------------------
    def set_launch(self, by, rows):
        _check(load().lbm_set_launch(self._h, int(by), int(rows)))

    def get_launch(self):
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(load().lbm_get_launch(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def set_timing(self, on=True):
        _check(load().lbm_set_timing(self._h, 1 if on else 0))

    @property
    def last_step_ms(self):
        r = ctypes.c_double()
        _check(load().lbm_last_step_ms(self._h, ctypes.byref(r)))
        return r.value


class Batch:
    """Many independent lattices advanced together (schedules: set_launch)."""

    def __init__(self, cases_grids, masks, params_list):
        L = load()
        n = len(cases_grids)
        self.n = n
        self._grids = (Grid * n)(*cases_grids)
        self._params = (Params * n)(*params_list)
        self._masks = [None if m is None else np.ascontiguousarray(m, dtype=np.uint8)
                       for m in masks]
        mp = (ctypes.c_void_p * n)(*[None if m is None else m.ctypes.data for m in self._masks])
        h = ctypes.c_void_p()
        _check(L.lbm_batch_create(n, self._grids, mp, self._params, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().lbm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_fields(self, c, rho=None, ux=None, uy=None):
        arrs = [_host_ptr(a, np.float64) for a in (rho, ux, uy)]
        _check(load().lbm_batch_init_fields(self._h, int(c), *[p for _, p in arrs]))

    def init_fields_device(self, c, rho=None, ux=None, uy=None):
        """As Lattice.init_fields_device, for case c."""
        _ready(rho, ux, uy)
        _check(load().lbm_batch_init_fields_device(self._h, int(c), _dev_ptr(rho), _dev_ptr(ux),
                                                   _dev_ptr(uy)))

    def set_stream(self, stream):
        raw = getattr(stream, "cuda_stream", stream)
        _check(load().lbm_batch_set_stream(self._h, ctypes.c_void_p(raw) if raw else None))

    def average_last_two(self):
        """Every enabled case: state = mean of its last two steps' states."""
        _check(load().lbm_batch_average_last_two(self._h))

    def set_launch(self, rows_per_item=0, schedule=0):
        """rows_per_item: block height 4, 8 or 16 (0 = 4); schedule 0 graph
        of per-step kernels case after case, 1 tiles interleaved across
        cases, 2 persistent dataflow kernel."""
        _check(load().lbm_batch_set_launch(self._h, int(rows_per_item), int(schedule)))

    def run(self, tol, max_steps):
        """Run until every case's residual < tol (checked every check_every
        steps) or max_steps.  Returns the steps each case took; a case that
        diverged has its step count negated (and self.diverged is set)."""
        steps = np.zeros(self.n, dtype=np.int64)
        rc = load().lbm_batch_run(self._h, float(tol), int(max_steps),
                                  steps.ctypes.data_as(ctypes.c_void_p))
        self.diverged = rc == LBM_EUNSTABLE
        if rc not in (LBM_OK, LBM_EUNSTABLE):
            _check(rc)
        return steps

    def residual(self, c):
        r = ctypes.c_double()
        _check(load().lbm_batch_residual(self._h, int(c), ctypes.byref(r)))
        return r.value

    def set_plateau(self, checks, factor=0.9):
        _check(load().lbm_batch_set_plateau(self._h, int(checks), float(factor)))

    def status(self):
        st = np.zeros(self.n, dtype=np.int32)
        _check(load().lbm_batch_status(self._h, st.ctypes.data_as(ctypes.c_void_p)))
        return st

    def set_enabled(self, enabled=None):
        if enabled is None:
            _check(load().lbm_batch_set_enabled(self._h, None))
        else:
            e = np.ascontiguousarray(enabled, dtype=np.int32)
            _check(load().lbm_batch_set_enabled(self._h, e.ctypes.data_as(ctypes.c_void_p)))

    def set_storage(self, storage):
        st = STORAGE_NAMES[storage] if isinstance(storage, str) else int(storage)
        _check(load().lbm_batch_set_storage(self._h, st))

    def fields(self, c, ny, nx):
        out = [np.zeros((ny, nx)) for _ in range(3)]
        _check(load().lbm_batch_fields(self._h, int(c),
                                       *[o.ctypes.data_as(ctypes.c_void_p) for o in out]))
        return tuple(out)
