"""The C ABI library without a GPU: it loads, exports every function the
header declares, and rejects invalid arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1806_10251_amd import lbm
    if not os.path.exists(lbm.LIB_PATH):
        pytest.skip("liblbm.so not built")
    return lbm, lbm.load()


def test_header_declares_the_binding_surface(lib):
    lbm, _ = lib
    assert declared_functions() == sorted(lbm.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    lbm, _ = lib
    raw = ctypes.CDLL(lbm.LIB_PATH)
    missing = [f for f in declared_functions() if not hasattr(raw, f)]
    assert not missing, missing


def declared_unet_functions():
    text = open(os.path.join(ROOT, "include", "unet.h")).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    return sorted(set(re.findall(r"\b(unet_\w+)\s*\(", text)))


def test_library_exports_every_network_symbol(lib):
    """include/unet.h: every declared function is exported by the same
    library and has a ctypes signature in the binding."""
    from paper_1806_10251_amd import unet
    lbm, _ = lib
    raw = ctypes.CDLL(lbm.LIB_PATH)
    names = declared_unet_functions()
    assert "unet_make_input_rect" in names and "unet_train_step" in names
    missing = [f for f in names if not hasattr(raw, f)]
    assert not missing, missing
    L = unet.load()
    for f in names:
        assert getattr(L, f).argtypes is not None, f


def test_launch_shapes_are_listed(lib):
    lbm, _ = lib
    shapes = lbm.launch_shapes()
    assert len(shapes) >= 4
    for by, rows in shapes:
        assert 64 * by <= 1024 and rows >= 1


def _create(L, lbm, nx=16, ny=16, sides=(1, 1, 1, 2), mask=None, **kw):
    grid = lbm.make_grid(nx, ny, sides)
    p = lbm.make_params(**{"nu": 0.01, "gamma": 0.5, "u_lid": 0.1, **kw})
    h = ctypes.c_void_p()
    mp = None if mask is None else np.ascontiguousarray(mask, np.uint8).ctypes.data
    return L.lbm_create(ctypes.byref(grid), mp, ctypes.byref(p), ctypes.byref(h))


@pytest.mark.parametrize("kw,sides", [
    (dict(gamma=0.0), (1, 1, 1, 2)),                 # gamma must be positive
    (dict(gamma=1.5), (1, 1, 1, 2)),                 # ... and at most 1
    (dict(nu=-0.1), (1, 1, 1, 2)),                   # omega4 outside (0, 2)
    (dict(), (0, 1, 1, 2)),                          # periodic W without periodic E
    (dict(storage="f16", storage_scale=3000.0), (1, 1, 1, 2)),   # scale not 2^k
    (dict(check_every=0), (1, 1, 1, 2)),
])
def test_invalid_configurations_are_rejected(lib, kw, sides):
    lbm, L = lib
    rc = _create(L, lbm, sides=sides, **kw)
    assert rc == lbm.LBM_EINVAL
    assert L.lbm_last_error()


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_lattices_over_4_gib_are_rejected(lib, storage):
    """One lattice is addressed with 32-bit byte offsets: 12000^2 nodes need
    5.3 GB in FP32 (nine framed planes) and are refused before any device
    work."""
    lbm, L = lib
    rc = _create(L, lbm, nx=12000, ny=12000, storage=storage)
    assert rc == lbm.LBM_EINVAL
    assert b"2^32 bytes" in L.lbm_last_error()


def test_all_solid_mask_is_rejected(lib):
    lbm, L = lib
    assert _create(L, lbm, mask=np.ones((16, 16))) == lbm.LBM_EINVAL


def test_null_handles_are_rejected(lib):
    lbm, L = lib
    r = ctypes.c_double()
    assert L.lbm_step(None, 1) == lbm.LBM_EINVAL
    assert L.lbm_residual(None, ctypes.byref(r)) == lbm.LBM_EINVAL
    assert L.lbm_batch_run(None, 1e-8, 10, None) == lbm.LBM_EINVAL
