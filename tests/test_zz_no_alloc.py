"""lbm_fields_noalloc (the entry point for callers that cannot allocate)
against lbm_fields, through the C ABI: two calls in a row on one lattice and
then on a smaller one, a lattice larger than one staging chunk (131072 nodes,
ragged last chunk), a subset of the fields, and the rejection of rows longer
than a chunk.  Collected last, so that a failure here hides no other test."""
import sys

import numpy as np
import pytest

from workloads import cavity_sides, periodic_sides

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


@pytest.mark.parametrize("nx,ny,storage,steps", [
    (300, 200, "f64", 40),      # one chunk
    (96, 64, "f32", 25),        # smaller, right after
    (1030, 530, "f32", 10),     # five chunks, last one ragged
    (70, 50, "bf16", 10),       # smaller again
])
def test_noalloc_fields_match_lbm_fields(lbm, nx, ny, storage, steps):
    _say(f"noalloc fields {nx}x{ny} {storage} {steps} steps")
    U = 0.1
    lat = lbm.Lattice(nx, ny, cavity_sides(), storage=storage, nu=U * nx / 400, gamma=0.5,
                      u_lid=U)
    lat.step(steps)
    for call in range(2):
        ref = lat.fields()
        out = lat.fields_noalloc()
        for a, b in zip(out, ref):
            np.testing.assert_array_equal(a, b)
        lat.step(1)
    ref = lat.fields()
    out = lat.fields_noalloc(rho=False, uy=False)
    assert out[0] is None and out[2] is None
    np.testing.assert_array_equal(out[1], ref[1])
    lat.close()


def test_noalloc_rejects_rows_longer_than_a_chunk(lbm):
    _say("noalloc rejection 131073 x 2")
    lat = lbm.Lattice(131073, 2, periodic_sides(), storage="f32", nu=0.05, gamma=1.0)
    with pytest.raises(lbm.LbmError) as e:
        lat.fields_noalloc()
    assert e.value.code == lbm.LBM_EINVAL
    assert "staging" in str(e.value)
    lat.close()
