"""MI355X-native GI-corrected preconditioned cascaded central-moment D2Q9 LBM.

Hot path: hand-written HIP kernels for gfx950 behind the C ABI of
``include/lbm.h`` (``liblbm.so``, built in-tree by ``build.py``).  The Python
modules here only marshal arguments (``lbm``), pick launch shapes
(``autotune``) and drive the warm-start network (``surrogate``).
"""
from .lbm import (Batch, Lattice, LbmError, UnstableError, launch_shapes, load,  # noqa: F401
                  make_grid, make_params)

__all__ = ["Lattice", "Batch", "LbmError", "UnstableError", "load", "launch_shapes",
           "make_grid", "make_params"]
