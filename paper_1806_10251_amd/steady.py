"""Run lattices to steady state: residual ||u^{n+1} - u^n|| / ||u^n|| < tol.

Two drivers with the same stopping rule (residual checked every check_every
steps): one lattice at a time (the plain method) and many lattices in one
persistent kernel (the batch).  Host logic only; every step runs in the HIP
library.

Precision: the one-step residual of an FP32-storage run stalls at its
rounding floor (about 1e-7 for cavities) and cannot reach 1e-8.  Half-way
bounce-back cavities carry non-decaying lattice-scale modes (present in the
uncorrected and the corrected scheme alike) that FP32 rounding keeps feeding,
so a later switch to FP64 does not remove the floor either.  Runs to 1e-8
therefore use FP64 storage from the start; FP32 runs can stop when their
residual stops improving (plateau rule) to report the floor.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import lbm as L


@dataclass
class SteadyResult:
    steps: int
    residual: float
    seconds: float
    status: str                      # "converged", "plateau", "max_steps" or "diverged"
    history: list = field(default_factory=list, repr=False)


def run_single(lat: L.Lattice, tol=1e-8, max_steps=2_000_000, check_every=100,
               plateau_checks=0, factor=0.9) -> SteadyResult:
    """Plain driver.  `lat` must have been created with this check_every.
    plateau_checks > 0 also stops when the residual has not dropped below
    factor * (best so far) for that many consecutive checks."""
    t0 = time.perf_counter()
    best, stall, steps = np.inf, 0, 0
    hist = []
    status = "max_steps"
    r = np.inf
    while steps < max_steps:
        lat.step(check_every)
        steps += check_every
        try:
            r = lat.residual
        except L.UnstableError:
            status = "diverged"
            break
        hist.append((steps, r))
        if steps < 2 * check_every:
            continue
        if r < tol:
            status = "converged"
            break
        if plateau_checks > 0:
            if r < best * factor:
                best, stall = r, 0
            else:
                stall += 1
                if stall >= plateau_checks:
                    status = "plateau"
                    break
    return SteadyResult(steps, float(r), time.perf_counter() - t0, status, hist)


def run_batch(batch: L.Batch, tol=1e-8, max_steps=2_000_000, plateau_checks=0, factor=0.9):
    """Batched driver.  Returns (steps, status, seconds): steps per case and
    status per case (1 converged, 2 plateau, 0 max_steps, 3 diverged)."""
    t0 = time.perf_counter()
    batch.set_enabled(None)
    batch.set_plateau(plateau_checks, factor)
    steps = batch.run(tol, max_steps)
    return np.abs(steps), batch.status(), time.perf_counter() - t0
