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


# ---------------------------------------------------------------------------
# Convergence acceleration by preconditioning (Sec. 6: the lid-driven cavity
# at Re = 3200 and the square cylinder at Re = 30 reach their steady states
# faster as gamma falls).
# ---------------------------------------------------------------------------

def sweep_lattice(kind, size, re, u, gamma, storage="f64", check_every=100):
    """One lattice of the sweep.  cavity: size x size fluid nodes, lid speed
    u, Re = u size / nu.  cylinder: square cylinder of side D = size on the
    channel centre line, 12.5 D from the inlet, in a 50 D x 8 D channel with
    a parabolic inlet of peak u, Re = u D / nu."""
    if kind == "cavity":
        nu = u * size / re
        sides = (L.WALL, L.WALL, L.WALL, L.LID)
        return L.Lattice(size, size, sides, storage=storage, check_every=check_every,
                         nu=nu, gamma=gamma, u_lid=u)
    if kind == "cylinder":
        D = size
        nx, ny = 50 * D, 8 * D
        x0, y0 = int(round(12.5 * D - D / 2)), ny // 2 - D // 2
        mask = np.zeros((ny, nx), np.uint8)
        mask[y0:y0 + D, x0:x0 + D] = 1
        sides = (L.INLET, L.OUTLET, L.WALL, L.WALL)
        return L.Lattice(nx, ny, sides, solid=mask, storage=storage, check_every=check_every,
                         nu=u * D / re, gamma=gamma, u_in_max=u)
    raise ValueError(f"unknown kind {kind!r}")


def gamma_sweep(kind, size, re, u, gammas, tols=(1e-6, 1e-8), storage="f64",
                max_steps=4_000_000, check_every=100):
    """Steps (and seconds) until the residual first falls below each of tols,
    for each gamma, from the state at rest.  Returns one dict per gamma."""
    out = []
    for g in gammas:
        lat = sweep_lattice(kind, size, re, u, g, storage=storage, check_every=check_every)
        res = run_single(lat, tol=min(tols), max_steps=max_steps, check_every=check_every)
        first = {}
        for t in tols:
            hit = next((s for s, r in res.history if s >= 2 * check_every and r < t), None)
            first[f"{t:g}"] = hit
        out.append({"kind": kind, "size": size, "re": re, "u": u, "gamma": g,
                    "storage": storage, "status": res.status, "steps": res.steps,
                    "residual": res.residual, "seconds": round(res.seconds, 3),
                    "steps_to": first})
        lat.close()
    return out


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="steps to steady state against gamma")
    ap.add_argument("cmd", choices=["sweep"])
    ap.add_argument("--kind", choices=["cavity", "cylinder"], default="cavity")
    ap.add_argument("--size", type=int, default=400, help="cavity side or cylinder D")
    ap.add_argument("--re", type=float, default=3200.0)
    ap.add_argument("--mach", type=float, default=0.05,
                    help="reference speed in lattice sound speeds (u = mach / sqrt 3)")
    ap.add_argument("--gammas", default="1,0.5,0.2,0.1,0.05")
    ap.add_argument("--tols", default="1e-6,1e-8")
    ap.add_argument("--storage", default="f64")
    ap.add_argument("--max-steps", type=int, default=4_000_000)
    a = ap.parse_args(argv)
    u = a.mach / np.sqrt(3.0)
    gammas = [float(x) for x in a.gammas.split(",")]
    tols = [float(x) for x in a.tols.split(",")]
    for g in gammas:
        row = gamma_sweep(a.kind, a.size, a.re, u, [g], tols, a.storage, a.max_steps)[0]
        print(json.dumps(row), flush=True)


if __name__ == "__main__":
    main()
