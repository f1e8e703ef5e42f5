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
# Time to steady state of a case mix: the plain method (one case after
# another), the batch, and the batch with the two-step filter and the
# learned warm start.
# ---------------------------------------------------------------------------

def case_kw(k):
    """Lattice parameters of a drawn case (workloads.draw_cases)."""
    kw = {"u_lid": k.u_ref} if k.kind == "cavity" else {"u_in_max": k.u_ref}
    return dict(nu=k.nu, gamma=k.gamma, **kw)


def batch_arm(cases, tol, max_steps, storage="f64", choice=None, warm_net=None, filter_at=(),
              plateau=(0, 0.9), segment=None, log=None):
    """One batched run of every case to tol from rest (or from the
    network's prediction, computed inside the timed region), with optional
    filter steps.  segment: run in windows of that many steps, retiring
    finished cases between windows and logging each window.  With the warm
    start the run always goes in windows (10 000 steps unless segment is
    given): a predicted case that diverges is reset to rest inside the
    running batch at the end of its window and runs again with the same
    filter and a full step budget (the cold start is the fallback); its
    steps include the failed attempt.  Returns (steps, status, seconds,
    [(ux, uy)] per case)."""
    import torch

    from . import autotune, surrogate
    n = len(cases)
    if warm_net is not None and segment is None:
        segment = 10_000
    grids = [L.make_grid(k.nx, k.ny, k.sides) for k in cases]
    params = [L.make_params(storage=storage, check_every=100, **case_kw(k)) for k in cases]
    b = L.Batch(grids, [k.mask for k in cases], params)
    if choice is not None:
        autotune.apply_batch_choice(b, choice)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if warm_net is not None:
        surrogate.warm_init(warm_net, cases)(0, n, b)
    done = 0
    for at in filter_at:
        b.run(0.0, at - done)
        done = at
        b.average_last_two()
    if segment is None:
        steps, st, _ = run_batch(b, tol=tol, max_steps=max_steps - done,
                                 plateau_checks=plateau[0], factor=plateau[1])
        total = np.where(st == 3, steps, steps + done)
    else:
        taken = np.full(n, done, np.int64)      # steps each case has run in this arm
        limit = np.full(n, max_steps, np.int64)
        total = np.full(n, -1, np.int64)
        st = np.zeros(n, np.int32)
        active = np.ones(n, bool)
        restarted = np.zeros(n, bool)
        may_restart = np.array([warm_net is not None and surrogate.covers(k, warm_net)
                                for k in cases])

        def restart(idx):
            # back to rest inside the batch, with the arm's filter steps
            for i in idx:
                b.init_fields(int(i))
                restarted[i] = True
                limit[i] = taken[i] + max_steps
            en = np.zeros(n, np.int32)
            en[idx] = 1
            b.set_enabled(en)
            d = 0
            for at in filter_at:
                b.run(0.0, at - d)
                d = at
                b.average_last_two()
            taken[idx] += d
            now = b.status() if filter_at else np.zeros(n, np.int32)
            for i in idx:
                if now[i] == 3:                  # diverges from rest as well
                    total[i], st[i], active[i] = taken[i], 3, False
            if log:
                log(f"[tts] {len(idx)} warm-started case(s) diverged; reset to rest in the batch")

        if warm_net is not None and filter_at:
            now = b.status()
            first = [i for i in range(n) if now[i] == 3 and may_restart[i]]
            if first:
                restart(np.array(first))
        while True:
            for i in np.flatnonzero(active):
                if taken[i] >= limit[i]:
                    total[i], st[i], active[i] = taken[i], 0, False
            if not active.any():
                break
            m = int(min(segment, (limit - taken)[active].min()))
            b.set_enabled(active.astype(np.int32))
            b.set_plateau(*plateau)
            steps = b.run(tol, m)
            now = b.status()
            again = []
            for i in np.flatnonzero(active):
                if now[i] in (1, 2, 3):
                    taken[i] += abs(int(steps[i]))
                    if now[i] == 3 and may_restart[i] and not restarted[i]:
                        again.append(i)
                        continue
                    total[i], st[i], active[i] = taken[i], now[i], False
                else:
                    taken[i] += m
            if again:
                restart(np.array(again))
            if log:
                log(f"[tts] window of {m} steps: {int((~active).sum())}/{n} cases retired, "
                    f"{time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    fields = [b.fields(i, k.ny, k.nx)[1:] for i, k in enumerate(cases)]
    b.close()
    return total, st, sec, fields


_STATUS = {1: "converged", 3: "diverged", 0: "max_steps", 2: "plateau"}


def plain_arm(cases, tol, max_steps, storage="f64", log=None):
    """Every case on its own lattice, one after another, from rest.
    Returns (steps, status codes as in run_batch, seconds, fields)."""
    import torch
    code = {v: k for k, v in _STATUS.items()}
    steps, status, fields, sec = [], [], [], 0.0
    for i, k in enumerate(cases):
        if log and i % 16 == 0:
            log(f"[tts] plain: case {i}/{len(cases)}, {sec:.1f} s")
        lat = L.Lattice(k.nx, k.ny, k.sides, solid=k.mask, storage=storage, check_every=100,
                        **case_kw(k))
        torch.cuda.synchronize()
        r = run_single(lat, tol=tol, max_steps=max_steps)
        fields.append(lat.fields()[1:])
        lat.close()
        sec += r.seconds
        steps.append(r.steps)
        status.append(code[r.status])
    return np.array(steps), np.array(status, np.int32), sec, fields


def max_error(cases, fields, ref, which):
    """max |u - u_ref| / U over the cases in which (None if empty)."""
    errs = [max(np.abs(fields[i][0] - ref[i][0]).max(), np.abs(fields[i][1] - ref[i][1]).max()) /
            cases[i].u_ref for i in which]
    return float(max(errs)) if errs else None


def arm_summary(name, cases, steps, status, sec, fields, ref=None, ref_ok=None, base_s=None):
    """JSON-ready summary of one arm: seconds, total steps, outcome counts,
    and the error against the reference fields over the cases converged in
    both."""
    out = {"arm": name, "seconds": round(sec, 3), "steps": int(np.sum(steps)),
           "status": {_STATUS[c]: int((status == c).sum()) for c in sorted(set(status.tolist()))}}
    if ref is not None:
        ok = [i for i in range(len(cases)) if status[i] == 1 and ref_ok[i]]
        out["max_err"] = max_error(cases, fields, ref, ok)
        out["compared_cases"] = len(ok)
    if base_s:
        out["speedup_vs_plain"] = round(base_s / sec, 3)
    return out


# ---------------------------------------------------------------------------
# Convergence acceleration by preconditioning# ---------------------------------------------------------------------------
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


def mix_time_to_steady(n_cases=256, side_lo=64, side_hi=512, seed=1806, tol=1e-8,
                       max_steps=100_000, storage="f64", arms=("plain", "batch"), weights=None,
                       segment=10_000, log=print):
    """Time to steady state of the seeded batched mix (workloads.draw_cases):
    each arm in `arms` runs every case to tol (at most max_steps steps) from
    rest or from the learned warm start.  Arms: "plain" (one lattice after
    another), "batch", "batch+filter" (two-step filter of the warm start on a
    cold start), "batch+surrogate" (warm start and filter).  Errors are
    max |u - u_ref| / U against the first arm's fields, over the cases
    converged in both.  Batch arms run in windows of `segment` steps.
    Returns a JSON-ready dict."""

    from . import autotune, surrogate
    from . import unet as U
    from workloads import draw_cases
    cases = draw_cases(n_cases, seed, side_lo=side_lo, side_hi=side_hi)
    nodes = int(sum(k.nx * k.ny for k in cases))
    log(f"[tts] {n_cases} cases, {nodes} nodes, storage {storage}, tol {tol:g}, "
        f"at most {max_steps} steps")
    grids = [L.make_grid(k.nx, k.ny, k.sides) for k in cases]
    masks = [k.mask for k in cases]
    params = [L.make_params(storage=storage, check_every=100, **case_kw(k)) for k in cases]
    choice, _ = autotune.tune_batch(grids, masks, params, steps=200)
    net = None
    if any(a == "batch+surrogate" for a in arms):
        net = U.UNet(max_batch=16, res=surrogate.RES, seed=0)
        surrogate.load_into(net, weights or surrogate.DEFAULT_WEIGHTS)
    results, ref, ref_ok, base_s = [], None, None, None
    for a in arms:
        seg = dict(segment=segment, log=log)
        if a == "plain":
            r = plain_arm(cases, tol, max_steps, storage, log=log)
        elif a == "batch":
            r = batch_arm(cases, tol, max_steps, storage, choice, **seg)
        elif a == "batch+filter":
            r = batch_arm(cases, tol, max_steps, storage, choice, filter_at=surrogate.WARM_FILTER,
                          **seg)
        elif a == "batch+surrogate":
            r = batch_arm(cases, tol, max_steps, storage, choice, warm_net=net,
                          filter_at=surrogate.WARM_FILTER, **seg)
        else:
            raise ValueError(f"unknown arm {a!r}")
        steps, st, sec, fields = r
        if ref is None:
            ref, ref_ok = fields, st == 1
        if a == "plain":
            base_s = sec
        results.append(arm_summary(a, cases, steps, st, sec, fields, ref, ref_ok, base_s))
        log(f"[tts] {results[-1]}")
    if net is not None:
        net.close()
    return {"cases": n_cases, "nodes": nodes, "seed": seed, "tol": tol, "storage": storage,
            "max_steps": max_steps,
            "sample": f"seeded mix (seed {seed}) of cavities s x s and channels 4s x s, s in "
                      f"[{side_lo}, {side_hi}], 1-4 rectangular obstacles covering 5-20%, Re in "
                      "[50, 1000], gamma log-uniform in [0.05, 1]",
            "batch_launch": {"block_height": choice[0], "schedule": choice[1]},
            "error_reference": f"fields of the {arms[0]} arm", "arms": results}


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="steps to steady state against gamma; time to "
                                             "steady state of the batched mix")
    ap.add_argument("cmd", choices=["sweep", "tts"])
    ap.add_argument("--cases", type=int, default=256, help="tts: number of cases")
    ap.add_argument("--side-lo", type=int, default=64)
    ap.add_argument("--side-hi", type=int, default=512)
    ap.add_argument("--seed", type=int, default=1806)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--arms", default="plain,batch,batch+filter,batch+surrogate")
    ap.add_argument("--kind", choices=["cavity", "cylinder"], default="cavity")
    ap.add_argument("--size", type=int, default=400, help="cavity side or cylinder D")
    ap.add_argument("--re", type=float, default=3200.0)
    ap.add_argument("--mach", type=float, default=0.05,
                    help="reference speed in lattice sound speeds (u = mach / sqrt 3)")
    ap.add_argument("--gammas", default="1,0.5,0.2,0.1,0.05")
    ap.add_argument("--tols", default="1e-6,1e-8")
    ap.add_argument("--storage", default="f64")
    ap.add_argument("--max-steps", type=int, default=None,
                    help="sweep: 4000000 by default; tts: 100000 by default")
    a = ap.parse_args(argv)
    if a.cmd == "tts":
        import sys
        import torch
        if not torch.cuda.is_available():
            sys.exit("needs a GPU")
        L.load()
        out = mix_time_to_steady(a.cases, a.side_lo, a.side_hi, a.seed, a.tol,
                                 a.max_steps or 100_000,
                                 a.storage, tuple(a.arms.split(",")),
                                 log=lambda m: print(m, file=sys.stderr, flush=True))
        print(json.dumps(out), flush=True)
        return
    u = a.mach / np.sqrt(3.0)
    gammas = [float(x) for x in a.gammas.split(",")]
    tols = [float(x) for x in a.tols.split(",")]
    for g in gammas:
        row = gamma_sweep(a.kind, a.size, a.re, u, [g], tols, a.storage,
                          a.max_steps or 4_000_000)[0]
        print(json.dumps(row), flush=True)


if __name__ == "__main__":
    main()
