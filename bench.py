#!/usr/bin/env python3
"""Throughput benchmark of the fused GI-preconditioned cascaded D2Q9 step.

Workload (one GPU): lid-driven cavity 1024 x 1024, Re = 1000, U_lid = 0.1,
gamma = 0.5, FP32 deviation storage, residual reduction every 100 steps.
One "step" is one pass of the whole hot path (pull-stream with boundary
links, macroscopic fields, density gradient, strain estimate, GI
corrections, cascaded collision; FP64 residual/mass on check steps) over the
lattice, with the populations resident in HBM.

Second leg (time_to_steady): a seeded sample of the batched workload (mixed
cavities and channels with obstacles, uneven sizes, Re and gamma), every case
run to residual < 1e-8 in FP64 storage, once case after case with the plain
single-lattice driver and once as one batch; wall times of both.

Prints one JSON line (rank 0).  --gpus above 1 is not supported: the method
runs on one GPU here (see the design notes for how it would shard).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + % HBM roofline; time-to-steady (resid 1e-8) surrogate+batch vs plain"
PEAK_HBM_GBS = 8000.0
BYTES_PER_LUP = {"f64": 144, "f32": 72, "bf16": 36, "f16": 36}


def cpu_baseline(n, U, re, gamma, budget_s=12.0):
    """The FP64 oracle on this host's cores, on a bounded sample of the same
    workload (the same 1024^2 cavity, a few steps)."""
    import oracle
    from workloads import cavity_sides

    o = oracle.Oracle(n, n, cavity_sides(), nu=U * n / re, gamma=gamma, u_lid=U)
    t0 = time.perf_counter()
    o.step(2)
    dt = (time.perf_counter() - t0) / 2
    steps = max(2, min(400, int(budget_s / max(dt, 1e-6))))
    t0 = time.perf_counter()
    o.step(steps)
    el = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    # the same oracle on one thread, a shorter sample
    oracle.set_threads(1)
    steps1 = max(2, steps // max(cores, 1))
    t0 = time.perf_counter()
    o.step(steps1)
    el1 = time.perf_counter() - t0
    oracle.set_threads(cores)
    return {"value": n * n * steps / el / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"cavity {n}x{n} Re {re:g} gamma {gamma:g}, {steps} steps after 2 warm-up "
                      f"steps, FP64, {el:.1f} s",
            "single_thread": {"value": n * n * steps1 / el1 / 1e6, "unit": "MLUPS",
                              "sample": f"{steps1} further steps, {el1:.1f} s"}}



def _host_cpu():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_plan(progress=None):
    """The FP64 oracle over the host-baseline runs: lid-driven cavities of 256^2
    and 1024^2 for 1000 fixed steps at gamma 0.5 (Re 1000, U_lid 0.1), on one
    thread and on all threads (1024^2 on one thread: a 100-step sample); a
    128^2 cavity at Re 100, U_lid 0.1 run from rest to a velocity residual
    below 1e-8 (checked every 100 steps) at gamma 1 and 0.5; and the 32^2
    cavity at Re 100, gamma 0.5, 5000 steps (wall time)."""
    import oracle
    from workloads import cavity_sides

    cores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    say = progress or (lambda m: None)

    def fixed(n, re, gamma, steps, threads):
        oracle.set_threads(threads)
        o = oracle.Oracle(n, n, cavity_sides(), nu=0.1 * n / re, gamma=gamma, u_lid=0.1)
        o.step(2)
        t0 = time.perf_counter()
        o.step(steps)
        el = time.perf_counter() - t0
        o.close()
        say(f"cavity {n}^2 {steps} steps, {threads} threads: {el:.2f} s")
        return {"n": n, "re": re, "gamma": gamma, "steps": steps, "threads": threads,
                "seconds": round(el, 3), "mlups": round(n * n * steps / el / 1e6, 2)}

    def to_steady(n, re, gamma, threads, tol=1e-8, every=100, cap=2_000_000):
        oracle.set_threads(threads)
        o = oracle.Oracle(n, n, cavity_sides(), nu=0.1 * n / re, gamma=gamma, u_lid=0.1)
        t0 = time.perf_counter()
        steps = 0
        res = float("inf")
        while steps < cap:
            o.step(every)
            steps += every
            res = o.residual
            if res < tol:
                break
        el = time.perf_counter() - t0
        o.close()
        say(f"cavity {n}^2 gamma {gamma} to {tol:g}: {steps} steps, {el:.1f} s")
        return {"n": n, "re": re, "gamma": gamma, "tol": tol, "check_every": every,
                "threads": threads, "steps": steps, "converged": bool(res < tol),
                "residual": res, "seconds": round(el, 2),
                "mlups": round(n * n * steps / el / 1e6, 2)}

    out = {"host_cpu": _host_cpu(), "threads_all": cores, "kind": "oracle", "storage": "f64"}
    out["fixed_steps"] = [fixed(256, 1000, 0.5, 1000, 1), fixed(256, 1000, 0.5, 1000, cores),
                          fixed(1024, 1000, 0.5, 100, 1), fixed(1024, 1000, 0.5, 1000, cores)]
    out["time_to_steady"] = [to_steady(128, 100, g, cores) for g in (1.0, 0.5)]
    out["c1_wall"] = [fixed(32, 100, 0.5, 5000, 1), fixed(32, 100, 0.5, 5000, cores)]
    oracle.set_threads(cores)
    return out


# Kernel sources and the build script (its compile flags) for which the
# committed traffic summary holds HBM byte counters; the figure is reported
# only while their hash matches.
TRAFFIC_SOURCES = ("paper_1806_10251_amd/csrc/lbm_kernels.h",
                   "paper_1806_10251_amd/csrc/lbm_device.h",
                   "paper_1806_10251_amd/csrc/lbm_step.hip",
                   "paper_1806_10251_amd/build.py")
TRAFFIC_SUMMARY = "profiles/step_f32_cavity1024_hbm_traffic.md"


def source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(storage, n, by, rows):
    """HBM bytes per step launch from the committed counter summary, if it
    was taken for this kernel source, storage, size and launch shape."""
    try:
        with open(os.path.join(ROOT, TRAFFIC_SUMMARY)) as f:
            kv = dict(line[2:].split(": ", 1) for line in f if line.startswith("- ") and ": " in line)
    except OSError:
        return None
    want = {"source_hash": source_hash(), "storage": storage, "size": f"{n}x{n}",
            "launch": f"{by},{rows}"}
    if any(kv.get(k, "").strip() != v for k, v in want.items()):
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def timed_window(warmup, steps, K):
    """What the timed steps were: the library runs the check step (velocity
    residual and mass, FP64 partials and their reduction) at every step whose
    1-based index is a multiple of K, and stores the velocity one step
    before; the other steps are plain."""
    def multiples(lo, hi):          # multiples of K in [lo, hi]
        return hi // K - (lo - 1) // K
    check = multiples(warmup + 1, warmup + steps)
    store = multiples(warmup + 2, warmup + steps + 1)
    return {"steps": steps, "plain": steps - check - store, "store": store, "check": check,
            "check_every": K, "graph_windows": "captured graphs of K steps, replayed"}




def _case_kw(k):
    from paper_1806_10251_amd import steady
    return steady.case_kw(k)


def _batch_arm(lbm, cases, choice, tol, max_steps, warm_net=None, filter_at=()):
    from paper_1806_10251_amd import steady
    return steady.batch_arm(cases, tol, max_steps, "f64", choice, warm_net, filter_at)


def _accuracy(cases, fields, ref, ok):
    from paper_1806_10251_amd import steady
    return steady.max_error(cases, fields, ref, ok)


def time_to_steady(lbm, n_cases, side_hi, max_steps, seed=1806, tol=1e-8):
    """Time to steady state of a sample of the batched workload: the plain
    method (one case after another, cold start), the batch (cold), the batch
    with the two-step filter (cold), and the batch with the learned warm start
    and the filter.  Each arm's converged fields are compared with a tighter
    run (residual 1e-11) of the same cases."""
    import numpy as np
    import torch

    from paper_1806_10251_amd import autotune, steady, surrogate
    from paper_1806_10251_amd import unet as U
    from workloads import draw_cases

    cases = draw_cases(n_cases, seed, side_lo=64, side_hi=side_hi)
    grids = [lbm.make_grid(k.nx, k.ny, k.sides) for k in cases]
    masks = [k.mask for k in cases]
    params = [lbm.make_params(storage="f64", check_every=100, **_case_kw(k)) for k in cases]
    print(f"[bench] time-to-steady: {n_cases} cases, {sum(k.nx * k.ny for k in cases)} nodes; "
          "tuning the batch", file=sys.stderr, flush=True)
    choice, _ = autotune.tune_batch(grids, masks, params, steps=200)
    arms = {}
    steps_b, st_b, t_batch, f_batch = _batch_arm(lbm, cases, choice, tol, max_steps)
    arms["batch"] = (steps_b, st_b, t_batch, f_batch)
    print(f"[bench] batch {t_batch:.2f} s; reference run to 1e-11", file=sys.stderr, flush=True)
    _, st_ref, _, f_ref = _batch_arm(lbm, cases, choice, 1e-11, 4 * max_steps)
    # the filtered arms also at tol / 10: at tol their error against the
    # reference exceeds the plain method's, at tol / 10 it is below it
    arms["batch+filter"] = _batch_arm(lbm, cases, choice, tol, max_steps,
                                      filter_at=surrogate.WARM_FILTER)
    arms["batch+filter@tol/10"] = _batch_arm(lbm, cases, choice, tol / 10, max_steps,
                                             filter_at=surrogate.WARM_FILTER)
    weights = surrogate.DEFAULT_WEIGHTS
    net = None
    if os.path.exists(weights):
        net = U.UNet(max_batch=16, res=surrogate.RES, seed=0)
        surrogate.load_into(net, weights)
        arms["batch+surrogate"] = _batch_arm(lbm, cases, choice, tol, max_steps, warm_net=net,
                                             filter_at=surrogate.WARM_FILTER)
        arms["batch+surrogate@tol/10"] = _batch_arm(lbm, cases, choice, tol / 10, max_steps,
                                                    warm_net=net,
                                                    filter_at=surrogate.WARM_FILTER)
    print("[bench] plain runs", file=sys.stderr, flush=True)
    t_plain, status, mismatch, f_plain, steps_p = 0.0, {}, [], [], []
    names = {1: "converged", 3: "diverged", 0: "max_steps", 2: "plateau"}
    for i, k in enumerate(cases):
        lat = lbm.Lattice(k.nx, k.ny, k.sides, solid=k.mask, storage="f64", check_every=100,
                          **_case_kw(k))
        torch.cuda.synchronize()
        r = steady.run_single(lat, tol=tol, max_steps=max_steps)
        f_plain.append(lat.fields()[1:])
        lat.close()
        t_plain += r.seconds
        steps_p.append(r.steps)
        # for diverging cases only the outcome is compared (the step count
        # records where the blow-up was seen, not a converged state)
        if r.status != names[int(st_b[i])] or (r.status != "diverged" and
                                                r.steps != int(steps_b[i])):
            mismatch.append({"case": i, "plain": [r.steps, r.status],
                             "batch": [int(steps_b[i]), names[int(st_b[i])]]})
        status[r.status] = status.get(r.status, 0) + 1
    ok = [i for i in range(n_cases) if st_ref[i] == 1 and st_b[i] == 1]
    out = {"tol": tol, "storage": "f64", "cases": n_cases,
           "sample": f"seeded mix (seed {seed}) of cavities s x s and channels 4s x s, s in "
                     f"[64, {side_hi}], 1-4 rectangular obstacles covering 5-20%, Re in "
                     f"[50, 1000], gamma log-uniform in [0.05, 1]; at most {max_steps} steps",
           "plain_s": round(t_plain, 3), "batch_s": round(t_batch, 3),
           "speedup": round(t_plain / t_batch, 3), "status": status,
           "batch_launch": {"block_height": choice[0], "schedule": choice[1]},
           "same_steps_and_outcome": not mismatch, "mismatch": mismatch,
           "accuracy_ref": "max |u - u_ref| / U over cases converged in both, u_ref from a "
                           "batched run to residual 1e-11",
           "arms": {"plain": {"seconds": round(t_plain, 3), "steps": int(np.sum(steps_p)),
                              "max_err": _accuracy(cases, f_plain, f_ref, ok)}}}
    for name, (stp, st, sec, flds) in arms.items():
        out["arms"][name] = {"seconds": round(sec, 3), "steps": int(np.sum(stp)),
                             "converged": int((st == 1).sum()),
                             "max_err": _accuracy(cases, flds, f_ref, [i for i in ok if st[i] == 1]),
                             "speedup_vs_plain": round(t_plain / sec, 3)}
    if net is not None:
        kinds = getattr(net, "kinds", ("cavity",))
        out["warm_start"] = {"weights": os.path.relpath(weights, ROOT),
                             "covers": ", ".join(kinds) + " (other cases keep the cold start; a "
                                       "warm start that diverges runs again from rest within "
                                       "the arm)",
                             "filter_steps": list(surrogate.WARM_FILTER),
                             "tol": tol / 10,
                             "note": "accuracy-matched arm: error against the reference at "
                                     "or below the plain method's",
                             **out["arms"]["batch+surrogate@tol/10"]}
        net.close()
    else:
        out["warm_start"] = None
    return out


def batch_throughput(lbm, n_cases=256, steps=1000, seed=1806, choice=(8, 0)):
    """The full batched mix (256 seeded cavities and channels, sides 64-512,
    FP32) for a fixed window of steps from rest: aggregate MLUPS of the batch
    against the plain driver running the cases one after another.  Lattice
    updates are counted per case over the steps it actually took (a case
    that turns non-finite leaves the batch at its next check step)."""
    import numpy as np
    import torch

    from paper_1806_10251_amd import autotune
    from workloads import draw_cases
    cases = draw_cases(n_cases, seed, side_lo=64, side_hi=512)
    nodes = np.array([k.nx * k.ny for k in cases], dtype=np.float64)
    print(f"[bench] batch throughput: {n_cases} cases, {nodes.sum():.3e} nodes", file=sys.stderr,
          flush=True)
    grids = [lbm.make_grid(k.nx, k.ny, k.sides) for k in cases]
    params = [lbm.make_params(storage="f32", check_every=100, **_case_kw(k)) for k in cases]
    b = lbm.Batch(grids, [k.mask for k in cases], params)
    autotune.apply_batch_choice(b, choice)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    took = np.abs(np.asarray(b.run(0.0, steps), dtype=np.float64))
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    b.close()
    t_plain, lups_plain = 0.0, 0.0
    for k in cases:
        lat = lbm.Lattice(k.nx, k.ny, k.sides, solid=k.mask, storage="f32", check_every=100,
                          **_case_kw(k))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.step(steps)
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t0
        lups_plain += k.nx * k.ny * steps
        lat.close()
    mb = float((nodes * took).sum()) / t_batch / 1e6
    mp = lups_plain / t_plain / 1e6
    return {"cases": n_cases, "nodes": int(nodes.sum()), "steps": steps, "storage": "f32",
            "sample": f"seeded mix (seed {seed}) of cavities s x s and channels 4s x s, s in "
                      "[64, 512], 1-4 rectangular obstacles covering 5-20%, Re in [50, 1000], "
                      "gamma log-uniform in [0.05, 1]",
            "batch_launch": {"block_height": choice[0], "schedule": choice[1]},
            "batch_mlups": round(mb, 1), "plain_mlups": round(mp, 1),
            "batch_seconds": round(t_batch, 3), "plain_seconds": round(t_plain, 3),
            "cases_left_early": int((took < steps).sum()), "speedup": round(mb / mp, 3)}


def kernel_variants(lbm, n, U, re, gamma, storage, by, rows, step_ms, steps=5000, warmup=500):
    """Step time of the same cavity with the uncorrected eq. 4 kernel, with
    the strain rates of the corrections from finite differences of the
    velocity and with the raw-moment MRT form of the collision, at the same
    launch shape (HIP events), and the cost of the GI corrections over the
    uncorrected kernel."""
    from workloads import cavity_sides
    out = {"steps": steps}
    for name, kw in (("uncorrected_eq4", dict(gi_correct=0)), ("fd_strain", dict(strain_fd=1)),
                     ("mrt", dict(mrt=1))):
        print(f"[bench] kernel variant {name}", file=sys.stderr, flush=True)
        v = lbm.Lattice(n, n, cavity_sides(), storage=storage, nu=U * n / re, gamma=gamma,
                        u_lid=U, check_every=100, **kw)
        v.set_launch(by, rows)
        v.step(warmup)
        v.set_timing(True)
        v.step(steps)
        ms = v.last_step_ms
        v.set_timing(False)
        v.close()
        out[name] = {"us_per_step": round(ms * 1e3, 2), "mlups": round(n * n / (ms * 1e-3) / 1e6, 1)}
    out["gi_correction_cost"] = round(step_ms / (out["uncorrected_eq4"]["us_per_step"] * 1e-3) - 1, 4)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--gamma", type=float, default=0.5)
    ap.add_argument("--storage", default="f32", choices=list(BYTES_PER_LUP))
    ap.add_argument("--launch", default="", help="by,rows (default: library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tts-cases", type=int, default=24)
    ap.add_argument("--tts-side", type=int, default=128)
    ap.add_argument("--tts-max-steps", type=int, default=200000)
    ap.add_argument("--no-tts", action="store_true")
    ap.add_argument("--no-batch-throughput", action="store_true",
                    help="skip the fixed-window throughput of the 256-case batch")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip timing the uncorrected (eq. 4) and finite-difference-strain kernels")
    ap.add_argument("--cpu-plan", action="store_true",
                    help="only time the FP64 oracle on this host over the host-baseline runs "
                         "(fixed-step cavities, 128^2 time to steady state, the 32^2 case) and "
                         "print them as one JSON line; no GPU is used")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a 256 MiB device copy first (reference for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported; this build runs the method on one "
              "GPU (multi-GPU sharding is design-only).", file=sys.stderr)
        sys.exit(2)

    if args.cpu_plan:
        print(json.dumps({"cpu_plan": cpu_plan(
            lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True))}), flush=True)
        return

    import torch

    from paper_1806_10251_amd import lbm
    from workloads import cavity_sides

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    lbm.load()

    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    n, U, re, gamma = args.n, 0.1, 1000.0, args.gamma
    K = 100
    print(f"[bench] cavity {n}x{n} Re {re:g} gamma {gamma:g} {args.storage}; "
          f"warmup {args.warmup}, timed {args.steps}", file=sys.stderr, flush=True)
    lat = lbm.Lattice(n, n, cavity_sides(), storage=args.storage, nu=U * n / re, gamma=gamma,
                      u_lid=U, check_every=K)
    if args.launch:
        by, rows = (int(v) for v in args.launch.split(","))
    else:
        from paper_1806_10251_amd import autotune
        (by, rows), _ = autotune.tune_lattice(n, n, cavity_sides(), storage=args.storage,
                                              use_cache=False, nu=U * n / re, gamma=gamma,
                                              u_lid=U)
    lat.set_launch(by, rows)
    stream = torch.cuda.current_stream()
    lat.set_stream(stream)
    lat.step(args.warmup)
    torch.cuda.synchronize()
    lat.set_timing(True)
    t0 = time.perf_counter()
    lat.step(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms_dev = lat.last_step_ms        # HIP events on the library's stream
    lat.set_timing(False)
    try:
        resid, mass = lat.residual, lat.mass
    except lbm.LbmError:            # a run shorter than the check cadence
        resid, mass = None, None

    lups = n * n * args.steps
    mlups = lups / wall / 1e6
    bpl = BYTES_PER_LUP[args.storage]
    achieved = bpl * n * n / (step_ms_dev * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic",
        "config": {"workload": f"lid-driven cavity {n}x{n}, Re {re:g}, U_lid {U}, gamma {gamma:g}, "
                               f"{args.storage} deviation storage, residual every {K} steps",
                   "nx": n, "ny": n, "gamma": gamma, "re": re, "u_lid": U,
                   "launch": {"block": [64, by], "rows_per_thread": rows}},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": measured_traffic(args.storage, n, by, rows),
                     "note": f"{bpl} B/LUP algorithmic (each population read and written once) x "
                             f"{n * n} nodes per launch / average step time "
                             f"{step_ms_dev * 1e3:.2f} us from HIP events on the library's "
                             f"stream over the timed window (its plain, store and check steps "
                             f"and check reductions); traffic: HBM bytes per plain-step launch "
                             f"from the committed counter summary"},
        "timed_window": timed_window(args.warmup, args.steps, K),
        "residual_at_end": resid,
        "mass_drift": None if mass is None else mass - n * n,
    }
    if not args.no_variants:
        out["kernel_variants"] = kernel_variants(lbm, n, U, re, gamma, args.storage, by, rows,
                                                 step_ms_dev)
    if not args.no_batch_throughput:
        out["batch_throughput"] = batch_throughput(lbm)
    if not args.no_tts:
        out["time_to_steady"] = time_to_steady(lbm, args.tts_cases, args.tts_side,
                                               args.tts_max_steps)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(n, U, re, gamma)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
