"""Autotuner for the launch shapes of the fused step and the batch kernel.

Single lattice: every (block height, rows per thread) pair the library
supports is timed on a scratch lattice of the same configuration with the
library's own HIP-event timer; the fastest is cached per (nx, ny, storage,
obstacles, outlet) in a JSON file ($LBM_TUNE_CACHE, default
~/.cache/lbm_tune.json).

Batch: block height (4, 8, 16 wavefronts) and schedule (graph of per-step
kernels with tiles case after case or interleaved, or the persistent
dataflow kernel) are timed on a scratch batch of the same cases.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import lbm as L


def _cache_path():
    return os.environ.get("LBM_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "lbm_tune.json"))


def _load_cache():
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save_cache(c):
    p = _cache_path()
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        tmp = p + ".tmp"
        with open(tmp, "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
        os.replace(tmp, p)
    except OSError:
        pass


def lattice_key(nx, ny, sides, solid, storage):
    has_solid = solid is not None and bool(np.asarray(solid).any())
    return f"{nx}x{ny}:{storage}:obst{int(has_solid)}:outlet{int(sides[1] == L.OUTLET)}"


def tune_lattice(nx, ny, sides, solid=None, steps=400, warmup=100, use_cache=True, **params):
    """Fastest (by, rows) for this lattice configuration; returns
    (shape, {shape: us_per_step})."""
    storage = params.get("storage", "f32")
    key = lattice_key(nx, ny, sides, solid, storage)
    cache = _load_cache() if use_cache else {}
    if key in cache:
        return tuple(cache[key]["shape"]), {tuple(json.loads(k)): v for k, v in
                                             cache[key]["table"].items()}
    p = dict(params)
    p["check_every"] = 100
    table = {}
    lat = L.Lattice(nx, ny, sides, solid=solid, **p)
    try:
        for shape in L.launch_shapes():
            lat.set_launch(*shape)
            lat.step(warmup)
            lat.set_timing(True)
            lat.step(steps)
            table[shape] = lat.last_step_ms * 1e3
            lat.set_timing(False)
    finally:
        lat.close()
    best = min(table, key=table.get)
    if use_cache:
        cache[key] = {"shape": list(best), "table": {json.dumps(list(k)): v for k, v in table.items()}}
        _save_cache(cache)
    return best, table


def tune_batch(grids, masks, params, steps=300, block_heights=(4, 8, 16),
               schedules=(0, 1, 2)):
    """Fastest (block height, schedule) for a batch of cases (schedules as
    in Batch.set_launch).  Returns (choice, table of seconds per step)."""
    b = L.Batch(grids, masks, params)
    table = {}
    try:
        for by in block_heights:
            for sched in schedules:
                b.set_launch(by, sched)
                b.run(0.0, 100)                   # warm-up
                t0 = time.perf_counter()
                b.run(0.0, steps)
                table[(by, sched)] = (time.perf_counter() - t0) / steps
    finally:
        b.close()
    best = min(table, key=table.get)
    return best, table


def apply_batch_choice(batch, choice):
    by, sched = choice
    batch.set_launch(by, sched)
