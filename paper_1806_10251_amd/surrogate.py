"""Learned warm start: training data from the method, training, inference.

Host driver only.  The steady fields that serve as training targets come
from the lattice Boltzmann library itself (batched FP64 runs to residual
1e-8); the network (unet.py, include/unet.h) is trained and run by the
library's BF16 MFMA kernels; the predicted (rho, u) initialise the lattice
at their equilibrium, so the iteration and its fixed point are unchanged and
only the starting point moves.  The cold start (rest state) remains the
fallback for every case the network does not cover (the kinds its weights
were trained on: square cavities and channels for the default weights) and
for a warm-started case that diverges (it runs again from rest).

Targets (per fluid node): (rho - 1) / (3 U^2), u_x / U, u_y / U (a
channel's density target is zero: velocity only).  The network works at a
fixed resolution (128 x 128); a lattice of any shape is described to it by
the solid fraction of each coarse cell, and its output is interpolated
bilinearly to the lattice (unet_fields_from_output_rect), for a cavity with
the fluid mean of rho - 1 removed so that the closed lattice keeps the cold
start's mass and with the staggered momenta that bounce-back lattices never
damp removed.  A warm-started state is also replaced, after its first step and
after 1000 steps, by the mean of its last two steps (Batch.average_last_two):
the prediction excites period-2 components that barely decay and would
otherwise dominate the one-step residual.

Command line (one GPU):
  python -m paper_1806_10251_amd.surrogate train --channels 1500 --epochs 60 --out weights.npy
  python -m paper_1806_10251_amd.surrogate bench-train   (training-step timing)
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np

from . import lbm as L
from . import steady
from . import unet as U

RES = 128
WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")
CAVITY_WEIGHTS = os.path.join(WEIGHTS_DIR, "unet_cavity128.npy")
MIX_WEIGHTS = os.path.join(WEIGHTS_DIR, "unet_mix128.npy")
DEFAULT_WEIGHTS = MIX_WEIGHTS if os.path.exists(MIX_WEIGHTS) else CAVITY_WEIGHTS


def cavity_cases(n, seed, side, re_lo=50.0, re_hi=500.0):
    """Seeded lid-driven cavities side x side with 1-4 rectangular obstacles,
    Re uniform in [re_lo, re_hi], gamma log-uniform in [0.05, 1]; speeds as
    for the batched case mix."""
    from workloads import draw_cases
    return draw_cases(n, seed, side_lo=side, side_hi=side, re_lo=re_lo, re_hi=re_hi,
                      channel_frac=0.0)


def channel_cases(n, seed, side, re_lo=50.0, re_hi=500.0):
    """Seeded channels 4 side x side (parabolic inlet, convective outlet)
    with 1-4 rectangular obstacles, otherwise drawn as cavity_cases."""
    from workloads import draw_cases
    return draw_cases(n, seed, side_lo=side, side_hi=side, re_lo=re_lo, re_hi=re_hi,
                      channel_frac=1.0)


def case_params(cases):
    """Network case parameters (Re, gamma, U, kind) per case."""
    return np.array([[k.re, k.gamma, k.u_ref,
                      U.KIND_CHANNEL if k.kind == "channel" else U.KIND_CAVITY] for k in cases],
                    np.float32)


def steady_fields(cases, tol=1e-8, max_steps=400000, chunk=512, init=None, filter_at=(),
                  log=None):
    """Run every case to the residual tol with the batch (FP64).  init(i0,
    i1, batch) may set initial fields of cases [i0, i1); filter_at: steps
    after which the state is replaced by the mean of its last two steps
    (Batch.average_last_two), before the run that checks the residual.
    Returns (rho, ux, uy, steps, status, seconds) with fields [n][ny][nx]
    (FP64, host); steps count from the start."""
    n = len(cases)
    ny, nx = cases[0].ny, cases[0].nx
    rho = np.zeros((n, ny, nx))
    ux, uy = np.zeros_like(rho), np.zeros_like(rho)
    steps = np.zeros(n, np.int64)
    status = np.zeros(n, np.int32)
    secs = 0.0
    for i0 in range(0, n, chunk):
        part = cases[i0:i0 + chunk]
        grids = [L.make_grid(k.nx, k.ny, k.sides) for k in part]
        params = [L.make_params(storage="f64", check_every=100, **steady.case_kw(k))
                  for k in part]
        b = L.Batch(grids, [k.mask for k in part], params)
        import torch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if init is not None:
            init(i0, i0 + len(part), b)
        done = 0
        for at in sorted(filter_at):
            if at > done:
                b.run(0.0, at - done)
                done = at
            b.average_last_two()
        s, st, _ = steady.run_batch(b, tol=tol, max_steps=max_steps - done)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        secs += sec
        steps[i0:i0 + len(part)] = np.where(st == 3, s, s + done)
        status[i0:i0 + len(part)] = st
        for j in range(len(part)):
            rho[i0 + j], ux[i0 + j], uy[i0 + j] = b.fields(j, ny, nx)
        b.close()
        if log:
            log(f"steady fields {i0 + len(part)}/{n}: {sec:.1f} s, "
                f"converged {(st == 1).sum()}/{len(part)}")
    return rho, ux, uy, steps, status, secs


def targets(cases, rho, ux, uy, res=None):
    """Training targets (rho - 1) / (3 U^2), u / U per fluid node and the
    fluid mask.  With res given and lattices of another size, both are taken
    to the network's res x res cells (the cells of the input map): the mean
    over the fluid nodes of a cell, which is fluid if it holds any."""
    cp = case_params(cases).astype(np.float64)
    Uv = cp[:, 2][:, None, None]
    t = np.stack([(rho - 1.0) / (3.0 * Uv ** 2), ux / Uv, uy / Uv], axis=-1)
    # Channels: velocity only.  Their pressure drop, (rho - 1) / (3 U^2) of
    # order 100 / Re times the blockage, is one to two orders of magnitude
    # above a cavity's pressure variations in these units and dominated the
    # loss (a first training run on both kinds stayed at a loss of about 150);
    # with a zero target the network returns rho ~ 1 for a channel.
    is_channel = np.array([k.kind == "channel" for k in cases])
    t[is_channel, ..., 0] = 0.0
    fluid = np.stack([(k.mask == 0) for k in cases]).astype(np.uint8)
    t = np.where(fluid[..., None] == 1, t, 0.0)
    n, ny, nx = fluid.shape
    if res is not None and (ny, nx) != (res, res):
        def cells(fine):
            lo = [I * fine // res for I in range(res)]
            return lo, [max((I + 1) * fine // res, lo[I] + 1) for I in range(res)]
        (lx, hx), (ly, hy) = cells(nx), cells(ny)
        tc = np.zeros((n, res, res, 3))
        fc = np.zeros((n, res, res), np.uint8)
        for J in range(res):
            for I in range(res):
                f = fluid[:, ly[J]:hy[J], lx[I]:hx[I]].reshape(n, -1).astype(np.float64)
                v = t[:, ly[J]:hy[J], lx[I]:hx[I]].reshape(n, -1, 3)
                cnt = f.sum(1)
                tc[:, J, I] = (v * f[..., None]).sum(1) / np.maximum(cnt, 1)[:, None]
                fc[:, J, I] = cnt > 0
        t, fluid = tc, fc
    return t.astype(np.float32), fluid


class Dataset:
    """Network inputs and targets resident on the device.  groups: one or
    more (cases, rho, ux, uy) of one lattice shape each."""

    def __init__(self, *groups):
        import torch
        if len(groups) == 4 and not isinstance(groups[0], tuple):
            groups = (tuple(groups),)
        xs, ts, fs = [], [], []
        for cases, rho, ux, uy in groups:
            t, fluid = targets(cases, rho, ux, uy, RES)
            solid = torch.tensor(np.stack([k.mask for k in cases]).astype(np.uint8),
                                 device="cuda")
            cp = torch.tensor(case_params(cases), device="cuda")
            xs.append(U.make_input(solid, cp, RES))
            ts.append(torch.tensor(t, device="cuda"))
            fs.append(torch.tensor(fluid, device="cuda"))
        self.x0 = torch.cat(xs)
        self.t = torch.cat(ts)
        self.fluid = torch.cat(fs)
        self.n = int(self.x0.shape[0])


def train(net, data, epochs, batch, lr=1e-3, lr_end=1e-4, seed=0, log=None):
    """Adam with a cosine learning-rate decay from lr to lr_end; mini-batches
    drawn without replacement each epoch.  Returns the loss per step."""
    import torch
    rng = np.random.default_rng(seed)
    steps_per_epoch = max(1, data.n // batch)
    total = epochs * steps_per_epoch
    hist = []
    k = 0
    for ep in range(epochs):
        perm = torch.tensor(rng.permutation(data.n), device="cuda")
        for s in range(steps_per_epoch):
            idx = perm[s * batch:(s + 1) * batch]
            rate = lr_end + 0.5 * (lr - lr_end) * (1 + math.cos(math.pi * k / max(1, total - 1)))
            loss = net.train_step(data.x0.index_select(0, idx).contiguous(),
                                  data.t.index_select(0, idx).contiguous(),
                                  data.fluid.index_select(0, idx).contiguous(), rate)
            hist.append(loss)
            k += 1
        if log:
            log(f"epoch {ep + 1}/{epochs}: loss {np.mean(hist[-steps_per_epoch:]):.4e}")
    return hist


def evaluate_loss(net, data, batch):
    """Mean loss over the data set without updating the network."""
    import torch
    losses = []
    for i0 in range(0, data.n, batch):
        idx = torch.arange(i0, min(data.n, i0 + batch), device="cuda")
        losses.append(net.backward(data.x0.index_select(0, idx).contiguous(),
                                   data.t.index_select(0, idx).contiguous(),
                                   data.fluid.index_select(0, idx).contiguous()) * len(idx))
    return float(np.sum(losses) / data.n)


def covers(case, net=None):
    """True for the cases the network predicts: the kinds its weights were
    trained on (net.kinds, set by load_into; square cavities when unknown)."""
    kinds = getattr(net, "kinds", ("cavity",)) if net is not None else ("cavity",)
    if case.kind == "cavity":
        return "cavity" in kinds and case.nx == case.ny
    return case.kind in kinds


def predict_fields(net, cases):
    """Predicted (rho, ux, uy) device tensors [ny][nx] per case; None for
    cases the network does not cover (covers(); they keep the cold start).
    Cases of one shape share a forward pass."""
    import torch
    out = [None] * len(cases)
    by_size = {}
    for i, k in enumerate(cases):
        if covers(k, net):
            by_size.setdefault((k.ny, k.nx), []).append(i)
    for fine, idx in by_size.items():
        group = [cases[i] for i in idx]
        solid = torch.tensor(np.stack([k.mask for k in group]).astype(np.uint8), device="cuda")
        cp = torch.tensor(case_params(group), device="cuda")
        x0 = U.make_input(solid, cp, RES)
        for i0 in range(0, len(group), net.max_batch):
            i1 = min(len(group), i0 + net.max_batch)
            o = net.forward(x0[i0:i1].contiguous())
            r, a, b = U.fields_from_output(o, cp[i0:i1].contiguous(), solid[i0:i1].contiguous())
            for j in range(i1 - i0):
                out[idx[i0 + j]] = (r[j].contiguous(), a[j].contiguous(), b[j].contiguous())
    return out


# Steps after which a warm-started state is replaced by the mean of its last
# two steps: the prediction excites period-2 components (eigenvalue near -1
# of the step map) that barely decay and dominate the one-step residual.
WARM_FILTER = (1, 1000)


def warm_init(net, cases):
    """An init callback for steady_fields (and for any batch built from
    `cases` in order): equilibrium at the prediction where there is one
    (use with filter_at=WARM_FILTER)."""
    pred = predict_fields(net, cases)

    def init(i0, i1, batch):
        for j in range(i1 - i0):
            p = pred[i0 + j]
            if p is not None:
                batch.init_fields_device(j, *p)
    return init


# (cin, cout, level) of the 15 convolutions, in network order
CONVS = [(32, 32, 0), (32, 32, 0), (32, 64, 1), (64, 64, 1), (64, 128, 2), (128, 128, 2),
         (128, 256, 3), (256, 256, 3), (384, 128, 2), (128, 128, 2), (192, 64, 1), (64, 64, 1),
         (96, 32, 0), (32, 32, 0), (32, 32, 0)]


def network_flops(res, batch=1):
    """(forward, training step) FLOPs of the convolutions: 2 * 9 * cin * cout
    per output pixel; a training step adds the input gradient (all layers
    but the first) and the weight gradient."""
    fwd = sum(2 * 9 * ci * co * (res >> lv) ** 2 for ci, co, lv in CONVS)
    first = 2 * 9 * 32 * 32 * res * res
    return batch * fwd, batch * (3 * fwd - first)


def bench_train(steps=50, batch=16, seed=0):
    """Time training steps on synthetic inputs (random geometry, smooth
    targets): returns (ms per step, TFLOP/s of the convolutions)."""
    import torch
    rng = np.random.default_rng(seed)
    solid = torch.tensor((rng.random((batch, RES, RES)) > 0.9).astype(np.uint8), device="cuda")
    cp = torch.tensor(np.tile([[200.0, 0.5, 0.1]], (batch, 1)).astype(np.float32), device="cuda")
    x0 = U.make_input(solid, cp, RES)
    c = (np.arange(RES) + 0.5) / RES
    X, Y = np.meshgrid(c, c)
    t = np.stack([np.sin(2 * np.pi * X), X * Y, Y - 0.5], axis=-1)
    t = torch.tensor(np.broadcast_to(t, (batch, RES, RES, 3)).astype(np.float32), device="cuda")
    fluid = (1 - solid).contiguous()
    net = U.UNet(max_batch=batch, res=RES, seed=seed)
    for _ in range(3):
        net.train_step(x0, t, fluid, 1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        net.train_step(x0, t, fluid, 1e-4)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    net.close()
    return ms, network_flops(RES, batch)[1] / (ms * 1e-3) / 1e12


def _kinds_path(path):
    return os.path.splitext(path)[0] + ".kinds.json"


def save(net, path, kinds=("cavity",)):
    """Parameters (.npy) and the case kinds they were trained on (.kinds.json)."""
    import json
    np.save(path, net.params())
    with open(_kinds_path(path), "w") as f:
        json.dump({"kinds": list(kinds)}, f)


def load_into(net, path):
    """Load parameters and record on `net` the kinds they cover (square
    cavities when the file has no kinds record)."""
    import json
    net.set_params(np.load(path, allow_pickle=False))
    try:
        with open(_kinds_path(path)) as f:
            net.kinds = tuple(json.load(f)["kinds"])
    except OSError:
        net.kinds = ("cavity",)


def _log(msg):
    print(f"[surrogate] {msg}", flush=True)


def evaluate(net, cases, tols=(1e-8, 1e-9, 1e-10), max_steps=600000, segment=20000,
             log=_log):
    """Held-out evaluation of the warm start: every arm runs all cases in one
    FP64 batch from the cold start or the prediction, with or without the
    residual filter (WARM_FILTER), to each residual tolerance; the error of
    an arm is max |u - u_ref| / U against a warm-start run to residual 1e-11.
    Returns one dict per arm."""
    import torch

    def arm(name, tol, warm, filter_at, cases=cases):
        n = len(cases)
        grids = [L.make_grid(k.nx, k.ny, k.sides) for k in cases]
        params = [L.make_params(storage="f64", check_every=100, nu=k.nu, gamma=k.gamma,
                                u_lid=k.u_ref) for k in cases]
        b = L.Batch(grids, [k.mask for k in cases], params)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if warm:
            warm_init(net, cases)(0, n, b)
        done = 0
        for at in filter_at:
            b.run(0.0, at - done)
            done = at
            b.average_last_two()
        total = np.full(n, -1, np.int64)
        status = np.zeros(n, np.int32)
        active = np.ones(n, bool)
        while done < max_steps and active.any():
            b.set_enabled(active.astype(np.int32))
            b.set_plateau(0, 0.9)
            m = min(segment, max_steps - done)
            steps = b.run(tol, m)
            st = b.status()
            for i in range(n):
                if active[i] and st[i] in (1, 3):
                    total[i] = done + abs(int(steps[i]))
                    status[i] = st[i]
                    active[i] = False
            done += m
            log(f"{name} {tol:g}: {done} steps, retired {(~active).sum()}/{n}, "
                f"{time.perf_counter() - t0:.1f} s")
        total[active] = done
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        fields = [b.fields(i, k.ny, k.nx)[1:] for i, k in enumerate(cases)]
        b.close()
        redo = [i for i in range(n) if warm and covers(cases[i], net) and status[i] == 3]
        if redo:
            # the cold start is the fallback for a warm start that diverges
            sec2, total2, status2, fields2 = arm(name + " (cold fallback)", tol, False, filter_at,
                                                 [cases[i] for i in redo])
            for j, i in enumerate(redo):
                total[i] += total2[j]
                status[i] = status2[j]
                fields[i] = fields2[j]
            sec += sec2
        return sec, total, status, fields

    _, _, st_ref, f_ref = arm("reference warm+filter", 1e-11, True, WARM_FILTER)
    ok = [i for i in range(len(cases)) if st_ref[i] == 1]
    plan = [("cold", tols[0], False, ())]
    for tol in tols:
        plan += [("cold+filter", tol, False, WARM_FILTER), ("warm+filter", tol, True, WARM_FILTER)]
    out = []
    for name, tol, warm, fa in plan:
        sec, total, status, f = arm(name, tol, warm, fa)
        err = float(max(max(np.abs(f[i][0] - f_ref[i][0]).max(),
                            np.abs(f[i][1] - f_ref[i][1]).max()) / cases[i].u_ref
                        for i in ok)) if ok else None
        out.append({"arm": name, "tol": tol, "seconds": round(sec, 2),
                    "steps_sum": int(total.sum()), "converged": int((status == 1).sum()),
                    "cases": len(cases), "reference_converged": len(ok),
                    "max_err_vs_ref": err})
        log("RESULT " + str(out[-1]))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--cases", type=int, default=2000)
    t.add_argument("--seed", type=int, default=20181)
    t.add_argument("--epochs", type=int, default=40)
    t.add_argument("--batch", type=int, default=16)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--max-steps", type=int, default=300000)
    t.add_argument("--channels", type=int, default=0,
                   help="also train on this many channels 4*128 x 128 (seed + 1)")
    t.add_argument("--channel-max-steps", type=int, default=60000)
    t.add_argument("--out", required=True)
    t.add_argument("--data-cache", default="")
    bt = sub.add_parser("bench-train")
    bt.add_argument("--steps", type=int, default=50)
    bt.add_argument("--batch", type=int, default=16)
    ev = sub.add_parser("evaluate", help="held-out warm-start evaluation (FP64 batches)")
    ev.add_argument("--cases", type=int, default=64)
    ev.add_argument("--side", type=int, default=512)
    ev.add_argument("--seed", type=int, default=5151)
    ev.add_argument("--weights", default=DEFAULT_WEIGHTS)
    ev.add_argument("--tols", default="1e-8,1e-9,1e-10")
    ev.add_argument("--max-steps", type=int, default=600000)
    args = ap.parse_args(argv)
    if args.cmd == "evaluate":
        import json
        import torch
        if not torch.cuda.is_available():
            sys.exit("needs a GPU")
        L.load()
        U.load()
        net = U.UNet(max_batch=16, res=RES, seed=0)
        load_into(net, args.weights)
        rows = evaluate(net, cavity_cases(args.cases, args.seed, args.side),
                        tols=tuple(float(t) for t in args.tols.split(",")),
                        max_steps=args.max_steps)
        print(json.dumps(rows), flush=True)
        return
    if args.cmd == "bench-train":
        import torch
        if not torch.cuda.is_available():
            sys.exit("needs a GPU")
        L.load()
        U.load()
        ms, tf = bench_train(args.steps, args.batch)
        print(f"[surrogate] training step (batch {args.batch}, {RES}x{RES}): {ms:.2f} ms, "
              f"{tf:.1f} TFLOP/s in the convolutions", flush=True)
        return

    import torch
    if not torch.cuda.is_available():
        sys.exit("needs a GPU")
    L.load()
    U.load()
    cases = cavity_cases(args.cases, args.seed, RES)
    if args.data_cache and os.path.exists(args.data_cache):
        z = np.load(args.data_cache, allow_pickle=False)
        rho, ux, uy, status = z["rho"], z["ux"], z["uy"], z["status"]
    else:
        rho, ux, uy, steps, status, sec = steady_fields(cases, max_steps=args.max_steps, log=_log)
        _log(f"generated {len(cases)} steady fields in {sec:.1f} s; converged "
             f"{(status == 1).sum()}, steps median {int(np.median(steps))}")
        if args.data_cache:
            np.savez(args.data_cache, rho=rho, ux=ux, uy=uy, status=status)
    keep = [i for i in range(len(cases)) if status[i] == 1]
    cases = [cases[i] for i in keep]
    groups = [(cases, rho[keep], ux[keep], uy[keep])]
    kinds = ["cavity"]
    if args.channels:
        ch = channel_cases(args.channels, args.seed + 1, RES)
        rho, ux, uy, steps, status, sec = steady_fields(ch, max_steps=args.channel_max_steps,
                                                        log=_log)
        _log(f"generated {len(ch)} steady channel fields in {sec:.1f} s; converged "
             f"{(status == 1).sum()}, steps median {int(np.median(steps))}")
        keep = [i for i in range(len(ch)) if status[i] == 1]
        groups.append(([ch[i] for i in keep], rho[keep], ux[keep], uy[keep]))
        kinds.append("channel")
        del rho, ux, uy
    data = Dataset(*groups)
    _log(f"training set: {data.n} cases")
    net = U.UNet(max_batch=args.batch, res=RES, seed=args.seed)
    t0 = time.perf_counter()
    hist = train(net, data, args.epochs, args.batch, lr=args.lr, seed=args.seed, log=_log)
    torch.cuda.synchronize()
    _log(f"trained {len(hist)} steps in {time.perf_counter() - t0:.1f} s; "
         f"final loss {np.mean(hist[-20:]):.4e}")
    save(net, args.out, kinds)


if __name__ == "__main__":
    main()
