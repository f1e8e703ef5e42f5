"""Learned warm start: training data from the method, training, inference.

Host driver only.  The steady fields that serve as training targets come
from the lattice Boltzmann library itself (batched FP64 runs to residual
1e-8); the network (unet.py, include/unet.h) is trained and run by the
library's BF16 MFMA kernels; the predicted (rho, u) initialise the lattice
at their equilibrium, so the iteration and its fixed point are unchanged and
only the starting point moves.  The cold start (rest state) remains the
fallback: a case whose warm start does not converge is rerun cold.

Targets (per fluid node): (rho - 1) / (3 U^2), u_x / U, u_y / U.  The
network works at a fixed resolution (128 x 128); a larger lattice is
described to it by the solid fraction of each coarse cell, and its output is
interpolated bilinearly to the lattice (unet_fields_from_output), with the
fluid mean of rho - 1 removed so that a closed cavity keeps the cold start's
mass.

Command line (one GPU):
  python -m paper_1806_10251_amd.surrogate train --out weights.npy
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


def cavity_cases(n, seed, side, re_lo=50.0, re_hi=500.0):
    """Seeded lid-driven cavities side x side with 1-4 rectangular obstacles,
    Re uniform in [re_lo, re_hi], gamma log-uniform in [0.05, 1]; speeds as
    for the batched case mix."""
    from workloads import draw_cases
    return draw_cases(n, seed, side_lo=side, side_hi=side, re_lo=re_lo, re_hi=re_hi,
                      channel_frac=0.0)


def case_params(cases):
    return np.array([[k.re, k.gamma, k.u_ref] for k in cases], np.float32)


def _lat_kw(k):
    return dict(nu=k.nu, gamma=k.gamma, u_lid=k.u_ref)


def steady_fields(cases, tol=1e-8, max_steps=400000, chunk=512, init=None, log=None):
    """Run every case to the residual tol with the batch (FP64).  init(i0,
    i1, batch) may set initial fields of cases [i0, i1).  Returns (rho, ux,
    uy, steps, status, seconds) with fields [n][ny][nx] (FP64, host)."""
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
        params = [L.make_params(storage="f64", check_every=100, **_lat_kw(k)) for k in part]
        b = L.Batch(grids, [k.mask for k in part], params)
        if init is not None:
            init(i0, i0 + len(part), b)
        s, st, sec = steady.run_batch(b, tol=tol, max_steps=max_steps)
        secs += sec
        steps[i0:i0 + len(part)] = s
        status[i0:i0 + len(part)] = st
        for j in range(len(part)):
            rho[i0 + j], ux[i0 + j], uy[i0 + j] = b.fields(j, ny, nx)
        b.close()
        if log:
            log(f"steady fields {i0 + len(part)}/{n}: {sec:.1f} s, "
                f"converged {(st == 1).sum()}/{len(part)}")
    return rho, ux, uy, steps, status, secs


def targets(cases, rho, ux, uy):
    cp = case_params(cases).astype(np.float64)
    Uv = cp[:, 2][:, None, None]
    t = np.stack([(rho - 1.0) / (3.0 * Uv ** 2), ux / Uv, uy / Uv], axis=-1)
    fluid = np.stack([(k.mask == 0) for k in cases]).astype(np.uint8)
    t = np.where(fluid[..., None] == 1, t, 0.0)
    return t.astype(np.float32), fluid


class Dataset:
    """Network inputs and targets resident on the device."""

    def __init__(self, cases, rho, ux, uy):
        import torch
        t, fluid = targets(cases, rho, ux, uy)
        solid = torch.tensor(np.stack([k.mask for k in cases]).astype(np.uint8), device="cuda")
        cp = torch.tensor(case_params(cases), device="cuda")
        self.x0 = U.make_input(solid, cp, RES)
        self.t = torch.tensor(t, device="cuda")
        self.fluid = torch.tensor(fluid, device="cuda")
        self.n = len(cases)


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


def predict_fields(net, cases):
    """Device tensors rho, ux, uy [n][fine][fine] for square cases."""
    import torch
    fine = cases[0].nx
    solid = torch.tensor(np.stack([k.mask for k in cases]).astype(np.uint8), device="cuda")
    cp = torch.tensor(case_params(cases), device="cuda")
    x0 = U.make_input(solid, cp, RES)
    rho = torch.empty((len(cases), fine, fine), device="cuda")
    ux, uy = torch.empty_like(rho), torch.empty_like(rho)
    for i0 in range(0, len(cases), net.max_batch):
        i1 = min(len(cases), i0 + net.max_batch)
        out = net.forward(x0[i0:i1].contiguous())
        r, a, b = U.fields_from_output(out, cp[i0:i1].contiguous(), solid[i0:i1].contiguous())
        rho[i0:i1], ux[i0:i1], uy[i0:i1] = r, a, b
    return rho, ux, uy


def warm_init(net, cases):
    """An init callback for steady_fields: equilibrium at the prediction."""
    rho, ux, uy = predict_fields(net, cases)

    def init(i0, i1, batch):
        for j in range(i1 - i0):
            batch.init_fields_device(j, rho[i0 + j].contiguous(), ux[i0 + j].contiguous(),
                                     uy[i0 + j].contiguous())
    return init


def save(net, path):
    np.save(path, net.params())


def load_into(net, path):
    net.set_params(np.load(path, allow_pickle=False))


def _log(msg):
    print(f"[surrogate] {msg}", flush=True)


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
    t.add_argument("--out", required=True)
    t.add_argument("--data-cache", default="")
    args = ap.parse_args(argv)

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
    data = Dataset(cases, rho[keep], ux[keep], uy[keep])
    net = U.UNet(max_batch=args.batch, res=RES, seed=args.seed)
    t0 = time.perf_counter()
    hist = train(net, data, args.epochs, args.batch, lr=args.lr, seed=args.seed, log=_log)
    torch.cuda.synchronize()
    _log(f"trained {len(hist)} steps in {time.perf_counter() - t0:.1f} s; "
         f"final loss {np.mean(hist[-20:]):.4e}")
    save(net, args.out)


if __name__ == "__main__":
    main()
