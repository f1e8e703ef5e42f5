"""Plain NumPy FP64 reference of the warm-start U-Net (layers, loss, Adam).

TEST INFRASTRUCTURE ONLY: used by the tests to check the HIP kernels; the
product path never imports it and it shares no code with the HIP library.

Every layer is written from its definition, in FP64, on NHWC arrays:

* 3x3 convolution with zero padding (cross-correlation, the CNN convention):
  y[n,i,j,o] = b[o] + sum_{a,b in {-1,0,1}} sum_c x[n,i+a,j+b,c] w[o,t(a,b),c]
  with the tap index t = 3(a+1) + (b+1) (row-major over (dy, dx));
* its gradients: dx = sum_t shift(dy, -offset_t) @ w[:,t,:],
  dw[o,t,c] = sum_p dy[p,o] x[p+offset_t,c], db[o] = sum_p dy[p,o];
* 2x2 average pooling, nearest 2x upsampling and their adjoints;
* masked mean-squared error over the first three output channels;
* Adam (Kingma & Ba, 2015, Algorithm 1).

``bf16()`` rounds to bfloat16 (round to nearest even, via float32), so that
tests can feed both sides identical rounded inputs and, optionally, round
stored activations the way the device does.
"""
from __future__ import annotations

import numpy as np

IN_CHANNELS = 32
OUT_CHANNELS = 32


def bf16(a):
    """Round to the nearest bfloat16 (ties to even); returns float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = rounded.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if nan.any():
        out[nan] = np.nan
    return out


def _shift(x, dy, dx):
    """s[n,i,j,:] = x[n,i+dy,j+dx,:] with zeros outside."""
    n, h, w, c = x.shape
    s = np.zeros_like(x)
    i0, i1 = max(0, -dy), min(h, h - dy)
    j0, j1 = max(0, -dx), min(w, w - dx)
    s[:, i0:i1, j0:j1, :] = x[:, i0 + dy:i1 + dy, j0 + dx:j1 + dx, :]
    return s


TAPS = [(a, b) for a in (-1, 0, 1) for b in (-1, 0, 1)]


def conv3x3(x, w, b=None):
    """x [n,h,w,cin], w [cout,9,cin], b [cout] -> [n,h,w,cout] (FP64)."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    y = np.zeros(x.shape[:3] + (w.shape[0],))
    for t, (a, c) in enumerate(TAPS):
        y += _shift(x, a, c) @ w[:, t, :].T
    if b is not None:
        y += np.asarray(b, np.float64)
    return y


def conv3x3_bwd_data(dy, w):
    dy = np.asarray(dy, np.float64)
    w = np.asarray(w, np.float64)
    dx = np.zeros(dy.shape[:3] + (w.shape[2],))
    for t, (a, c) in enumerate(TAPS):
        dx += _shift(dy, -a, -c) @ w[:, t, :]
    return dx


def conv3x3_bwd_weight(dy, x):
    dy = np.asarray(dy, np.float64)
    x = np.asarray(x, np.float64)
    cout, cin = dy.shape[3], x.shape[3]
    dyf = dy.reshape(-1, cout)
    dw = np.zeros((cout, 9, cin))
    for t, (a, c) in enumerate(TAPS):
        dw[:, t, :] = dyf.T @ _shift(x, a, c).reshape(-1, cin)
    return dw, dyf.sum(axis=0)


def pool2(x):
    n, h, w, c = x.shape
    return x.reshape(n, h // 2, 2, w // 2, 2, c).mean(axis=(2, 4))


def pool2_bwd(dy):
    return np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2) / 4.0


def up2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up2_bwd(dy):
    n, h, w, c = dy.shape
    return dy.reshape(n, h // 2, 2, w // 2, 2, c).sum(axis=(2, 4))


def mse_loss(out, target, fluid):
    """Mean over fluid pixels and the first three channels; returns (loss,
    d loss / d out)."""
    out = np.asarray(out, np.float64)
    m = np.asarray(fluid, bool)
    nf = m.sum()
    d = out[..., :3] - np.asarray(target, np.float64)
    d = d * m[..., None]
    loss = (d ** 2).sum() / (3.0 * nf)
    g = np.zeros_like(out)
    g[..., :3] = 2.0 * d / (3.0 * nf)
    return loss, g


def adam(p, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# --- the network --------------------------------------------------------------
# Conv layers in order: (name of input, cin, name of output, cout, relu).
# Encoder level l: two convolutions, then 2x2 pooling of the second one's
# output; decoder: upsample, concatenate [upsampled, skip], two convolutions;
# last: a linear 3x3 convolution to OUT_CHANNELS.
LAYERS = [
    ("x0", 32, "e0a", 32, True), ("e0a", 32, "e0", 32, True),
    ("p1", 32, "e1a", 64, True), ("e1a", 64, "e1", 64, True),
    ("p2", 64, "e2a", 128, True), ("e2a", 128, "e2", 128, True),
    ("p3", 128, "b3a", 256, True), ("b3a", 256, "b3", 256, True),
    ("cat2", 384, "d2a", 128, True), ("d2a", 128, "d2", 128, True),
    ("cat1", 192, "d1a", 64, True), ("d1a", 64, "d1", 64, True),
    ("cat0", 96, "d0a", 32, True), ("d0a", 32, "d0", 32, True),
    ("d0", 32, "out", OUT_CHANNELS, False),
]


def param_layout():
    """(weight offset, bias offset, cin, cout) per layer; weights then bias."""
    off, lay = 0, []
    for _, cin, _, cout, _ in LAYERS:
        lay.append((off, off + 9 * cin * cout, cin, cout))
        off += 9 * cin * cout + cout
    return lay, off


def unpack(params):
    lay, _ = param_layout()
    return [(params[w:w + 9 * ci * co].reshape(co, 9, ci), params[b:b + co])
            for w, b, ci, co in lay]


def forward(params, x0, round_acts=False):
    """Returns (output, activations).  round_acts: round every stored
    activation to bf16 (as the device stores them) and the weights too."""
    r = bf16 if round_acts else (lambda a: a)
    wb = [(r(w), b) for w, b in unpack(params)]
    act = {"x0": r(x0)}

    def conv(k):
        src, _, dst, _, relu = LAYERS[k]
        y = conv3x3(act[src], *wb[k])
        if relu:
            y = np.maximum(y, 0.0)
        act[dst] = y if dst == "out" else r(y)

    conv(0), conv(1)
    act["p1"] = r(pool2(act["e0"]))
    conv(2), conv(3)
    act["p2"] = r(pool2(act["e1"]))
    conv(4), conv(5)
    act["p3"] = r(pool2(act["e2"]))
    conv(6), conv(7)
    act["cat2"] = np.concatenate([up2(act["b3"]), act["e2"]], axis=3)
    conv(8), conv(9)
    act["cat1"] = np.concatenate([up2(act["d2"]), act["e1"]], axis=3)
    conv(10), conv(11)
    act["cat0"] = np.concatenate([up2(act["d1"]), act["e0"]], axis=3)
    conv(12), conv(13)
    conv(14)
    return act["out"], act


def backward(params, x0, target, fluid, round_acts=False):
    """Loss and gradient (same layout as params) of the masked MSE."""
    out, act = forward(params, x0, round_acts)
    loss, gout = mse_loss(out, target, fluid)
    r = bf16 if round_acts else (lambda a: a)
    wb = [(r(w), b) for w, b in unpack(params)]
    grads = [None] * len(LAYERS)
    g = {"out": gout}

    def back(k, need_dx=True):
        src, _, dst, _, relu = LAYERS[k]
        d = g[dst]
        if relu:
            d = d * (act[dst] > 0)
        grads[k] = conv3x3_bwd_weight(d, act[src])
        if need_dx:
            g[src] = conv3x3_bwd_data(d, wb[k][0])

    back(14), back(13), back(12)
    g["d1"], g["e0"] = up2_bwd(g["cat0"][..., :64]), g["cat0"][..., 64:]
    back(11), back(10)
    g["d2"], g["e1"] = up2_bwd(g["cat1"][..., :128]), g["cat1"][..., 128:]
    back(9), back(8)
    g["b3"], g["e2"] = up2_bwd(g["cat2"][..., :256]), g["cat2"][..., 256:]
    back(7), back(6)
    g["e2"] = g["e2"] + pool2_bwd(g["p3"])
    back(5), back(4)
    g["e1"] = g["e1"] + pool2_bwd(g["p2"])
    back(3), back(2)
    g["e0"] = g["e0"] + pool2_bwd(g["p1"])
    back(1), back(0, need_dx=False)
    flat = np.zeros_like(np.asarray(params, np.float64))
    lay, _ = param_layout()
    for (w_off, b_off, ci, co), (dw, db) in zip(lay, grads):
        flat[w_off:w_off + 9 * ci * co] = dw.ravel()
        flat[b_off:b_off + co] = db
    return loss, flat


KIND_CAVITY, KIND_CHANNEL = 0, 1


def _kinds(case_params):
    cp = np.asarray(case_params, np.float64)
    if cp.shape[1] > 3:
        return cp[:, 3].astype(int)
    return np.full(cp.shape[0], KIND_CAVITY)


def make_input(solid, case_params, res):
    """Network input as defined for the device (channels 0-7 used).  solid
    [n][ny][nx]; case_params rows (Re, gamma, U) for cavities or
    (Re, gamma, U, kind).  Channel 6 marks the driven boundary: the top row
    of a cavity, the left column of a channel."""
    solid = np.asarray(solid)
    n, ny, nx = solid.shape

    def cells(fine):
        lo = [I * fine // res for I in range(res)]
        hi = [max((I + 1) * fine // res, lo[I] + 1) for I in range(res)]
        return lo, hi
    lx, hx = cells(nx)
    ly, hy = cells(ny)
    frac = np.array([[[solid[k, ly[J]:hy[J], lx[I]:hx[I]].astype(np.float64).mean()
                       for I in range(res)] for J in range(res)] for k in range(n)])
    x = np.zeros((n, res, res, IN_CHANNELS))
    cp = np.asarray(case_params, np.float64)
    c = (np.arange(res) + 0.5) / res
    x[..., 0] = frac
    x[..., 1] = cp[:, 0, None, None] / 500.0
    x[..., 2] = cp[:, 1, None, None]
    x[..., 3] = cp[:, 2, None, None] / 0.1
    x[..., 4] = c[None, None, :]
    x[..., 5] = c[None, :, None]
    for k, kind in enumerate(_kinds(case_params)):
        if kind == KIND_CHANNEL:
            x[k, :, 0, 6] = 1.0
        else:
            x[k, res - 1, :, 6] = 1.0
    x[..., 7] = 1.0
    return x


def fields_from_output(out, case_params, solid):
    """Lattice fields from the network output: bilinear interpolation of the
    coarse pixel-centred output to the fine node centres (clamped at the
    border, along x with nx and along y with ny), rho = 1 + 3 U^2 o0,
    u = U (o1, o2); solid nodes rho = 1, u = 0.  For a cavity, the fluid
    mean of rho - 1 is then removed and, with it removed, the staggered
    momenta: u_x -= (-1)^i sum((-1)^i rho u_x) / sum(rho) over the fluid
    (likewise u_y with (-1)^j); these two sums change sign every step of a
    bounce-back lattice and must start at zero.  A channel keeps the
    interpolated prediction."""
    out = np.asarray(out, np.float64)
    solid = np.asarray(solid, bool)
    n, res = out.shape[0], out.shape[1]
    ny, nx = solid.shape[1], solid.shape[2]
    kinds = _kinds(case_params)

    def axis(fine):
        c = np.clip((np.arange(fine) + 0.5) * res / fine - 0.5, 0, res - 1)
        i0 = np.minimum(c.astype(int), max(res - 2, 0))
        return i0, np.minimum(i0 + 1, res - 1), c - i0
    x0, x1, fx = axis(nx)
    y0, y1, fy = axis(ny)
    rho = np.empty((n, ny, nx))
    ux, uy = np.empty_like(rho), np.empty_like(rho)
    for k in range(n):
        U = float(case_params[k][2])
        o = out[k]
        ry = (1 - fy)[:, None, None] * o[y0] + fy[:, None, None] * o[y1]   # along y (rows)
        v = (1 - fx)[None, :, None] * ry[:, x0] + fx[None, :, None] * ry[:, x1]
        r = 1 + 3 * U * U * v[..., 0]
        a, b = U * v[..., 1], U * v[..., 2]
        s = solid[k]
        r[s], a[s], b[s] = 1.0, 0.0, 0.0
        if kinds[k] == KIND_CAVITY:
            r[~s] -= (r[~s] - 1).mean()
            sx = np.where(np.arange(nx) % 2 == 0, 1.0, -1.0)[None, :]
            sy = np.where(np.arange(ny) % 2 == 0, 1.0, -1.0)[:, None]
            R = r[~s].sum()
            cx = (sx * r * a)[~s].sum() / R
            cy = (sy * r * b)[~s].sum() / R
            a = np.where(s, 0.0, a - sx * cx)
            b = np.where(s, 0.0, b - sy * cy)
        rho[k], ux[k], uy[k] = r, a, b
    return rho, ux, uy
