"""ctypes binding of the U-Net warm-start kernels (include/unet.h).

Argument marshalling only: tensors are torch CUDA tensors (bf16 or float32,
NHWC, contiguous) whose device pointers are passed to the library; every
computation runs in the library's HIP kernels.  Raises when the library is
missing (there is no fallback).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import lbm as _lbm

IN_CHANNELS = 32
OUT_CHANNELS = 32

_lib = None


class UnetError(RuntimeError):
    pass


def load():
    global _lib
    if _lib is not None:
        return _lib
    L = _lbm.load()
    vp, i32, i64, dbl, u64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                              ctypes.c_uint64)
    P = ctypes.POINTER
    sig = {
        "unet_conv3x3_fwd": [vp, i32, vp, vp, vp, i32, i32, i32, i32, i32, i32, i32, i32, vp],
        "unet_conv3x3_bwd_data": [vp, i32, vp, vp, i32, i32, i32, i32, i32, i32, vp, vp],
        "unet_wgrad_work_floats": [i32, i32, i32, i32, i32],
        "unet_conv3x3_bwd_weight": [vp, i32, vp, i32, vp, vp, i32, i32, i32, i32, i32, vp, vp],
        "unet_relu_bwd": [vp, i32, vp, i32, i64, i32, vp],
        "unet_pool2_fwd": [vp, i32, vp, i32, i32, i32, i32, i32, vp],
        "unet_pool2_bwd": [vp, i32, vp, i32, vp, i32, i32, i32, i32, i32, vp],
        "unet_up2_fwd": [vp, i32, vp, i32, i32, i32, i32, i32, vp],
        "unet_up2_bwd": [vp, i32, vp, i32, i32, i32, i32, i32, vp],
        "unet_loss_work_doubles": [i64],
        "unet_mse_loss": [vp, i32, vp, vp, i64, vp, P(dbl), vp, vp],
        "unet_adam": [vp, vp, vp, vp, vp, i64, dbl, dbl, dbl, dbl, i64, vp],
        "unet_make_input": [vp, i32, vp, i32, i32, vp, vp],
        "unet_fields_from_output": [vp, i32, i32, i32, vp, vp, i32, vp, vp, vp, vp],
        "unet_make_input_rect": [vp, i32, i32, vp, i32, i32, vp, vp],
        "unet_fields_from_output_rect": [vp, i32, i32, i32, vp, vp, i32, i32, vp, vp, vp, vp],
        "unet_create": [i32, i32, u64, P(vp)],
        "unet_destroy": [vp],
        "unet_set_stream": [vp, vp],
        "unet_num_params": [vp, P(i64)],
        "unet_get_params": [vp, vp],
        "unet_set_params": [vp, vp],
        "unet_get_grads": [vp, vp],
        "unet_forward": [vp, vp, i32, vp],
        "unet_backward": [vp, vp, vp, vp, i32, P(dbl)],
        "unet_train_step": [vp, vp, vp, vp, i32, dbl, P(dbl)],
        "unet_last_error": [],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.unet_wgrad_work_floats.restype = ctypes.c_int64
    L.unet_loss_work_doubles.restype = ctypes.c_int64
    L.unet_last_error.restype = ctypes.c_char_p
    L.unet_destroy.restype = None
    _lib = L
    return L


def _check(rc):
    if rc != 0:
        msg = load().unet_last_error().decode(errors="replace")
        raise UnetError(f"{msg} (code {rc})")


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# --- layers (tests and tools) -------------------------------------------------

def conv3x3_fwd(x, w, bias, cout, relu=False, out_f32=False, y=None):
    """x: bf16 [n,h,w,ldx]; w: bf16 [cout,9,cin] (cin = w.shape[2])."""
    import torch
    n, h, wd, ldx = x.shape
    cin = w.shape[2]
    if y is None:
        y = torch.empty((n, h, wd, cout), device=x.device,
                        dtype=torch.float32 if out_f32 else torch.bfloat16)
    _check(load().unet_conv3x3_fwd(_p(x), ldx, _p(w), _p(bias), _p(y), y.shape[3], n, h, wd, cin,
                                   cout, int(relu), int(out_f32), _stream()))
    return y


def conv3x3_bwd_data(dy, w, cin):
    import torch
    n, h, wd, lddy = dy.shape
    cout = w.shape[0]
    dx = torch.empty((n, h, wd, cin), device=dy.device, dtype=torch.bfloat16)
    work = torch.empty(9 * cin * cout, device=dy.device, dtype=torch.bfloat16)
    _check(load().unet_conv3x3_bwd_data(_p(dy), lddy, _p(w), _p(dx), cin, n, h, wd, cin, cout,
                                        _p(work), _stream()))
    return dx


def conv3x3_bwd_weight(dy, x, cin, cout):
    import torch
    n, h, wd, lddy = dy.shape
    ldx = x.shape[3]
    dw = torch.empty((cout, 9, cin), device=dy.device, dtype=torch.float32)
    db = torch.empty(cout, device=dy.device, dtype=torch.float32)
    nw = load().unet_wgrad_work_floats(n, h, wd, cin, cout)
    work = torch.empty(int(nw), device=dy.device, dtype=torch.float32)
    _check(load().unet_conv3x3_bwd_weight(_p(dy), lddy, _p(x), ldx, _p(dw), _p(db), n, h, wd, cin,
                                          cout, _p(work), _stream()))
    return dw, db


def relu_bwd(d, y):
    n, h, wd, c = d.shape
    _check(load().unet_relu_bwd(_p(d), c, _p(y), y.shape[3], n * h * wd, c, _stream()))
    return d


def pool2_fwd(x):
    import torch
    n, h, wd, c = x.shape
    y = torch.empty((n, h // 2, wd // 2, c), device=x.device, dtype=torch.bfloat16)
    _check(load().unet_pool2_fwd(_p(x), c, _p(y), c, n, h, wd, c, _stream()))
    return y


def pool2_bwd(dy, add=None):
    import torch
    n, h, wd, c = dy.shape
    dx = torch.empty((n, 2 * h, 2 * wd, c), device=dy.device, dtype=torch.bfloat16)
    _check(load().unet_pool2_bwd(_p(dy), c, _p(add), c, _p(dx), c, n, 2 * h, 2 * wd, c,
                                 _stream()))
    return dx


def up2_fwd(x):
    import torch
    n, h, wd, c = x.shape
    y = torch.empty((n, 2 * h, 2 * wd, c), device=x.device, dtype=torch.bfloat16)
    _check(load().unet_up2_fwd(_p(x), c, _p(y), c, n, h, wd, c, _stream()))
    return y


def up2_bwd(dy):
    import torch
    n, h, wd, c = dy.shape
    dx = torch.empty((n, h // 2, wd // 2, c), device=dy.device, dtype=torch.bfloat16)
    _check(load().unet_up2_bwd(_p(dy), c, _p(dx), c, n, h // 2, wd // 2, c, _stream()))
    return dx


def mse_loss(out, target, fluid):
    """out f32 [n,h,w,ldo]; target f32 [n,h,w,3]; fluid u8 [n,h,w]."""
    import torch
    n, h, wd, ldo = out.shape
    npix = n * h * wd
    dout = torch.empty_like(out, dtype=torch.bfloat16)
    work = torch.empty(int(load().unet_loss_work_doubles(npix)), device=out.device,
                       dtype=torch.float64)
    loss = ctypes.c_double()
    _check(load().unet_mse_loss(_p(out), ldo, _p(target), _p(fluid), npix, _p(dout),
                                ctypes.byref(loss), _p(work), _stream()))
    return loss.value, dout


def adam(p, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, pb=None):
    _check(load().unet_adam(_p(p), _p(m), _p(v), _p(g), _p(pb), p.numel(), lr, beta1, beta2, eps,
                            int(t), _stream()))


KIND_CAVITY, KIND_CHANNEL = 0, 1


def make_input(solid, case_params, res):
    """solid u8 [n,ny,nx]; case_params f32 [n,3] = (Re, gamma, U) for square
    cavities, or [n,4] = (Re, gamma, U, kind) for any shape and kind."""
    import torch
    n, ny, nx = solid.shape
    x0 = torch.empty((n, res, res, IN_CHANNELS), device=solid.device, dtype=torch.bfloat16)
    if case_params.shape[1] == 4:
        _check(load().unet_make_input_rect(_p(solid), nx, ny, _p(case_params), n, res, _p(x0),
                                           _stream()))
    else:
        if nx != ny:
            raise ValueError("three case parameters describe square cavities only")
        _check(load().unet_make_input(_p(solid), nx, _p(case_params), n, res, _p(x0), _stream()))
    return x0


def fields_from_output(out, case_params, solid):
    """out f32 [n,res,res,ldo]; solid u8 [n,ny,nx]; case_params as for
    make_input -> rho, ux, uy f32 [n,ny,nx]."""
    import torch
    n, res, _, ldo = out.shape
    ny, nx = solid.shape[1], solid.shape[2]
    rho = torch.empty((n, ny, nx), device=out.device, dtype=torch.float32)
    ux = torch.empty_like(rho)
    uy = torch.empty_like(rho)
    if case_params.shape[1] == 4:
        _check(load().unet_fields_from_output_rect(_p(out), ldo, n, res, _p(case_params),
                                                   _p(solid), nx, ny, _p(rho), _p(ux), _p(uy),
                                                   _stream()))
    else:
        if nx != ny:
            raise ValueError("three case parameters describe square cavities only")
        _check(load().unet_fields_from_output(_p(out), ldo, n, res, _p(case_params), _p(solid),
                                              nx, _p(rho), _p(ux), _p(uy), _stream()))
    return rho, ux, uy


# --- the network ---------------------------------------------------------------

class UNet:
    """The warm-start network (4 levels, 32..256 channels) on the device."""

    def __init__(self, max_batch, res, seed=0):
        h = ctypes.c_void_p()
        _check(load().unet_create(int(max_batch), int(res), ctypes.c_uint64(seed),
                                  ctypes.byref(h)))
        self._h = h
        self.max_batch, self.res = int(max_batch), int(res)
        import torch
        self.set_stream(torch.cuda.current_stream())
        n = ctypes.c_int64()
        _check(load().unet_num_params(self._h, ctypes.byref(n)))
        self.num_params = n.value

    def close(self):
        if getattr(self, "_h", None):
            load().unet_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        raw = getattr(stream, "cuda_stream", stream)
        _check(load().unet_set_stream(self._h, ctypes.c_void_p(raw) if raw else None))

    def params(self):
        a = np.empty(self.num_params, dtype=np.float32)
        _check(load().unet_get_params(self._h, a.ctypes.data_as(ctypes.c_void_p)))
        return a

    def set_params(self, a):
        a = np.ascontiguousarray(a, dtype=np.float32)
        assert a.size == self.num_params
        _check(load().unet_set_params(self._h, a.ctypes.data_as(ctypes.c_void_p)))

    def grads(self):
        a = np.empty(self.num_params, dtype=np.float32)
        _check(load().unet_get_grads(self._h, a.ctypes.data_as(ctypes.c_void_p)))
        return a

    def forward(self, x0, out=None):
        import torch
        n = x0.shape[0]
        if out is None:
            out = torch.empty((n, self.res, self.res, OUT_CHANNELS), device=x0.device,
                              dtype=torch.float32)
        _check(load().unet_forward(self._h, _p(x0), n, _p(out)))
        return out

    def backward(self, x0, target, fluid):
        loss = ctypes.c_double()
        _check(load().unet_backward(self._h, _p(x0), _p(target), _p(fluid), x0.shape[0],
                                    ctypes.byref(loss)))
        return loss.value

    def train_step(self, x0, target, fluid, lr):
        loss = ctypes.c_double()
        _check(load().unet_train_step(self._h, _p(x0), _p(target), _p(fluid), x0.shape[0],
                                      float(lr), ctypes.byref(loss)))
        return loss.value
