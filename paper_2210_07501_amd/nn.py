"""Thin ctypes binding of the warm-start network kernels (include/lbm_nn.h,
inside liblbm.so), same names as the C ABI.

Argument marshalling only: tensors are PyTorch CUDA tensors (their device
addresses are passed), the stream is torch's current one.  bf16 buffers are
torch.bfloat16 tensors.  Raises if the library has not been built.
"""
from __future__ import annotations

import ctypes

from . import lbm as _lbm

EXPORTS = ("nn_conv3x3_fwd", "nn_set_conv_walk", "nn_conv3x3_bwd_data", "nn_conv3x3_wgrad_workspace", "nn_conv3x3_bwd_weight",
           "nn_relu_bwd", "nn_add", "nn_pool2", "nn_up2", "nn_mse", "nn_mse_noalloc", "nn_adam", "nn_cast_weights", "nn_features",
           "nn_to_fields", "nn_targets", "nn_velocity_scale")

_loaded = None


def load():
    global _loaded
    if _loaded is not None:
        return _loaded
    L = _lbm.load()
    vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    pp = ctypes.POINTER(_lbm.lbm_params)
    L.nn_conv3x3_fwd.argtypes = [vp, vp, vp, vp, vp, i32, i32, i32, i32, i32, i32, i32, vp]
    L.nn_conv3x3_bwd_data.argtypes = [vp, vp, vp, i32, i32, i32, i32, i32, vp]
    L.nn_set_conv_walk.argtypes = [i32]
    L.nn_conv3x3_wgrad_workspace.argtypes = [i32, i32, i32, i32, i32, ctypes.POINTER(i64)]
    L.nn_conv3x3_bwd_weight.argtypes = [vp, vp, vp, vp, vp, i64, i32, i32, i32, i32, i32, i32, vp]
    L.nn_relu_bwd.argtypes = [vp, vp, vp, i64, vp]
    L.nn_add.argtypes = [vp, vp, vp, i64, vp]
    L.nn_pool2.argtypes = [i32, vp, vp, i32, i32, i32, i32, vp]
    L.nn_up2.argtypes = [i32, vp, vp, i32, i32, i32, i32, vp]
    L.nn_mse.argtypes = [vp, vp, vp, i32, i64, i32, vp, vp, i64, vp]
    L.nn_mse_noalloc.argtypes = [vp, vp, vp, i32, i64, i32, vp, vp]
    L.nn_adam.argtypes = [vp, vp, vp, vp, vp, vp, i64, i32, i32, i64, f32, f32, f32, f32, f32, vp]
    L.nn_cast_weights.argtypes = [vp, vp, vp, i32, i32, vp]
    L.nn_features.argtypes = [pp, i32, vp, i32, vp]
    L.nn_to_fields.argtypes = [pp, i32, vp, vp, i32, vp]
    L.nn_targets.argtypes = [pp, i32, vp, vp, vp]
    L.nn_velocity_scale.argtypes = [pp]
    L.nn_velocity_scale.restype = ctypes.c_double
    for name in EXPORTS:
        if name != "nn_velocity_scale":
            getattr(L, name).restype = ctypes.c_int
    _loaded = L
    return L


def _p(t):
    """Device address of a tensor (None -> NULL)."""
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream or None)


def _check(rc, where):
    if rc != 0:
        raise _lbm.LBMError(rc, where)


def _params(cfgs):
    return (_lbm.lbm_params * len(cfgs))(*[_lbm.make_params(c) for c in cfgs])


def nn_set_conv_walk(steps):
    _check(load().nn_set_conv_walk(int(steps)), "nn_set_conv_walk")


def nn_conv3x3_fwd(x, w, bias, y, y32, y32_channels, n, h, wd, ci, co, relu):
    _check(load().nn_conv3x3_fwd(_p(x), _p(w), _p(bias), _p(y), _p(y32), int(y32_channels), n, h, wd, ci, co,
                                 int(relu), _stream()), "nn_conv3x3_fwd")


def nn_conv3x3_bwd_data(dy, wflip, dx, n, h, wd, ci, co):
    _check(load().nn_conv3x3_bwd_data(_p(dy), _p(wflip), _p(dx), n, h, wd, ci, co, _stream()), "nn_conv3x3_bwd_data")


def nn_conv3x3_wgrad_workspace(n, h, wd, ci, co):
    b = ctypes.c_int64()
    _check(load().nn_conv3x3_wgrad_workspace(n, h, wd, ci, co, ctypes.byref(b)), "nn_conv3x3_wgrad_workspace")
    return int(b.value)


def nn_conv3x3_bwd_weight(x, dy, dw, db, work, accumulate, n, h, wd, ci, co):
    nbytes = work.numel() * work.element_size()
    _check(load().nn_conv3x3_bwd_weight(_p(x), _p(dy), _p(dw), _p(db), _p(work), nbytes, int(accumulate), n, h, wd,
                                        ci, co, _stream()), "nn_conv3x3_bwd_weight")


def nn_relu_bwd(dy, y, dx):
    _check(load().nn_relu_bwd(_p(dy), _p(y), _p(dx), dy.numel(), _stream()), "nn_relu_bwd")


def nn_add(a, b, out):
    _check(load().nn_add(_p(a), _p(b), _p(out), a.numel(), _stream()), "nn_add")


def nn_pool2(backward, src, dst, n, h, wd, c):
    _check(load().nn_pool2(int(backward), _p(src), _p(dst), n, h, wd, c, _stream()), "nn_pool2")


def nn_up2(backward, src, dst, n, h, wd, c):
    _check(load().nn_up2(int(backward), _p(src), _p(dst), n, h, wd, c, _stream()), "nn_up2")


def nn_mse(pred, target, dpred, cpad, npix, nch, loss, work):
    nbytes = work.numel() * work.element_size()
    _check(load().nn_mse(_p(pred), _p(target), _p(dpred), int(cpad), int(npix), int(nch), _p(loss), _p(work),
                         nbytes, _stream()), "nn_mse")


def nn_mse_noalloc(pred, target, dpred, cpad, npix, nch, loss):
    _check(load().nn_mse_noalloc(_p(pred), _p(target), _p(dpred), int(cpad), int(npix), int(nch), _p(loss),
                                 _stream()), "nn_mse_noalloc")


def nn_adam(w, w16, wflip, g, m, v, co, ci, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
    _check(load().nn_adam(_p(w), _p(w16), _p(wflip), _p(g), _p(m), _p(v), w.numel(), int(co), int(ci), int(step),
                          float(lr), float(beta1), float(beta2), float(eps), float(weight_decay), _stream()),
           "nn_adam")


def nn_cast_weights(w, w16, wflip, co, ci):
    _check(load().nn_cast_weights(_p(w), _p(w16), _p(wflip), int(co), int(ci), _stream()), "nn_cast_weights")


def nn_features(cfgs, x, cpad):
    _check(load().nn_features(_params(cfgs), len(cfgs), _p(x), int(cpad), _stream()), "nn_features")


def nn_to_fields(cfgs, pred, fields, phi_from_net=False):
    _check(load().nn_to_fields(_params(cfgs), len(cfgs), _p(pred), _p(fields), int(bool(phi_from_net)), _stream()),
           "nn_to_fields")


def nn_targets(cfgs, fields, target):
    _check(load().nn_targets(_params(cfgs), len(cfgs), _p(fields), _p(target), _stream()), "nn_targets")


def nn_velocity_scale(cfg):
    p = _lbm.make_params(cfg)
    return float(load().nn_velocity_scale(ctypes.byref(p)))
