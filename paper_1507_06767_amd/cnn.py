"""ctypes binding of include/lbm_cnn.h: same names, argument marshalling only.

Tensors are torch tensors on the GPU; their dtype, contiguity, device and
size are checked here against what the C function will touch, so that no
kernel reads or writes past a buffer.  Every function returns the C status
(0 on success) and enqueues its kernels on `stream` (torch's current stream
when None).
"""
from __future__ import annotations

import ctypes

import torch

from . import abi

LBM_CNN_TAPS = 27
LBM_CNN_LOSS_FLOATS = 257
LBM_CNN_HYPER_FLOATS = 8
LBM_CNN_MAX_LAYERS = 8


class lbm_cnn_layer(ctypes.Structure):
    _fields_ = [("w", ctypes.c_void_p), ("b", ctypes.c_void_p), ("work", ctypes.c_void_p),
                ("mw", ctypes.c_void_p), ("vw", ctypes.c_void_p), ("mb", ctypes.c_void_p), ("vb", ctypes.c_void_p),
                ("packed", ctypes.c_void_p), ("packed_flip", ctypes.c_void_p), ("gw", ctypes.c_void_p),
                ("gb", ctypes.c_void_p), ("co", ctypes.c_int32), ("ci", ctypes.c_int32)]

_lib = abi._lib
_P = ctypes.c_void_p
_I32, _I64, _F = ctypes.c_int32, ctypes.c_int64, ctypes.c_float
_SIG = {
    "lbm_cnn_packed_size": ([_I32, _I32], _I64),
    "lbm_cnn_pack_weights": ([_P, _I32, _I32, _I32, _P, _P], _I32),
    "lbm_cnn_conv3d_forward": ([_P, _I32, _I32, _I32, _I32, _I32, _P, _I32, _P, _I32, _P, _P, _P], _I32),
    "lbm_cnn_wgrad_workspace": ([_I32, _I32, _I32, _I32, _I32, _I32], _I64),
    "lbm_cnn_conv3d_wgrad": ([_P, _P, _I32, _I32, _I32, _I32, _I32, _I32, _P, _P, _P, _P], _I32),
    "lbm_cnn_relu_backward": ([_P, _P, _I64, _P], _I32),
    "lbm_cnn_mse": ([_P, _I32, _P, _I64, _P, _P, _P], _I32),
    "lbm_cnn_adam": ([_P, _P, _P, _P, _I64, _F, _F, _F, _F, _I32, _P], _I32),
    "lbm_cnn_adam_begin": ([_P, _F, _F, _F, _F, _P], _I32),
    "lbm_cnn_adam_dev": ([_P, _P, _P, _P, _I64, _P, _P], _I32),
    "lbm_cnn_adam_layer": ([_P] * 8 + [_I32, _I32, _P, _P, _P, _P], _I32),
    "lbm_cnn_conv3d_wgrad_partials": ([_P, _P, _I32, _I32, _I32, _I32, _I32, _I32, _P, _P], _I32),
    "lbm_cnn_backward_layer": ([_P, _P, _I32, _I32, _I32, _I32, _I32, _I32, _P, _P, _P, _P, _P], _I32),
    "lbm_cnn_adam_layer_fold": ([_P, _P, _P, _I32, _I32, _I32, _I32, _P, _P, _P, _P, _I32, _I32, _P, _P, _P, _P,
                                 _P, _P], _I32),
    "lbm_cnn_adam_layers_fold": ([_I32, ctypes.POINTER(lbm_cnn_layer), _I32, _I32, _I32, _I32, _P, _P], _I32),
}
for _name, (_args, _res) in _SIG.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res


def pad4(c: int) -> int:
    return (c + 3) // 4 * 4


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ptr(t, dtype, numel, name, align=4):
    if t is None:
        return None
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous {dtype} CUDA tensor")
    if t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, needs {numel}")
    if t.data_ptr() % align:
        raise ValueError(f"{name} is not {align}-byte aligned")
    return t.data_ptr()


def lbm_cnn_packed_size(co: int, ci: int) -> int:
    return int(_lib.lbm_cnn_packed_size(int(co), int(ci)))


def lbm_cnn_pack_weights(w, co, ci, flip, packed, stream=None):
    size = lbm_cnn_packed_size(ci, co) if flip else lbm_cnn_packed_size(co, ci)
    return _lib.lbm_cnn_pack_weights(_ptr(w, torch.float32, co * LBM_CNN_TAPS * ci, "w"), int(co), int(ci),
                                     int(bool(flip)), _ptr(packed, torch.int16, size, "packed", 8),
                                     _stream(stream))


def lbm_cnn_conv3d_forward(x, n, d, h, wd, ci, packed, co, bias, relu, mask, y, stream=None):
    nv = n * d * h * wd
    return _lib.lbm_cnn_conv3d_forward(
        _ptr(x, torch.float32, nv * pad4(ci), "x", 16), n, d, h, wd, ci,
        _ptr(packed, torch.int16, lbm_cnn_packed_size(co, ci), "packed", 8), co,
        _ptr(bias, torch.float32, co, "bias"), int(bool(relu)),
        _ptr(mask, torch.float32, nv * pad4(co), "mask"),
        _ptr(y, torch.float32, nv * pad4(co), "y", 16), _stream(stream))


def lbm_cnn_wgrad_workspace(n, d, h, wd, ci, co) -> int:
    return int(_lib.lbm_cnn_wgrad_workspace(n, d, h, wd, ci, co))


def lbm_cnn_conv3d_wgrad(x, gz, n, d, h, wd, ci, co, work, gw, gb, stream=None):
    nv = n * d * h * wd
    ws = lbm_cnn_wgrad_workspace(n, d, h, wd, ci, co) // 4
    return _lib.lbm_cnn_conv3d_wgrad(
        _ptr(x, torch.float32, nv * pad4(ci), "x"), _ptr(gz, torch.float32, nv * pad4(co), "gz"),
        n, d, h, wd, ci, co, _ptr(work, torch.float32, ws, "work"),
        _ptr(gw, torch.float32, co * LBM_CNN_TAPS * ci, "gw"), _ptr(gb, torch.float32, co, "gb"),
        _stream(stream))


def lbm_cnn_conv3d_wgrad_partials(x, gz, n, d, h, wd, ci, co, work, stream=None):
    nv = n * d * h * wd
    ws = lbm_cnn_wgrad_workspace(n, d, h, wd, ci, co) // 4
    return _lib.lbm_cnn_conv3d_wgrad_partials(
        _ptr(x, torch.float32, nv * pad4(ci), "x"), _ptr(gz, torch.float32, nv * pad4(co), "gz"),
        n, d, h, wd, ci, co, _ptr(work, torch.float32, ws, "work"), _stream(stream))


def lbm_cnn_backward_layer(x, gz, n, d, h, wd, ci, co, work, packed_flip, mask, gin, stream=None):
    nv = n * d * h * wd
    ws = lbm_cnn_wgrad_workspace(n, d, h, wd, ci, co) // 4
    return _lib.lbm_cnn_backward_layer(
        _ptr(x, torch.float32, nv * pad4(ci), "x"), _ptr(gz, torch.float32, nv * pad4(co), "gz", 16),
        n, d, h, wd, ci, co, _ptr(work, torch.float32, ws, "work"),
        _ptr(packed_flip, torch.int16, lbm_cnn_packed_size(ci, co), "packed_flip", 8),
        _ptr(mask, torch.float32, nv * pad4(ci), "mask"), _ptr(gin, torch.float32, nv * pad4(ci), "gin", 16),
        _stream(stream))


def lbm_cnn_relu_backward(a, g, count, stream=None):
    return _lib.lbm_cnn_relu_backward(_ptr(a, torch.float32, count, "a"), _ptr(g, torch.float32, count, "g"),
                                      int(count), _stream(stream))


def lbm_cnn_mse(y, ystride, target, count, g, loss, stream=None):
    return _lib.lbm_cnn_mse(_ptr(y, torch.float32, count * ystride, "y"), int(ystride),
                            _ptr(target, torch.float32, count, "target"), int(count),
                            _ptr(g, torch.float32, count * ystride, "g"),
                            _ptr(loss, torch.float32, LBM_CNN_LOSS_FLOATS, "loss"),
                            _stream(stream))


def lbm_cnn_adam(w, g, m, v, count, lr, beta1, beta2, eps, t, stream=None):
    return _lib.lbm_cnn_adam(*(_ptr(a, torch.float32, count, nm) for a, nm in ((w, "w"), (g, "g"), (m, "m"),
                                                                               (v, "v"))),
                             int(count), float(lr), float(beta1), float(beta2), float(eps), int(t), _stream(stream))


def lbm_cnn_adam_begin(hyper, lr, beta1, beta2, eps, stream=None):
    return _lib.lbm_cnn_adam_begin(_ptr(hyper, torch.float32, LBM_CNN_HYPER_FLOATS, "hyper"), float(lr),
                                   float(beta1), float(beta2), float(eps), _stream(stream))


def lbm_cnn_adam_dev(w, g, m, v, count, hyper, stream=None):
    return _lib.lbm_cnn_adam_dev(*(_ptr(a, torch.float32, count, nm) for a, nm in ((w, "w"), (g, "g"), (m, "m"),
                                                                                   (v, "v"))),
                                 int(count), _ptr(hyper, torch.float32, LBM_CNN_HYPER_FLOATS, "hyper"),
                                 _stream(stream))


def lbm_cnn_adam_layer(w, b, gw, gb, mw, vw, mb, vb, co, ci, packed, packed_flip, hyper, stream=None):
    nw, nb = co * LBM_CNN_TAPS * ci, co
    args = [_ptr(w, torch.float32, nw, "w"), _ptr(b, torch.float32, nb, "b"), _ptr(gw, torch.float32, nw, "gw"),
            _ptr(gb, torch.float32, nb, "gb"), _ptr(mw, torch.float32, nw, "mw"), _ptr(vw, torch.float32, nw, "vw"),
            _ptr(mb, torch.float32, nb, "mb"), _ptr(vb, torch.float32, nb, "vb")]
    return _lib.lbm_cnn_adam_layer(*args, int(co), int(ci),
                                   _ptr(packed, torch.int16, lbm_cnn_packed_size(co, ci), "packed", 8),
                                   _ptr(packed_flip, torch.int16, lbm_cnn_packed_size(ci, co), "packed_flip", 8),
                                   _ptr(hyper, torch.float32, LBM_CNN_HYPER_FLOATS, "hyper"), _stream(stream))


def lbm_cnn_adam_layer_fold(w, b, work, n, d, h, wd, mw, vw, mb, vb, co, ci, packed, packed_flip, hyper,
                            gw=None, gb=None, stream=None):
    nw, nb = co * LBM_CNN_TAPS * ci, co
    ws = lbm_cnn_wgrad_workspace(n, d, h, wd, ci, co) // 4
    return _lib.lbm_cnn_adam_layer_fold(
        _ptr(w, torch.float32, nw, "w"), _ptr(b, torch.float32, nb, "b"), _ptr(work, torch.float32, ws, "work"),
        n, d, h, wd, _ptr(mw, torch.float32, nw, "mw"), _ptr(vw, torch.float32, nw, "vw"),
        _ptr(mb, torch.float32, nb, "mb"), _ptr(vb, torch.float32, nb, "vb"), int(co), int(ci),
        _ptr(packed, torch.int16, lbm_cnn_packed_size(co, ci), "packed", 8),
        _ptr(packed_flip, torch.int16, lbm_cnn_packed_size(ci, co), "packed_flip", 8),
        _ptr(hyper, torch.float32, LBM_CNN_HYPER_FLOATS, "hyper"), _ptr(gw, torch.float32, nw, "gw"),
        _ptr(gb, torch.float32, nb, "gb"), _stream(stream))


def lbm_cnn_adam_layers_fold(layers, n, d, h, wd, hyper, stream=None):
    """layers: a sequence of dicts with the arguments of
    lbm_cnn_adam_layer_fold (w, b, work, mw, vw, mb, vb, packed, packed_flip,
    gw, gb, co, ci; gw, gb may be None)."""
    if not 1 <= len(layers) <= LBM_CNN_MAX_LAYERS:
        raise ValueError(f"1 to {LBM_CNN_MAX_LAYERS} layers")
    arr = (lbm_cnn_layer * len(layers))()
    for k, L in enumerate(layers):
        co, ci = int(L["co"]), int(L["ci"])
        nw, nb = co * LBM_CNN_TAPS * ci, co
        ws = lbm_cnn_wgrad_workspace(n, d, h, wd, ci, co) // 4
        arr[k] = lbm_cnn_layer(
            _ptr(L["w"], torch.float32, nw, "w"), _ptr(L["b"], torch.float32, nb, "b"),
            _ptr(L["work"], torch.float32, ws, "work"), _ptr(L["mw"], torch.float32, nw, "mw"),
            _ptr(L["vw"], torch.float32, nw, "vw"), _ptr(L["mb"], torch.float32, nb, "mb"),
            _ptr(L["vb"], torch.float32, nb, "vb"),
            _ptr(L["packed"], torch.int16, lbm_cnn_packed_size(co, ci), "packed", 8),
            _ptr(L["packed_flip"], torch.int16, lbm_cnn_packed_size(ci, co), "packed_flip", 8),
            _ptr(L.get("gw"), torch.float32, nw, "gw"), _ptr(L.get("gb"), torch.float32, nb, "gb"), co, ci)
    return _lib.lbm_cnn_adam_layers_fold(len(layers), arr, n, d, h, wd,
                                         _ptr(hyper, torch.float32, LBM_CNN_HYPER_FLOATS, "hyper"), _stream(stream))
