"""Python binding of the learned upsampler (include/sg_upsampler.h).

Argument marshalling only: every step runs in the HIP kernels of libsg.so.
Tensors are torch CUDA tensors (device pointers), weights numpy float32.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import sg

_lib = sg.lib()
_P = C.c_void_p
_lib.sg_up_param_count.restype = C.c_int64
_lib.sg_up_create.argtypes = [C.c_int32, C.c_int64, C.POINTER(_P)]
_lib.sg_up_destroy.argtypes = [_P]
_lib.sg_up_set_weights.argtypes = [_P, C.POINTER(C.c_float), C.c_int64]
_lib.sg_up_get_weights.argtypes = [_P, C.POINTER(C.c_float), C.c_int64]
_lib.sg_up_forward.argtypes = [_P, C.c_int32, C.c_int32, C.c_int32, _P, _P, _P, C.c_double, _P,
                               _P, C.POINTER(C.c_double), _P]
_lib.sg_up_gradients.argtypes = [_P, C.c_int32, C.c_int32, C.c_int32, _P, _P, C.c_double, _P,
                                 C.c_double, C.POINTER(C.c_float), C.POINTER(C.c_double), _P]
_lib.sg_up_train_step.argtypes = [_P, C.c_int32, C.c_int32, C.c_int32, _P, _P, C.c_double, _P,
                                  C.c_double, C.c_double, C.POINTER(C.c_double), _P]
_lib.sg_up_read_buffer.argtypes = [_P, C.c_int32, _P, C.c_int64]
_lib.sg_up_set_fused.argtypes = [_P, C.c_int32]
_lib.sg_up_forward_flag.argtypes = [_P, C.c_int32, C.c_int32, C.c_int32, _P, _P, _P, C.c_double,
                                    _P, _P, C.c_double, _P, _P]
for _f in ("sg_up_create", "sg_up_destroy", "sg_up_set_weights", "sg_up_get_weights",
           "sg_up_forward", "sg_up_gradients", "sg_up_train_step", "sg_up_read_buffer",
           "sg_up_set_fused", "sg_up_forward_flag"):
    getattr(_lib, _f).restype = C.c_int

LAYERS = ((8, 32), (32, 32), (32, 32), (32, 32))


def param_count() -> int:
    return int(_lib.sg_up_param_count())


def pack(params) -> np.ndarray:
    """[(w [9, cin, 32], b [32]) per layer] -> packed float32 vector."""
    return np.concatenate([np.concatenate([np.asarray(w, np.float32).ravel(),
                                           np.asarray(b, np.float32).ravel()])
                           for w, b in params]).astype(np.float32)


def unpack(vec):
    out, o = [], 0
    for ci, co in LAYERS:
        n = 9 * ci * co
        out.append((vec[o:o + n].reshape(9, ci, co), vec[o + n:o + n + co]))
        o += n + co
    return out


def _dp(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Upsampler:
    def __init__(self, max_pixels: int, device: int = 0):
        h = C.c_void_p()
        sg._check(_lib.sg_up_create(int(device), int(max_pixels), C.byref(h)), "sg_up_create")
        self.h = h

    def close(self):
        if self.h is not None:
            sg._check(_lib.sg_up_destroy(self.h), "sg_up_destroy")
            self.h = None

    def set_weights(self, vec):
        v = np.ascontiguousarray(vec, dtype=np.float32)
        sg._check(_lib.sg_up_set_weights(self.h, v.ctypes.data_as(C.POINTER(C.c_float)), len(v)),
                  "sg_up_set_weights")

    def set_fused(self, fused: bool):
        """Inference in one fused kernel (default) or layer by layer."""
        sg._check(_lib.sg_up_set_fused(self.h, int(bool(fused))), "sg_up_set_fused")

    def get_weights(self) -> np.ndarray:
        v = np.zeros(param_count(), np.float32)
        sg._check(_lib.sg_up_get_weights(self.h, v.ctypes.data_as(C.POINTER(C.c_float)), len(v)),
                  "sg_up_get_weights")
        return v

    def forward(self, rgba, depth, depth_scale, out_rgba, out_err=None, predict=False,
                stream=None, content=None):
        """content: None, or the input's content mask (uint8 device tensor
        [n][(h + 7) // 8][(w + 7) // 8], as the render fills tile_any)."""
        n, h, w = rgba.shape[:3]
        mse = (C.c_double * n)() if predict else None
        sg._check(_lib.sg_up_forward(self.h, n, h, w, _dp(rgba), _dp(depth), _dp(content),
                                     float(depth_scale), _dp(out_rgba), _dp(out_err), mse,
                                     sg._stream(stream)), "sg_up_forward")
        return np.array(mse[:]) if predict else None

    def forward_flag(self, rgba, depth, depth_scale, out_rgba, threshold_db, fallback,
                     out_err=None, stream=None, content=None):
        """Inference and the fallback decision on the device: fallback (a
        one-element int32 device tensor) = 1 when the predicted PSNR of the
        batch is below threshold_db. Asynchronous."""
        n, h, w = rgba.shape[:3]
        sg._check(_lib.sg_up_forward_flag(self.h, n, h, w, _dp(rgba), _dp(depth), _dp(content),
                                          float(depth_scale), _dp(out_rgba), _dp(out_err),
                                          float(threshold_db), _dp(fallback),
                                          sg._stream(stream)), "sg_up_forward_flag")

    def gradients(self, rgba, depth, depth_scale, target, err_weight=1.0, stream=None):
        n, h, w = rgba.shape[:3]
        g = np.zeros(param_count(), np.float32)
        loss = C.c_double()
        sg._check(_lib.sg_up_gradients(self.h, n, h, w, _dp(rgba), _dp(depth), float(depth_scale),
                                       _dp(target), float(err_weight),
                                       g.ctypes.data_as(C.POINTER(C.c_float)), C.byref(loss),
                                       sg._stream(stream)), "sg_up_gradients")
        return float(loss.value), g

    def train_step(self, rgba, depth, depth_scale, target, lr, err_weight=1.0, want_loss=False,
                   stream=None):
        n, h, w = rgba.shape[:3]
        loss = C.c_double() if want_loss else None
        sg._check(_lib.sg_up_train_step(self.h, n, h, w, _dp(rgba), _dp(depth),
                                        float(depth_scale), _dp(target), float(err_weight),
                                        float(lr), C.byref(loss) if want_loss else None,
                                        sg._stream(stream)), "sg_up_train_step")
        return float(loss.value) if want_loss else None

    def read_buffer(self, which: int, shape, dtype):
        import torch
        n = int(np.prod(shape))
        nbytes = n * (2 if dtype == "bf16" else 4)
        raw = np.zeros(nbytes, np.uint8)
        sg._check(_lib.sg_up_read_buffer(self.h, int(which), C.c_void_p(raw.ctypes.data),
                                         nbytes), "sg_up_read_buffer")
        if dtype == "bf16":
            return torch.from_numpy(raw.view(np.int16).copy()).view(torch.bfloat16).float() \
                .numpy().astype(np.float64).reshape(shape)
        return raw.view(np.float32).astype(np.float64).reshape(shape)
