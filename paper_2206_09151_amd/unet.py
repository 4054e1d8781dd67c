"""ctypes binding of the artefact-correction network (include/tomo_unet.h): argument
marshalling only; every step runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes

import torch

from . import tomo

_LIB = tomo.lib()
_vp, _i32, _f = ctypes.c_void_p, ctypes.c_int32, ctypes.c_float
_LIB.tomo_unet_param_count.argtypes = []
_LIB.tomo_unet_param_count.restype = _i32
_LIB.tomo_unet_create.argtypes = [_i32, ctypes.POINTER(_vp)]
_LIB.tomo_unet_forward.argtypes = [_vp, _vp, _vp, _vp, _vp]
_LIB.tomo_unet_gradient.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp]
_LIB.tomo_unet_adam.argtypes = [_vp, _vp, _vp, _vp, _vp, _i32, _f, _f, _f, _f, _vp]
_LIB.tomo_unet_error.argtypes = [_vp]
_LIB.tomo_unet_error.restype = ctypes.c_char_p
_LIB.tomo_unet_destroy.argtypes = [_vp]
for _name in ("tomo_unet_create", "tomo_unet_forward", "tomo_unet_gradient", "tomo_unet_adam", "tomo_unet_destroy"):
    getattr(_LIB, _name).restype = ctypes.c_int

EXPORTED = ["tomo_unet_param_count", "tomo_unet_create", "tomo_unet_forward", "tomo_unet_gradient",
            "tomo_unet_adam", "tomo_unet_error", "tomo_unet_destroy"]


def param_count() -> int:
    return int(_LIB.tomo_unet_param_count())


class Net:
    """Workspace of the network for volumes of edge n."""

    def __init__(self, n: int):
        out = ctypes.c_void_p()
        st = _LIB.tomo_unet_create(int(n), ctypes.byref(out))
        if st != tomo.OK:
            raise tomo.TomoError(st, _LIB.tomo_unet_error(None).decode())
        self._h = out
        self.n = n

    def _check(self, st):
        if st != tomo.OK:
            raise tomo.TomoError(st, _LIB.tomo_unet_error(self._h).decode())

    def _s(self, stream):
        return ctypes.c_void_p(tomo._stream_ptr(stream))

    # every buffer is checked for its element type and size before the call: the kernels
    # read and write exactly n^3 voxels and param_count() parameters
    def _vol(self, t, name):
        return tomo._dptr(t, torch.float32, 4 * self.n ** 3, name)

    def _par(self, t, name):
        return tomo._dptr(t, torch.float32, 4 * param_count(), name)

    def forward(self, params, x, y, stream=None):
        self._check(_LIB.tomo_unet_forward(self._h, self._par(params, "params"), self._vol(x, "x"), self._vol(y, "y"),
                                           self._s(stream)))

    def gradient(self, params, x, target, grad, loss, stream=None):
        self._check(_LIB.tomo_unet_gradient(self._h, self._par(params, "params"), self._vol(x, "x"),
                                            self._vol(target, "target"), self._par(grad, "grad"),
                                            tomo._dptr(loss, torch.float64, 8, "loss"), self._s(stream)))

    def adam(self, params, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self._check(_LIB.tomo_unet_adam(self._h, self._par(params, "params"), self._par(grad, "grad"),
                                        self._par(m, "m"), self._par(v, "v"),
                                        int(step), float(lr), float(beta1), float(beta2), float(eps),
                                        self._s(stream)))

    def destroy(self):
        if getattr(self, "_h", None):
            _LIB.tomo_unet_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
