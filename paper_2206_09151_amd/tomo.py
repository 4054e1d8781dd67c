"""ctypes binding of libtomo.so (include/tomo.h): argument marshalling only.

Device memory and streams come from PyTorch (ROCm); every step of the
reconstruction runs in the library's HIP kernels.  Importing this module
raises if the built library is missing -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
# PyTorch is imported before the library is loaded so that libtomo.so binds to the HIP
# runtime torch already loaded (same soname): one runtime owns the streams and the
# device memory that are passed across the boundary.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtomo.so")

OK, EINVAL, ENOMEM, EDEVICE, EDOMAIN, EUNSUPPORTED = range(6)
RAMP_AXIS, RAMP_ISO, SAMPLING = 0, 1, 2
F32, BF16, F16 = 0, 1, 2
_MODES = {"ramp_axis": RAMP_AXIS, "ramp_iso": RAMP_ISO, "sampling": SAMPLING}

EXPORTED = [
    "tomo_plan", "tomo_backpropagate", "tomo_grid", "tomo_reconstruct", "tomo_reconstruct_async", "tomo_sync",
    "tomo_filtered_spectra", "tomo_workspace_bytes", "tomo_batch_capacity", "tomo_stack_bytes",
    "tomo_status_string", "tomo_last_error", "tomo_plan_error", "tomo_destroy",
    "tomo_timing_enable", "tomo_timing_read", "tomo_fourier_reconstruct", "tomo_fourier_reconstruct_async",
    "tomo_fourier_entries",
    "tomo_batch_create", "tomo_batch_launch", "tomo_batch_sync", "tomo_batch_error", "tomo_batch_destroy",
    "tomo_grid_rows", "tomo_backpropagate_noalloc",
]
KERNEL_KINDS = ("spectra", "planes", "grid", "fgrid", "finverse")
NOALLOC_SCRATCH_BYTES = 32 << 20    # TOMO_NOALLOC_SCRATCH_BYTES
FOURIER_OPERATOR, FOURIER_SPLAT = 1, 2
EQ11, EQ12 = 11, 12


class TomoParams(ctypes.Structure):
    _fields_ = [
        ("n_vox", ctypes.c_int32), ("n_pix", ctypes.c_int32), ("n_planes", ctypes.c_int32),
        ("n_angles", ctypes.c_int32),
        ("voxel_size", ctypes.c_double), ("wavelength", ctypes.c_double), ("sigma", ctypes.c_double),
        ("epsilon", ctypes.c_double), ("eps_sampling", ctypes.c_double), ("i_in", ctypes.c_double),
        ("ewald", ctypes.c_int32), ("weight_mode", ctypes.c_int32), ("plane_dtype", ctypes.c_int32),
        ("angle_batch", ctypes.c_int32), ("fourier", ctypes.c_int32), ("tune", ctypes.c_int32),
        ("max_workspace_bytes", ctypes.c_size_t),
    ]


class TomoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libtomo.so not built at {path}; run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    dptr = ctypes.POINTER(ctypes.c_double)
    lib.tomo_plan.argtypes = [ctypes.POINTER(TomoParams), dptr, dptr, dptr, vp, ctypes.POINTER(vp)]
    lib.tomo_backpropagate.argtypes = [vp, vp, i32, i32, vp, vp]
    lib.tomo_backpropagate_noalloc.argtypes = [vp, vp, i32, i32, vp, vp]
    lib.tomo_grid.argtypes = [vp, vp, i32, i32, vp, vp]
    lib.tomo_reconstruct.argtypes = [vp, vp, vp, vp]
    lib.tomo_reconstruct_async.argtypes = [vp, vp, vp, vp]
    lib.tomo_sync.argtypes = [vp, vp]
    lib.tomo_filtered_spectra.argtypes = [vp, vp, i32, i32, vp, vp]
    lib.tomo_workspace_bytes.argtypes = [ctypes.POINTER(TomoParams)]
    lib.tomo_workspace_bytes.restype = sz
    lib.tomo_batch_capacity.argtypes = [vp]
    lib.tomo_stack_bytes.argtypes = [vp, i32]
    lib.tomo_stack_bytes.restype = sz
    lib.tomo_status_string.argtypes = [ctypes.c_int]
    lib.tomo_status_string.restype = ctypes.c_char_p
    lib.tomo_last_error.argtypes = [vp]
    lib.tomo_last_error.restype = ctypes.c_char_p
    lib.tomo_plan_error.argtypes = []
    lib.tomo_plan_error.restype = ctypes.c_char_p
    lib.tomo_destroy.argtypes = [vp]
    lib.tomo_timing_enable.argtypes = [vp, i32]
    lib.tomo_timing_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), i32]
    lib.tomo_fourier_reconstruct.argtypes = [vp, vp, i32, ctypes.c_double, vp, vp]
    lib.tomo_fourier_reconstruct_async.argtypes = [vp, vp, i32, ctypes.c_double, vp, vp]
    lib.tomo_grid_rows.argtypes = [vp]
    lib.tomo_grid_rows.restype = i32
    lib.tomo_fourier_entries.argtypes = [vp]
    lib.tomo_fourier_entries.restype = sz
    lib.tomo_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), i32, i32,
                                      ctypes.POINTER(vp)]
    lib.tomo_batch_launch.argtypes = [vp, vp]
    lib.tomo_batch_sync.argtypes = [vp, vp]
    lib.tomo_batch_error.argtypes = [vp]
    lib.tomo_batch_error.restype = ctypes.c_char_p
    lib.tomo_batch_destroy.argtypes = [vp]
    for name in ("tomo_batch_create", "tomo_batch_launch", "tomo_batch_sync", "tomo_batch_destroy"):
        getattr(lib, name).restype = ctypes.c_int
    for name in ("tomo_plan", "tomo_backpropagate", "tomo_backpropagate_noalloc", "tomo_grid", "tomo_reconstruct", "tomo_reconstruct_async", "tomo_sync",
                 "tomo_filtered_spectra", "tomo_destroy", "tomo_batch_capacity", "tomo_timing_enable",
                 "tomo_timing_read", "tomo_fourier_reconstruct", "tomo_fourier_reconstruct_async"):
        getattr(lib, name).restype = ctypes.c_int
    return lib


_LIB = load_library()


def lib() -> ctypes.CDLL:
    return _LIB


@dataclass
class Params:
    """Problem constants as the paper states them (SI units); see include/tomo.h."""
    n_vox: int
    n_angles: int
    voxel_size: float
    wavelength: float
    sigma: float
    epsilon: float
    n_pix: int = 0
    n_planes: int = 0
    ewald: int = 1
    weight_mode: str = "ramp_axis"
    eps_sampling: float = 1e-3
    i_in: float = 1.0
    plane_dtype: int = F32
    angle_batch: int = 0
    fourier: int = 0
    tune: int = 0
    max_workspace_bytes: int = 0

    def to_c(self) -> TomoParams:
        mode = _MODES[self.weight_mode] if isinstance(self.weight_mode, str) else int(self.weight_mode)
        return TomoParams(self.n_vox, self.n_pix, self.n_planes, self.n_angles, self.voxel_size,
                          self.wavelength, self.sigma, self.epsilon, self.eps_sampling, self.i_in,
                          self.ewald, mode, self.plane_dtype, self.angle_batch, self.fourier,
                          self.tune, self.max_workspace_bytes)


def _stream_ptr(stream) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _dptr(t, dtype=None, min_bytes: int = 0, name: str = "tensor") -> int:
    """Device address of a contiguous device tensor, after checking its element type and
    that it holds at least min_bytes: the kernels read and write exactly the sizes the
    plan implies, so a short or mistyped buffer is refused here, before any launch."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name}: expected {dtype}, got {t.dtype}")
    have = t.numel() * t.element_size()
    if have < min_bytes:
        raise ValueError(f"{name}: holds {have} bytes, the call needs {min_bytes}")
    return t.data_ptr()


def workspace_bytes(params: Params) -> int:
    return int(_LIB.tomo_workspace_bytes(ctypes.byref(params.to_c())))


class Plan:
    """A reconstruction plan: geometry, filter tables and workspace on the device."""

    def __init__(self, params: Params, dirs, dist, vaxes=None, stream=None):
        self.params = params
        d = np.ascontiguousarray(dirs, dtype=np.float64)
        r = np.ascontiguousarray(np.broadcast_to(np.asarray(dist, dtype=np.float64), (d.shape[0],)))
        if d.ndim != 2 or d.shape[1] != 3 or d.shape[0] != params.n_angles:
            raise ValueError("dirs must be [n_angles, 3]")
        va = None if vaxes is None else np.ascontiguousarray(vaxes, dtype=np.float64)
        if va is not None and va.shape != d.shape:
            raise ValueError("vaxes must be [n_angles, 3]")
        dp = ctypes.POINTER(ctypes.c_double)
        out = ctypes.c_void_p()
        self._c = params.to_c()
        st = _LIB.tomo_plan(ctypes.byref(self._c), d.ctypes.data_as(dp),
                            None if va is None else va.ctypes.data_as(dp), r.ctypes.data_as(dp),
                            ctypes.c_void_p(_stream_ptr(stream)), ctypes.byref(out))
        if st != OK:
            raise TomoError(st, _LIB.tomo_plan_error().decode())
        self._h = out
        self.n = params.n_angles
        self.N = params.n_vox
        self.M = params.n_pix or params.n_vox
        self.K = (params.n_planes or params.n_vox) if params.ewald else 1

    # ---------------------------------------------------------------- helpers
    def _check(self, st: int):
        if st != OK:
            raise TomoError(st, _LIB.tomo_last_error(self._h).decode())

    def _images(self, t, nb: int) -> int:
        return _dptr(t, torch.float32, 4 * nb * self.M * self.M, "images")

    def _volume(self, t) -> int:
        return _dptr(t, torch.float32, 4 * self.N ** 3, "volume")

    def _planes(self, t, nb: int) -> int:
        return _dptr(t, self.stack_dtype, int(_LIB.tomo_stack_bytes(self._h, nb)), "planes")

    @property
    def grid_rows(self) -> int:
        """Voxel rows per thread of the gridding kernel (autotuned with Params.tune)."""
        return int(_LIB.tomo_grid_rows(self._h))

    @property
    def fourier_entries(self) -> int:
        """Non-zero entries of the Fourier-space gridding operator (fourier = 1)."""
        return int(_LIB.tomo_fourier_entries(self._h))

    @property
    def batch(self) -> int:
        return int(_LIB.tomo_batch_capacity(self._h))

    def stack_shape(self, nb: int) -> tuple:
        return (nb, self.M, self.K, self.M)

    @property
    def stack_dtype(self):
        """torch dtype of the plane stack (plane_dtype)."""
        return {F32: torch.float32, BF16: torch.bfloat16, F16: torch.float16}[self.params.plane_dtype]

    # ---------------------------------------------------------------- entry points
    def backpropagate(self, images, first: int, nb: int, planes, stream=None):
        nb = int(nb)
        self._check(_LIB.tomo_backpropagate(self._h, self._images(images, max(nb, 0)), first, nb,
                                            self._planes(planes, max(nb, 0)), ctypes.c_void_p(_stream_ptr(stream))))

    def backpropagate_noalloc(self, images, first: int, nb: int, planes, stream=None):
        """backpropagate without any allocation: the spectra live in the library's static
        per-GPU workspace (at most NOALLOC_SCRATCH_BYTES / (16 M^2) views per call)."""
        nb = int(nb)
        self._check(_LIB.tomo_backpropagate_noalloc(self._h, self._images(images, max(nb, 0)), first, nb,
                                                    self._planes(planes, max(nb, 0)),
                                                    ctypes.c_void_p(_stream_ptr(stream))))

    def grid(self, planes, first: int, nb: int, volume, stream=None):
        nb = int(nb)
        self._check(_LIB.tomo_grid(self._h, self._planes(planes, max(nb, 0)), first, nb, self._volume(volume),
                                   ctypes.c_void_p(_stream_ptr(stream))))

    def reconstruct(self, images, volume, stream=None):
        self._check(_LIB.tomo_reconstruct(self._h, self._images(images, self.n), self._volume(volume),
                                          ctypes.c_void_p(_stream_ptr(stream))))

    def reconstruct_async(self, images, volume, stream=None):
        """Enqueue a whole reconstruction without waiting; domain errors surface at sync()."""
        self._check(_LIB.tomo_reconstruct_async(self._h, self._images(images, self.n), self._volume(volume),
                                                ctypes.c_void_p(_stream_ptr(stream))))

    def sync(self, stream=None):
        self._check(_LIB.tomo_sync(self._h, ctypes.c_void_p(_stream_ptr(stream))))

    def filtered_spectra(self, images, first: int, nb: int, out, stream=None):
        nb = int(nb)
        self._check(_LIB.tomo_filtered_spectra(self._h, self._images(images, max(nb, 0)), first, nb,
                                               _dptr(out, torch.float32, 8 * max(nb, 0) * self.M * self.M, "out"),
                                               ctypes.c_void_p(_stream_ptr(stream))))

    def fourier_reconstruct(self, images, volume, variant: int = EQ11, nsr: float = 0.0, stream=None):
        """The Fourier-space form (eq. 11 or eq. 12 by 3D gridding, NSR filter)."""
        self._check(_LIB.tomo_fourier_reconstruct(self._h, self._images(images, self.n), int(variant), float(nsr),
                                                  self._volume(volume), ctypes.c_void_p(_stream_ptr(stream))))

    def fourier_reconstruct_async(self, images, volume, variant: int = EQ11, nsr: float = 0.0, stream=None):
        """fourier_reconstruct enqueued without waiting; domain errors surface at sync()."""
        self._check(_LIB.tomo_fourier_reconstruct_async(self._h, self._images(images, self.n), int(variant),
                                                        float(nsr), self._volume(volume),
                                                        ctypes.c_void_p(_stream_ptr(stream))))

    def timing(self, enable: bool):
        self._check(_LIB.tomo_timing_enable(self._h, 1 if enable else 0))

    def timing_read(self, reset: bool = True) -> dict:
        """Per-kernel totals since the last reset: {kind: (total_ms, launches)}."""
        ms = (ctypes.c_double * len(KERNEL_KINDS))()
        cnt = (ctypes.c_int64 * len(KERNEL_KINDS))()
        self._check(_LIB.tomo_timing_read(self._h, ms, cnt, 1 if reset else 0))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNEL_KINDS)}

    def destroy(self):
        if getattr(self, "_h", None):
            _LIB.tomo_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Batch:
    """Independent reconstructions (one plan each) recorded into one HIP graph."""

    def __init__(self, plans, images, volumes, lanes: int = 0):
        if not (len(plans) == len(images) == len(volumes)) or not plans:
            raise ValueError("plans, images and volumes must be non-empty lists of one length")
        n = len(plans)
        self._keep = (list(plans), list(images), list(volumes))   # buffers bound into the graph
        hp = (ctypes.c_void_p * n)(*[p._h for p in plans])
        hi = (ctypes.c_void_p * n)(*[p._images(t, p.n) for p, t in zip(plans, images)])
        hv = (ctypes.c_void_p * n)(*[p._volume(t) for p, t in zip(plans, volumes)])
        out = ctypes.c_void_p()
        st = _LIB.tomo_batch_create(hp, hi, hv, n, int(lanes), ctypes.byref(out))
        if st != OK:
            raise TomoError(st, _LIB.tomo_plan_error().decode())
        self._h = out

    def _check(self, st: int):
        if st != OK:
            raise TomoError(st, _LIB.tomo_batch_error(self._h).decode())

    def launch(self, stream=None):
        self._check(_LIB.tomo_batch_launch(self._h, ctypes.c_void_p(_stream_ptr(stream))))

    def sync(self, stream=None):
        self._check(_LIB.tomo_batch_sync(self._h, ctypes.c_void_p(_stream_ptr(stream))))

    def destroy(self):
        if getattr(self, "_h", None):
            _LIB.tomo_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
