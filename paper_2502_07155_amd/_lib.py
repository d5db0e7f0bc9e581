"""ctypes loader for libblnfft.so (the HIP library built in-tree by ``build.py``).

Loading fails loudly when the library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libblnfft.so")

# bl_status values (include/blnfft.h)
BL_OK, BL_EINVAL, BL_EDOMAIN, BL_ENOMEM, BL_EDEVICE, BL_ESTATE, BL_EUNSUPPORTED = range(7)
WINDOWS = {"sinh": 0, "ckb": 1}
METHODS = {"shannon": 0, "nfft": 1}
PRECISIONS = {"f64": 0, "f32": 1, "f32c": 2, "f32d": 3}

EXPORTS = [
    "bl_plan_create", "bl_set_nodes", "bl_precompute_weights", "bl_forward", "bl_samples",
    "bl_interpolate",
    "bl_get_theta",
    "bl_adjoint", "bl_adjoint_noalloc", "bl_grad_x", "bl_plan_stats", "bl_plan_destroy", "bl_window_transform",
    "bl_batch_create", "bl_batch_set_nodes", "bl_batch_forward", "bl_batch_destroy",
    "bl_status_string", "bl_last_error", "bl_version",
]


class BLNFFTError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {message} (status {status})")
        self.status = status


class Stats(ctypes.Structure):
    _fields_ = [
        ("n_nodes", ctypes.c_int64),
        ("n_outside", ctypes.c_int64),
        ("n_chunks", ctypes.c_int64),
        ("tile", ctypes.c_int64 * 3),
        ("chunk_cap", ctypes.c_int64),
        ("workspace_bytes", ctypes.c_int64),
        ("beta", ctypes.c_double),
        ("weight_fit_err", ctypes.c_double),
        ("fft_lines", ctypes.c_int64 * 6),
        ("fft_radix", ctypes.c_int64 * 6),
        ("tuned", ctypes.c_int64 * 2),
    ]


_lib = None


def load() -> ctypes.CDLL:
    """Return the loaded library, loading it on first use."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing; build it with "
                          "`python -m paper_2502_07155_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "bl_plan_create": [P(vp), i32, i64, i64, i32, i32, dbl, i32, i32, vp],
        "bl_set_nodes": [vp, i64, vp],
        "bl_precompute_weights": [vp, i32],
        "bl_forward": [vp, vp, vp],
        "bl_samples": [vp, vp],
        "bl_interpolate": [vp, vp, vp],
        "bl_get_theta": [vp, vp],
        "bl_adjoint": [vp, vp, vp],
        "bl_adjoint_noalloc": [vp, vp, vp],
        "bl_grad_x": [vp, vp, vp],
        "bl_plan_stats": [vp, P(Stats)],
        "bl_plan_destroy": [vp],
        "bl_window_transform": [i32, i32, i64, i64, i32, dbl, i64, P(dbl), P(dbl)],
        "bl_batch_create": [P(vp), i32, P(i64), P(i64), P(i32), P(i64), i32, vp],
        "bl_batch_set_nodes": [vp, vp],
        "bl_batch_forward": [vp, vp, vp],
        "bl_batch_destroy": [vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    for name in ("bl_status_string",):
        getattr(lib, name).argtypes = [ctypes.c_int]
        getattr(lib, name).restype = ctypes.c_char_p
    for name in ("bl_last_error", "bl_version"):
        getattr(lib, name).argtypes = []
        getattr(lib, name).restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(status: int, where: str) -> None:
    if status != BL_OK:
        lib = load()
        msg = lib.bl_last_error().decode(errors="replace")
        raise BLNFFTError(status, where, msg or lib.bl_status_string(status).decode())
