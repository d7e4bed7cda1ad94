"""Multi-core CPU baseline of the benchmark (OpenMP C in sat_omp.c): the integral image of an
8-bit image built in row bands on every host core, then uint32 window sums by corner lookup.

A comparison point only: the tests check it against the oracle; the product library and the
oracle never import it.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None
_i64 = ctypes.c_int64
_p = ctypes.c_void_p


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        lib.omp_sat_build_u8.argtypes = [_p, _i64, _i64, _i64, _p, _i64, ctypes.c_int]
        lib.omp_sat_build_u8.restype = ctypes.c_int
        lib.omp_window_sum_u32.argtypes = [_p] + [_i64] * 6 + [_p, _i64, ctypes.c_int]
        lib.omp_window_sum_u32.restype = ctypes.c_int
        _lib = lib
    return _lib


def sat_u8(img, threads=0, out=None):
    """uint64 integral image of a 2-D uint8 array (rows may be padded); returns (table, threads)."""
    img = np.asarray(img)
    if img.ndim != 2 or img.dtype != np.uint8 or img.strides[1] != 1:
        raise ValueError("image must be a 2-D uint8 array with unit column stride")
    H, W = img.shape
    S = out if out is not None else np.empty((H, W), np.uint64)
    n = _load().omp_sat_build_u8(img.ctypes.data, H, W, img.strides[0], S.ctypes.data, S.strides[0] // 8, threads)
    if n < 0:
        raise MemoryError("omp_sat_build_u8: scratch allocation failed")
    return S, n


def window_sum_u32(S, h, w, s=1, threads=0, out=None):
    """uint32 sums of every h x w window at stride s from table S; returns (sums, threads)."""
    H, W = S.shape
    oh, ow = (H - h) // s + 1, (W - w) // s + 1
    o = out if out is not None else np.empty((oh, ow), np.uint32)
    n = _load().omp_window_sum_u32(S.ctypes.data, H, W, S.strides[0] // 8, h, w, s, o.ctypes.data,
                                   o.strides[0] // 4, threads)
    if n < 0:
        raise ValueError("window does not fit the image")
    return o, n
