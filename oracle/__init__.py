"""Python view of the C oracle for the integral-image sliding-window method.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of the benchmark
use this module to produce expected values.  The product library never imports it, and it
imports nothing from the product package.

Every function takes numpy arrays, calls the serial C code in sat_oracle.c and returns numpy
arrays.  Images are 2-D uint8 or uint16 arrays whose rows may be padded (any row stride that is a
whole number of elements); tables and outputs come back dense.
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
        path = os.environ.get("SAT_ORACLE_LIBRARY") or _build.LIB   # another build of sat_oracle.c (sanitizers)
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        lib = ctypes.CDLL(path)
        lib.oracle_window_shape.argtypes = [_i64] * 5 + [_p, _p]
        lib.oracle_sat.argtypes = [_p, ctypes.c_int, _i64, _i64, _i64, _p, _p]
        lib.oracle_window_sum_sat.argtypes = [_p] + [_i64] * 5 + [_p]
        lib.oracle_window_sum_direct.argtypes = [_p, ctypes.c_int] + [_i64] * 6 + [ctypes.c_int, _p]
        lib.oracle_window_at.argtypes = [_p, ctypes.c_int] + [_i64] * 5 + [_p, _p]
        lib.oracle_window_at.restype = None
        lib.oracle_mean_std.argtypes = [_p, _p, _i64, ctypes.c_uint64, _p, _p]
        lib.oracle_mean_std.restype = None
        lib.oracle_coverage_total.argtypes = [_p, ctypes.c_int] + [_i64] * 6
        lib.oracle_coverage_total.restype = ctypes.c_uint64
        lib.oracle_column_totals.argtypes = [_p, ctypes.c_int, _i64, _i64, _i64, _p, _p, _p, _p]
        lib.oracle_sat_power.argtypes = [_p, ctypes.c_int, _i64, _i64, _i64, ctypes.c_int, _p]
        lib.oracle_window_powers.argtypes = [_p, ctypes.c_int] + [_i64] * 5 + [ctypes.c_int, _p]
        lib.oracle_window_powers.restype = None
        lib.oracle_moments.argtypes = [_p, _p, _p, _p, _i64, ctypes.c_uint64, _p, _p, _p, _p]
        lib.oracle_moments.restype = None
        lib.oracle_stream.argtypes = ([_p, ctypes.c_int, _i64, _i64, _i64, ctypes.c_int, _i64, _p, _p,
                                       _i64, _p, _p, _p, _i64, _p, _p, _p])
        lib.oracle_stream_open.argtypes = [_p, ctypes.c_int, _i64, _i64, _i64, ctypes.c_int, _i64, _p, _p, _i64,
                                           _i64, _p]
        lib.oracle_stream_open.restype = _p
        lib.oracle_stream_next.argtypes = [_p, _i64, _p, _p, _p, _p]
        lib.oracle_stream_close.argtypes = [_p]
        lib.oracle_stream_close.restype = None
        _lib = lib
    return _lib


def _image(img):
    img = np.asarray(img)
    if img.ndim != 2 or img.dtype not in (np.uint8, np.uint16):
        raise ValueError("image must be a 2-D uint8 or uint16 array")
    if img.strides[1] != img.itemsize or img.strides[0] % img.itemsize or img.strides[0] < 0:
        img = np.ascontiguousarray(img)
    pitch = img.strides[0] // img.itemsize
    return img, img.itemsize, pitch


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def window_shape(H, W, h, w, s=1):
    """Output shape (rows, cols) of the valid region, or None if the window does not fit."""
    oh, ow = ctypes.c_int64(), ctypes.c_int64()
    if _load().oracle_window_shape(H, W, h, w, s, ctypes.byref(oh), ctypes.byref(ow)):
        return None
    return oh.value, ow.value


def sat(img, squares=False):
    """Inclusive integral image (uint64, dense); with squares=True also the table of I^2."""
    img, bpp, pitch = _image(img)
    H, W = img.shape
    S = np.empty((H, W), np.uint64)
    Q = np.empty((H, W), np.uint64) if squares else None
    rc = _load().oracle_sat(_ptr(img), bpp, H, W, pitch, _ptr(S), _ptr(Q) if squares else None)
    if rc:
        raise ValueError("oracle_sat rejected its arguments")
    return (S, Q) if squares else S


def column_totals(img, squares=False, carry=None, carry_sq=None):
    """Column totals of the image added to `carry` (uint64, zero if None): T[x] = carry[x] +
    sum_y img[y, x] (mod 2^64).  Returns T, or (T, T2) with the totals of the squared pixels."""
    img, bpp, pitch = _image(img)
    H, W = img.shape
    c = None if carry is None else np.ascontiguousarray(carry, dtype=np.uint64)
    cq = None if carry_sq is None else np.ascontiguousarray(carry_sq, dtype=np.uint64)
    for a in (c, cq):
        if a is not None and a.shape != (W,):
            raise ValueError("carry must have W entries")
    T = np.empty(W, np.uint64)
    T2 = np.empty(W, np.uint64) if squares else None
    if _load().oracle_column_totals(_ptr(img), bpp, H, W, pitch, _ptr(c) if c is not None else None,
                                    _ptr(cq) if cq is not None else None, _ptr(T),
                                    _ptr(T2) if T2 is not None else None):
        raise ValueError("oracle_column_totals: bad arguments")
    return (T, T2) if squares else T


def window_sum_sat(S, h, w, s=1):
    """Window sums by four-corner lookup into a dense uint64 table S (uint64 output)."""
    S = np.ascontiguousarray(S, dtype=np.uint64)
    H, W = S.shape
    shape = window_shape(H, W, h, w, s)
    if shape is None:
        raise ValueError("window does not fit")
    out = np.empty(shape, np.uint64)
    if _load().oracle_window_sum_sat(_ptr(S), H, W, h, w, s, _ptr(out)):
        raise ValueError("oracle_window_sum_sat rejected its arguments")
    return out


def window_sum_direct(img, h, w, s=1, squares=False):
    """Window sums by direct summation of every window (uint64 output)."""
    img, bpp, pitch = _image(img)
    H, W = img.shape
    shape = window_shape(H, W, h, w, s)
    if shape is None:
        raise ValueError("window does not fit")
    out = np.empty(shape, np.uint64)
    if _load().oracle_window_sum_direct(_ptr(img), bpp, H, W, pitch, h, w, s, int(squares), _ptr(out)):
        raise ValueError("oracle_window_sum_direct rejected its arguments")
    return out


def window_at(img, y0, x0, h, w):
    """(sum, sum of squares) of one window, summed directly."""
    img, bpp, pitch = _image(img)
    a, b = ctypes.c_uint64(), ctypes.c_uint64()
    _load().oracle_window_at(_ptr(img), bpp, pitch, y0, x0, h, w, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def mean_std(sums, sum_sqs, n):
    """FP64 window mean and population std from exact integer sums over n pixels."""
    sums = np.ascontiguousarray(sums, dtype=np.uint64)
    sum_sqs = np.ascontiguousarray(sum_sqs, dtype=np.uint64)
    if sums.shape != sum_sqs.shape:
        raise ValueError("shape mismatch")
    mean = np.empty(sums.shape, np.float64)
    std = np.empty(sums.shape, np.float64)
    _load().oracle_mean_std(_ptr(sums), _ptr(sum_sqs), sums.size, int(n), _ptr(mean), _ptr(std))
    return mean, std


def window_stats(img, h, w, s=1):
    """(sum, mean, std) of every window: integral images, corner lookups, then mean_std."""
    S, Q = sat(img, squares=True)
    sums = window_sum_sat(S, h, w, s)
    sqs = window_sum_sat(Q, h, w, s)
    mean, std = mean_std(sums, sqs, h * w)
    return sums, mean, std


def coverage_total(img, h, w, s=1):
    """Sum of all window sums (mod 2^64), from pixels weighted by how many windows hold them."""
    img, bpp, pitch = _image(img)
    H, W = img.shape
    return int(_load().oracle_coverage_total(_ptr(img), bpp, H, W, pitch, h, w, s))


def stream(img, windows, s, rows, sat_rows=(), squares=False):
    """Serial integral image over a large image keeping only a ring of rows.

    windows: list of (h, w); rows: list (one per window) of ascending output-row indices.
    Returns (outs, sat_out, total): outs[i] is a (len(rows[i]), ow_i) uint64 array, sat_out a
    (len(sat_rows), W) uint64 array of table rows, total the last table entry (mod 2^64).
    """
    img, bpp, pitch = _image(img)
    H, W = img.shape
    nwin = len(windows)
    wh = np.array([w[0] for w in windows], np.int64)
    ww = np.array([w[1] for w in windows], np.int64)
    nrows = np.array([len(r) for r in rows], np.int64)
    flat = np.concatenate([np.asarray(r, np.int64) for r in rows]) if nwin else np.zeros(0, np.int64)
    ows = []
    for (h, w) in windows:
        shape = window_shape(H, W, h, w, s)
        if shape is None:
            raise ValueError("window does not fit")
        ows.append(shape[1])
    out = np.zeros(int(sum(n * o for n, o in zip(nrows, ows))), np.uint64)
    srows = np.asarray(sat_rows, np.int64)
    sat_out = np.zeros((len(srows), W), np.uint64)
    total = ctypes.c_uint64()
    rc = _load().oracle_stream(_ptr(img), bpp, H, W, pitch, int(squares), nwin, _ptr(wh), _ptr(ww), s,
                               _ptr(nrows), _ptr(flat), _ptr(out), len(srows), _ptr(srows),
                               _ptr(sat_out), ctypes.byref(total))
    if rc:
        raise ValueError("oracle_stream failed (%d)" % rc)
    outs, pos = [], 0
    for n, o in zip(nrows, ows):
        outs.append(out[pos:pos + n * o].reshape(n, o))
        pos += n * o
    return outs, sat_out, total.value


class Stream:
    """The streamed table (oracle_stream's recurrence) started at image row r0 and advanced band by
    band: table row r0-1 is the running sum along x of `carry`, the column totals of rows 0..r0-1
    (uint64, W entries; None when r0 == 0).  Several streams started at different rows cover one
    image independently.

        st = Stream(img, [(100, 100), (250, 250)], s=1, r0=r0, carry=carry)
        sat_rows, outs = st.next(r1)   # table rows st.cur..r1-1; per window (k_first, rows)
        st.close()

    For window i, next() returns the output rows whose windows lie in rows r0..r1-1 and were not
    returned before, as (index of the first, a (n, ow_i) uint64 array).  `img` is the whole
    image (it is held, not copied, while the stream is open).
    """

    def __init__(self, img, windows, s=1, r0=0, carry=None, squares=False):
        self._img, bpp, pitch = _image(img)
        self.H, self.W = self._img.shape
        self.windows = [(int(h), int(w)) for h, w in windows]
        self.s = int(s)
        self.cur = int(r0)
        self.ows = []
        for h, w in self.windows:
            shape = window_shape(self.H, self.W, h, w, self.s)
            if shape is None:
                raise ValueError("window does not fit")
            self.ows.append(shape[1])
        self._carry = None if carry is None else np.ascontiguousarray(carry, dtype=np.uint64)
        if self._carry is not None and self._carry.shape != (self.W,):
            raise ValueError("carry must have W entries")
        n = len(self.windows)
        wh = np.array([h for h, _ in self.windows] or [0], np.int64)
        ww = np.array([w for _, w in self.windows] or [0], np.int64)
        self._h = _load().oracle_stream_open(_ptr(self._img), bpp, self.H, self.W, pitch, int(squares), n,
                                             _ptr(wh), _ptr(ww), self.s, self.cur,
                                             _ptr(self._carry) if self._carry is not None else None)
        if not self._h:
            raise ValueError("oracle_stream_open rejected its arguments")

    def next(self, r1, want_sat=True):
        """Advance through row r1-1: (table rows cur..r1-1 as an (r1-cur, W) uint64 array or None,
        [(k_first, outputs) per window])."""
        if self._h is None:
            raise ValueError("stream closed")
        r1 = int(r1)
        if r1 < self.cur or r1 > self.H:
            raise ValueError("r1 out of range")
        n = len(self.windows)
        sat = np.empty((r1 - self.cur, self.W), np.uint64) if want_sat else None
        cap = (r1 - self.cur + self.s - 1) // self.s + 1
        bufs = [np.empty((cap, ow), np.uint64) for ow in self.ows]
        ptrs = (ctypes.c_void_p * max(n, 1))(*[b.ctypes.data for b in bufs])
        k_first = np.zeros(max(n, 1), np.int64)
        n_out = np.zeros(max(n, 1), np.int64)
        if _load().oracle_stream_next(self._h, r1, _ptr(sat) if sat is not None else None, ptrs, _ptr(k_first),
                                      _ptr(n_out)):
            raise ValueError("oracle_stream_next rejected its arguments")
        self.cur = r1
        return sat, [(int(k_first[i]), bufs[i][:int(n_out[i])]) for i in range(n)]

    def close(self):
        if self._h is not None:
            _load().oracle_stream_close(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- higher window moments (tables of pixel powers; the method applied to I^k)

def sat_power(img, k):
    """Inclusive integral image of pixel^k (k = 1..4), uint64, wrapping mod 2^64."""
    img, bpp, pitch = _image(img)
    H, W = img.shape
    T = np.empty((H, W), np.uint64)
    if _load().oracle_sat_power(_ptr(img), bpp, H, W, pitch, int(k), _ptr(T)):
        raise ValueError("oracle_sat_power rejected its arguments")
    return T


def window_powers(img, y0, x0, h, w, k):
    """[sum of pixel^1, ..., sum of pixel^k] over one window, summed directly (mod 2^64)."""
    img, bpp, pitch = _image(img)
    out = np.zeros(k, np.uint64)
    _load().oracle_window_powers(_ptr(img), bpp, pitch, y0, x0, h, w, int(k), _ptr(out))
    return [int(v) for v in out]


def moments(s1, s2, n, s3=None, s4=None):
    """(mean, std, skew, kurt) in FP64 from exact window power sums over n pixels: population
    moments, skewness m3/m2^1.5, excess kurtosis m4/m2^2 - 3 (NaN where m2 = 0); skew needs s3,
    kurt needs s3 and s4 (None otherwise)."""
    arrs = [np.ascontiguousarray(a, dtype=np.uint64) for a in (s1, s2)]
    if s4 is not None and s3 is None:
        raise ValueError("kurtosis needs s3 as well")
    s3a = np.ascontiguousarray(s3, dtype=np.uint64) if s3 is not None else None
    s4a = np.ascontiguousarray(s4, dtype=np.uint64) if s4 is not None else None
    shape = arrs[0].shape
    for a in [arrs[1], s3a, s4a]:
        if a is not None and a.shape != shape:
            raise ValueError("shape mismatch")
    mean, std = np.empty(shape, np.float64), np.empty(shape, np.float64)
    skew = np.empty(shape, np.float64) if s3a is not None else None
    kurt = np.empty(shape, np.float64) if s4a is not None else None
    _load().oracle_moments(_ptr(arrs[0]), _ptr(arrs[1]), _ptr(s3a) if s3a is not None else None,
                           _ptr(s4a) if s4a is not None else None, arrs[0].size, int(n), _ptr(mean), _ptr(std),
                           _ptr(skew) if skew is not None else None, _ptr(kurt) if kurt is not None else None)
    return mean, std, skew, kurt


def window_moments(img, h, w, s=1, k=4):
    """Power sums (list of k uint64 arrays) and (mean, std, skew, kurt) of every window: tables of
    pixel^1..pixel^k, corner lookups, then moments (skew needs k >= 3, kurt k = 4)."""
    sums = [window_sum_sat(sat_power(img, j), h, w, s) for j in range(1, k + 1)]
    stats = moments(sums[0], sums[1], h * w, sums[2] if k >= 3 else None, sums[3] if k >= 4 else None)
    return sums, stats
