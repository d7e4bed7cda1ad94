"""ctypes declarations of libsat.so (include/sat.h).  Argument marshalling only.

The library is loaded on first use.  If it is missing the call fails with an error naming the
build step; there is no other implementation to fall back to.
"""
import ctypes
import os
import threading

# SAT_LIBRARY names another build of the same library (the tests' sanitizer build of the host code).
LIB_PATH = os.environ.get("SAT_LIBRARY") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsat.so")

SAT_OK, SAT_ERR_ARG, SAT_ERR_WINDOW, SAT_ERR_OVERFLOW, SAT_ERR_WORKSPACE, SAT_ERR_HIP, SAT_ERR_DEVICE = range(7)
STATUS_NAMES = {0: "SAT_OK", 1: "SAT_ERR_ARG", 2: "SAT_ERR_WINDOW", 3: "SAT_ERR_OVERFLOW",
                4: "SAT_ERR_WORKSPACE", 5: "SAT_ERR_HIP", 6: "SAT_ERR_DEVICE"}
SAT_U8, SAT_U16, SAT_U32, SAT_U64, SAT_F64 = 1, 2, 3, 4, 5


class SatError(RuntimeError):
    """A libsat call returned an error status."""

    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


class BatchItem(ctypes.Structure):
    _fields_ = [("image", ctypes.c_void_p), ("H", ctypes.c_int64), ("W", ctypes.c_int64),
                ("image_pitch", ctypes.c_int64), ("sat", ctypes.c_void_p), ("sat_sq", ctypes.c_void_p),
                ("sat_pitch", ctypes.c_int64), ("sum_out", ctypes.c_void_p), ("mean_out", ctypes.c_void_p),
                ("std_out", ctypes.c_void_p), ("out_pitch", ctypes.c_int64)]


_lib = None
_lock = threading.Lock()
_i64, _p, _i32, _sz = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
_st = ctypes.c_int


def load(path: str = LIB_PATH):
    """Load libsat.so and declare its signatures (idempotent)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise RuntimeError("libsat.so is not built (%s); run `python -m paper_2410_16291_amd.build` "
                               "or __graft_entry__.build()" % path)
        # torch first: libsat's libamdhip64 dependency then binds to the HIP runtime torch already
        # loaded.  Loaded the other way round, the process holds two runtimes and torch's sees no
        # device.
        import torch  # noqa: F401
        lib = ctypes.CDLL(path)
        sig = {
            "window_out_shape": (_st, [_i64, _i64, _i64, _i64, _i64, _p, _p]),
            "sat_build_workspace_bytes": (_sz, [_i64, _i64, ctypes.c_int, ctypes.c_int]),
            "sat_build": (_st, [_p, ctypes.c_int, _i64, _i64, _i64, _p, _p, _i64, _p, _sz, _p]),
            "sat_build_noalloc": (_st, [_p, ctypes.c_int, _i64, _i64, _i64, _p, _p, _i64, _p]),
            "sat_build_band": (_st, [_p, ctypes.c_int, _i64, _i64, _i64, _p, _p, _i64, _p, _p, _i64, _p, _p, _p,
                                     _sz, _p]),
            "sat_column_totals": (_st, [_p, ctypes.c_int, _i64, _i64, _i64, _p, _p, _p, _p, _p]),
            "window_sum": (_st, [_p, ctypes.c_int, _i64, _i64, _i64, _i64, _i64, _i64, _p, ctypes.c_int,
                                 _i64, _p]),
            "window_mean_std": (_st, [_p, _p, _i64, _i64, _i64, _i64, _i64, _i64, _p, _p, _p, _i64, _p]),
            "window_sum_multi": (_st, [_p, ctypes.c_int, _i64, _i64, _i64, _i32, _p, _p, _i64, _p,
                                       ctypes.c_int, _p, _p]),
            "sat_batch_workspace_bytes": (_sz, [_p, _i32, ctypes.c_int, ctypes.c_int]),
            "sat_build_batched": (_st, [_p, _i32, ctypes.c_int, _p, _sz, _p]),
            "window_mean_std_batched": (_st, [_p, _i32, _i64, _i64, _i64, _p, _sz, _p]),
            "sat_build_stats_workspace_bytes": (_sz, [_p, _i32, ctypes.c_int]),
            "sat_build_stats_batched": (_st, [_p, _i32, ctypes.c_int, _i64, _i64, _i64, _p, _sz, _p]),
            "sat_workspace_check": (_st, [_p, _p]),
            "sat_upload": (_st, [_p, _p, _sz, _p]),
            "sat_last_error": (ctypes.c_char_p, []),
            "sat_variant_count": (_i32, [_i32]),
            "sat_variant_name": (ctypes.c_char_p, [_i32, _i32]),
            "sat_force_variant": (_st, [_i32, _i32]),
            "sat_variant_supported": (_i32, [_i32, _i32, ctypes.c_int, _i32]),
            "sat_powers_workspace_bytes": (_sz, [_i64, _i64, ctypes.c_int, _i32]),
            "sat_build_powers": (_st, [_p, ctypes.c_int, _i64, _i64, _i64, _i32, _p, _i64, _p, _sz, _p]),
            "window_moments": (_st, [_p, _i32, ctypes.c_int, _i64, _i64, _i64, _i64, _i64, _i64, _p, _p, _p, _p,
                                     _i64, _p]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


def check(status: int) -> None:
    """Raise SatError for a non-zero status, with the library's message."""
    if status != SAT_OK:
        raise SatError(status, load().sat_last_error().decode())
