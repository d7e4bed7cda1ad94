"""torch-tensor face of libsat: sat_build, window_sum, window_mean_std, window_sum_multi.

torch supplies device memory and the stream; every step of the computation runs in the HIP
kernels behind the C ABI.  Tables are uint64 tensors of shape (H, W) that may be views of a
wider allocation (row pitch = stride(0)); outputs likewise.
"""
from __future__ import annotations

import ctypes
from typing import Dict, List, Optional, Sequence, Tuple

import torch

from . import _lib
from ._lib import SAT_F64, SAT_U8, SAT_U16, SAT_U32, SAT_U64, BatchItem, check

_PIXEL = {torch.uint8: SAT_U8, torch.uint16: SAT_U16}
_MAXPIX = {"u8": 255, "u16": 65535, "u32": (1 << 32) - 1}
_PIXCODE = {"u8": SAT_U8, "u16": SAT_U16, "u32": SAT_U32}

# Per (device, stream) workspace cache: a build workspace may not be shared by two builds in
# flight, and builds on one stream are ordered, so one buffer per stream suffices.
_workspaces: Dict[Tuple[int, int], torch.Tensor] = {}


def _stream_handle(device: torch.device, stream: Optional[torch.cuda.Stream]) -> int:
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return s.cuda_stream


def _require_cuda(t: torch.Tensor, name: str) -> None:
    if not t.is_cuda:
        raise ValueError("%s must be a device (cuda) tensor" % name)
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("%s must be 2-D with unit column stride" % name)


def workspace(nbytes: int, device: torch.device, stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """A cached device workspace of at least nbytes for builds on this stream.

    The buffer is allocated on the stream the builds run on, so torch's caching allocator orders
    its reuse after them.  A larger request replaces the cached buffer; the old one is first
    recorded on that stream, so its memory is not handed out again before the launches that used
    it have run."""
    s = stream if stream is not None else torch.cuda.current_stream(device)
    key = (device.index if device.index is not None else torch.cuda.current_device(), s.cuda_stream)
    ws = _workspaces.get(key)
    if ws is None or ws.numel() < nbytes:
        with torch.cuda.stream(s):
            new = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        if ws is not None:
            ws.record_stream(s)
        _workspaces[key] = ws = new
    return ws


def table_pitch(W: int) -> int:
    """Row pitch (elements) used for tables allocated here: width rounded up to 16 elements."""
    return (W + 15) // 16 * 16


def empty_table(H: int, W: int, device, pitch: Optional[int] = None) -> torch.Tensor:
    pitch = table_pitch(W) if pitch is None else pitch
    return torch.empty((H, pitch), dtype=torch.uint64, device=device)[:, :W]


def image_pitch(W: int, dtype: torch.dtype) -> int:
    """Row pitch (elements) of images allocated here: a whole number of 128-byte lines, so every
    row starts 16-byte aligned and the build stages its tiles with 16-byte loads."""
    per_line = 128 // dtype.itemsize
    return (W + per_line - 1) // per_line * per_line


def empty_image(H: int, W: int, dtype: torch.dtype, device) -> torch.Tensor:
    """A zeroed H x W image (uint8 or uint16) on the line-aligned row pitch of image_pitch."""
    return torch.zeros((H, image_pitch(W, dtype)), dtype=dtype, device=device)[:, :W]


def out_pitch(ow: int, dtype: torch.dtype) -> int:
    """Row pitch (elements) of outputs allocated here: a whole number of 128-byte lines, so that
    no two output rows share a cache line (a partly written line costs HBM a read-modify-write)."""
    per_line = 128 // dtype.itemsize
    return (ow + per_line - 1) // per_line * per_line


def empty_out(oh: int, ow: int, dtype: torch.dtype, device) -> torch.Tensor:
    """An oh x ow output with the line-aligned row pitch of out_pitch (a view of a wider buffer)."""
    return torch.empty((oh, out_pitch(ow, dtype)), dtype=dtype, device=device)[:, :ow]


def build_workspace_bytes(H: int, W: int, pixel_type: int, squares: bool) -> int:
    n = _lib.load().sat_build_workspace_bytes(H, W, pixel_type, int(squares))
    if n == 0:
        raise ValueError("invalid image size %dx%d" % (H, W))
    return n


def sat_build(image: torch.Tensor, squares: bool = False, sat: Optional[torch.Tensor] = None,
              sat_sq: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None,
              stream: Optional[torch.cuda.Stream] = None):
    """Integral image of a 2-D uint8/uint16 device image; with squares=True also of its squares.

    Returns S, or (S, Q).  S[y, x] = sum of image[:y+1, :x+1] (mod 2^64).
    """
    _require_cuda(image, "image")
    if image.dtype not in _PIXEL:
        raise ValueError("image dtype must be uint8 or uint16")
    H, W = image.shape
    dev = image.device
    S = sat if sat is not None else empty_table(H, W, dev)
    Q = sat_sq if sat_sq is not None else (empty_table(H, W, dev, S.stride(0)) if squares else None)
    _require_cuda(S, "sat")
    if Q is not None:
        _require_cuda(Q, "sat_sq")
        if Q.stride(0) != S.stride(0):
            raise ValueError("sat and sat_sq must share a row pitch")
    ptype = _PIXEL[image.dtype]
    need = build_workspace_bytes(H, W, ptype, Q is not None)
    wsb = ws if ws is not None else workspace(need, dev, stream)
    check(_lib.load().sat_build(image.data_ptr(), ptype, H, W, image.stride(0), S.data_ptr(),
                                Q.data_ptr() if Q is not None else None, S.stride(0), wsb.data_ptr(),
                                wsb.numel(), _stream_handle(dev, stream)))
    return (S, Q) if squares or sat_sq is not None else S


def _vector(t: Optional[torch.Tensor], W: int, name: str) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("%s must be a device (cuda) tensor" % name)
    if t.dtype not in (torch.uint64, torch.int64) or t.dim() != 1 or t.numel() != W or t.stride(0) != 1:
        raise ValueError("%s must be a contiguous 64-bit vector of %d elements" % (name, W))
    return t.data_ptr()


def empty_totals(W: int, device) -> torch.Tensor:
    """A device vector for W column totals."""
    return torch.empty(W, dtype=torch.uint64, device=device)


def column_totals(image: torch.Tensor, squares: bool = False, carry: Optional[torch.Tensor] = None,
                  carry_sq: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
                  out_sq: Optional[torch.Tensor] = None, stream: Optional[torch.cuda.Stream] = None):
    """Column totals of a 2-D uint8/uint16 device image added to `carry` (zero if None):
    out[x] = carry[x] + sum_y image[y, x] (mod 2^64); with squares=True also of the squared pixels.
    `out` may be `carry` itself.  Returns T, or (T, TQ)."""
    _require_cuda(image, "image")
    if image.dtype not in _PIXEL:
        raise ValueError("image dtype must be uint8 or uint16")
    H, W = image.shape
    dev = image.device
    T = out if out is not None else empty_totals(W, dev)
    TQ = out_sq if out_sq is not None else (empty_totals(W, dev) if squares else None)
    check(_lib.load().sat_column_totals(image.data_ptr(), _PIXEL[image.dtype], H, W, image.stride(0),
                                        _vector(carry, W, "carry"), _vector(carry_sq, W, "carry_sq"),
                                        _vector(T, W, "out"), _vector(TQ, W, "out_sq"),
                                        _stream_handle(dev, stream)))
    return (T, TQ) if TQ is not None else T


def sat_build_band(image: torch.Tensor, carry: Optional[torch.Tensor] = None, rows_above: int = 0,
                   squares: bool = False, carry_sq: Optional[torch.Tensor] = None,
                   sat: Optional[torch.Tensor] = None, sat_sq: Optional[torch.Tensor] = None,
                   totals: bool = True, total: Optional[torch.Tensor] = None,
                   total_sq: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None,
                   stream: Optional[torch.cuda.Stream] = None):
    """Table rows rows_above .. rows_above+H-1 of a taller image from its band of rows `image` and
    `carry`, the column totals of the rows_above rows above the band (None: no rows above).

    With totals=True the band's column totals through its last row (carry included: the carry of
    the band below) are returned as well; `total` may be `carry` itself to advance it in place.
    Returns (S, T), or (S, Q, T, TQ) with squares=True (T, TQ None with totals=False)."""
    _require_cuda(image, "image")
    if image.dtype not in _PIXEL:
        raise ValueError("image dtype must be uint8 or uint16")
    H, W = image.shape
    dev = image.device
    S = sat if sat is not None else empty_table(H, W, dev)
    Q = sat_sq if sat_sq is not None else (empty_table(H, W, dev, S.stride(0)) if squares else None)
    _require_cuda(S, "sat")
    if Q is not None:
        _require_cuda(Q, "sat_sq")
        if Q.stride(0) != S.stride(0):
            raise ValueError("sat and sat_sq must share a row pitch")
    T = total if total is not None else (empty_totals(W, dev) if totals else None)
    TQ = total_sq if total_sq is not None else (empty_totals(W, dev) if totals and Q is not None else None)
    ptype = _PIXEL[image.dtype]
    need = build_workspace_bytes(H, W, ptype, Q is not None)
    wsb = ws if ws is not None else workspace(need, dev, stream)
    check(_lib.load().sat_build_band(image.data_ptr(), ptype, H, W, image.stride(0), _vector(carry, W, "carry"),
                                     _vector(carry_sq, W, "carry_sq"), rows_above, S.data_ptr(),
                                     Q.data_ptr() if Q is not None else None, S.stride(0), _vector(T, W, "total"),
                                     _vector(TQ, W, "total_sq"), wsb.data_ptr(), wsb.numel(),
                                     _stream_handle(dev, stream)))
    return (S, Q, T, TQ) if Q is not None else (S, T)


def out_shape(H: int, W: int, h: int, w: int, stride: int = 1) -> Tuple[int, int]:
    oh, ow = ctypes.c_int64(), ctypes.c_int64()
    check(_lib.load().window_out_shape(H, W, h, w, stride, ctypes.byref(oh), ctypes.byref(ow)))
    return oh.value, ow.value


def default_out_dtype(h: int, w: int, pixel_type: str) -> torch.dtype:
    return torch.uint32 if h * w * _MAXPIX[pixel_type] <= 0xFFFFFFFF else torch.uint64


def window_sum(S: torch.Tensor, h: int, w: int, stride: int = 1, pixel_type: str = "u16",
               out_dtype: Optional[torch.dtype] = None, out: Optional[torch.Tensor] = None,
               stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """Sum of every h x w window (valid region, step `stride`) by four-corner lookup into S."""
    _require_cuda(S, "sat")
    H, W = S.shape
    oh, ow = out_shape(H, W, h, w, stride)
    if out is None:
        out_dtype = out_dtype or default_out_dtype(h, w, pixel_type)
        out = empty_out(oh, ow, out_dtype, S.device)
    _require_cuda(out, "out")
    if tuple(out.shape) != (oh, ow) or out.stride(1) != 1:
        raise ValueError("out must be %d x %d with unit column stride" % (oh, ow))
    code = {torch.uint32: SAT_U32, torch.uint64: SAT_U64}.get(out.dtype)
    if code is None:
        raise ValueError("out dtype must be uint32 or uint64")
    check(_lib.load().window_sum(S.data_ptr(), _PIXCODE[pixel_type], H, W, S.stride(0), h, w, stride,
                                 out.data_ptr(), code, out.stride(0), _stream_handle(S.device, stream)))
    return out


def window_sum_multi(S: torch.Tensor, windows: Sequence[Tuple[int, int]], stride: int = 1,
                     pixel_type: str = "u16", out_dtype: Optional[torch.dtype] = None,
                     outs: Optional[Sequence[torch.Tensor]] = None,
                     stream: Optional[torch.cuda.Stream] = None) -> List[torch.Tensor]:
    """window_sum for several (h, w) windows in one pass over S (`outs`: preallocated outputs,
    one per window, all of one dtype)."""
    _require_cuda(S, "sat")
    H, W = S.shape
    n = len(windows)
    if outs is not None:
        outs = list(outs)
        if len(outs) != n:
            raise ValueError("one output per window")
        out_dtype = outs[0].dtype
        for o, (h, w) in zip(outs, windows):
            _require_cuda(o, "out")
            if o.dtype != out_dtype or tuple(o.shape) != out_shape(H, W, h, w, stride) or o.stride(1) != 1:
                raise ValueError("outs must match the windows' output shapes, share one dtype and have unit "
                                 "column stride")
    else:
        if out_dtype is None:
            big = any(default_out_dtype(h, w, pixel_type) == torch.uint64 for h, w in windows)
            out_dtype = torch.uint64 if big else torch.uint32
        outs = [empty_out(*out_shape(H, W, h, w, stride), out_dtype, S.device) for h, w in windows]
    hs = (ctypes.c_int64 * n)(*[h for h, _ in windows])
    ws = (ctypes.c_int64 * n)(*[w for _, w in windows])
    ptrs = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    pitches = (ctypes.c_int64 * n)(*[o.stride(0) for o in outs])
    code = SAT_U32 if out_dtype == torch.uint32 else SAT_U64
    check(_lib.load().window_sum_multi(S.data_ptr(), _PIXCODE[pixel_type], H, W, S.stride(0), n, hs, ws, stride,
                                       ptrs, code, pitches, _stream_handle(S.device, stream)))
    return outs


def window_mean_std(S: torch.Tensor, Q: torch.Tensor, h: int, w: int, stride: int = 1, with_sum: bool = True,
                    outs: Optional[Tuple[Optional[torch.Tensor], torch.Tensor, torch.Tensor]] = None,
                    stream: Optional[torch.cuda.Stream] = None):
    """(sum or None, mean, std) of every window from the tables of pixels and squared pixels
    (`outs`: preallocated (sum or None, mean, std) sharing one row pitch)."""
    _require_cuda(S, "sat")
    _require_cuda(Q, "sat_sq")
    if Q.shape != S.shape or Q.stride(0) != S.stride(0):
        raise ValueError("sat and sat_sq must have the same shape and pitch")
    H, W = S.shape
    oh, ow = out_shape(H, W, h, w, stride)
    if outs is None:
        s1 = empty_out(oh, ow, torch.uint64, S.device) if with_sum else None
        mean = empty_out(oh, ow, torch.float64, S.device)
        std = empty_out(oh, ow, torch.float64, S.device)
    else:
        s1, mean, std = outs
        for t in ([s1] if s1 is not None else []) + [mean, std]:
            _require_cuda(t, "out")
            if tuple(t.shape) != (oh, ow) or t.stride(0) != mean.stride(0):
                raise ValueError("outputs must be %d x %d and share one row pitch" % (oh, ow))
        if (s1 is not None and s1.dtype != torch.uint64) or mean.dtype != torch.float64 or std.dtype != torch.float64:
            raise ValueError("outputs must be uint64 (sum) and float64 (mean, std)")
    pitch = mean.stride(0)
    check(_lib.load().window_mean_std(S.data_ptr(), Q.data_ptr(), H, W, S.stride(0), h, w, stride,
                                      s1.data_ptr() if s1 is not None else None, mean.data_ptr(), std.data_ptr(),
                                      pitch, _stream_handle(S.device, stream)))
    return s1, mean, std


# ---------------------------------------------------------------- higher window moments

MOMENTS = ("mean", "std", "skew", "kurt")    # statistic i needs the tables of pixel^1 .. pixel^(i+1)


def powers_workspace_bytes(H: int, W: int, pixel_type: int, k: int) -> int:
    n = _lib.load().sat_powers_workspace_bytes(H, W, pixel_type, k)
    if n == 0:
        raise ValueError("invalid size %dx%d, pixel type or k = %d" % (H, W, k))
    return n


def sat_build_powers(image: torch.Tensor, k: int, tables: Optional[List[torch.Tensor]] = None,
                     ws: Optional[torch.Tensor] = None, stream: Optional[torch.cuda.Stream] = None) -> List[torch.Tensor]:
    """Tables of pixel^1 .. pixel^k (k = 1..4) of a 2-D uint8/uint16 device image, one pass:
    tables[p-1][y, x] = sum of image[:y+1, :x+1]^p (mod 2^64).  `tables`: k preallocated uint64
    tables sharing one row pitch."""
    _require_cuda(image, "image")
    if image.dtype not in _PIXEL:
        raise ValueError("image dtype must be uint8 or uint16")
    H, W = image.shape
    dev = image.device
    if tables is None:
        first = empty_table(H, W, dev)
        tables = [first] + [empty_table(H, W, dev, first.stride(0)) for _ in range(k - 1)]
    if len(tables) != k:
        raise ValueError("need %d tables" % k)
    for t in tables:
        _require_cuda(t, "table")
        if tuple(t.shape) != (H, W) or t.dtype != torch.uint64 or t.stride(0) != tables[0].stride(0):
            raise ValueError("tables must be %d x %d uint64 sharing one row pitch" % (H, W))
    ptype = _PIXEL[image.dtype]
    wsb = ws if ws is not None else workspace(powers_workspace_bytes(H, W, ptype, k), dev, stream)
    ptrs = (ctypes.c_void_p * k)(*[t.data_ptr() for t in tables])
    check(_lib.load().sat_build_powers(image.data_ptr(), ptype, H, W, image.stride(0), k, ptrs, tables[0].stride(0),
                                       wsb.data_ptr(), wsb.numel(), _stream_handle(dev, stream)))
    return list(tables)


def window_moments(tables: List[torch.Tensor], h: int, w: int, stride: int = 1, *, pixel_type: str,
                   stats: Tuple[str, ...] = MOMENTS, outs: Optional[dict] = None,
                   stream: Optional[torch.cuda.Stream] = None) -> dict:
    """{name: float64 output} for `stats` (a subset of mean, std, skew, kurt: population moments,
    skewness and excess kurtosis, NaN for constant windows) of every window, from the tables of
    pixel^1 .. pixel^k (sat_build_powers; k at least the order of the highest statistic).
    pixel_type ("u8" or "u16", the image the tables came from) is required: it bounds the sums
    for the overflow checks."""
    for t in tables:
        _require_cuda(t, "table")
        if t.shape != tables[0].shape or t.stride(0) != tables[0].stride(0):
            raise ValueError("tables must share shape and row pitch")
    bad = [s for s in stats if s not in MOMENTS]
    if bad or not stats:
        raise ValueError("stats must be a non-empty subset of %s" % (MOMENTS,))
    H, W = tables[0].shape
    oh, ow = out_shape(H, W, h, w, stride)
    given = outs or {}
    outs = {n: given[n] if n in given else empty_out(oh, ow, torch.float64, tables[0].device) for n in stats}
    pitch = None
    for name, t in outs.items():
        _require_cuda(t, "out")
        if tuple(t.shape) != (oh, ow) or t.dtype != torch.float64 or (pitch is not None and t.stride(0) != pitch):
            raise ValueError("outputs must be %d x %d float64 sharing one row pitch" % (oh, ow))
        pitch = t.stride(0)
    k = len(tables)
    ptrs = (ctypes.c_void_p * k)(*[t.data_ptr() for t in tables])
    arg = [outs[n].data_ptr() if n in outs else None for n in MOMENTS]
    check(_lib.load().window_moments(ptrs, k, _PIXCODE[pixel_type], H, W, tables[0].stride(0), h, w, stride,
                                     arg[0], arg[1], arg[2], arg[3], pitch, _stream_handle(tables[0].device, stream)))
    return {n: outs[n] for n in stats}


def upload(host: torch.Tensor, dst: torch.Tensor, stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """Copy the pinned host tensor `host` into the device tensor `dst` (both contiguous, the same
    number of bytes) with a kernel on `stream`: the call returns once the kernel is enqueued,
    whatever other copies are in flight.  `host` must stay alive until the copy has run."""
    if host.device.type != "cpu" or not host.is_pinned():
        raise ValueError("host must be a pinned CPU tensor")
    if not dst.is_cuda:
        raise ValueError("dst must be a device (cuda) tensor")
    if not host.is_contiguous() or not dst.is_contiguous():
        raise ValueError("host and dst must be contiguous")
    n = host.numel() * host.element_size()
    if n != dst.numel() * dst.element_size():
        raise ValueError("host and dst must hold the same number of bytes")
    check(_lib.load().sat_upload(host.data_ptr(), dst.data_ptr(), n, _stream_handle(dst.device, stream)))
    return dst


def workspace_check(ws: torch.Tensor, stream: Optional[torch.cuda.Stream] = None) -> None:
    """Synchronise and raise if a build that used `ws` reported a lookback fault."""
    check(_lib.load().sat_workspace_check(ws.data_ptr(), _stream_handle(ws.device, stream)))


def variants(kind: int, pixel_type: Optional[str] = None, squares: bool = False) -> List[str]:
    """Names of the compiled build (kind 0) or gather (kind 1) variants; with `pixel_type`, only
    those that run on such images (with the squared table if `squares`)."""
    lib = _lib.load()
    names = [lib.sat_variant_name(kind, i).decode() for i in range(lib.sat_variant_count(kind))]
    if pixel_type is None:
        return names
    code = _PIXCODE[pixel_type]
    return [n for i, n in enumerate(names) if lib.sat_variant_supported(kind, i, code, int(squares))]


def force_variant(kind: int, index: int) -> None:
    """Make later calls on this thread use build (kind 0) or gather (kind 1) variant `index`."""
    check(_lib.load().sat_force_variant(kind, index))


# ---------------------------------------------------------------- batches

def batch_items(images: Sequence[torch.Tensor], tables: Sequence[Tuple[torch.Tensor, Optional[torch.Tensor]]],
                outs: Optional[Sequence[Tuple[Optional[torch.Tensor], torch.Tensor, torch.Tensor]]] = None):
    n = len(tables)
    arr = (BatchItem * n)()
    for i, (S, Q) in enumerate(tables):
        it = arr[i]
        if images is not None:
            img = images[i]
            it.image, it.image_pitch = img.data_ptr(), img.stride(0)
        it.H, it.W = S.shape
        it.sat, it.sat_sq, it.sat_pitch = S.data_ptr(), (Q.data_ptr() if Q is not None else None), S.stride(0)
        if outs is not None:
            s1, mean, std = outs[i]
            it.sum_out = s1.data_ptr() if s1 is not None else None
            it.mean_out, it.std_out, it.out_pitch = mean.data_ptr(), std.data_ptr(), mean.stride(0)
    return arr
