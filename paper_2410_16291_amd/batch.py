"""Many uneven-sized images in one launch: tables for all of them, then window statistics.

sat_build_batched hands the (image, strip) work items of every image to one persistent kernel;
window_mean_std_batched covers the work items of every image's windows in one grid;
sat_build_stats_batched does both in one persistent launch, the statistics of each image
starting as soon as its tables are stored.  `variant` names a compiled kernel variant (see
autotune) to use for the call; None keeps the library's own choice.
"""
from __future__ import annotations

from typing import List, Optional, Sequence, Tuple

import torch

from . import _lib
from .api import _PIXEL, _require_cuda, _stream_handle, empty_out, empty_table, out_shape, workspace
from ._lib import check

Tables = List[Tuple[torch.Tensor, Optional[torch.Tensor]]]
Stats = List[Tuple[Optional[torch.Tensor], torch.Tensor, torch.Tensor]]


def alloc_tables(images: Sequence[torch.Tensor], squares: bool = False) -> Tables:
    """(S, Q or None) of the right shape for every image (line-aligned pitches)."""
    out = []
    for img in images:
        H, W = img.shape
        S = empty_table(H, W, img.device)
        Q = empty_table(H, W, img.device, S.stride(0)) if squares else None
        out.append((S, Q))
    return out


def alloc_stats(tables: Sequence[Tuple[torch.Tensor, Optional[torch.Tensor]]], h: int, w: int, stride: int = 1,
                with_sum: bool = True) -> Stats:
    """(sum or None, mean, std) outputs for every table's windows."""
    outs = []
    for S, _ in tables:
        oh, ow = out_shape(S.shape[0], S.shape[1], h, w, stride)
        s1 = empty_out(oh, ow, torch.uint64, S.device) if with_sum else None
        outs.append((s1, empty_out(oh, ow, torch.float64, S.device), empty_out(oh, ow, torch.float64, S.device)))
    return outs


def build_batched(images: Sequence[torch.Tensor], squares: bool = False, tables: Optional[Tables] = None,
                  variant: Optional[str] = None, stream: Optional[torch.cuda.Stream] = None) -> Tables:
    """Tables (S, Q or None) of every image, built by one persistent launch."""
    if not images:
        return []
    dtype = images[0].dtype
    if dtype not in _PIXEL or any(i.dtype != dtype for i in images):
        raise ValueError("all images must share one dtype, uint8 or uint16")
    for i in images:
        _require_cuda(i, "image")
    dev = images[0].device
    if tables is None:
        tables = alloc_tables(images, squares)
    if len(tables) != len(images):
        raise ValueError("one (S, Q) pair per image")
    for img, (S, Q) in zip(images, tables):
        if tuple(S.shape) != tuple(img.shape) or (squares and (Q is None or Q.shape != S.shape)):
            raise ValueError("tables must match the images' shapes")
    from .api import batch_items
    from .autotune import forced
    items = batch_items(images, tables)
    lib = _lib.load()
    with forced(0, variant):
        need = lib.sat_batch_workspace_bytes(items, len(images), _PIXEL[dtype], int(squares))
        ws = workspace(need, dev, stream)
        check(lib.sat_build_batched(items, len(images), _PIXEL[dtype], ws.data_ptr(), ws.numel(),
                                    _stream_handle(dev, stream)))
    return tables


def mean_std_batched(tables: Sequence[Tuple[torch.Tensor, torch.Tensor]], h: int, w: int, stride: int = 1,
                     with_sum: bool = True, outs: Optional[Stats] = None, variant: Optional[str] = None,
                     stream: Optional[torch.cuda.Stream] = None) -> Stats:
    """[(sum or None, mean, std)] of every image's windows, one launch for all images."""
    if not tables:
        return []
    dev = tables[0][0].device
    for S, Q in tables:
        _require_cuda(S, "sat")
        _require_cuda(Q, "sat_sq")
    if outs is None:
        outs = alloc_stats(tables, h, w, stride, with_sum)
    from .api import batch_items
    from .autotune import forced
    items = batch_items(None, tables, outs)
    lib = _lib.load()
    need = 256 + len(tables) * 256
    ws = workspace(need, dev, stream)
    with forced(1, variant):
        check(lib.window_mean_std_batched(items, len(tables), h, w, stride, ws.data_ptr(), ws.numel(),
                                          _stream_handle(dev, stream)))
    return outs


def build_stats_batched(images: Sequence[torch.Tensor], h: int, w: int, stride: int = 1, with_sum: bool = True,
                        tables: Optional[Tables] = None, outs: Optional[Stats] = None,
                        build_variant: Optional[str] = None, gather_variant: Optional[str] = None,
                        stream: Optional[torch.cuda.Stream] = None) -> Tuple[Tables, Stats]:
    """Tables (S, Q) of every image and the (sum or None, mean, std) of every image's h x w windows
    at `stride`, in one persistent launch."""
    if not images:
        return [], []
    dtype = images[0].dtype
    if dtype not in _PIXEL or any(i.dtype != dtype for i in images):
        raise ValueError("all images must share one dtype, uint8 or uint16")
    for i in images:
        _require_cuda(i, "image")
    dev = images[0].device
    if tables is None:
        tables = alloc_tables(images, True)
    if len(tables) != len(images) or any(Q is None for _, Q in tables):
        raise ValueError("one (S, Q) pair per image, squares included")
    for img, (S, Q) in zip(images, tables):
        if tuple(S.shape) != tuple(img.shape) or Q.shape != S.shape:
            raise ValueError("tables must match the images' shapes")
    if outs is None:
        outs = alloc_stats(tables, h, w, stride, with_sum)
    from .api import batch_items
    from .autotune import forced
    items = batch_items(images, tables, outs)
    lib = _lib.load()
    with forced(0, build_variant), forced(1, gather_variant):
        need = lib.sat_build_stats_workspace_bytes(items, len(images), _PIXEL[dtype])
        if need == 0:
            raise ValueError("invalid image sizes")
        ws = workspace(need, dev, stream)
        check(lib.sat_build_stats_batched(items, len(images), _PIXEL[dtype], h, w, stride, ws.data_ptr(), ws.numel(),
                                          _stream_handle(dev, stream)))
    return tables, outs
