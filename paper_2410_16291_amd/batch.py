"""Many uneven-sized images in one launch: tables for all of them, then window statistics.

sat_build_batched hands (image, strip) work items of every image to one persistent kernel;
window_mean_std_batched covers (image, output row, chunk) items of every image in one grid.
"""
from __future__ import annotations

from typing import List, Optional, Sequence, Tuple

import torch

from . import _lib
from .api import _PIXEL, _require_cuda, _stream_handle, empty_out, empty_table, out_shape, workspace
from ._lib import check


def build_batched(images: Sequence[torch.Tensor], squares: bool = False,
                  stream: Optional[torch.cuda.Stream] = None) -> List[Tuple[torch.Tensor, Optional[torch.Tensor]]]:
    """Tables (S, Q or None) of every image, built by one persistent launch."""
    if not images:
        return []
    dtype = images[0].dtype
    if dtype not in _PIXEL or any(i.dtype != dtype for i in images):
        raise ValueError("all images must share one dtype, uint8 or uint16")
    for i in images:
        _require_cuda(i, "image")
    dev = images[0].device
    tables = []
    for img in images:
        H, W = img.shape
        S = empty_table(H, W, dev)
        Q = empty_table(H, W, dev, S.stride(0)) if squares else None
        tables.append((S, Q))
    from .api import batch_items
    items = batch_items(images, tables)
    lib = _lib.load()
    need = lib.sat_batch_workspace_bytes(items, len(images), _PIXEL[dtype], int(squares))
    ws = workspace(need, dev, stream)
    check(lib.sat_build_batched(items, len(images), _PIXEL[dtype], ws.data_ptr(), ws.numel(),
                                _stream_handle(dev, stream)))
    return tables


def mean_std_batched(tables: Sequence[Tuple[torch.Tensor, torch.Tensor]], h: int, w: int, stride: int = 1,
                     with_sum: bool = True, stream: Optional[torch.cuda.Stream] = None):
    """[(sum or None, mean, std)] of every image's windows, one launch for all images."""
    if not tables:
        return []
    dev = tables[0][0].device
    outs = []
    for S, Q in tables:
        _require_cuda(S, "sat")
        _require_cuda(Q, "sat_sq")
        oh, ow = out_shape(S.shape[0], S.shape[1], h, w, stride)
        s1 = empty_out(oh, ow, torch.uint64, dev) if with_sum else None
        outs.append((s1, empty_out(oh, ow, torch.float64, dev), empty_out(oh, ow, torch.float64, dev)))
    from .api import batch_items
    items = batch_items(None, tables, outs)
    lib = _lib.load()
    need = 256 + len(tables) * 256
    ws = workspace(need, dev, stream)
    check(lib.window_mean_std_batched(items, len(tables), h, w, stride, ws.data_ptr(), ws.numel(),
                                      _stream_handle(dev, stream)))
    return outs
