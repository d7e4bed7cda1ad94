"""Window sums of images whose integral image does not fit in HBM, or that stream from the host.

The image is processed in bands of rows.  For the band of rows [b0, b1) the device builds the
integral image of rows [r0, b1) only, r0 = b0 - (h_max - 1) rounded down to the stride grid: a
local table.  A window sum is a difference of table values along both axes, so the sum of any
window lying inside rows [r0, b1) is the same from the local table as from the table of the
whole image.  The band emits exactly the output rows whose windows end inside it (their last row
in [b0, b1)); every such window starts at or after r0.  The full table is never materialised: the
device holds one band's image rows, its local table and its output rows at a time.

Image rows come from a callback (host numpy rows, a memory map, a generator, pinned host tensors
or device tensors); pageable host rows are staged through pinned buffers, and every band is
uploaded on a copy stream while the previous band is being computed.  All window sizes of a band
come from one pass over its table (window_sum_multi).  Output rows go to a callback as device
tensors, on the compute stream, valid once that stream is synchronised; `banded_window_sums`
collects them into host arrays.

Cost over the whole-image path: the h_max - 1 overlap rows are built again for every band, and
their outputs are discarded: about (h_max - 1) / band_rows extra table rows per band.

`build_table_streamed` is the other use of bands: the whole image's table in HBM, built band by
band as the image arrives.  There the bands do not overlap; each band's build starts from the
column totals of the rows above it and leaves those through its own last row for the next band.
"""
from __future__ import annotations

from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import api


def _check_windows(H: int, W: int, windows: Sequence[Tuple[int, int]], stride: int):
    if not windows:
        raise ValueError("at least one window")
    for h, w in windows:
        if h < 1 or w < 1 or h > H or w > W:
            raise ValueError("window %dx%d does not fit a %dx%d image" % (h, w, H, W))
    if stride < 1:
        raise ValueError("stride must be >= 1")


def band_plan(H: int, h_max: int, stride: int, band_rows: int) -> List[Tuple[int, int, int]]:
    """[(r0, b0, b1)]: the band of rows [b0, b1) and the first image row r0 its local table starts
    at (b0 - h_max + 1 rounded down to a multiple of the stride, at least 0)."""
    if band_rows < 1:
        raise ValueError("band_rows must be >= 1")
    plan = []
    b0 = 0
    while b0 < H:
        b1 = min(H, b0 + band_rows)
        r0 = max(0, b0 - (h_max - 1))
        r0 -= r0 % stride
        plan.append((r0, b0, b1))
        b0 = b1
    return plan


def band_outputs(r0: int, b0: int, b1: int, H: int, h: int, stride: int) -> Tuple[int, int]:
    """Output rows [k0, k1) of an h-tall window whose last row lies in [b0, b1), and the output
    row of the local table (rows from r0) that k0 corresponds to."""
    oh = (H - h) // stride + 1
    # last row of output k is k*stride + h - 1; it lies in [b0, b1) for k in [k0, k1)
    k0 = max(0, -(-(b0 - h + 1) // stride))
    k1 = min(oh, (b1 - h) // stride + 1) if b1 - h >= 0 else 0
    return k0, max(k0, k1)


class _Uploader:
    """Two device image buffers of rows_max x W and two pinned staging buffers: stage() puts image
    rows [r0, r1) into buffer `slot` on the copy stream (host rows through a pinned buffer), after
    the compute stream has released that buffer."""

    def __init__(self, rows_max: int, W: int, pixel_type: str, dev: torch.device):
        self.W = W
        self.np_dtype = np.uint8 if pixel_type == "u8" else np.uint16
        self.t_dtype = torch.uint8 if pixel_type == "u8" else torch.uint16
        self.copy = torch.cuda.Stream(dev)
        self.dimg = [torch.empty((rows_max, W), dtype=self.t_dtype, device=dev) for _ in range(2)]
        self.pinned = [torch.empty((rows_max, W), dtype=torch.uint8 if self.np_dtype == np.uint8 else torch.int16,
                                   pin_memory=True) for _ in range(2)]
        self.uploaded = [torch.cuda.Event() for _ in range(2)]
        self.consumed = [torch.cuda.Event() for _ in range(2)]

    def start(self, compute: torch.cuda.Stream) -> None:
        for e in self.consumed:
            e.record(compute)

    def stage(self, slot: int, r0: int, r1: int, read_rows: Callable) -> None:
        rows = read_rows(r0, r1)
        n = r1 - r0
        if isinstance(rows, torch.Tensor) and (rows.is_cuda or rows.is_pinned()):
            if tuple(rows.shape) != (n, self.W):
                raise ValueError("read_rows returned shape %s, expected %s" % (tuple(rows.shape), (n, self.W)))
            with torch.cuda.stream(self.copy):
                self.copy.wait_event(self.consumed[slot])
                if rows.dtype == self.t_dtype:
                    self.dimg[slot][:n].copy_(rows, non_blocking=True)
                else:                                   # a signed view of the same bytes
                    self.dimg[slot][:n].view(rows.dtype).copy_(rows, non_blocking=True)
                self.uploaded[slot].record(self.copy)
            return
        if isinstance(rows, torch.Tensor):
            rows = rows.numpy()
        a = np.ascontiguousarray(rows, dtype=self.np_dtype)
        if a.shape != (n, self.W):
            raise ValueError("read_rows returned shape %s, expected %s" % (a.shape, (n, self.W)))
        self.consumed[slot].synchronize()            # the pinned buffer's last upload is done with it
        host = self.pinned[slot][:n]
        host.numpy()[...] = a.view(host.numpy().dtype)
        with torch.cuda.stream(self.copy):
            self.copy.wait_event(self.consumed[slot])
            dst = self.dimg[slot][:n]
            dst.view(host.dtype).copy_(host, non_blocking=True)
            self.uploaded[slot].record(self.copy)

    def acquire(self, compute: torch.cuda.Stream, slot: int, n: int) -> torch.Tensor:
        compute.wait_event(self.uploaded[slot])
        return self.dimg[slot][:n]

    def release(self, compute: torch.cuda.Stream, slot: int) -> None:
        self.consumed[slot].record(compute)


class BandedWindowSums:
    """Streams an H x W image through the device in bands and produces window sums.

    read_rows(r0, r1) -> image rows [r0, r1) as a (r1-r0, W) numpy array, pinned host tensor or
    device tensor.
    on_rows(i, k0, rows) receives, for window i, the device tensor of its output rows [k0, k0+n).
    """

    def __init__(self, H: int, W: int, windows: Sequence[Tuple[int, int]], stride: int = 1,
                 pixel_type: str = "u8", band_rows: int = 8192, device="cuda:0",
                 out_dtype: Optional[torch.dtype] = None):
        _check_windows(H, W, windows, stride)
        self.H, self.W = H, W
        self.windows = [(int(h), int(w)) for h, w in windows]
        self.stride = stride
        self.pixel_type = pixel_type
        self.dev = torch.device(device)
        self.h_max = max(h for h, _ in self.windows)
        self.band_rows = band_rows
        self.plan = band_plan(H, self.h_max, stride, band_rows)
        big = any(api.default_out_dtype(h, w, pixel_type) == torch.uint64 for h, w in self.windows)
        self.out_dtype = out_dtype or (torch.uint64 if big else torch.uint32)
        self.compute = torch.cuda.Stream(self.dev)
        rows_max = max(b1 - r0 for r0, _, b1 in self.plan)
        self.rows_max = rows_max
        self.up = _Uploader(rows_max, W, pixel_type, self.dev)      # double-buffered image bands
        self.dimg = self.up.dimg
        self.table = api.empty_table(rows_max, W, self.dev)
        self.bpp = 1 if pixel_type == "u8" else 2

    def run(self, read_rows: Callable, on_rows: Callable) -> None:
        plan = self.plan
        self.up.start(self.compute)
        self.up.stage(0, plan[0][0], plan[0][2], read_rows)
        for bi, (r0, b0, b1) in enumerate(plan):
            slot = bi & 1
            if bi + 1 < len(plan):
                nr0, _, nb1 = plan[bi + 1]
                self.up.stage(slot ^ 1, nr0, nb1, read_rows)
            n = b1 - r0
            img = self.up.acquire(self.compute, slot, n)
            S = self.table[:n]
            ws = api.workspace(api.build_workspace_bytes(n, self.W, self.bpp, False), self.dev, self.compute)
            api.sat_build(img, sat=S, ws=ws, stream=self.compute)
            self.up.release(self.compute, slot)
            # every window with output rows in this band, in one pass over the band's table
            todo = []
            for i, (h, w) in enumerate(self.windows):
                k0, k1 = band_outputs(r0, b0, b1, self.H, h, self.stride)
                if k1 > k0 and h <= n:
                    todo.append((i, k0, k1))
            if not todo:
                continue
            with torch.cuda.stream(self.compute):
                outs = api.window_sum_multi(S, [self.windows[i] for i, _, _ in todo], self.stride,
                                            pixel_type=self.pixel_type, out_dtype=self.out_dtype,
                                            stream=self.compute)
                for (i, k0, k1), out in zip(todo, outs):
                    lk0 = k0 - r0 // self.stride       # output row of the local table
                    on_rows(i, k0, out[lk0:lk0 + (k1 - k0)])
        self.compute.synchronize()


def banded_window_sums(read_rows: Callable, H: int, W: int, windows: Sequence[Tuple[int, int]], stride: int = 1,
                       pixel_type: str = "u8", band_rows: int = 8192, device="cuda:0",
                       out_dtype: Optional[torch.dtype] = None) -> List[np.ndarray]:
    """Window sums of every window size of `windows` as host arrays, computed band by band."""
    job = BandedWindowSums(H, W, windows, stride, pixel_type, band_rows, device, out_dtype)
    host = []
    for h, w in job.windows:
        oh, ow = api.out_shape(H, W, h, w, stride)
        host.append(np.zeros((oh, ow), np.uint32 if job.out_dtype == torch.uint32 else np.uint64))
    pending = []

    def on_rows(i, k0, rows):
        signed = rows.view(torch.int32 if job.out_dtype == torch.uint32 else torch.int64)
        pending.append((i, k0, signed.to("cpu", non_blocking=False)))

    job.run(read_rows, on_rows)
    for i, k0, t in pending:
        a = t.numpy()
        host[i][k0:k0 + a.shape[0]] = a.view(host[i].dtype)
    return host


def build_table_streamed(read_rows: Callable, H: int, W: int, pixel_type: str = "u8", squares: bool = False,
                         band_rows: int = 8192, device="cuda:0", sat: Optional[torch.Tensor] = None,
                         sat_sq: Optional[torch.Tensor] = None):
    """The integral image of the whole H x W image (and of its squares) in HBM, from image rows
    that arrive band by band (read_rows as for BandedWindowSums).  Each band's table rows are
    built from the band and the column totals of the rows above it (sat_build_band), which the
    band's build advances in place for the next band; bands are uploaded on a copy stream while
    the previous band builds.  The device holds the table, two image bands and the W-word totals.
    Returns S, or (S, Q)."""
    if H < 1 or W < 1 or band_rows < 1:
        raise ValueError("H, W and band_rows must be >= 1")
    dev = torch.device(device)
    S = sat if sat is not None else api.empty_table(H, W, dev)
    Q = sat_sq if sat_sq is not None else (api.empty_table(H, W, dev, S.stride(0)) if squares else None)
    bpp = 1 if pixel_type == "u8" else 2
    bands = [(b0, min(H, b0 + band_rows)) for b0 in range(0, H, band_rows)]
    rows_max = max(b1 - b0 for b0, b1 in bands)
    compute = torch.cuda.Stream(dev)
    up = _Uploader(rows_max, W, pixel_type, dev)
    carry = api.empty_totals(W, dev)
    carry_sq = api.empty_totals(W, dev) if Q is not None else None
    # the build variant (and so the workspace it needs) depends on the band height
    need = max(api.build_workspace_bytes(n, W, bpp, Q is not None) for n in {b1 - b0 for b0, b1 in bands})
    ws = api.workspace(need, dev, compute)
    up.start(compute)
    up.stage(0, bands[0][0], bands[0][1], read_rows)
    for bi, (b0, b1) in enumerate(bands):
        slot = bi & 1
        if bi + 1 < len(bands):
            up.stage(slot ^ 1, bands[bi + 1][0], bands[bi + 1][1], read_rows)
        img = up.acquire(compute, slot, b1 - b0)
        first = bi == 0
        api.sat_build_band(img, carry=None if first else carry, rows_above=b0, squares=Q is not None,
                           carry_sq=None if first or Q is None else carry_sq, sat=S[b0:b1],
                           sat_sq=Q[b0:b1] if Q is not None else None, total=carry, total_sq=carry_sq, ws=ws,
                           stream=compute)
        up.release(compute, slot)
    compute.synchronize()
    return (S, Q) if Q is not None else S
