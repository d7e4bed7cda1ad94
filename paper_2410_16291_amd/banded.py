"""Window sums of images whose integral image does not fit in HBM, or that stream from the host.

The image is processed in bands of rows.  Each band's rows of the image's table are built from
the band's image rows and the column totals of every row above it (sat_build_band), which the
build advances for the next band: the table values are those of the whole image's table, and no
image row is built twice.  A window that ends inside the band [b0, b1) may start up to h_max - 1
rows above b0, and its sum needs the table row just above its first row, so the device keeps the
last table rows of the bands before (a ring of h_max + stride - 1 rows, copied forward on the
device after each band) in front of the band's rows: the gather runs over one contiguous view of
table rows [v0, b1), v0 the first row any output of the band needs on the stride grid.  The band
emits exactly the output rows whose windows end inside it.  The full table is never
materialised: the device holds two ring-plus-band tables, the band's image rows when they come
from the host, and its output rows.

Image rows come from a callback (host numpy rows, a memory map, a generator, pinned host tensors
or device tensors).  Device rows are built in place.  Host rows are uploaded into device buffers
on rows of whole 128-byte lines (pageable rows staged through pinned buffers) on a copy stream,
each band while the previous band is being computed.  All window sizes of a band come from one
pass over its table view (window_sum_multi), on a second stream, so that one band's gather
overlaps the next band's build.  Output rows go to a callback as device tensors, on the gather
stream, valid once that stream is synchronised; `banded_window_sums` collects them into host
arrays.

Cost over the whole-image path: per band, the copy of the ring's rows, and the outputs of the
view's first rows (windows that end above the band), which the gather computes and drops.

`build_table_streamed` is the other use of bands: the whole image's table in HBM, built band by
band as the image arrives, with the same carried column totals.
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
    """[(v0, b0, b1)]: the band of rows [b0, b1) and the first table row v0 of the view its gather
    runs on: b0 - h_max rounded down to a multiple of the stride (the row above the first row of
    any window the band emits), or 0.  b0 - v0 is at most h_max + stride - 1."""
    if band_rows < 1:
        raise ValueError("band_rows must be >= 1")
    plan = []
    b0 = 0
    while b0 < H:
        b1 = min(H, b0 + band_rows)
        v0 = max(0, (b0 - h_max) // stride * stride)
        plan.append((v0, b0, b1))
        b0 = b1
    return plan


def band_outputs(v0: int, b0: int, b1: int, H: int, h: int, stride: int) -> Tuple[int, int]:
    """Output rows [k0, k1) of an h-tall window whose last row lies in [b0, b1) (output row k of
    the image is output row k - v0 / stride of the band's view)."""
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
        # rows on whole 128-byte lines: the builds take the same plans as on a resident image
        self.dimg = [api.empty_image(rows_max, W, self.t_dtype, dev) for _ in range(2)]
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
    device tensor (built in place: unit column stride, any row pitch).
    on_rows(i, k0, rows) receives, for window i, the device tensor of its output rows [k0, k0+n),
    on the gather stream (current while on_rows runs), valid once that stream is synchronised.
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
        self.compute = torch.cuda.Stream(self.dev)           # builds (and uploads' hand-over)
        self.gather = torch.cuda.Stream(self.dev)            # gathers
        self.rows_max = max(b1 - b0 for _, b0, b1 in self.plan)
        self.ring = self.h_max + stride - 1          # table rows kept in front of each band
        self.up = None                               # host-row uploads, made on first use
        # two ring-plus-band tables, alternating: band i's ring rows are copied into the other
        self.tables = [api.empty_table(self.ring + self.rows_max, W, self.dev) for _ in range(2)]
        self.carry = api.empty_totals(W, self.dev)
        self.bpp = 1 if pixel_type == "u8" else 2
        self.t_dtype = torch.uint8 if pixel_type == "u8" else torch.uint16

    def _device_rows(self, rows, n: int) -> Optional[torch.Tensor]:
        """`rows` itself when it is a device band the build can read in place, else None."""
        if not (isinstance(rows, torch.Tensor) and rows.is_cuda):
            return None
        if tuple(rows.shape) != (n, self.W):
            raise ValueError("read_rows returned shape %s, expected %s" % (tuple(rows.shape), (n, self.W)))
        if rows.dtype not in (self.t_dtype, torch.int16 if self.bpp == 2 else torch.int8):
            raise ValueError("read_rows returned %s rows for %s pixels" % (rows.dtype, self.pixel_type))
        if rows.stride(1) != 1:
            return None
        return rows if rows.dtype == self.t_dtype else rows.view(self.t_dtype)

    def run(self, read_rows: Callable, on_rows: Callable) -> None:
        """Builds run on the compute stream, gathers on a second stream: band i's gather overlaps
        band i+1's build, whose strips alone do not fill the GPU.  The two tables alternate; a
        table is written again (the next ring, then the band two later) only after the gather
        that read it has finished."""
        plan, R, W = self.plan, self.ring, self.W
        A, B = self.compute, self.gather
        pending = None          # host rows: staged through the uploader
        first_rows = read_rows(plan[0][1], plan[0][2])
        dev_rows = self._device_rows(first_rows, plan[0][2] - plan[0][1])
        if dev_rows is None:
            if self.up is None:
                self.up = _Uploader(self.rows_max, W, self.pixel_type, self.dev)
            self.up.start(A)
            self.up.stage(0, plan[0][1], plan[0][2], lambda a, b: first_rows)
            pending = 0
        B.wait_stream(A)
        gathered = [None, None]          # event: the last gather that read table 0 / 1 is done
        for bi, (v0, b0, b1) in enumerate(plan):
            n = b1 - b0
            slot = bi & 1
            if pending is not None:
                if bi + 1 < len(plan):
                    self.up.stage(slot ^ 1, plan[bi + 1][1], plan[bi + 1][2], read_rows)
                img = self.up.acquire(A, slot, n)
            else:
                img = dev_rows if bi == 0 else self._device_rows(read_rows(b0, b1), n)
                if img is None:
                    raise ValueError("read_rows must return device rows for every band once it has for one")
            T = self.tables[slot]
            # the band's table rows, after the ring's R rows (global row y at index y - b0 + R);
            # table `slot` was last read by the gather of band bi - 2, which the copy of band bi - 1
            # below already waited for
            with torch.cuda.stream(A):
                ws = api.workspace(api.build_workspace_bytes(n, W, self.bpp, False), self.dev, A)
                api.sat_build_band(img, carry=None if bi == 0 else self.carry, rows_above=b0,
                                   sat=T[R:R + n], total=self.carry, ws=ws, stream=A)
                built = torch.cuda.Event()
                built.record(A)
                if pending is not None:
                    self.up.release(A, slot)
                if bi + 1 < len(plan):
                    # the next band's ring: this table's rows [n, n + R), global rows [b1 - R, b1),
                    # into the other table once the gather of band bi - 1 has read it
                    if gathered[slot ^ 1] is not None:
                        A.wait_event(gathered[slot ^ 1])
                    self.tables[slot ^ 1][:R].copy_(T[n:n + R])
            todo = []
            for i, (h, w) in enumerate(self.windows):
                k0, k1 = band_outputs(v0, b0, b1, self.H, h, self.stride)
                if k1 > k0:
                    todo.append((i, k0, k1))
            if not todo:
                continue
            with torch.cuda.stream(B):
                B.wait_event(built)
                view = T[v0 - b0 + R:R + n]
                hs = [self.windows[i] for i, _, _ in todo]
                if any(h > view.shape[0] for h, _ in hs):
                    raise AssertionError("band view shorter than a window it emits")
                outs = api.window_sum_multi(view, hs, self.stride, pixel_type=self.pixel_type,
                                            out_dtype=self.out_dtype, stream=B)
                done = torch.cuda.Event()
                done.record(B)
                gathered[slot] = done
                for (i, k0, k1), out in zip(todo, outs):
                    lk0 = k0 - v0 // self.stride       # output row of the view
                    on_rows(i, k0, out[lk0:lk0 + (k1 - k0)])
        A.wait_stream(B)
        A.synchronize()


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
