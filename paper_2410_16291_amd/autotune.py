"""Kernel-shape selection by measurement: the tile/scan shapes of the table build and the gather.

The library compiles several build variants (pixels per lane, rows per wave, waves per
workgroup, lookback / reduce-then-scan / helper-wave column scans) and several gather variants
(chain walks with 1, 2 or 4 outputs per thread, row-pair kernels over bands of 2 to 8 column
chunks).  Which one is fastest depends on the image sizes, the pixel type, the squared table and
the window, so the tuner times every candidate on the caller's own work (one warm-up and `reps`
timed runs each, HIP events on the launch stream): the build variant, then the strip height of
the chosen variant (its own, three quarters, half), the gather variant, and for statistics
whether tables and statistics go in one launch or two.  It keeps the fastest of each and caches
the choices per device (name, architecture, CU count) and shape class (image count, total pixels
and rows, pixel type, squares, window, stride) in a JSON file; later calls in the same class reuse
them without timing.

    tuner = Tuner()
    choice = tuner.tune_batch(images, squares=True, win=(64, 64), stride=4)
    Tuner.run_batch(choice, images, True, (64, 64), 4, tables, outs)
"""
from __future__ import annotations

import contextlib
import json
import math
import os
import re
from typing import Callable, Dict, Iterable, List, Optional, Sequence, Tuple

import torch

from . import api

DEFAULT_CACHE = os.environ.get("SAT_TUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "sat_mi355x_tune.json"))


def device_key(device) -> str:
    p = torch.cuda.get_device_properties(device)
    return "%s|%s|%d" % (p.name, getattr(p, "gcnArchName", ""), p.multi_processor_count)


def shape_class(sizes: Iterable[Tuple[int, int]], pixel_bytes: int, squares: bool,
                win: Optional[Tuple[int, int]] = None, stride: int = 1) -> str:
    """Images by count and total pixels (powers of two), pixel type, squared table, window."""
    sizes = list(sizes)
    px = sum(h * w for h, w in sizes)
    rows = sum(h for h, _ in sizes)
    key = "n%d_px2^%d_rows2^%d_b%d_%s" % (1 << max(0, math.ceil(math.log2(len(sizes)))) if sizes else 0,
                                         round(math.log2(max(px, 1))), round(math.log2(max(rows, 1))),
                                         pixel_bytes, "sq" if squares else "s")
    if win is not None:
        key += "_w%dx%d_s%d" % (win[0], win[1], stride)
    return key


@contextlib.contextmanager
def forced_strip(rows: Optional[int]):
    """Run the body with batched builds on this thread using strips of `rows` rows (None: the
    variant's own height)."""
    if rows is None:
        yield
        return
    api.force_variant(2, int(rows))
    try:
        yield
    finally:
        api.force_variant(2, -1)


@contextlib.contextmanager
def forced_segments(n: Optional[int]):
    """Run the body with helper-wave builds of one image on this thread split into `n` column
    segments per strip (None: the built-in choice)."""
    if n is None:
        yield
        return
    api.force_variant(4, int(n))
    try:
        yield
    finally:
        api.force_variant(4, 0)


def strip_height(name: str) -> Optional[int]:
    """Full strip height (rows per wave x waves) of a build variant, from its name."""
    m = re.search(r"rw(\d+)_nw(\d+)", name)
    return int(m.group(1)) * int(m.group(2)) if m else None


@contextlib.contextmanager
def forced(kind: int, name: Optional[str]):
    """Run the body with variant `name` of `kind` (0 build, 1 gather) forced on this thread."""
    if name is None:
        yield
        return
    names = api.variants(kind)
    if name not in names:
        raise ValueError("unknown %s variant %r" % ("build" if kind == 0 else "gather", name))
    api.force_variant(kind, names.index(name))
    try:
        yield
    finally:
        api.force_variant(kind, -1)


def time_ms(run: Callable[[], None], reps: int = 3, stream: Optional[torch.cuda.Stream] = None) -> float:
    """Median event time of `run` on the current stream after one untimed run."""
    s = stream or torch.cuda.current_stream()
    run()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(s)
        run()
        b.record(s)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


class Tuner:
    """Times candidate variants and remembers the fastest per device and shape class."""

    def __init__(self, path: Optional[str] = DEFAULT_CACHE, reps: int = 3):
        self.path = path
        self.reps = reps
        self.cache: Dict[str, dict] = {}
        if path and os.path.exists(path):
            try:
                with open(path) as f:
                    self.cache = json.load(f)
            except (OSError, ValueError):
                self.cache = {}

    def _save(self) -> None:
        if not self.path:
            return
        os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.cache, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    def lookup(self, kind: int, key: str) -> Optional[str]:
        entry = self.cache.get("%d|%s" % (kind, key))
        return entry["best"] if entry else None

    def tune(self, kind: int, key: str, run: Callable[[], None], candidates: Optional[Sequence[str]] = None,
             retune: bool = False) -> Tuple[str, Dict[str, float]]:
        """Fastest of `candidates` (default: every compiled variant of `kind`) for `run`."""
        ck = "%d|%s" % (kind, key)
        if not retune and ck in self.cache:
            return self.cache[ck]["best"], self.cache[ck]["ms"]
        names = list(candidates) if candidates is not None else api.variants(kind)
        times = {}
        for name in names:
            with forced(kind, name):
                times[name] = round(time_ms(run, self.reps), 4)
        best = min(times, key=times.get)
        self.cache[ck] = {"best": best, "ms": times}
        self._save()
        return best, times

    def tune_batch(self, images: Sequence[torch.Tensor], squares: bool, win: Tuple[int, int], stride: int,
                   retune: bool = False) -> dict:
        """Build and mean/std (or sum) variants for this batch, timed on the batch itself."""
        from . import batch
        dev = images[0].device
        pb = images[0].element_size()
        sizes = [tuple(i.shape) for i in images]
        dkey = device_key(dev)
        bkey = dkey + "|" + shape_class(sizes, pb, squares)
        tables = batch.alloc_tables(images, squares)
        build, build_ms = self.tune(0, bkey, lambda: batch.build_batched(images, squares, tables=tables),
                                    candidates=api.variants(0, "u8" if pb == 1 else "u16", squares), retune=retune)
        gkey = dkey + "|" + shape_class(sizes, pb, squares, win, stride)
        if squares:
            outs = batch.alloc_stats(tables, win[0], win[1], stride)
            run = lambda: batch.mean_std_batched(tables, win[0], win[1], stride, outs=outs)   # noqa: E731
        else:
            run = lambda: [api.window_sum(S, win[0], win[1], stride,                          # noqa: E731
                                          pixel_type="u8" if pb == 1 else "u16") for S, _ in tables]
        gather, gather_ms = self.tune(1, gkey, run, retune=retune)
        # strip height of the chosen build variant: its own, three quarters and half of it
        strip, strip_ms = None, {}
        th = strip_height(build)
        if th:
            skey = bkey + "|" + build
            ck = "2|" + skey
            if not retune and ck in self.cache:
                strip, strip_ms = self.cache[ck]["best"], self.cache[ck]["ms"]
            else:
                cands = [th] + sorted({h for h in (th * 3 // 4, th // 2) if 8 <= h < th}, reverse=True)
                for h in cands:
                    with forced(0, build), forced_strip(h):
                        strip_ms[str(h)] = round(time_ms(lambda: batch.build_batched(images, squares, tables=tables),
                                                         self.reps), 4)
                best = min(strip_ms, key=strip_ms.get)
                strip = int(best)
                self.cache[ck] = {"best": strip, "ms": strip_ms}
                self._save()
            strip = None if strip == th else strip
        # tables and statistics fused in one launch, or the two launches (statistics only)
        fused, fused_ms = False, {}
        if squares:
            fkey = "3|" + gkey + "|" + build + "|" + gather + "|" + str(strip)
            if not retune and fkey in self.cache:
                fused, fused_ms = self.cache[fkey]["best"], self.cache[fkey]["ms"]
            else:
                def two():
                    batch.build_batched(images, squares, tables=tables)
                    batch.mean_std_batched(tables, win[0], win[1], stride, outs=outs)

                def one():
                    batch.build_stats_batched(images, win[0], win[1], stride, tables=tables, outs=outs)
                with forced(0, build), forced(1, gather), forced_strip(strip):
                    fused_ms = {"two_launches": round(time_ms(two, self.reps), 4),
                                "one_launch": round(time_ms(one, self.reps), 4)}
                fused = fused_ms["one_launch"] < fused_ms["two_launches"]
                self.cache[fkey] = {"best": fused, "ms": fused_ms}
                self._save()
        return {"build": build, "gather": gather, "build_ms": build_ms, "gather_ms": gather_ms,
                "strip_h": strip, "strip_ms": strip_ms, "fused": fused, "fused_ms": fused_ms,
                "build_key": bkey, "gather_key": gkey}

    @staticmethod
    def run_batch(choice: dict, images, squares: bool, win: Tuple[int, int], stride: int, tables, outs) -> None:
        """The batch with a tune_batch choice: its variants, strip height and launch form."""
        from . import batch
        with forced(0, choice["build"]), forced(1, choice["gather"]), forced_strip(choice.get("strip_h")):
            if choice.get("fused"):
                batch.build_stats_batched(images, win[0], win[1], stride, tables=tables, outs=outs)
            else:
                batch.build_batched(images, squares, tables=tables)
                batch.mean_std_batched(tables, win[0], win[1], stride, outs=outs)
