"""Whole-output comparison with the oracle, band by band, for images too large for one serial
oracle pass in memory or in time (the 70000 x 85000 workload and its row shards).

The image's rows are split into parts; one worker thread per part runs an oracle.Stream started
at the part's first row (seeded with the oracle's column totals of the rows above, summed part by
part) and advances it a band of rows at a time.  Every table row of the part, and every output row
whose window starts in the part, is compared element by element with the same rows fetched from
the device through the caller's getters.  Host memory stays bounded by a few bands per worker.

Getters (each returns a numpy array; rows are half-open ranges):
  table(a, b)          table rows a..b-1, shape (b-a, W)
  out(i, k0, k1)       output rows k0..k1-1 of window i
  stats(k0, k1)        (mean, std) rows k0..k1-1 of the window `stats_window` indexes, whose
                       squared-pixel sums equal its sums (0/1 images: the table is its own table
                       of squares)
"""
import os
import threading
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle

STD_RTOL = 1e-12


def default_workers():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def check_std(got, ref, what):
    zero = ref == 0
    assert np.all(got[zero] == 0.0), what
    rel = np.abs(got[~zero] - ref[~zero]) / ref[~zero]
    assert rel.size == 0 or rel.max() <= STD_RTOL, (what, float(rel.max()))


def compare(img, windows, s, table=None, out=None, stats=None, stats_window=None, parts=None, band=256,
            workers=None, progress=None):
    """Compare every table row (if `table`), every output row of every window (if `out`) and every
    mean/std row of window `stats_window` (if `stats`) with the oracle.  Returns a summary dict of
    what was compared; raises AssertionError at the first difference."""
    H, W = img.shape
    windows = [(int(h), int(w)) for h, w in windows]
    hmax = max([h for h, _ in windows] + [1])
    workers = workers or default_workers()
    n_parts = parts or workers
    bounds = [H * i // n_parts for i in range(n_parts + 1)]
    bounds = sorted(set(bounds))
    segs = list(zip(bounds[:-1], bounds[1:]))
    shapes = [oracle.window_shape(H, W, h, w, s) for h, w in windows]
    lock = threading.Lock()
    counts = {"table_rows": 0, "out_rows": [0] * len(windows), "stat_rows": 0, "parts_done": 0}
    t_start = time.perf_counter()

    def say(msg):
        if progress:
            progress("[%6.1f s] %s" % (time.perf_counter() - t_start, msg))

    # column totals of each part, then the totals of all rows above each part
    with ThreadPoolExecutor(workers) as ex:
        totals = list(ex.map(lambda ab: oracle.column_totals(img[ab[0]:ab[1]]), segs))
    carries, run = [], np.zeros(W, np.uint64)
    for t in totals:
        carries.append(run.copy())
        run = run + t
    say("column totals of %d parts" % len(segs))

    def part(idx):
        a, b = segs[idx]
        end = min(H, b + hmax - 1)
        st = oracle.Stream(img, windows, s, r0=a, carry=carries[idx] if a > 0 else None)
        try:
            cur = a
            while cur < end:
                r1 = min(end, cur + band)
                ref_rows, per = st.next(r1, want_sat=table is not None and cur < b)
                if table is not None and cur < b:
                    e = min(r1, b)
                    got = table(cur, e)
                    if not np.array_equal(got, ref_rows[:e - cur]):
                        bad = np.argwhere(got != ref_rows[:e - cur])[0]
                        raise AssertionError("table row %d col %d differs" % (cur + bad[0], bad[1]))
                    with lock:
                        counts["table_rows"] += e - cur
                for i, (k0, block) in enumerate(per):
                    # keep the output rows whose window starts in this part
                    ks = [k for k in range(k0, k0 + block.shape[0]) if a <= k * s < b]
                    if not ks:
                        continue
                    lo, hi = ks[0], ks[-1] + 1
                    ref = block[lo - k0:hi - k0]
                    if out is not None:
                        got = out(i, lo, hi)
                        if not np.array_equal(got, ref):
                            bad = np.argwhere(got != ref)[0]
                            raise AssertionError("window %s output row %d col %d differs" %
                                                 (windows[i], lo + bad[0], bad[1]))
                        with lock:
                            counts["out_rows"][i] += hi - lo
                    if stats is not None and i == stats_window:
                        n = windows[i][0] * windows[i][1]
                        ref_mean, ref_std = oracle.mean_std(ref, ref, n)
                        g_mean, g_std = stats(lo, hi)
                        if not np.array_equal(g_mean, ref_mean):
                            bad = np.argwhere(g_mean != ref_mean)[0]
                            raise AssertionError("mean row %d col %d differs" % (lo + bad[0], bad[1]))
                        check_std(g_std, ref_std, "std rows %d..%d" % (lo, hi))
                        with lock:
                            counts["stat_rows"] += hi - lo
                cur = r1
        finally:
            st.close()
        with lock:
            counts["parts_done"] += 1
            done = counts["parts_done"]
        say("part %d (rows %d..%d) compared; %d of %d parts done" % (idx, a, b - 1, done, len(segs)))

    with ThreadPoolExecutor(workers) as ex:
        for f in [ex.submit(part, i) for i in range(len(segs))]:
            f.result()
    if table is not None:
        assert counts["table_rows"] == H
    if out is not None:
        for i, (oh, _) in enumerate(shapes):
            assert counts["out_rows"][i] == oh, (windows[i], counts["out_rows"][i], oh)
    if stats is not None:
        assert counts["stat_rows"] == shapes[stats_window][0]
    counts["seconds"] = round(time.perf_counter() - t_start, 1)
    return counts
