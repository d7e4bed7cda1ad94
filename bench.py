"""Throughput of the integral-image hot path on one MI355X.

One step = the whole path over one synthetic full-scale image: build the uint64 integral image of
a 70000 x 85000 uint8 cell-centroid mask (Thomas cluster process), then the sums of every
100x100, 250x250 and 500x500 window at stride 1 from that one table (uint32 outputs), all three
window sizes in one pass over the table.  The image, the table and the outputs stay resident in
HBM; the timed region contains only the kernels.  Prints ONE JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--rows H --cols W]

`value` is Gpixels/s of image processed per second of whole-step time.  `roofline` reports the
dominant kernel's algorithmic bytes over its average launch duration (HIP events around each
launch, on the launch stream, inside the timed region) against the 8 TB/s HBM peak, and the HBM
traffic rocprofv3 counted for that kernel when the committed counter summary was taken from the
current kernel source.  `cpu_baseline` times the oracle on a bounded band of rows of the same
image on all host cores (and on one core), beside a multi-core OpenMP baseline, scaled to the same
unit.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Gpix/s SAT+window sums at 70k×85k, % HBM peak; served p50/p99 latency"
WINDOWS = (100, 250, 500)
GATHER_SRC = os.path.join(ROOT, "paper_2410_16291_amd", "csrc", "sat_gather.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "window_sum_multi_70000x85000_traffic.md")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--rows", type=int, default=70000)
    ap.add_argument("--cols", type=int, default=85000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-separate", action="store_true",
                    help="skip the context timing of one window size per call")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-image section")
    ap.add_argument("--batch-images", type=int, default=64)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving section")
    ap.add_argument("--no-banded", action="store_true", help="skip the banded (out-of-core) section")
    ap.add_argument("--no-moments", action="store_true", help="skip the higher-moments section")
    ap.add_argument("--no-meanstd", action="store_true", help="skip the 8192^2 16-bit mean/std section")
    ap.add_argument("--no-shard", action="store_true", help="skip the one-GPU row-shard section")
    ap.add_argument("--moments-size", type=int, default=32768)
    ap.add_argument("--band-rows", type=int, default=8192)
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="length of the 50 req/s request stream")
    ap.add_argument("--burst-seconds", type=float, default=3.0, help="length of the 500 req/s burst")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the baseline sample")
    ap.add_argument("--json-out", default=None)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run plain int64 copies of known size (1 GiB read + 1 GiB written, "
                         "contiguous and row-strided) for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE")
    return ap.parse_args()


def alg_bytes_build(H, W):
    """Read the uint8 image once, write the uint64 table once."""
    return H * W * (1 + 8)


def alg_bytes_windows(H, W, hs, out_bytes=4):
    """Every table entry the corner lookups of all windows touch, read once, plus every output
    written once (stride 1, square windows)."""
    rows = cols = 0
    for h in hs:
        oh, ow = H - h + 1, W - h + 1
        rows = max(rows, min(H, (oh - 1) + (H - (h - 1))) if oh > 1 else (2 if h < H else 1))
        cols = max(cols, min(W, (ow - 1) + (W - (h - 1))) if ow > 1 else (2 if h < W else 1))
    return rows * cols * 8 + sum((H - h + 1) * (W - h + 1) * out_bytes for h in hs)


def source_digest(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def committed_traffic(H, W):
    """HBM bytes per launch of the fused gather from the committed counter summary, if that
    summary was taken from the current kernel source at this size; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    text = open(TRAFFIC_FILE).read()
    m_src = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
    m_val = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    m_size = re.search(r"workload_rows_cols:\s*(\d+)x(\d+)", text)
    if not (m_src and m_val and m_size):
        return None
    if m_src.group(1) != source_digest(GATHER_SRC) or (int(m_size.group(1)), int(m_size.group(2))) != (H, W):
        return None
    return float(m_val.group(1))


def host_cpu():
    """(CPU model name, logical CPUs this process may run on)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return model, n


def cpu_baseline(H, W, seconds_target):
    """The oracle on the first rows of the same image (table + the three windows), timed three ways
    on the host: the oracle on all host cores (the sample's rows in parts, each part streamed by the
    oracle from the column totals of the rows above it, one thread per part), the oracle on one
    core, and the multi-core OpenMP baseline (row-band table build, then the window sums)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import cpu_baseline as omp
    import oracle
    from paper_2410_16291_amd import synth

    model, ncpu = host_cpu()
    threads = max(1, min(ncpu, int(os.environ.get("OMP_NUM_THREADS", ncpu) or ncpu)))
    ys, xs = synth.thomas_points(H, W, seed=2)
    hmax = max(WINDOWS)
    wins = [(h, h) for h in WINDOWS]

    def slab(R):
        a = np.zeros((R, W), np.uint8)
        keep = ys < R
        a[ys[keep], xs[keep]] = 1
        return a

    def one_core(img):
        t0 = time.perf_counter()
        S = oracle.sat(img)
        for h in WINDOWS:
            if h <= img.shape[0]:
                oracle.window_sum_sat(S, h, h, 1)
        return time.perf_counter() - t0

    def all_cores(img, parts):
        """The oracle's own stream, started at each part's first row from the column totals of the
        rows above (oracle.column_totals), every output row of each part's windows emitted."""
        R = img.shape[0]
        bounds = [R * i // parts for i in range(parts + 1)]
        segs = list(zip(bounds[:-1], bounds[1:]))
        t0 = time.perf_counter()
        with ThreadPoolExecutor(parts) as ex:
            totals = list(ex.map(lambda ab: oracle.column_totals(img[ab[0]:ab[1]]), segs))
        carries, run = [], np.zeros(W, np.uint64)
        for t in totals:
            carries.append(run.copy())
            run = run + t

        def part(i):
            a, b = segs[i]
            st = oracle.Stream(img, wins, 1, r0=a, carry=carries[i] if a else None)
            end, cur = min(R, b + hmax - 1), a
            while cur < end:
                cur = min(end, cur + 512)
                st.next(cur, want_sat=False)
            st.close()

        with ThreadPoolExecutor(parts) as ex:
            list(ex.map(part, range(len(segs))))
        return time.perf_counter() - t0

    def openmp(img, S, outs):
        t0 = time.perf_counter()
        _, n = omp.sat_u8(img, threads, out=S)
        for h, o in zip(WINDOWS, outs):
            omp.window_sum_u32(S, h, h, 1, threads, out=o)
        return time.perf_counter() - t0, n

    share = seconds_target / 3.0
    # one core: scale a 1024-row trial to the time share
    t = one_core(slab(1024))
    R1 = int(min(H, max(2 * hmax, 1024 * share / max(t, 1e-3))))
    t1 = one_core(slab(R1))
    # all cores: parts of at least 4 * hmax rows so the rows each part re-reads below it stay small
    R = int(min(H, max(threads * 4 * hmax, 16384)))
    img = slab(R)
    t = all_cores(img, threads)
    reps = max(1, min(5, int(share / max(t, 1e-3))))
    tp = min(all_cores(img, threads) for _ in range(reps))
    # OpenMP: the same sample, buffers reused (the first run touches their pages)
    Ro = min(R, 8192)
    imgo = np.ascontiguousarray(img[:Ro])
    S = np.empty((Ro, W), np.uint64)
    outs = [np.empty((Ro - h + 1, W - h + 1), np.uint32) for h in WINDOWS]
    t, n_omp = openmp(imgo, S, outs)
    reps = max(1, min(5, int(share / max(t, 1e-3))))
    to = min(openmp(imgo, S, outs)[0] for _ in range(reps))
    return {"value": round(R * W / tp / 1e9, 5), "unit": "Gpix/s", "cores": threads, "kind": "oracle",
            "sample": "rows 0..%d of the %dx%d image (%.1f Mpx) in %d parts, one thread each: the serial "
                      "oracle's streamed table and the window sums %s by corner lookup (uint64) from the "
                      "oracle's column totals of the rows above each part; best of %d runs, %.2f s" %
                      (R - 1, H, W, R * W / 1e6, threads, "/".join(map(str, WINDOWS)), reps, tp),
            "cpu_model": model, "host_cpus": ncpu,
            "one_core": {"value": round(R1 * W / t1 / 1e9, 5), "cores": 1, "kind": "oracle",
                         "sample": "rows 0..%d (%.1f Mpx): serial table build + the three window sums, "
                                   "one thread, %.1f s" % (R1 - 1, R1 * W / 1e6, t1)},
            "openmp": {"value": round(Ro * W / to / 1e9, 5), "cores": n_omp, "kind": "openmp",
                       "sample": "rows 0..%d (%.1f Mpx): row-band table build on %d threads, then the "
                                 "three uint32 window sums, buffers reused; best of %d runs, %.3f s" %
                                 (Ro - 1, Ro * W / 1e6, n_omp, reps, to)}}


def batched_section(torch, dev, n_images):
    """Many uneven images: one batched build + one batched mean/std launch, against the same
    work as one build and one mean/std call per image, and against the autotuned variants."""
    from paper_2410_16291_amd import api, autotune, batch, synth

    sizes = synth.uneven_sizes(n_images, 1000, 12000, seed=3)
    imgs = [synth.lognormal_u16_device(H, W, 3000 + i, dev) for i, (H, W) in enumerate(sizes)]
    px = sum(H * W for H, W in sizes)
    h = w = 64
    stride = 4
    tables = batch.alloc_tables(imgs, squares=True)
    outs = batch.alloc_stats(tables, h, w, stride)
    ws = api.workspace(max(api.build_workspace_bytes(H, W, 2, True) for H, W in sizes), dev)
    torch.cuda.synchronize()

    def per_image():
        for img, (S, Q), o in zip(imgs, tables, outs):
            api.sat_build(img, sat=S, sat_sq=Q, ws=ws)
            api.window_mean_std(S, Q, h, w, stride, outs=o)

    def batched(build=None, gather=None):
        batch.build_batched(imgs, True, tables=tables, variant=build)
        batch.mean_std_batched(tables, h, w, stride, outs=outs, variant=gather)

    t_per = autotune.time_ms(per_image, reps=3)
    t_bat = autotune.time_ms(batched, reps=3)
    t_fused = autotune.time_ms(lambda: batch.build_stats_batched(imgs, h, w, stride, tables=tables, outs=outs),
                               reps=3)
    tuner = autotune.Tuner(path=None, reps=3)
    t0 = time.perf_counter()
    choice = tuner.tune_batch(imgs, squares=True, win=(h, w), stride=stride)
    tune_s = time.perf_counter() - t0
    t_tuned = autotune.time_ms(lambda: autotune.Tuner.run_batch(choice, imgs, True, (h, w), stride, tables, outs),
                               reps=3)
    alg = px * (2 + 16 + 1) + sum(o[1].numel() * 24 for o in outs)   # image, S+Q, rows read, outputs
    res = {"workload": "%d uint16 log-normal images (mu 6, sigma 1), sides uniform on 1000..12000 (seed 3); "
                       "tables of pixels and squares; 64x64 windows at stride 4: sum, mean, std" % n_images,
           "images": n_images, "gpix": round(px / 1e9, 4),
           "per_image_calls_ms": round(t_per, 3), "per_image_gpix_s": round(px / t_per / 1e6, 2),
           "batched_ms": round(t_bat, 3), "batched_gpix_s": round(px / t_bat / 1e6, 2),
           "fused_ms": round(t_fused, 3), "fused_gpix_s": round(px / t_fused / 1e6, 2),
           "fused_alg_GB_s": round(alg / (t_fused * 1e-3) / 1e9, 1),
           "tuned": {"build": choice["build"], "gather": choice["gather"], "strip_h": choice["strip_h"],
                     "one_launch": choice["fused"], "candidates_ms": {"strip_h": choice["strip_ms"],
                                                                       "launches": choice["fused_ms"]},
                     "ms": round(t_tuned, 3),
                     "gpix_s": round(px / t_tuned / 1e6, 2), "tuning_s": round(tune_s, 2)},
           "speedup_batched_vs_per_image": round(t_per / t_bat, 3),
           "speedup_tuned_vs_per_image": round(t_per / t_tuned, 3),
           "tuned_alg_GB_s": round(alg / (t_tuned * 1e-3) / 1e9, 1)}
    del imgs, tables, outs
    torch.cuda.synchronize()
    return res


def timed_ms(torch, stream, fn, reps):
    """Mean HIP-event time of `fn` on `stream` over `reps` runs after one untimed run."""
    import numpy as np
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.mean(ts))


def meanstd_section(torch, dev, n, reps):
    """An n x n uint16 log-normal image (mu 6, sigma 1): tables of pixels and squares, then the
    sum, mean and std of every 64 x 64 window at stride 1.  Algorithmic bytes: image + S + Q for
    the build (18 B/px); S and Q read once and 24 B per output for the statistics."""
    from paper_2410_16291_amd import api, synth
    h = 64
    img = api.empty_image(n, n, torch.uint16, dev)
    img.copy_(synth.lognormal_u16_device(n, n, 1, dev))
    S = api.empty_table(n, n, dev)
    Q = api.empty_table(n, n, dev, S.stride(0))
    ws = torch.empty(api.build_workspace_bytes(n, n, 2, True), dtype=torch.uint8, device=dev)
    oh, ow = api.out_shape(n, n, h, h, 1)
    outs = (api.empty_out(oh, ow, torch.uint64, dev), api.empty_out(oh, ow, torch.float64, dev),
            api.empty_out(oh, ow, torch.float64, dev))
    stream = torch.cuda.current_stream(dev)
    t_build = timed_ms(torch, stream, lambda: api.sat_build(img, sat=S, sat_sq=Q, ws=ws), reps)
    api.workspace_check(ws)
    t_stats = timed_ms(torch, stream, lambda: api.window_mean_std(S, Q, h, h, 1, outs=outs), reps)
    alg_b = n * n * 18
    alg_g = n * n * 16 + oh * ow * 24
    res = {"workload": "%dx%d uint16 log-normal intensities (mu 6, sigma 1, seed 1); tables of pixels and squares; "
                       "sum, mean and std of every %dx%d window at stride 1" % (n, n, h, h),
           "build_ms": round(t_build, 4), "build_GB_s": round(alg_b / (t_build * 1e-3) / 1e9, 1),
           "build_frac_hbm_peak": round(alg_b / (t_build * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "mean_std_ms": round(t_stats, 4), "mean_std_GB_s": round(alg_g / (t_stats * 1e-3) / 1e9, 1),
           "mean_std_frac_hbm_peak": round(alg_g / (t_stats * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "gpix_s": round(n * n / ((t_build + t_stats) * 1e-3) / 1e9, 2)}
    del img, S, Q, ws, outs
    torch.cuda.empty_cache()
    return res


def moments_section(torch, dev, n, reps):
    """Tables of pixel^1..pixel^4 of an n x n 8-bit intensity image in one pass, then the mean, std,
    skewness and excess kurtosis of every 64 x 64 window at stride 1 (HIP events on the launch
    stream, inputs resident).  Algorithmic bytes: the image and four tables for the build
    (1 + 32 B/px); four tables read once and four float64 outputs for the gather."""
    from paper_2410_16291_amd import api, synth
    h = 64
    img = api.empty_image(n, n, torch.uint8, dev)
    img.copy_(synth.lognormal_u16_device(n, n, 5, dev, mu=4.0, sigma=0.9).view(torch.int16).clamp_(0, 255).to(torch.uint8))
    first = api.empty_table(n, n, dev)
    tables = [first] + [api.empty_table(n, n, dev, first.stride(0)) for _ in range(3)]
    ws = torch.empty(api.powers_workspace_bytes(n, n, 1, 4), dtype=torch.uint8, device=dev)
    oh, ow = api.out_shape(n, n, h, h, 1)
    outs = {k: api.empty_out(oh, ow, torch.float64, dev) for k in api.MOMENTS}
    stream = torch.cuda.current_stream(dev)
    t_build = timed_ms(torch, stream, lambda: api.sat_build_powers(img, 4, tables=tables, ws=ws), reps)
    api.workspace_check(ws)
    t_gather = timed_ms(torch, stream, lambda: api.window_moments(tables, h, h, 1, pixel_type="u8", outs=outs), reps)
    alg_b = n * n * (1 + 32)
    alg_g = n * n * 32 + oh * ow * 32
    res = {"workload": "%dx%d uint8 log-normal intensities (mu 4, sigma 0.9, seed 5, clipped to 255); tables of "
                       "pixel^1..pixel^4; mean, std, skewness, excess kurtosis of every %dx%d window at stride 1"
                       % (n, n, h, h),
           "build_powers_ms": round(t_build, 4), "build_alg_GB": round(alg_b / 1e9, 3),
           "build_GB_s": round(alg_b / (t_build * 1e-3) / 1e9, 1),
           "build_frac_hbm_peak": round(alg_b / (t_build * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "moments_ms": round(t_gather, 4), "moments_alg_GB": round(alg_g / 1e9, 3),
           "moments_GB_s": round(alg_g / (t_gather * 1e-3) / 1e9, 1),
           "moments_frac_hbm_peak": round(alg_g / (t_gather * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "gpix_s": round(n * n / ((t_build + t_gather) * 1e-3) / 1e9, 2)}
    del img, tables, ws, outs
    torch.cuda.empty_cache()
    return res


def serving_section(torch, dev, seconds, burst_seconds):
    """Poisson request streams against resident tables: the nominal 50 req/s mix, and a burst at
    500 req/s served with 4 slots (continuous batching) and with 1 slot (one request at a time)."""
    from paper_2410_16291_amd import serve, synth

    def run(rate, duration, slots):
        reqs = synth.request_stream(rate=rate, duration=duration, seed=4)
        ex = serve.GpuExecutor(dev, slots)
        srv = serve.Server(ex, budget_bytes=200e9, slots=slots)
        rep = srv.run(reqs, idle=lambda: time.sleep(2e-5))
        torch.cuda.synchronize()
        ex.close()
        del srv, ex
        torch.cuda.empty_cache()
        return rep.as_dict()

    # No warm-up run: the first requests of the stream pay the first launch of each kernel.
    out = {"workload": "Poisson arrivals; 20% builds of uint8 Thomas-cluster masks with sides uniform on "
                       "2000..16000, uploaded by a copy kernel from pinned host buffers a producer thread "
                       "fills ahead of arrival (H2D timed apart from the build), 80% window queries (sides "
                       "16..512, strides 1..8, 25% mean/std) on resident tables; tables, images and outputs "
                       "placed in one 200 GB device arena allocated before the stream; seed 4",
           "nominal_50_per_s": dict(run(50.0, seconds, 4), rate=50.0, slots=4)}
    if burst_seconds > 0:
        out["burst_500_per_s_4_slots"] = dict(run(500.0, burst_seconds, 4), rate=500.0, slots=4)
        out["burst_500_per_s_1_slot"] = dict(run(500.0, burst_seconds, 1), rate=500.0, slots=1)
    return out


def banded_section(torch, dev, H, W, band_rows):
    """The same window sums computed band by band, the table never materialised: the image
    streamed from pinned host memory (PCIe included) and from device memory.  Then the whole table
    built in HBM as the image streams in from pinned host memory."""
    from paper_2410_16291_amd import api, banded, synth

    mask = synth.thomas_mask(H, W, seed=2)
    host = torch.empty((H, W), dtype=torch.uint8, pin_memory=True)
    host.numpy()[...] = mask
    del mask
    wins = [(h, h) for h in WINDOWS]
    res = {"workload": "the %dx%d mask above in bands of %d rows, each band's table rows built from the "
                       "column totals of the rows above, the last 500 table rows carried to the next band "
                       "on the device; windows 100/250/500 at stride 1; outputs left on the device; "
                       "from_device: the image resident in HBM on 128-byte row lines, built in place"
                       % (H, W, band_rows),
           "band_rows": band_rows}
    for name, src in (("from_pinned_host", host), ("from_device", None)):
        if src is None:
            src = api.empty_image(H, W, torch.uint8, dev)
            src.copy_(host)
        job = banded.BandedWindowSums(H, W, wins, 1, "u8", band_rows, dev)
        job.run(lambda r0, r1: src[r0:r1], lambda i, k0, rows: None)        # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        job.run(lambda r0, r1: src[r0:r1], lambda i, k0, rows: None)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[name] = {"ms": round(dt * 1e3, 2), "gpix_s": round(H * W / dt / 1e9, 2), "bands": len(job.plan),
                     "device_GB": round((sum(t.untyped_storage().nbytes() for t in (job.up.dimg if job.up else []))
                                         + sum(t.untyped_storage().nbytes() for t in job.tables)) / 1e9, 2)}
        del job, src
        torch.cuda.empty_cache()
    # the whole table in HBM, built band by band as the image streams in (no overlap rows: each
    # band starts from the column totals of the rows above)
    S = api.empty_table(H, W, dev)
    banded.build_table_streamed(lambda r0, r1: host[r0:r1], H, W, "u8", band_rows=band_rows, device=dev, sat=S)
    t0 = time.perf_counter()
    banded.build_table_streamed(lambda r0, r1: host[r0:r1], H, W, "u8", band_rows=band_rows, device=dev, sat=S)
    dt = time.perf_counter() - t0
    res["table_from_pinned_host"] = {"ms": round(dt * 1e3, 2), "gpix_s": round(H * W / dt / 1e9, 2)}
    del S, host
    torch.cuda.empty_cache()
    return res


def shard_section(torch, dev, H, W, shards, reps):
    """One GPU's share of the image split by rows over `shards` GPUs, at its real shape: the
    column totals of its rows (what it would contribute to the exchange of totals), then its band
    build seeded with the totals of the rows above (what the exchange would return), next to the
    plain build of the same rows.  A middle shard of the bench mask; HIP events on the launch
    stream, inputs resident.  Algorithmic bytes: the shard's image for the totals, its image and
    table for the builds (plus the W-word vectors)."""
    from paper_2410_16291_amd import api, synth

    rows = H // shards
    k = shards // 2
    r0, r1 = k * rows, (k + 1) * rows
    ys, xs = synth.thomas_points(H, W, seed=2)
    img = api.empty_image(H, W, torch.uint8, dev)
    img[torch.from_numpy(ys).to(dev), torch.from_numpy(xs).to(dev)] = 1
    carry = api.column_totals(img[:r0])
    band = img[r0:r1]
    S = api.empty_table(rows, W, dev)
    T = api.empty_totals(W, dev)
    own = api.empty_totals(W, dev)
    ws = torch.empty(api.build_workspace_bytes(rows, W, 1, False), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    t_tot = timed_ms(torch, stream, lambda: api.column_totals(band, out=own), reps)
    t_band = timed_ms(torch, stream, lambda: api.sat_build_band(band, carry=carry, rows_above=r0, sat=S, total=T,
                                                                ws=ws), reps)
    api.workspace_check(ws)
    t_plain = timed_ms(torch, stream, lambda: api.sat_build(band, sat=S, ws=ws), reps)
    px = rows * W
    alg_tot = px + 16 * W
    alg_band = 9 * px + 16 * W
    res = {"workload": "rows %d..%d of the %dx%d mask above (one of %d row shards), 128-byte row pitch"
                       % (r0, r1 - 1, H, W, shards),
           "column_totals_ms": round(t_tot, 4), "column_totals_GB_s": round(alg_tot / (t_tot * 1e-3) / 1e9, 1),
           "column_totals_frac_hbm_peak": round(alg_tot / (t_tot * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "band_build_ms": round(t_band, 4), "band_build_GB_s": round(alg_band / (t_band * 1e-3) / 1e9, 1),
           "band_build_frac_hbm_peak": round(alg_band / (t_band * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "plain_build_ms": round(t_plain, 4),
           "share_gpix_s": round(px / ((t_tot + t_band) * 1e-3) / 1e9, 2)}
    del img, band, carry, S, T, own, ws
    torch.cuda.empty_cache()
    return res


def calibrate_copy(torch, dev):
    """Plain copies of known size for the counter scale: 1 GiB read and 1 GiB written each."""
    n = 1 << 27
    a = torch.ones(n, dtype=torch.int64, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)                                   # contiguous: the runtime's copy kernel
    cols = 1 << 14
    a2 = torch.ones((n // cols, cols + 16), dtype=torch.int64, device=dev)[:, :cols]
    b2 = torch.empty((n // cols, cols), dtype=torch.int64, device=dev)
    b2.copy_(a2)                                 # row-strided: one 8-byte load per lane
    torch.cuda.synchronize()
    del a, b, a2, b2


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the path has no multi-GPU implementation (it would shard "
              "an image by strips of rows, one per GPU); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2410_16291_amd import api, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    H, W = args.rows, args.cols
    wins = [(h, h) for h in WINDOWS]

    # --- synthetic input, made resident in HBM before any timing
    ys, xs = synth.thomas_points(H, W, seed=2)
    img = api.empty_image(H, W, torch.uint8, dev)          # rows on 128-byte lines, like the table
    img[torch.from_numpy(ys).to(dev), torch.from_numpy(xs).to(dev)] = 1
    S = api.empty_table(H, W, dev)
    ws = torch.empty(api.build_workspace_bytes(H, W, 1, False), dtype=torch.uint8, device=dev)
    outs = [api.empty_out(*api.out_shape(H, W, h, w, 1), torch.uint32, dev) for h, w in wins]
    torch.cuda.synchronize()
    if args.calibrate_copy:
        calibrate_copy(torch, dev)
    stream = torch.cuda.current_stream(dev)

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        return e

    def step(marks=None):
        if marks is not None:
            marks["build"].append(ev())
        api.sat_build(img, sat=S, ws=ws)
        if marks is not None:
            marks["build"].append(ev())
        api.window_sum_multi(S, wins, 1, pixel_type="u8", outs=outs)
        if marks is not None:
            marks["gather"].append(ev())

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    api.workspace_check(ws)

    # --- timed region: exactly K steps; events around every launch on the launch stream
    marks = {"build": [], "gather": []}
    torch.cuda.synchronize()
    t0 = ev()
    for _ in range(args.steps):
        step(marks)
    t1 = ev()
    torch.cuda.synchronize()
    total_ms = t0.elapsed_time(t1)
    api.workspace_check(ws)
    b = marks["build"]
    build_ms = float(np.mean([b[2 * i].elapsed_time(b[2 * i + 1]) for i in range(args.steps)]))
    gather_ms = float(np.mean([b[2 * i + 1].elapsed_time(marks["gather"][i]) for i in range(args.steps)]))

    ms_step = total_ms / args.steps
    value = H * W / (ms_step * 1e-3) / 1e9
    alg = {"sat_build": alg_bytes_build(H, W), "window_sum_multi": alg_bytes_windows(H, W, WINDOWS)}
    per = {"sat_build": build_ms, "window_sum_multi": gather_ms}
    kernels = {k: {"ms": round(per[k], 4), "alg_GB": round(alg[k] / 1e9, 3),
                   "GB_s": round(alg[k] / (per[k] * 1e-3) / 1e9, 1),
                   "frac_hbm_peak": round(alg[k] / (per[k] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)} for k in per}
    dom = max(per, key=lambda k: per[k])
    achieved = alg[dom] / (per[dom] * 1e-3) / 1e9
    traffic = committed_traffic(H, W) if dom == "window_sum_multi" else None

    # --- context: the same window sums as one call per window size (not part of the step)
    separate = None
    if not args.no_separate:
        separate = {}
        for (h, w), o in zip(wins, outs):
            api.window_sum(S, h, w, 1, pixel_type="u8", out=o)
            ts = []
            for _ in range(3):
                a = ev()
                api.window_sum(S, h, w, 1, pixel_type="u8", out=o)
                ts.append((a, ev()))
            torch.cuda.synchronize()
            separate["window_sum_%dx%d" % (h, w)] = round(float(np.mean([x.elapsed_time(y) for x, y in ts])), 4)

    res = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gpix/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "%dx%d uint8 Thomas-cluster centroid mask (parent density 2e-6/px, 200 "
                               "children, sigma 40 px, seed 2); uint64 integral image; sums of every "
                               "100x100, 250x250 and 500x500 window at stride 1 from one table in one "
                               "pass, uint32 outputs" % (H, W), "rows": H, "cols": W,
                   "windows": list(WINDOWS), "stride": 1,
                   "row_pitch_bytes": {"image": img.stride(0) * img.element_size(),
                                       "table": S.stride(0) * 8, "outputs": outs[0].stride(0) * 4}},
        "hbm_frac_step": round(sum(alg.values()) / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "step_alg_GB": round(sum(alg.values()) / 1e9, 3),
        "kernels": kernels,
        "separate_window_calls_ms": separate,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic / 1e9, 3),
                     "traffic_unit": "GB per launch (HBM reads + writes)"},
    }
    del img, S, ws, outs
    torch.cuda.empty_cache()
    if not args.no_batched:
        res["batched"] = batched_section(torch, dev, args.batch_images)
    if not args.no_banded:
        res["banded"] = banded_section(torch, dev, H, W, args.band_rows)
    if not args.no_shard:
        res["row_shard"] = shard_section(torch, dev, H, W, 8, 10)
    if not args.no_meanstd:
        res["mean_std_8192"] = meanstd_section(torch, dev, 8192, 10)
    if not args.no_moments:
        res["moments"] = moments_section(torch, dev, args.moments_size, 5)
    if not args.no_serve:
        torch.cuda.empty_cache()
        res["serving"] = serving_section(torch, dev, args.serve_seconds, args.burst_seconds)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(H, W, args.cpu_seconds)
    line = json.dumps(res)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(line + "\n")
    print(line, flush=True)


if __name__ == "__main__":
    main()
