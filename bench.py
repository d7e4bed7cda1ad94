"""Throughput of the integral-image hot path on one MI355X.

One step = the whole path over one synthetic full-scale image: build the uint64 integral image of
a 70000 x 85000 uint8 cell-centroid mask (Thomas cluster process), then the window sums of
100x100, 250x250 and 500x500 windows at stride 1 from that one table (uint32 outputs).  The
image, the table and the outputs stay resident in HBM; the timed region contains only the
kernels.  Prints ONE JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--rows H --cols W]

`value` is Gpixels/s of image processed per second of whole-step time.  `roofline` reports the
dominant kernel's algorithmic bytes over its measured average duration (HIP events on the
launch stream) against the 8 TB/s HBM peak; `cpu_baseline` times the oracle (serial C, one
core) on a bounded band of the same image and scales it to the same unit.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Gpix/s SAT+window sums at 70k×85k, % HBM peak; served p50/p99 latency"
WINDOWS = (100, 250, 500)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--rows", type=int, default=70000)
    ap.add_argument("--cols", type=int, default=85000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the baseline sample")
    ap.add_argument("--json-out", default=None)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 4 GiB device copy before timing (a known-size kernel for "
                         "scaling rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def alg_bytes_build(H, W):
    """Read the uint8 image once, write the uint64 table once."""
    return H * W * (1 + 8)


def alg_bytes_window(H, W, h, w, out_bytes=4):
    """Every table entry the corner lookups touch, read once, plus every output written once."""
    oh, ow = H - h + 1, W - w + 1
    rows = min(H, (oh - 1) + (H - (h - 1))) if oh > 1 else (2 if h < H else 1)
    cols = min(W, (ow - 1) + (W - (w - 1))) if ow > 1 else (2 if w < W else 1)
    return rows * cols * 8 + oh * ow * out_bytes


def cpu_baseline(H, W, seconds_target):
    """The oracle (serial C) on the first rows of the same image: table + the three windows."""
    import numpy as np

    import oracle
    from paper_2410_16291_amd import synth

    ys, xs = synth.thomas_points(H, W, seed=2)

    def run(R):
        slab = np.zeros((R, W), np.uint8)
        keep = ys < R
        slab[ys[keep], xs[keep]] = 1
        t0 = time.perf_counter()
        S = oracle.sat(slab)
        for h in WINDOWS:
            if h <= R:
                oracle.window_sum_sat(S, h, h, 1)
        return time.perf_counter() - t0

    R = 1024
    t = run(R)
    R2 = int(min(H, max(1024, R * seconds_target / max(t, 1e-3))))
    R2 = max(R2, 2 * max(WINDOWS))
    t2 = run(R2)
    return {"value": round(R2 * W / t2 / 1e9, 5), "unit": "Gpix/s", "cores": 1, "kind": "oracle",
            "sample": "rows 0..%d of the %dx%d image (%.1f Mpx): serial table build + window sums %s "
                      "by corner lookup, uint64, one thread, %.1f s" % (R2 - 1, H, W, R2 * W / 1e6,
                                                                       "/".join(map(str, WINDOWS)), t2)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(how the path would shard is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2410_16291_amd import api, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    H, W = args.rows, args.cols

    # --- synthetic input, made resident in HBM before any timing
    ys, xs = synth.thomas_points(H, W, seed=2)
    img = torch.zeros((H, W), dtype=torch.uint8, device=dev)
    idx = torch.from_numpy(ys * W + xs).to(dev)
    img.view(-1)[idx] = 1
    del idx
    S = api.empty_table(H, W, dev)
    ws = torch.empty(api.build_workspace_bytes(H, W, 1, False), dtype=torch.uint8, device=dev)
    outs = {h: torch.empty(api.out_shape(H, W, h, h, 1), dtype=torch.uint32, device=dev) for h in WINDOWS}
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream(dev)
    if args.calibrate_copy:
        a = torch.ones(4 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    def step(events=None):
        if events is not None:
            events["build"][0].append(torch.cuda.Event(enable_timing=True))
            events["build"][0][-1].record(stream)
        api.sat_build(img, sat=S, ws=ws)
        if events is not None:
            events["build"][1].append(torch.cuda.Event(enable_timing=True))
            events["build"][1][-1].record(stream)
        for h in WINDOWS:
            if events is not None:
                events[h][0].append(torch.cuda.Event(enable_timing=True))
                events[h][0][-1].record(stream)
            api.window_sum(S, h, h, 1, pixel_type="u8", out=outs[h])
            if events is not None:
                events[h][1].append(torch.cuda.Event(enable_timing=True))
                events[h][1][-1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    api.workspace_check(ws)

    # --- timed region: exactly K steps, whole-step clock
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(args.steps):
        step()
    t1.record(stream)
    torch.cuda.synchronize()
    total_ms = t0.elapsed_time(t1)
    api.workspace_check(ws)

    # --- per-kernel durations (a second pass with an event around every call)
    ev = {k: ([], []) for k in ("build",) + WINDOWS}
    for _ in range(args.steps):
        step(ev)
    torch.cuda.synchronize()
    per = {k: float(np.mean([a.elapsed_time(b) for a, b in zip(*ev[k])])) for k in ev}

    ms_step = total_ms / args.steps
    value = H * W / (ms_step * 1e-3) / 1e9
    alg = {"build": alg_bytes_build(H, W)}
    for h in WINDOWS:
        alg[h] = alg_bytes_window(H, W, h, h)
    step_bytes = sum(alg.values())
    kernels = {}
    for k in per:
        name = "sat_build" if k == "build" else "window_sum_%dx%d" % (k, k)
        kernels[name] = {"ms": round(per[k], 4), "alg_GB": round(alg[k] / 1e9, 3),
                         "GB_s": round(alg[k] / (per[k] * 1e-3) / 1e9, 1),
                         "frac_hbm_peak": round(alg[k] / (per[k] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    dom = max(per, key=lambda k: per[k])
    dom_name = "sat_build" if dom == "build" else "window_sum_%dx%d" % (dom, dom)
    achieved = alg[dom] / (per[dom] * 1e-3) / 1e9

    res = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gpix/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "%dx%d uint8 Thomas-cluster centroid mask (parent density 2e-6/px, 200 "
                               "children, sigma 40 px, seed 2); uint64 integral image; window sums "
                               "100x100, 250x250, 500x500 at stride 1 from one table, uint32 outputs"
                               % (H, W), "rows": H, "cols": W, "windows": list(WINDOWS), "stride": 1},
        "hbm_frac_step": round(step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "step_alg_GB": round(step_bytes / 1e9, 3),
        "kernels": kernels,
        "roofline": {"bound": "hbm", "kernel": dom_name, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None},
    }
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(H, W, args.cpu_seconds)
    line = json.dumps(res)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(line + "\n")
    print(line, flush=True)


if __name__ == "__main__":
    main()
