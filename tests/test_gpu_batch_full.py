"""The batched workload at its full size, element by element against the oracle: 64 uint16
log-normal images with sides uniform on 1000..12000 (about 2.5 Gpx), tables of pixels and squares
in one persistent build launch, then the sum, mean and std of every 64 x 64 window at stride 4 in
one launch -- with the library's built-in kernel choice, the autotuner's choice, and the fastest
build and gather variants the tuner timed after its choice -- and tables and statistics fused in
one launch (sat_build_stats_batched).  Every
table entry and every output of every image is compared; images are checked in parallel, one
image per worker at a time, to bound host memory."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
from paper_2410_16291_amd import api, autotune, batch, synth
from gpu_util import to_host

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

STD_RTOL = 1e-12
H_WIN = W_WIN = 64
STRIDE = 4


def check_std(got, ref, what):
    zero = ref == 0
    assert np.all(got[zero] == 0.0), what
    rel = np.abs(got[~zero] - ref[~zero]) / ref[~zero]
    assert rel.size == 0 or rel.max() <= STD_RTOL, (what, float(rel.max()))


def workers():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(8, n))


def test_batched_64_images_every_output_default_and_tuned(capsys):
    def say(msg):
        with capsys.disabled():
            print("batched 64: " + msg, flush=True)

    dev = torch.device("cuda:0")
    sizes = synth.uneven_sizes(64, 1000, 12000, seed=3)
    imgs = [synth.lognormal_u16_device(H, W, 3000 + i, dev) for i, (H, W) in enumerate(sizes)]
    say("%d images, %.2f Gpx" % (len(imgs), sum(H * W for H, W in sizes) / 1e9))

    # the library's own choice
    runs = {}
    t = batch.build_batched(imgs, True)
    runs["default"] = (t, batch.mean_std_batched(t, H_WIN, W_WIN, STRIDE))
    torch.cuda.synchronize()

    # the tuner's choice, and the fastest build and gather variants after it
    choice = autotune.Tuner(path=None, reps=1).tune_batch(imgs, squares=True, win=(H_WIN, W_WIN), stride=STRIDE)
    second = {}
    for kind in ("build", "gather"):
        others = {k: v for k, v in choice[kind + "_ms"].items() if k != choice[kind]}
        second[kind] = min(others, key=others.get) if others else choice[kind]
    for name, (bv, gv) in (("tuned", (choice["build"], choice["gather"])),
                           ("runner-up", (second["build"], second["gather"]))):
        say("%s: build %s, gather %s" % (name, bv, gv))
        t = batch.build_batched(imgs, True, variant=bv)
        runs[name] = (t, batch.mean_std_batched(t, H_WIN, W_WIN, STRIDE, variant=gv))
        torch.cuda.synchronize()
    say("fused: tables and statistics in one launch")
    runs["fused"] = batch.build_stats_batched(imgs, H_WIN, W_WIN, STRIDE)
    torch.cuda.synchronize()
    api.workspace_check(api.workspace(0, dev))
    for name, (tables, _) in runs.items():
        for i, (S, Q) in enumerate(tables):
            assert tuple(S.shape) == sizes[i] and tuple(Q.shape) == sizes[i], (name, i)

    def one(i):
        img_np = to_host(imgs[i])
        ref_S, ref_Q = oracle.sat(img_np, squares=True)
        sums = oracle.window_sum_sat(ref_S, H_WIN, W_WIN, STRIDE)
        ref_mean, ref_std = oracle.mean_std(sums, oracle.window_sum_sat(ref_Q, H_WIN, W_WIN, STRIDE), H_WIN * W_WIN)
        for name, (tables, outs) in runs.items():
            S, Q = tables[i]
            assert np.array_equal(to_host(S), ref_S), (name, i, "S")
            assert np.array_equal(to_host(Q), ref_Q), (name, i, "Q")
            s1, mean, std = outs[i]
            assert np.array_equal(to_host(s1), sums), (name, i, "sum")
            assert np.array_equal(to_host(mean), ref_mean), (name, i, "mean")
            check_std(to_host(std), ref_std, (name, i, "std"))
        return sizes[i][0] * sizes[i][1]

    done = 0
    with ThreadPoolExecutor(workers()) as ex:
        for k, px in enumerate(ex.map(one, range(len(imgs)))):
            done += px
            if k % 16 == 15:
                say("%d images compared (%.2f Gpx)" % (k + 1, done / 1e9))
    say("every table entry and output of every run equals the oracle")
