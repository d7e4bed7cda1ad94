"""Seeded generators: deterministic, with the shapes and distributions they promise."""
import numpy as np

from paper_2410_16291_amd import synth


def test_poisson_counts():
    a = synth.poisson_counts(512, 512, 0.05, seed=0)
    b = synth.poisson_counts(512, 512, 0.05, seed=0)
    assert a.dtype == np.uint8 and a.shape == (512, 512)
    assert np.array_equal(a, b)
    assert abs(a.mean() - 0.05) < 0.005
    assert abs((a == 0).mean() - np.exp(-0.05)) < 0.005


def test_lognormal_u16():
    a = synth.lognormal_u16(1000, 1500, seed=1)
    assert a.dtype == np.uint16 and np.array_equal(a, synth.lognormal_u16(1000, 1500, seed=1))
    assert 380 < np.median(a) < 430            # exp(6) = 403
    assert 600 < a.mean() < 730                # exp(6.5) = 665


def test_thomas_mask():
    H, W = 4000, 5000
    m = synth.thomas_mask(H, W, seed=2)
    assert m.dtype == np.uint8 and set(np.unique(m)) <= {0, 1}
    assert np.array_equal(m, synth.thomas_mask(H, W, seed=2))
    ys, xs = synth.thomas_points(H, W, seed=2)
    assert len(ys) <= 200 * 80                 # ~40 parents expected
    assert m.sum() <= len(ys) and m.sum() > 0.9 * len(ys)


def test_uneven_batch_and_requests():
    sizes = synth.uneven_sizes(64, seed=3)
    assert len(sizes) == 64 and all(1000 <= h <= 12000 and 1000 <= w <= 12000 for h, w in sizes)
    imgs = synth.uneven_batch(3, lo=10, hi=40, seed=3)
    assert [i.dtype for i in imgs] == [np.uint16] * 3
    reqs = synth.request_stream(rate=50, duration=10, seed=4)
    assert reqs[0].kind == "build" and 350 < len(reqs) < 650
    assert all(a.t_arrival <= b.t_arrival for a, b in zip(reqs, reqs[1:]))
    assert all(16 <= r.win_h <= 512 and 1 <= r.stride <= 8 for r in reqs if r.kind == "query")
