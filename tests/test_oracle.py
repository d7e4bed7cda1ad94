"""Pins for the C oracle: each check rests on something other than the oracle itself.

  - a hand-worked example (tests/golden/worked_3x4.json) built from the definitions;
  - closed forms of the table for constant and ramp images;
  - library special cases: numpy cumulative sums, numpy sliding-window sums;
  - brute force (the naive per-window summation of Sec. II-A) for every window and stride on
    small random images;
  - identities that hold at any size (last entry is the total, full-image window, translation,
    transpose, 180-degree rotation, stride subsampling, additivity, linearity mod 2^64);
  - mean and std against exact rational arithmetic (fractions / statistics.pvariance).
"""
import json
import math
import os
import statistics
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_img(rng, H, W, dtype=np.uint8, hi=None):
    hi = hi if hi is not None else (256 if dtype == np.uint8 else 65536)
    return rng.integers(0, hi, (H, W)).astype(dtype)


# ---------------------------------------------------------------- hand-worked example

def test_golden_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "worked_3x4.json")))
    img = np.array(g["image"], np.uint8)
    S, Q = oracle.sat(img, squares=True)
    assert S.tolist() == g["sat"]
    assert Q.tolist() == g["sat_sq"]
    for win in g["windows"]:
        out = oracle.window_sum_sat(S, win["h"], win["w"], win["s"])
        assert out.tolist() == win["sum"], win
        direct = oracle.window_sum_direct(img, win["h"], win["w"], win["s"])
        assert direct.tolist() == win["sum"], win
    ms = g["mean_std"]
    sums, mean, std = oracle.window_stats(img, ms["h"], ms["w"], ms["s"])
    k, l = ms["at"]
    assert mean[k, l] == ms["mean"]
    assert std[k, l] == math.sqrt(ms["std_squared_times_4"]) / 2.0


# ---------------------------------------------------------------- table: closed forms, library

@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_sat_matches_cumsum(dtype):
    rng = np.random.default_rng(10)
    for (H, W) in [(1, 1), (1, 37), (29, 1), (17, 23), (64, 65)]:
        img = rand_img(rng, H, W, dtype)
        S, Q = oracle.sat(img, squares=True)
        ref = np.cumsum(np.cumsum(img.astype(np.uint64), 0), 1)
        refq = np.cumsum(np.cumsum(img.astype(np.uint64) ** 2, 0), 1)
        assert np.array_equal(S, ref)
        assert np.array_equal(Q, refq)


def test_sat_closed_forms():
    H, W = 13, 17
    y = np.arange(H, dtype=np.uint64)[:, None]
    x = np.arange(W, dtype=np.uint64)[None, :]
    ones = np.ones((H, W), np.uint8)
    assert np.array_equal(oracle.sat(ones), (y + 1) * (x + 1))
    ramp_x = np.broadcast_to(np.arange(W, dtype=np.uint8)[None, :], (H, W)).copy()
    assert np.array_equal(oracle.sat(ramp_x), (y + 1) * (x * (x + 1) // 2))
    ramp_y = np.broadcast_to(np.arange(H, dtype=np.uint8)[:, None], (H, W)).copy()
    assert np.array_equal(oracle.sat(ramp_y), (x + 1) * (y * (y + 1) // 2))


def test_sat_padded_pitch_and_max_values():
    rng = np.random.default_rng(11)
    base = rand_img(rng, 21, 40, np.uint16)
    view = base[:, 3:30]                       # row pitch 40, width 27, misaligned start
    assert np.array_equal(oracle.sat(view), oracle.sat(np.ascontiguousarray(view)))
    for dtype, m in [(np.uint8, 255), (np.uint16, 65535)]:
        img = np.full((9, 11), m, dtype)
        S, Q = oracle.sat(img, squares=True)
        assert int(S[-1, -1]) == 99 * m
        assert int(Q[-1, -1]) == 99 * m * m


def test_last_entry_is_total():
    rng = np.random.default_rng(12)
    img = rand_img(rng, 77, 91, np.uint16)
    assert int(oracle.sat(img)[-1, -1]) == int(img.astype(np.uint64).sum())


# ---------------------------------------------------------------- window sums

def test_window_sums_match_brute_force_all_windows():
    rng = np.random.default_rng(13)
    img = rand_img(rng, 14, 17, np.uint8)
    S = oracle.sat(img)
    for h in range(1, 15):
        for w in range(1, 18):
            for s in (1, 2, 3, 5, 16):
                a = oracle.window_sum_sat(S, h, w, s)
                b = oracle.window_sum_direct(img, h, w, s)
                assert a.shape == ((14 - h) // s + 1, (17 - w) // s + 1)
                assert np.array_equal(a, b), (h, w, s)


def test_window_sums_match_brute_force_sampled_48():
    rng = np.random.default_rng(14)
    for dtype in (np.uint8, np.uint16):
        img = rand_img(rng, 48, 45, dtype)
        S, Q = oracle.sat(img, squares=True)
        for _ in range(60):
            h, w, s = int(rng.integers(1, 49)), int(rng.integers(1, 46)), int(rng.integers(1, 9))
            assert np.array_equal(oracle.window_sum_sat(S, h, w, s), oracle.window_sum_direct(img, h, w, s))
            assert np.array_equal(oracle.window_sum_sat(Q, h, w, s),
                                  oracle.window_sum_direct(img, h, w, s, squares=True))


def test_window_sums_match_numpy_sliding_window():
    rng = np.random.default_rng(15)
    img = rand_img(rng, 40, 52, np.uint16)
    S = oracle.sat(img)
    for (h, w, s) in [(1, 1, 1), (3, 7, 1), (8, 8, 2), (40, 52, 1), (5, 51, 3), (39, 2, 4)]:
        ref = np.lib.stride_tricks.sliding_window_view(img.astype(np.uint64), (h, w)).sum((-2, -1))[::s, ::s]
        assert np.array_equal(oracle.window_sum_sat(S, h, w, s), ref)


def test_window_shape_and_rejection():
    assert oracle.window_shape(512, 512, 32, 32, 1) == (481, 481)
    assert oracle.window_shape(70000, 85000, 500, 500, 1) == (69501, 84501)
    assert oracle.window_shape(10, 10, 3, 4, 3) == (3, 3)
    assert oracle.window_shape(10, 10, 11, 1, 1) is None
    assert oracle.window_shape(10, 10, 1, 1, 0) is None
    assert oracle.window_shape(10, 10, 0, 1, 1) is None


def test_all_ones_and_full_window():
    img = np.ones((20, 30), np.uint8)
    S = oracle.sat(img)
    assert np.all(oracle.window_sum_sat(S, 4, 7, 1) == 28)
    rng = np.random.default_rng(16)
    img = rand_img(rng, 20, 30, np.uint16)
    full = oracle.window_sum_sat(oracle.sat(img), 20, 30, 1)
    assert full.shape == (1, 1) and int(full[0, 0]) == int(img.astype(np.uint64).sum())


def test_translation_invariance():
    rng = np.random.default_rng(17)
    img = rand_img(rng, 15, 19, np.uint8)
    h, w, s = 4, 5, 2
    base = oracle.window_sum_sat(oracle.sat(img), h, w, s)
    for (a, b) in [(2, 4), (6, 0), (0, 8)]:
        canvas = np.zeros((15 + a + 3, 19 + b + 5), np.uint8)
        canvas[a:a + 15, b:b + 19] = img
        big = oracle.window_sum_sat(oracle.sat(canvas), h, w, s)
        ka, kb = a // s, b // s
        assert np.array_equal(big[ka:ka + base.shape[0], kb:kb + base.shape[1]], base)


def test_transpose_and_rotation():
    rng = np.random.default_rng(18)
    img = rand_img(rng, 23, 31, np.uint16)
    h, w = 5, 9
    out = oracle.window_sum_sat(oracle.sat(img), h, w, 1)
    out_t = oracle.window_sum_sat(oracle.sat(np.ascontiguousarray(img.T)), w, h, 1)
    assert np.array_equal(out_t, out.T)
    out_r = oracle.window_sum_sat(oracle.sat(np.ascontiguousarray(img[::-1, ::-1])), h, w, 1)
    assert np.array_equal(out_r, out[::-1, ::-1])


def test_stride_subsamples_stride_one():
    rng = np.random.default_rng(19)
    img = rand_img(rng, 33, 41, np.uint8)
    S = oracle.sat(img)
    one = oracle.window_sum_sat(S, 6, 4, 1)
    for s in (2, 3, 7):
        assert np.array_equal(oracle.window_sum_sat(S, 6, 4, s), one[::s, ::s])


def test_additivity():
    rng = np.random.default_rng(20)
    img = rand_img(rng, 25, 40, np.uint16)
    S = oracle.sat(img)
    h, w1, w2 = 6, 5, 9
    a = oracle.window_sum_sat(S, h, w1, 1)
    b = oracle.window_sum_sat(S, h, w2, 1)
    c = oracle.window_sum_sat(S, h, w1 + w2, 1)
    assert np.array_equal(a[:, :c.shape[1]] + b[:, w1:w1 + c.shape[1]], c)
    h1, h2 = 4, 7
    a = oracle.window_sum_sat(S, h1, w1, 1)
    b = oracle.window_sum_sat(S, h2, w1, 1)
    c = oracle.window_sum_sat(S, h1 + h2, w1, 1)
    assert np.array_equal(a[:c.shape[0]] + b[h1:h1 + c.shape[0]], c)


def test_linearity_and_wraparound_mod_2_64():
    rng = np.random.default_rng(21)
    i1 = rand_img(rng, 17, 22, np.uint8)
    i2 = rand_img(rng, 17, 22, np.uint8)
    both = (i1.astype(np.uint16) + i2.astype(np.uint16)).astype(np.uint16)
    assert np.array_equal(oracle.sat(both), oracle.sat(i1) + oracle.sat(i2))
    # Adding the table of a constant image c (c*(y+1)*(x+1)) with c near 2^64 wraps every entry;
    # the corner lookup must still add exactly c*h*w mod 2^64 to each window.
    S = oracle.sat(i1)
    y = np.arange(17, dtype=np.uint64)[:, None]
    x = np.arange(22, dtype=np.uint64)[None, :]
    c = np.uint64((1 << 64) - 977)
    with np.errstate(over="ignore"):
        shifted = S + c * (y + 1) * (x + 1)
        expect = oracle.window_sum_sat(S, 5, 6, 2) + c * np.uint64(30)
    assert np.array_equal(oracle.window_sum_sat(shifted, 5, 6, 2), expect)


def test_coverage_total_equals_sum_of_outputs():
    rng = np.random.default_rng(22)
    img = rand_img(rng, 37, 29, np.uint16)
    for (h, w, s) in [(1, 1, 1), (5, 4, 1), (9, 9, 3), (37, 29, 1)]:
        out = oracle.window_sum_sat(oracle.sat(img), h, w, s)
        assert oracle.coverage_total(img, h, w, s) == int(out.sum(dtype=np.uint64))


def test_stream_matches_full_tables():
    rng = np.random.default_rng(23)
    img = rand_img(rng, 120, 75, np.uint8)
    S, Q = oracle.sat(img, squares=True)
    windows = [(1, 1), (7, 9), (30, 75), (120, 10)]
    s = 2
    rows = []
    for (h, w) in windows:
        oh, _ = oracle.window_shape(120, 75, h, w, s)
        rows.append(sorted(set([0, oh - 1, oh // 2])))
    sat_rows = [0, 1, 59, 119]
    outs, sat_out, total = oracle.stream(img, windows, s, rows, sat_rows)
    for (h, w), r, o in zip(windows, rows, outs):
        assert np.array_equal(o, oracle.window_sum_sat(S, h, w, s)[r])
    assert np.array_equal(sat_out, S[sat_rows])
    assert total == int(S[-1, -1])
    outs_q, _, total_q = oracle.stream(img, windows[:2], s, rows[:2], squares=True)
    assert np.array_equal(outs_q[1], oracle.window_sum_sat(Q, 7, 9, s)[rows[1]])
    assert total_q == int(Q[-1, -1])


# ---------------------------------------------------------------- mean and std

def test_mean_std_exact_rationals():
    rng = np.random.default_rng(24)
    for dtype in (np.uint8, np.uint16):
        img = rand_img(rng, 9, 11, dtype)
        for (h, w, s) in [(1, 1, 1), (2, 3, 1), (4, 4, 2), (9, 11, 1), (3, 1, 2)]:
            sums, mean, std = oracle.window_stats(img, h, w, s)
            for k in range(sums.shape[0]):
                for l in range(sums.shape[1]):
                    vals = [int(v) for v in img[k * s:k * s + h, l * s:l * s + w].ravel()]
                    assert int(sums[k, l]) == sum(vals)
                    assert mean[k, l] == float(Fraction(sum(vals), len(vals)))   # correctly rounded
                    var = statistics.pvariance(vals)                                # exact Fraction
                    ref = math.sqrt(Fraction(var))
                    assert abs(std[k, l] - ref) <= 4e-16 * max(ref, 1e-300), (h, w, s, k, l)


def test_std_zero_and_binary_windows():
    img = np.full((6, 7), 200, np.uint8)
    _, mean, std = oracle.window_stats(img, 3, 2, 1)
    assert np.all(std == 0.0) and np.all(mean == 200.0)
    rng = np.random.default_rng(25)
    mask = (rng.random((30, 30)) < 0.3).astype(np.uint8)
    h, w = 5, 6
    sums, mean, std = oracle.window_stats(mask, h, w, 1)
    p = sums.astype(np.float64) / (h * w)
    assert np.allclose(std, np.sqrt(p * (1 - p)), rtol=1e-14, atol=0)
    assert np.array_equal(mean, p)


def test_std_large_mean_small_spread():
    # var << mean^2: a naive Q/n - mean^2 in double loses every digit here; the exact numerator
    # does not.  Window {65535 x (n-1), 65534}: var = (n-1)/n^2.
    img = np.full((8, 8), 65535, np.uint16)
    img[3, 4] = 65534
    _, _, std = oracle.window_stats(img, 8, 8, 1)
    n = 64
    assert abs(std[0, 0] - math.sqrt(n - 1) / n) <= 4e-16 * (math.sqrt(n - 1) / n)
