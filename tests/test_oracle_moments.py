"""Pins of the oracle's higher window moments (tables of pixel powers, then skewness and excess
kurtosis from exact power sums), against things other than its own formulas: brute-force power
sums, scipy's moment statistics, the central-moment definition evaluated in exact rationals, and
closed forms of two-valued and symmetric windows."""
import math
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

import oracle


def exact_table(img, k):
    """Inclusive 2-D prefix sum of pixel^k in Python integers, reduced mod 2^64."""
    a = img.astype(object) ** k
    return (np.cumsum(np.cumsum(a, axis=0), axis=1) % (1 << 64)).astype(np.uint64)


@pytest.mark.parametrize("dtype,hi,k_max", [(np.uint8, 256, 4), (np.uint16, 65536, 3)])
def test_power_tables_are_prefix_sums_of_powers(dtype, hi, k_max):
    rng = np.random.default_rng(40)
    img = rng.integers(0, hi, (23, 37)).astype(dtype)
    assert np.array_equal(oracle.sat_power(img, 1), oracle.sat(img))
    assert np.array_equal(oracle.sat_power(img, 2), oracle.sat(img, squares=True)[1])
    for k in range(1, k_max + 1):
        assert np.array_equal(oracle.sat_power(img, k), exact_table(img, k)), k


def test_power_tables_wrap_mod_2_64():
    img = np.full((300, 300), 255, np.uint8)          # total of pixel^4: 9e4 * 255^4 > 2^64
    T = oracle.sat_power(img, 4)
    assert int(T[-1, -1]) == (300 * 300 * 255 ** 4) % (1 << 64)
    # a window sum below 2^64 is still exact by corner differences of the wrapped table
    out = oracle.window_sum_sat(T, 100, 100, 50)
    assert np.all(out == np.uint64(100 * 100 * 255 ** 4))


def test_window_power_sums_by_corner_lookup_match_direct_sums():
    rng = np.random.default_rng(41)
    img = rng.integers(0, 256, (31, 29)).astype(np.uint8)
    sums, _ = oracle.window_moments(img, 6, 5, 3, k=4)
    for (y, x) in [(0, 0), (3, 6), (24, 24)]:
        ref = oracle.window_powers(img, y, x, 6, 5, 4)
        brute = [int((img[y:y + 6, x:x + 5].astype(object) ** j).sum()) for j in range(1, 5)]
        assert ref == brute
        assert [int(s[y // 3, x // 3]) for s in sums] == ref


def test_moments_match_scipy():
    stats = pytest.importorskip("scipy.stats")
    rng = np.random.default_rng(42)
    for dtype, hi, k in [(np.uint8, 256, 4), (np.uint16, 65536, 3)]:
        img = rng.lognormal(3.0, 0.8, (40, 50)).clip(0, hi - 1).astype(dtype)
        h, w, s = 9, 11, 4
        _, (mean, std, skew, kurt) = oracle.window_moments(img, h, w, s, k=k)
        for (a, b) in [(0, 0), (3, 5), (7, 9)]:
            win = img[a * s:a * s + h, b * s:b * s + w].astype(np.float64).ravel()
            assert mean[a, b] == pytest.approx(win.mean(), rel=1e-14)
            assert std[a, b] == pytest.approx(win.std(), rel=1e-12)
            assert skew[a, b] == pytest.approx(stats.skew(win, bias=True), rel=1e-9, abs=1e-12)
            if k == 4:
                assert kurt[a, b] == pytest.approx(stats.kurtosis(win, fisher=True, bias=True), rel=1e-9, abs=1e-12)


def central_moments_exact(values):
    """m2, m3, m4 (population) by their definition, in exact rationals."""
    n = len(values)
    mu = Fraction(sum(values), n)
    m = [sum((Fraction(v) - mu) ** j for v in values) / n for j in (2, 3, 4)]
    return m


def test_moments_match_the_central_definition_in_exact_arithmetic():
    getcontext().prec = 60
    rng = np.random.default_rng(43)
    img = rng.integers(0, 256, (12, 12)).astype(np.uint8)
    img[2:6, 2:6] = rng.integers(200, 256, (4, 4))          # a bright cluster: skewed windows
    _, (mean, std, skew, kurt) = oracle.window_moments(img, 5, 4, 1, k=4)
    for (y, x) in [(0, 0), (1, 1), (4, 7), (7, 8)]:
        vals = [int(v) for v in img[y:y + 5, x:x + 4].ravel()]
        m2, m3, m4 = central_moments_exact(vals)
        d2 = Decimal(m2.numerator) / Decimal(m2.denominator)
        d3 = Decimal(m3.numerator) / Decimal(m3.denominator)
        g1 = d3 / (d2 * d2.sqrt())
        g2 = (m4 / (m2 * m2)) - 3
        assert float(skew[y, x]) == pytest.approx(float(g1), rel=1e-14, abs=1e-15)
        assert float(kurt[y, x]) == pytest.approx(float(Decimal(g2.numerator) / Decimal(g2.denominator)),
                                                  rel=1e-14, abs=1e-15)
        assert float(std[y, x]) == pytest.approx(math.sqrt(m2), rel=1e-15)


@pytest.mark.parametrize("ones", [1, 3, 8, 12, 15])
def test_two_valued_windows_follow_the_bernoulli_closed_forms(ones):
    n = 16
    img = np.zeros((4, 4), np.uint8)
    img.ravel()[:ones] = 1
    _, (mean, std, skew, kurt) = oracle.window_moments(img, 4, 4, 1, k=4)
    p = ones / n
    q = 1 - p
    assert mean[0, 0] == pytest.approx(p, rel=1e-15)
    assert std[0, 0] == pytest.approx(math.sqrt(p * q), rel=1e-15)
    assert skew[0, 0] == pytest.approx((1 - 2 * p) / math.sqrt(p * q), rel=1e-14, abs=1e-15)
    assert kurt[0, 0] == pytest.approx((1 - 6 * p * q) / (p * q), rel=1e-14, abs=1e-15)


def test_constant_windows_have_no_shape_and_symmetric_ones_no_skew():
    img = np.full((6, 6), 7, np.uint16)
    _, (mean, std, skew, kurt) = oracle.window_moments(img, 3, 3, 1, k=3)
    assert np.all(mean == 7.0) and np.all(std == 0.0)
    assert np.all(np.isnan(skew)) and kurt is None
    sym = np.array([[10, 20, 30], [20, 30, 40], [30, 40, 50]], np.uint8)   # symmetric about 30
    _, (mean, std, skew, kurt) = oracle.window_moments(sym, 3, 3, 1, k=4)
    assert mean[0, 0] == 30.0 and skew[0, 0] == 0.0
    vals = [int(v) for v in sym.ravel()]
    m2, _, m4 = central_moments_exact(vals)
    assert kurt[0, 0] == pytest.approx(float(m4 / (m2 * m2)) - 3, rel=1e-15)
