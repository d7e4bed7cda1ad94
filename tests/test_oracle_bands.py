"""Pins for the oracle's column totals and for the band reading of the integral image.

The band build computes row r0 + y of a taller image's table from the band's rows and the column
totals of the rows above it (Sec. II-B: the table is a prefix sum down the columns of row-wise
prefix sums).  Its expected values in the GPU tests are rows of the whole image's oracle table; the
totals output is compared with oracle.column_totals, pinned here against brute force, against the
oracle's table by a separate route (differences of its last row), and against numpy sums.  The
identity the band build rests on is checked here on the oracle alone.
"""
import numpy as np
import pytest

import oracle


def rand_img(rng, H, W, dtype=np.uint8):
    return rng.integers(0, 256 if dtype == np.uint8 else 65536, (H, W)).astype(dtype)


def test_column_totals_brute_force():
    rng = np.random.default_rng(3)
    img = rand_img(rng, 7, 5)
    carry = rng.integers(0, 1 << 40, 5).astype(np.uint64)
    carry_sq = rng.integers(0, 1 << 40, 5).astype(np.uint64)
    T, T2 = oracle.column_totals(img, squares=True, carry=carry, carry_sq=carry_sq)
    for x in range(5):
        assert int(T[x]) == int(carry[x]) + sum(int(img[y, x]) for y in range(7))
        assert int(T2[x]) == int(carry_sq[x]) + sum(int(img[y, x]) ** 2 for y in range(7))


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_column_totals_are_differences_of_the_last_table_row(dtype):
    """The table's last row is the running sum along x of the column totals."""
    rng = np.random.default_rng(4)
    img = rand_img(rng, 300, 257, dtype)
    S, Q = oracle.sat(img, squares=True)
    T, T2 = oracle.column_totals(img, squares=True)
    assert np.array_equal(np.diff(S[-1], prepend=np.uint64(0)), T)
    assert np.array_equal(np.diff(Q[-1], prepend=np.uint64(0)), T2)
    assert np.array_equal(T, img.astype(np.uint64).sum(axis=0))


def test_column_totals_padded_pitch_and_wrap():
    rng = np.random.default_rng(5)
    base = rand_img(rng, 40, 70, np.uint16)
    img = base[:, 3:61]                              # a pitched view
    carry = np.full(58, np.iinfo(np.uint64).max, np.uint64)   # wraps mod 2^64
    T = oracle.column_totals(img, carry=carry)
    ref = (img.astype(np.uint64).sum(axis=0) - np.uint64(1))  # carry = -1 mod 2^64
    assert np.array_equal(T, ref)


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_band_rows_follow_from_the_band_and_the_totals_above(dtype):
    """Row r0 + y of the whole table = table of the band + running sum along x of the totals of
    the rows above; the totals chain band by band."""
    rng = np.random.default_rng(6)
    img = rand_img(rng, 211, 97, dtype)
    S, Q = oracle.sat(img, squares=True)
    carry = carry_sq = None
    r0 = 0
    for r1 in (1, 64, 65, 150, 211):
        band = img[r0:r1]
        Sb, Qb = oracle.sat(band, squares=True)
        above = np.zeros(97, np.uint64) if carry is None else np.cumsum(carry, dtype=np.uint64)
        above_sq = np.zeros(97, np.uint64) if carry_sq is None else np.cumsum(carry_sq, dtype=np.uint64)
        assert np.array_equal(Sb + above[None, :], S[r0:r1])
        assert np.array_equal(Qb + above_sq[None, :], Q[r0:r1])
        carry, carry_sq = oracle.column_totals(band, squares=True, carry=carry, carry_sq=carry_sq)
        r0 = r1
    T, T2 = oracle.column_totals(img, squares=True)
    assert np.array_equal(carry, T) and np.array_equal(carry_sq, T2)


def test_column_totals_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.column_totals(np.zeros((3, 4), np.uint8), carry=np.zeros(3, np.uint64))
    with pytest.raises(ValueError):
        oracle.column_totals(np.zeros((3, 4), np.int32))
