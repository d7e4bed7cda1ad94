"""Pins for the oracle's resumable stream (oracle.Stream), the form the full-size GPU parity tests
use: the table and the window sums computed band by band from any starting row, with the rows
above that row summarised by their column totals (Sec. II-B: a table row is the running sum
along x of the column totals above and at it).

Expected values here come from numpy alone (nested cumulative sums; sums over sliding window
views), not from the oracle's other routines, so a mistake shared by the stream and the
whole-image oracle still fails.
"""
import numpy as np
import pytest

import oracle


def numpy_table(img, squares=False):
    v = img.astype(np.uint64)
    if squares:
        v = v * v
    return np.cumsum(np.cumsum(v, axis=0, dtype=np.uint64), axis=1, dtype=np.uint64)


def numpy_windows(img, h, w, s, squares=False):
    v = img.astype(np.uint64)
    if squares:
        v = v * v
    return np.lib.stride_tricks.sliding_window_view(v, (h, w)).sum(axis=(-2, -1), dtype=np.uint64)[::s, ::s]


def numpy_carry(img, r0, squares=False):
    v = img[:r0].astype(np.uint64)
    if squares:
        v = v * v
    return v.sum(axis=0, dtype=np.uint64)


def run_stream(img, wins, s, r0, stops, squares=False):
    """Advance a stream started at r0 through each row in `stops`; return the table rows and,
    per window, {k: output row}."""
    carry = numpy_carry(img, r0, squares) if r0 > 0 else None
    st = oracle.Stream(img, wins, s, r0=r0, carry=carry, squares=squares)
    rows, outs = [], [dict() for _ in wins]
    for r1 in stops:
        sat, per = st.next(r1)
        rows.append(sat)
        for i, (k0, block) in enumerate(per):
            for j in range(block.shape[0]):
                assert k0 + j not in outs[i]
                outs[i][k0 + j] = block[j]
    st.close()
    return np.concatenate(rows) if rows else None, outs


@pytest.mark.parametrize("dtype,squares", [(np.uint8, False), (np.uint16, False), (np.uint16, True)])
def test_stream_from_any_row_matches_numpy(dtype, squares):
    rng = np.random.default_rng(31)
    H, W = 97, 41
    img = rng.integers(0, 256 if dtype == np.uint8 else 65536, (H, W)).astype(dtype)
    table = numpy_table(img, squares)
    wins = [(1, 1), (7, 5), (20, 41), (33, 2)]
    for s in (1, 2, 5):
        refs = [numpy_windows(img, h, w, s, squares) for h, w in wins]
        for r0 in (0, 1, 2, 6, 19, 20, 21, 50, 96):
            stops = sorted(set([r0, min(H, r0 + 1), min(H, r0 + 13), min(H, r0 + 40), H]))
            sat, outs = run_stream(img, wins, s, r0, stops, squares)
            assert np.array_equal(sat, table[r0:]), (s, r0)
            for (h, w), ref, got in zip(wins, refs, outs):
                ks = [k for k in range(ref.shape[0]) if k * s >= r0]     # windows at or below r0
                assert sorted(got) == ks, (h, w, s, r0)
                for k in ks:
                    assert np.array_equal(got[k], ref[k]), (h, w, s, r0, k)


def test_partition_of_rows_covers_every_output_once():
    """Streams started at the boundaries of a partition of the rows, each run up to the next
    boundary plus the tallest window, emit every table row and every output row; keeping only
    the output rows whose top row lies in a stream's own part gives each exactly once."""
    rng = np.random.default_rng(32)
    H, W = 150, 33
    img = (rng.random((H, W)) < 0.3).astype(np.uint8)
    wins = [(10, 10), (25, 7), (50, 33)]
    hmax = max(h for h, _ in wins)
    table = numpy_table(img)
    for s in (1, 3):
        refs = [numpy_windows(img, h, w, s) for h, w in wins]
        bounds = [0, 1, 37, 38, 90, 149, H]
        got_rows = np.zeros((H, W), np.uint64)
        seen = [dict() for _ in wins]
        for a, b in zip(bounds[:-1], bounds[1:]):
            end = min(H, b + hmax - 1)
            sat, outs = run_stream(img, wins, s, a, sorted(set([a, b, end])))
            got_rows[a:b] = sat[:b - a]
            for i, o in enumerate(outs):
                for k, row in o.items():
                    if a <= k * s < b:
                        assert k not in seen[i]
                        seen[i][k] = row
        assert np.array_equal(got_rows, table)
        for ref, got in zip(refs, seen):
            assert sorted(got) == list(range(ref.shape[0]))
            for k, row in got.items():
                assert np.array_equal(row, ref[k])


def test_stream_wraps_mod_2_64_with_a_large_carry():
    rng = np.random.default_rng(33)
    img = rng.integers(0, 65536, (30, 9)).astype(np.uint16)
    carry = np.full(9, np.iinfo(np.uint64).max - 5, np.uint64)       # totals of rows "above" wrap
    st = oracle.Stream(img, [(4, 3)], 1, r0=10, carry=carry)
    sat, ((k0, out),) = st.next(30)
    st.close()
    above = np.cumsum(carry, dtype=np.uint64)
    local = numpy_table(img[10:])
    assert np.array_equal(sat, local + above[None, :])
    assert k0 == 10 and np.array_equal(out, numpy_windows(img, 4, 3, 1)[10:])


def test_stream_edges_and_rejections():
    img = np.arange(12, dtype=np.uint8).reshape(3, 4)
    st = oracle.Stream(img, [(3, 4)], 1, r0=0)
    sat, ((k0, out),) = st.next(0)                  # nothing yet
    assert sat.shape == (0, 4) and out.shape == (0, 1)
    sat, ((k0, out),) = st.next(3)
    assert k0 == 0 and int(out[0, 0]) == int(img.sum())
    with pytest.raises(ValueError):
        st.next(2)                                  # backwards
    st.close()
    st = oracle.Stream(img, [(1, 1)], 1, r0=3, carry=img.astype(np.uint64).sum(0))
    sat, ((k0, out),) = st.next(3)                  # started at the end: nothing to emit
    assert sat.shape == (0, 4) and out.shape == (0, 4)
    st.close()
    with pytest.raises(ValueError):
        oracle.Stream(img, [(4, 1)], 1)             # window taller than the image
    with pytest.raises(ValueError):
        oracle.Stream(img, [(1, 1)], 1, r0=1)       # rows above but no carry
