"""The band-by-band comparison harness used by the full-size GPU parity tests, run on the CPU
against numpy's tables and window sums: it must accept them, cover every row once, and report a
single planted difference in a table row, an output row or a deviation."""
import numpy as np
import pytest

import banded_compare


def numpy_reference(img, wins, s):
    v = img.astype(np.uint64)
    table = np.cumsum(np.cumsum(v, axis=0, dtype=np.uint64), axis=1, dtype=np.uint64)
    outs = [np.lib.stride_tricks.sliding_window_view(v, (h, w)).sum(axis=(-2, -1), dtype=np.uint64)[::s, ::s]
            for h, w in wins]
    return table, outs


def numpy_stats(sums, n):
    mean = sums / np.float64(n)
    var = (np.float64(n) * sums.astype(np.float64) - sums.astype(np.float64) ** 2)   # Q = S for 0/1
    return mean, np.sqrt(np.maximum(var, 0.0)) / np.float64(n)


@pytest.mark.parametrize("s", [1, 3])
def test_harness_accepts_numpy_results_and_covers_every_row(s):
    rng = np.random.default_rng(41)
    img = (rng.random((301, 77)) < 0.2).astype(np.uint8)
    wins = [(10, 10), (25, 25), (50, 50)]
    table, outs = numpy_reference(img, wins, s)
    mean, std = numpy_stats(outs[1], 25 * 25)
    counts = banded_compare.compare(
        img, wins, s, table=lambda a, b: table[a:b], out=lambda i, k0, k1: outs[i][k0:k1].astype(np.uint32),
        stats=lambda k0, k1: (mean[k0:k1], std[k0:k1]), stats_window=1, parts=7, band=19, workers=3)
    assert counts["table_rows"] == 301
    assert counts["out_rows"] == [o.shape[0] for o in outs]
    assert counts["stat_rows"] == outs[1].shape[0]


@pytest.mark.parametrize("where", ["table", "out", "std"])
def test_harness_reports_one_planted_difference(where):
    rng = np.random.default_rng(42)
    img = (rng.random((200, 60)) < 0.3).astype(np.uint8)
    wins = [(8, 8), (40, 40)]
    table, outs = numpy_reference(img, wins, 1)
    mean, std = numpy_stats(outs[0], 64)
    if where == "table":
        table[133, 59] += np.uint64(1)
    elif where == "out":
        outs[1][77, 3] -= np.uint64(1)
    else:
        k = int(np.argmax(std[150]))
        std[150, k] *= 1 + 1e-11
    with pytest.raises(AssertionError):
        banded_compare.compare(img, wins, 1, table=lambda a, b: table[a:b], out=lambda i, k0, k1: outs[i][k0:k1],
                               stats=lambda k0, k1: (mean[k0:k1], std[k0:k1]), stats_window=0, parts=4, band=50,
                               workers=2)
