"""Band arithmetic of the out-of-core path, on the CPU: every output row is produced by exactly one
band, from a view of table rows that holds the row above its window (or starts at image row 0),
on the view's stride grid, with at most h_max + stride - 1 rows carried from the bands above."""
import itertools

import pytest

from paper_2410_16291_amd.banded import band_outputs, band_plan


@pytest.mark.parametrize("H,h_max,stride,band_rows", [(1, 1, 1, 1), (10, 3, 1, 1), (100, 7, 3, 10), (100, 100, 1, 7),
                                                       (517, 64, 4, 64), (1000, 250, 5, 333), (999, 1, 2, 1000)])
def test_every_output_row_once_and_window_inside_local_rows(H, h_max, stride, band_rows):
    plan = band_plan(H, h_max, stride, band_rows)
    # bands tile [0, H) in order
    assert plan[0][1] == 0 and plan[-1][2] == H
    for (_, _, b1), (_, b0n, _) in zip(plan, plan[1:]):
        assert b1 == b0n
    for r0, b0, b1 in plan:
        assert r0 % stride == 0 and 0 <= r0 <= b0 < b1 <= H
        assert b0 - r0 <= h_max + stride - 1                   # the ring the device keeps
    for h in sorted({1, h_max, max(1, h_max // 2)}):
        oh = (H - h) // stride + 1
        seen = []
        for r0, b0, b1 in plan:
            k0, k1 = band_outputs(r0, b0, b1, H, h, stride)
            for k in range(k0, k1):
                top, last = k * stride, k * stride + h - 1
                assert b0 <= last < b1                          # emitted by the band holding its last row
                assert top == 0 or r0 <= top - 1                # the row above the window is in the view
                assert (top - r0) % stride == 0                 # on the view's stride grid
            seen.extend(range(k0, k1))
        assert seen == list(range(oh))


def test_band_plan_rejects_empty_bands():
    with pytest.raises(ValueError):
        band_plan(10, 3, 1, 0)
