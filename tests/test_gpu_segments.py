"""Helper-wave builds with each strip split into column segments, against the oracle's tables.

A segment that starts mid-row takes its rows' totals left of it, and the table value above its
strip at the column left of it, from a pre-pass over the image (the table's column at each
segment boundary).  Segment counts are forced (sat_force_variant kind 4) over 8- and 16-bit
images with and without squares, ragged widths and heights (a short last strip, a short last
segment), both helper pipelines, rows that allow no 16-byte loads (the pre-pass's scalar path),
and band builds seeded by the column totals of the rows above (the carry's part of each boundary
column).  Tables must be bit-exact; every build's fault word must be clear.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2410_16291_amd import api
from paper_2410_16291_amd.autotune import forced, forced_segments
from gpu_util import to_device, to_host

pytestmark = pytest.mark.gpu

CASES = [
    # (H, W, dtype, squares, segment counts)
    (300, 5000, np.uint8, False, [2, 3, 5, 8]),          # three-stage helper, 8 px/lane
    (777, 4099, np.uint16, True, [2, 4, 7]),             # 16-bit with squares, ragged rows and columns
    (130, 40000, np.uint8, False, [3, 8]),               # wider than 32768: two-stage helper
    (1000, 3000, np.uint8, True, [2, 6]),
    (65, 2600, np.uint16, False, [4]),                   # 16-bit, 32-bit lookback words, short strip
]


def aligned(img_np, dtype):
    tdt = torch.uint8 if dtype == np.uint8 else torch.uint16
    H, W = img_np.shape
    img = api.empty_image(H, W, tdt, "cuda:0")          # rows on 128-byte lines: the helper plans
    img.copy_(to_device(img_np))
    return img


def check(res, ref, squares, tag):
    if squares:
        assert np.array_equal(to_host(res[0]), ref[0]), tag
        assert np.array_equal(to_host(res[1]), ref[1]), tag
    else:
        assert np.array_equal(to_host(res), ref), tag


@pytest.mark.parametrize("H,W,dtype,squares,nsegs", CASES,
                         ids=["%dx%d-%s%s" % (c[0], c[1], np.dtype(c[2]).name, "-sq" if c[3] else "") for c in CASES])
def test_segmented_build_matches_oracle(H, W, dtype, squares, nsegs):
    rng = np.random.default_rng(H * 7 + W)
    hi = 256 if dtype == np.uint8 else 65536
    img_np = rng.integers(0, hi, (H, W)).astype(dtype)
    img = aligned(img_np, dtype)
    ref = oracle.sat(img_np, squares=squares)
    ws = torch.empty(api.build_workspace_bytes(H, W, np.dtype(dtype).itemsize, squares), dtype=torch.uint8,
                     device="cuda:0")
    for n in nsegs:
        print("case: segmented build", H, W, np.dtype(dtype).name, squares, n, flush=True)
        with forced_segments(n):
            res = api.sat_build(img, squares=squares, ws=ws)
        api.workspace_check(ws)
        check(res, ref, squares, (H, W, n))


def test_segments_on_rows_without_16_byte_loads():
    """A forced helper variant on an image with an odd row pitch: the pre-pass reads pixel by
    pixel."""
    H, W = 200, 3001
    img_np = np.random.default_rng(5).integers(0, 256, (H, W)).astype(np.uint8)
    img = to_device(img_np)                               # contiguous: pitch 3001 bytes
    ref = oracle.sat(img_np)
    for name in ("helper_nt_px4_rw16_nw4", "helper3_nt_px4_rw16_nw4"):
        for n in (2, 5):
            print("case: segmented build, odd pitch", name, n, flush=True)
            ws = torch.empty(api.build_workspace_bytes(H, W, 1, False), dtype=torch.uint8, device="cuda:0")
            with forced(0, name), forced_segments(n):
                S = api.sat_build(img, ws=ws)
            api.workspace_check(ws)
            assert np.array_equal(to_host(S), ref), (name, n)


@pytest.mark.parametrize("squares", [False, True])
def test_segmented_band_build_with_carry(squares):
    """Rows 400..899 of a 900-row image built as a band from the oracle's column totals of the
    rows above: each boundary column starts from the carry left of it."""
    H, W, r = 900, 4500, 400
    img_np = np.random.default_rng(9).integers(0, 256, (H, W)).astype(np.uint8)
    ref = oracle.sat(img_np, squares=squares)
    tot = oracle.column_totals(img_np[:r], squares=squares)
    band = aligned(img_np[r:], np.uint8)
    carry = to_device(tot[0] if squares else tot)
    carry_sq = to_device(tot[1]) if squares else None
    for n in (2, 3, 8):
        print("case: segmented band build", squares, n, flush=True)
        ws = torch.empty(api.build_workspace_bytes(H - r, W, 1, squares), dtype=torch.uint8, device="cuda:0")
        with forced_segments(n):
            out = api.sat_build_band(band, carry=carry, rows_above=r, squares=squares, carry_sq=carry_sq, ws=ws)
        api.workspace_check(ws)
        if squares:
            S, Q, T, TQ = out
            assert np.array_equal(to_host(S), ref[0][r:]) and np.array_equal(to_host(Q), ref[1][r:]), n
            assert np.array_equal(to_host(T), oracle.column_totals(img_np, squares=True)[0]), n
        else:
            S, T = out
            assert np.array_equal(to_host(S), ref[r:]), n
            assert np.array_equal(to_host(T), oracle.column_totals(img_np)), n
