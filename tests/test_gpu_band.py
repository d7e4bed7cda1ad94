"""Band builds and column totals: HIP path vs the oracle through the C ABI (needs an MI355X).

A band build of image rows [r0, r1), seeded with the column totals of rows [0, r0), must give rows
r0 .. r1-1 of the whole image's table bit for bit, and the column totals of rows [0, r1).  The
expected tables are rows of the oracle's table of the whole image; the expected totals are the
oracle's column totals.  Covered: every build variant, 8- and 16-bit pixels with squares, bands
of one row up to whole images, carries chained in place, carries at their largest, the fault
word for a carry beyond its bound, streamed whole-image builds from host rows, and the
70000 x 85000 mask as eight row shards of one GPU's size.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2410_16291_amd import api, banded, synth
from paper_2410_16291_amd._lib import SAT_ERR_DEVICE, SatError
from gpu_util import padded_image, to_device, to_host

pytestmark = pytest.mark.gpu


def host_u64(t):
    return to_host(t).astype(np.uint64)


# ------------------------------------------------------------------ column totals

TOTAL_CASES = [
    # (H, W, pitch_extra, offset)
    (1, 1, 0, 0), (3, 1025, 0, 0), (700, 4099, 5, 1), (20000, 300, 0, 0), (64, 1024, 0, 0), (257, 2048, 0, 0),
]


@pytest.mark.parametrize("dtype,hi", [(np.uint8, 256), (np.uint16, 65536)])
@pytest.mark.parametrize("H,W,extra,offset", TOTAL_CASES)
def test_column_totals_match_oracle(dtype, hi, H, W, extra, offset):
    print("case: column totals", np.dtype(dtype).name, H, W, extra, offset, flush=True)
    rng = np.random.default_rng(H * 3 + W)
    img_np = rng.integers(0, hi, (H, W)).astype(dtype)
    img = padded_image(img_np, W + extra, offset) if (extra or offset) else to_device(img_np)
    carry_np = rng.integers(0, 1 << 40, W).astype(np.uint64)
    carry_sq_np = rng.integers(0, 1 << 40, W).astype(np.uint64)
    T, TQ = api.column_totals(img, squares=True, carry=to_device(carry_np), carry_sq=to_device(carry_sq_np))
    ref_T, ref_TQ = oracle.column_totals(img_np, squares=True, carry=carry_np, carry_sq=carry_sq_np)
    assert np.array_equal(host_u64(T), ref_T)
    assert np.array_equal(host_u64(TQ), ref_TQ)
    assert np.array_equal(host_u64(api.column_totals(img)), oracle.column_totals(img_np))
    c = to_device(carry_np)                               # accumulate in place
    api.column_totals(img, carry=c, out=c)
    assert np.array_equal(host_u64(c), oracle.column_totals(img_np, carry=carry_np))


def test_column_totals_pitched_rows_with_a_ragged_tile():
    """16-byte aligned rows (128-byte pitch): whole tiles take 16-byte loads, the last is ragged."""
    for dtype, hi, W in [(np.uint8, 256, 5000), (np.uint16, 65536, 2600)]:
        rng = np.random.default_rng(W)
        img_np = rng.integers(0, hi, (3001, W)).astype(dtype)
        img = api.empty_image(3001, W, torch.uint8 if dtype == np.uint8 else torch.uint16, "cuda:0")
        img.copy_(to_device(img_np))
        T, TQ = api.column_totals(img, squares=True)
        ref_T, ref_TQ = oracle.column_totals(img_np, squares=True)
        assert np.array_equal(host_u64(T), ref_T) and np.array_equal(host_u64(TQ), ref_TQ)


@pytest.mark.parametrize("dtype,value", [(np.uint8, 255), (np.uint16, 65535)])
def test_column_totals_tiles_at_their_row_limit(dtype, value):
    """A 140-million-row column: the totals kernel's tiles reach their 65536-row cap (16384 rows per
    wave), the largest lane sums it forms, here all of the largest pixel value."""
    H = 140_000_000
    print("case: column totals, one column of", H, "rows,", np.dtype(dtype).name, flush=True)
    tdt = torch.uint8 if dtype == np.uint8 else torch.uint16
    img = torch.full((H, 1), value if dtype == np.uint8 else -1, dtype=torch.uint8 if dtype == np.uint8 else
                     torch.int16, device="cuda:0").view(tdt)
    T, TQ = api.column_totals(img, squares=True)
    ref_T, ref_TQ = oracle.column_totals(np.full((H, 1), value, dtype), squares=True)
    assert np.array_equal(host_u64(T), ref_T) and np.array_equal(host_u64(TQ), ref_TQ)
    assert int(ref_T[0]) == value * H and int(ref_TQ[0]) == value * value * H


# ------------------------------------------------------------------ band builds

SPLITS = [0, 1, 97, 500, 1099, 1100]   # bands of 1, 96, 403, 599 and 1 rows of a 1100-row image


def check_bands(img_np, img, squares):
    """Build the image band by band with the totals chained in place; compare every band with
    the rows of the oracle's whole table and the final totals with the oracle's.  The workspace is
    sized per band for the variant the build will use (the forced one, if any)."""
    W = img_np.shape[1]
    bpp = img_np.itemsize
    ref = oracle.sat(img_np, squares=squares)
    ref_S, ref_Q = ref if squares else (ref, None)
    carry = api.empty_totals(W, img.device)
    carry_sq = api.empty_totals(W, img.device) if squares else None
    for r0, r1 in zip(SPLITS[:-1], SPLITS[1:]):
        first = r0 == 0
        ws = torch.empty(api.build_workspace_bytes(r1 - r0, W, bpp, squares), dtype=torch.uint8, device=img.device)
        res = api.sat_build_band(img[r0:r1], carry=None if first else carry, rows_above=r0, squares=squares,
                                 carry_sq=None if first or not squares else carry_sq, total=carry,
                                 total_sq=carry_sq, ws=ws)
        api.workspace_check(ws)
        assert np.array_equal(to_host(res[0]), ref_S[r0:r1]), (r0, r1)
        if squares:
            assert np.array_equal(to_host(res[1]), ref_Q[r0:r1]), (r0, r1)
    ref_T = oracle.column_totals(img_np, squares=squares)
    if squares:
        assert np.array_equal(host_u64(carry), ref_T[0]) and np.array_equal(host_u64(carry_sq), ref_T[1])
    else:
        assert np.array_equal(host_u64(carry), ref_T)


def test_band_build_every_variant():
    """Every build variant: 16-bit pixels with squares (where compiled) and 8-bit pixels on packed
    and on 16-byte aligned rows, 1100 x 2600 in bands of 1 to 599 rows."""
    rng = np.random.default_rng(41)
    img_np = rng.integers(0, 65536, (1100, 2600)).astype(np.uint16)
    img = to_device(img_np)
    img8_np = (img_np >> 8).astype(np.uint8)
    img8s = [to_device(img8_np), padded_image(img8_np, 2608, 0)]
    u16_sq, u8_sq = set(api.variants(0, "u16", True)), set(api.variants(0, "u8", True))
    try:
        for v, name in enumerate(api.variants(0)):
            print("case: band build, variant", name, flush=True)
            api.force_variant(0, v)
            if name in u16_sq:
                check_bands(img_np, img, True)
            for im in img8s:
                check_bands(img8_np, im, name in u8_sq)
    finally:
        api.force_variant(0, -1)


def test_band_build_with_oracle_carry_and_largest_carries():
    """A band seeded with the oracle's totals of the rows above; then carries at the largest value
    their rows_above allows (2^31 - 1 rows of 255, of 255^2): exact against the oracle's band table
    plus the running sum of the carry."""
    rng = np.random.default_rng(42)
    img_np = rng.integers(0, 256, (900, 777)).astype(np.uint8)
    S = oracle.sat(img_np)
    above_np = oracle.column_totals(img_np[:300])
    got, T = api.sat_build_band(to_device(img_np[300:]), carry=to_device(above_np), rows_above=300)
    assert np.array_equal(to_host(got), S[300:])
    assert np.array_equal(host_u64(T), oracle.column_totals(img_np))
    R = (1 << 31) - 1
    carry = np.full(777, R * 255, np.uint64)
    carry_sq = np.full(777, R * 255 * 255, np.uint64)
    band = img_np[:200]
    ws = torch.empty(api.build_workspace_bytes(200, 777, 1, True), dtype=torch.uint8, device="cuda:0")
    Sb, Qb, Tb, TQb = api.sat_build_band(to_device(band), carry=to_device(carry), rows_above=R, squares=True,
                                         carry_sq=to_device(carry_sq), ws=ws)
    api.workspace_check(ws)
    ref_S, ref_Q = oracle.sat(band, squares=True)
    assert np.array_equal(to_host(Sb), ref_S + np.cumsum(carry, dtype=np.uint64)[None, :])
    assert np.array_equal(to_host(Qb), ref_Q + np.cumsum(carry_sq, dtype=np.uint64)[None, :])
    ref_T, ref_TQ = oracle.column_totals(band, squares=True, carry=carry, carry_sq=carry_sq)
    assert np.array_equal(host_u64(Tb), ref_T) and np.array_equal(host_u64(TQb), ref_TQ)


def test_carry_beyond_its_bound_sets_the_fault_word():
    """A carry above 2^62 - 1 - H * 255 cannot be column totals of rows above (the host cannot see
    device values): the build completes, and the workspace check reports it."""
    img = to_device(np.ones((100, 300), np.uint8))
    carry = torch.full((300,), (1 << 62) - 50, dtype=torch.int64, device="cuda:0").view(torch.uint64)
    ws = torch.empty(api.build_workspace_bytes(100, 300, 1, False), dtype=torch.uint8, device="cuda:0")
    api.sat_build_band(img, carry=carry, ws=ws, totals=False)
    with pytest.raises(SatError) as e:
        api.workspace_check(ws)
    assert e.value.status == SAT_ERR_DEVICE
    api.sat_build(img, ws=ws)                       # the next build clears the fault word
    api.workspace_check(ws)


@pytest.mark.parametrize("band_rows", [1, 7, 1000, 5000])
def test_streamed_whole_table_from_host_rows(band_rows):
    print("case: streamed table, band rows", band_rows, flush=True)
    rng = np.random.default_rng(band_rows)
    img_np = rng.integers(0, 256, (3001, 777)).astype(np.uint8)
    S = banded.build_table_streamed(lambda r0, r1: img_np[r0:r1], 3001, 777, "u8", band_rows=band_rows)
    assert np.array_equal(to_host(S), oracle.sat(img_np))


def test_streamed_whole_table_u16_with_squares():
    img_np = synth.lognormal_u16(2500, 1300, 6.0, 1.0, seed=44)
    S, Q = banded.build_table_streamed(lambda r0, r1: img_np[r0:r1], 2500, 1300, "u16", squares=True,
                                       band_rows=333)
    ref_S, ref_Q = oracle.sat(img_np, squares=True)
    assert np.array_equal(to_host(S), ref_S) and np.array_equal(to_host(Q), ref_Q)


@pytest.mark.slow
def test_full_scale_eight_row_shards_of_70000x85000(capsys):
    """The bench image as eight shards of 8750 rows, each built as one GPU would build its share:
    its carry is the column totals of the rows above (sat_column_totals), its band build writes its
    rows of the table and its totals.  Every row of the assembled table is compared with the
    streamed oracle, band by band; every shard's totals match the oracle's totals chained over the
    shards."""
    import banded_compare
    H, W, n = 70000, 85000, 8
    dev = torch.device("cuda:0")

    def say(msg):
        with capsys.disabled():
            print("full scale shards: " + msg, flush=True)

    say("host mask")
    img_np = synth.thomas_mask(H, W, seed=2)
    img = api.empty_image(H, W, torch.uint8, dev)          # the bench's layout: rows on 128-byte lines
    img.copy_(torch.from_numpy(img_np))
    S = api.empty_table(H, W, dev)
    shard = H // n
    ws = torch.empty(api.build_workspace_bytes(shard, W, 1, False), dtype=torch.uint8, device=dev)
    totals = []
    for k in range(n):
        r0, r1 = k * shard, (k + 1) * shard
        carry = api.column_totals(img[:r0]) if r0 else None
        _, T = api.sat_build_band(img[r0:r1], carry=carry, rows_above=r0, sat=S[r0:r1], ws=ws)
        api.workspace_check(ws)
        totals.append(T)
    del img, ws
    torch.cuda.synchronize()
    say("shards built; comparing every table row with the streamed oracle")
    counts = banded_compare.compare(img_np, [], 1, table=lambda a, b: to_host(S[a:b]), progress=say)
    assert counts["table_rows"] == H
    c = None
    for k in range(n):
        r0, r1 = k * shard, (k + 1) * shard
        c = oracle.column_totals(img_np[r0:r1], carry=c)
        assert np.array_equal(host_u64(totals[k]), c), k
