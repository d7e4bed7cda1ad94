"""Tables of pixel powers and higher window moments: HIP path vs the oracle through the C ABI
(needs an MI355X).  Power tables are compared bit for bit.  Every statistic is bit-exact too: both
sides form the same exact integer numerators and take the same correctly rounded steps
(conversion to double, square root, products, division), with NaN exactly where the oracle has
NaN (constant windows).  Both gather paths (chain walks and row pairs) are compared."""
import numpy as np
import pytest
import torch

import oracle
from paper_2410_16291_amd import api, autotune, synth
from gpu_util import padded_image, to_device, to_host

pytestmark = pytest.mark.gpu

RTOL = 1e-12


def check_close(got, ref, name):
    """Bit-exact where defined, NaN where the oracle has NaN; reports the relative error against
    the 1e-12 bar first so that a failure says how far off it is."""
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(got), nan), name
    g, r = got[~nan], ref[~nan]
    zero = r == 0
    assert np.all(g[zero] == 0.0), name
    rel = np.abs(g[~zero] - r[~zero]) / np.abs(r[~zero])
    assert rel.size == 0 or rel.max() <= RTOL, (name, rel.max())
    assert np.array_equal(g, r), (name, int(np.sum(g != r)), g.size)


POWER_CASES = [
    # (H, W, pitch_extra, offset): image shape, extra pitch elements, misaligning element offset
    (1, 1, 0, 0), (3, 200, 0, 0), (65, 129, 0, 0), (1000, 1300, 0, 0), (257, 4099, 5, 1),
    (700, 1024, 0, 0), (2000, 777, 3, 0),
    (300, 2048, 0, 0), (300, 2000, 0, 0),     # 16-byte tile DMA over 8 blocks; ragged last block
]


@pytest.mark.parametrize("dtype,hi,k", [(np.uint8, 256, 4), (np.uint16, 65536, 3)])
@pytest.mark.parametrize("H,W,extra,offset", POWER_CASES)
def test_power_tables_bit_exact(dtype, hi, k, H, W, extra, offset):
    print("case: power tables", np.dtype(dtype).name, k, H, W, extra, offset, flush=True)
    rng = np.random.default_rng(H * 7 + W)
    img_np = rng.integers(0, hi, (H, W)).astype(dtype)
    img = padded_image(img_np, W + extra, offset) if (extra or offset) else to_device(img_np)
    ws = torch.empty(api.powers_workspace_bytes(H, W, 1 if dtype == np.uint8 else 2, k), dtype=torch.uint8,
                     device="cuda:0")
    tables = api.sat_build_powers(img, k, ws=ws)
    api.workspace_check(ws)
    for p, T in enumerate(tables, start=1):
        assert np.array_equal(to_host(T), oracle.sat_power(img_np, p)), p


def test_power_tables_many_strips_and_rounds():
    """More strips than resident workgroups (balanced strip heights, several rounds), 128-byte
    pitched rows (16-byte tile DMA), and k = 2 against sat_build's two tables."""
    for dtype, hi, k, H, W in [(np.uint8, 256, 4, 40001, 300), (np.uint16, 65536, 3, 16384, 520)]:
        print("case: power tables, rounds", np.dtype(dtype).name, H, W, flush=True)
        rng = np.random.default_rng(H)
        img_np = rng.integers(0, hi, (H, W)).astype(dtype)
        img = api.empty_image(H, W, torch.uint8 if dtype == np.uint8 else torch.uint16, "cuda:0")
        img.copy_(to_device(img_np))
        tables = api.sat_build_powers(img, k)
        torch.cuda.synchronize()
        for p, T in enumerate(tables, start=1):
            assert np.array_equal(to_host(T), oracle.sat_power(img_np, p)), p
        S, Q = api.sat_build(img, squares=True)
        S2, Q2 = api.sat_build_powers(img, 2)
        assert torch.equal(S.view(torch.int64), S2.view(torch.int64))
        assert torch.equal(Q.view(torch.int64), Q2.view(torch.int64))


# windows from 1 x 1 to 300 x 420 at strides 1 to 4
MOMENT_CASES = [(1, 1, 1), (5, 7, 1), (16, 16, 4), (33, 9, 3), (64, 64, 1), (66, 66, 1), (70, 70, 1), (1, 200, 2),
                (300, 420, 1)]
# built-in (LDS-staged chain walk for up to three tables at stride 1, register chain walk
# otherwise), register chain walk, row pairs
PATHS = [None, "chain_v4", "rowpair_v4_banded"]


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("h,w,s", MOMENT_CASES)
def test_window_moments_match_oracle_u8(h, w, s, path):
    print("case: moments u8", h, w, s, path, flush=True)
    img_np = synth.lognormal_u16(300, 420, 4.0, 0.9, rng=np.random.default_rng(h * 100 + w)).clip(0, 255).astype(np.uint8)
    img_np[40:90, 100:160] = 255                                  # saturated patch: constant windows
    img = to_device(img_np)
    tables = api.sat_build_powers(img, 4)
    with autotune.forced(1, path):
        got = api.window_moments(tables, h, w, s, pixel_type="u8")
    torch.cuda.synchronize()
    _, ref = oracle.window_moments(img_np, h, w, s, k=4)
    assert np.array_equal(to_host(got["mean"]), ref[0])
    for name, r in zip(("std", "skew", "kurt"), ref[1:]):
        check_close(to_host(got[name]), r, name)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("h,w,s", [(8, 8, 1), (31, 17, 2), (256, 256, 16), (40, 40, 8)])
def test_window_moments_match_oracle_u16(h, w, s, path):
    print("case: moments u16", h, w, s, path, flush=True)
    img_np = synth.lognormal_u16(520, 610, 6.0, 1.0, rng=np.random.default_rng(h + w))
    img = to_device(img_np)
    tables = api.sat_build_powers(img, 3)
    with autotune.forced(1, path):
        got = api.window_moments(tables, h, w, s, pixel_type="u16", stats=("mean", "std", "skew"))
    torch.cuda.synchronize()
    _, ref = oracle.window_moments(img_np, h, w, s, k=3)
    assert np.array_equal(to_host(got["mean"]), ref[0])
    check_close(to_host(got["std"]), ref[1], "std")
    check_close(to_host(got["skew"]), ref[2], "skew")


def test_moments_single_statistic_and_closed_forms():
    """Only the kurtosis requested (nothing else written); a 0/1 image whose windows follow the
    Bernoulli closed forms; a constant image gives NaN shape statistics."""
    rng = np.random.default_rng(77)
    img_np = (rng.random((200, 300)) < 0.3).astype(np.uint8)
    img = to_device(img_np)
    tables = api.sat_build_powers(img, 4)
    got = api.window_moments(tables, 10, 10, 5, pixel_type="u8", stats=("kurt",))
    assert list(got) == ["kurt"]
    _, ref = oracle.window_moments(img_np, 10, 10, 5, k=4)
    check_close(to_host(got["kurt"]), ref[3], "kurt")
    p = ref[0]
    pq = p * (1 - p)
    ok = pq > 0
    assert np.allclose(to_host(got["kurt"])[ok], ((1 - 6 * pq) / pq)[ok], rtol=1e-12)
    flat = to_device(np.full((50, 60), 9, np.uint8))
    got = api.window_moments(api.sat_build_powers(flat, 4), 7, 7, 1, pixel_type="u8")
    torch.cuda.synchronize()
    assert np.all(to_host(got["mean"]) == 9.0) and np.all(to_host(got["std"]) == 0.0)
    assert np.all(np.isnan(to_host(got["skew"]))) and np.all(np.isnan(to_host(got["kurt"])))


def test_moments_4096_u8_64x64():
    """A 4096 x 4096 8-bit image, 64 x 64 windows at stride 1: all 4033^2 outputs of all four
    statistics against the oracle."""
    print("case: moments 4096^2 u8 64x64", flush=True)
    img_np = synth.lognormal_u16(4096, 4096, 4.0, 0.9, rng=np.random.default_rng(5)).clip(0, 255).astype(np.uint8)
    img = api.empty_image(4096, 4096, torch.uint8, "cuda:0")
    img.copy_(to_device(img_np))
    tables = api.sat_build_powers(img, 4)
    got = api.window_moments(tables, 64, 64, 1, pixel_type="u8")
    torch.cuda.synchronize()
    _, ref = oracle.window_moments(img_np, 64, 64, 1, k=4)
    assert np.array_equal(to_host(got["mean"]), ref[0])
    for name, r in zip(("std", "skew", "kurt"), ref[1:]):
        check_close(to_host(got[name]), r, name)


@pytest.mark.parametrize("stats", [("mean",), ("std",), ("mean", "std"), ("mean", "std", "skew")])
def test_lds_walk_up_to_three_tables(stats):
    """The LDS-staged chain walk (stride 1, up to three tables): windows from 1 x 1 to 2 x 1500
    (spans of 5 to 8 loaded columns per thread), an image with ragged chunks, against the oracle."""
    img_np = synth.lognormal_u16(700, 2900, 4.0, 0.9, rng=np.random.default_rng(31)).clip(0, 255).astype(np.uint8)
    img = to_device(img_np)
    k = {"mean": 1, "std": 2, "skew": 3}[stats[-1]]
    tables = api.sat_build_powers(img, 3)
    for h, w in [(1, 1), (64, 64), (300, 420), (5, 700), (2, 1500)]:
        print("case: lds moments", stats, h, w, flush=True)
        got = api.window_moments(tables[:k], h, w, 1, pixel_type="u8", stats=stats)
        torch.cuda.synchronize()
        _, ref = oracle.window_moments(img_np, h, w, 1, k=3)
        for name in stats:
            r = ref[{"mean": 0, "std": 1, "skew": 2}[name]]
            if name == "mean":
                assert np.array_equal(to_host(got[name]), r), (h, w)
            else:
                check_close(to_host(got[name]), r, name)
