"""HIP path vs the oracle, element by element, through the C ABI (needs an MI355X).

Integer results (tables, window sums, counts) must be bit-exact; the FP64 mean must be
bit-exact (one correctly rounded division of exact operands on both sides); the FP64 std must be
within 1e-12 relative (exactly 0 where the oracle gives 0).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2410_16291_amd import api, synth
from gpu_util import padded_image, to_device, to_host

pytestmark = pytest.mark.gpu

STD_RTOL = 1e-12


def check_std(got, ref):
    zero = ref == 0
    assert np.all(got[zero] == 0.0)
    rel = np.abs(got[~zero] - ref[~zero]) / ref[~zero]
    assert rel.size == 0 or rel.max() <= STD_RTOL, rel.max()


def gpu_stats(img_np, h, w, s, squares_only=False):
    img = to_device(img_np)
    S, Q = api.sat_build(img, squares=True)
    s1, mean, std = api.window_mean_std(S, Q, h, w, s)
    torch.cuda.synchronize()
    return S, Q, s1, mean, std


# ------------------------------------------------------------------ the paper-shaped small cases

def test_cfg_small_poisson_512():
    print("case: 512x512 u8 poisson, 32x32 stride 1", flush=True)
    img_np = synth.poisson_counts(512, 512, 0.05, seed=0)
    img = to_device(img_np)
    S = api.sat_build(img)
    out = api.window_sum(S, 32, 32, 1, pixel_type="u8")
    torch.cuda.synchronize()
    assert out.dtype == torch.uint32 and tuple(out.shape) == (481, 481)
    ref_S = oracle.sat(img_np)
    assert np.array_equal(to_host(S), ref_S)
    ref = oracle.window_sum_sat(ref_S, 32, 32, 1)
    assert np.array_equal(to_host(out).astype(np.uint64), ref)
    assert np.array_equal(ref, oracle.window_sum_direct(img_np, 32, 32, 1))


def test_cfg_lognormal_8192_mean_std():
    print("case: 8192x8192 u16 lognormal, S and Q, 64x64 stride 1", flush=True)
    img_np = synth.lognormal_u16(8192, 8192, seed=1)
    S, Q, s1, mean, std = gpu_stats(img_np, 64, 64, 1)
    ref_S, ref_Q = oracle.sat(img_np, squares=True)
    assert np.array_equal(to_host(S), ref_S)
    assert np.array_equal(to_host(Q), ref_Q)
    del S, Q
    sums = oracle.window_sum_sat(ref_S, 64, 64, 1)
    sqs = oracle.window_sum_sat(ref_Q, 64, 64, 1)
    del ref_S, ref_Q
    ref_mean, ref_std = oracle.mean_std(sums, sqs, 64 * 64)
    assert np.array_equal(to_host(s1), sums)
    assert np.array_equal(to_host(mean), ref_mean)
    check_std(to_host(std), ref_std)


# ------------------------------------------------------------------ shapes and edges

SHAPES = [(1, 1), (1, 300), (300, 1), (17, 257), (64, 256), (65, 255), (129, 513), (200, 1000), (333, 77)]


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
@pytest.mark.parametrize("shape", SHAPES)
def test_build_shapes_bit_exact(shape, dtype):
    print("case: build", shape, np.dtype(dtype).name, flush=True)
    rng = np.random.default_rng(hash(shape) % 1000)
    hi = 256 if dtype == np.uint8 else 65536
    img_np = rng.integers(0, hi, shape).astype(dtype)
    S, Q = api.sat_build(to_device(img_np), squares=True)
    ref_S, ref_Q = oracle.sat(img_np, squares=True)
    assert np.array_equal(to_host(S), ref_S)
    assert np.array_equal(to_host(Q), ref_Q)


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_windows_and_strides(dtype):
    rng = np.random.default_rng(7)
    hi = 256 if dtype == np.uint8 else 65536
    img_np = rng.integers(0, hi, (301, 517)).astype(dtype)
    S, Q = api.sat_build(to_device(img_np), squares=True)
    ref_S, ref_Q = oracle.sat(img_np, squares=True)
    ptype = "u8" if dtype == np.uint8 else "u16"
    cases = [(1, 1, 1), (301, 517, 1), (301, 1, 1), (1, 517, 2), (32, 32, 1), (64, 64, 4), (7, 300, 3),
             (300, 7, 5), (100, 250, 8), (13, 17, 16)]
    for (h, w, s) in cases:
        print("case: window", h, w, s, ptype, flush=True)
        out = api.window_sum(S, h, w, s, pixel_type=ptype, out_dtype=torch.uint64)
        ref = oracle.window_sum_sat(ref_S, h, w, s)
        assert np.array_equal(to_host(out), ref), (h, w, s)
        if h * w * (hi - 1) <= 0xFFFFFFFF:
            out32 = api.window_sum(S, h, w, s, pixel_type=ptype, out_dtype=torch.uint32)
            assert np.array_equal(to_host(out32).astype(np.uint64), ref), (h, w, s)
        s1, mean, std = api.window_mean_std(S, Q, h, w, s)
        sqs = oracle.window_sum_sat(ref_Q, h, w, s)
        ref_mean, ref_std = oracle.mean_std(ref, sqs, h * w)
        assert np.array_equal(to_host(s1), ref)
        assert np.array_equal(to_host(mean), ref_mean)
        check_std(to_host(std), ref_std)
    # spot check against direct summation of the image itself
    out = to_host(api.window_sum(S, 9, 11, 2, pixel_type=ptype, out_dtype=torch.uint64))
    assert np.array_equal(out, oracle.window_sum_direct(img_np, 9, 11, 2))


@pytest.mark.parametrize("dtype,offset,pitch_extra", [(np.uint8, 3, 5), (np.uint8, 1, 0), (np.uint16, 1, 3),
                                                      (np.uint16, 2, 1)])
def test_unaligned_image_and_odd_table_pitch(dtype, offset, pitch_extra):
    print("case: unaligned", np.dtype(dtype).name, offset, pitch_extra, flush=True)
    rng = np.random.default_rng(8)
    H, W = 150, 700
    hi = 256 if dtype == np.uint8 else 65536
    img_np = rng.integers(0, hi, (H, W)).astype(dtype)
    img = padded_image(img_np, W + pitch_extra, offset)
    assert img.data_ptr() % 4 != 0 or pitch_extra % 4 != 0
    big = torch.empty((H, W + 1), dtype=torch.uint64, device="cuda:0")     # odd pitch: scalar stores
    S = big[:, :W]
    bigq = torch.empty((H, W + 1), dtype=torch.uint64, device="cuda:0")
    Q = bigq[:, :W]
    api.sat_build(img, sat=S, sat_sq=Q)
    ref_S, ref_Q = oracle.sat(img_np, squares=True)
    assert np.array_equal(to_host(S), ref_S)
    assert np.array_equal(to_host(Q), ref_Q)
    out = api.window_sum(S, 5, 9, 1, pixel_type="u16", out_dtype=torch.uint64)
    assert np.array_equal(to_host(out), oracle.window_sum_sat(ref_S, 5, 9, 1))


def test_max_pixel_values():
    for dtype, m in [(np.uint8, 255), (np.uint16, 65535)]:
        img_np = np.full((257, 1031), m, dtype)
        S, Q = api.sat_build(to_device(img_np), squares=True)
        ref_S, ref_Q = oracle.sat(img_np, squares=True)
        assert np.array_equal(to_host(S), ref_S)
        assert np.array_equal(to_host(Q), ref_Q)
        s1, mean, std = api.window_mean_std(S, Q, 64, 64, 1)
        assert np.all(to_host(std) == 0.0) and np.all(to_host(mean) == float(m))


# ------------------------------------------------------------------ variants, stress, fault word

def test_every_build_variant_bit_exact():
    """Every build variant on 16-bit pixels with squares (5200-byte rows) and on 8-bit pixels with
    8-byte aligned rows (2600 bytes: dword DMA in the helper-wave variants) and 16-byte aligned
    rows (pitch 2608); a variant not compiled for a pixel type is refused with SAT_ERR_ARG."""
    from paper_2410_16291_amd._lib import SAT_ERR_ARG, SatError
    rng = np.random.default_rng(9)
    img_np = rng.integers(0, 65536, (1100, 2600)).astype(np.uint16)
    ref_S, ref_Q = oracle.sat(img_np, squares=True)
    img = to_device(img_np)
    img8_np = (img_np & 0xFF).astype(np.uint8)
    ref8_S, ref8_Q = oracle.sat(img8_np, squares=True)
    img8s = [to_device(img8_np), padded_image(img8_np, 2608, 0)]
    names = api.variants(0)
    u16_sq, u8, u8_sq = set(api.variants(0, "u16", True)), set(api.variants(0, "u8")), set(api.variants(0, "u8", True))
    assert u8 == set(names)                                   # every variant runs plain 8-bit builds
    try:
        for v, name in enumerate(names):
            print("case: build variant", name, flush=True)
            api.force_variant(0, v)
            ws = torch.empty(api.build_workspace_bytes(1100, 2600, 2, True), dtype=torch.uint8, device="cuda:0")
            if name in u16_sq:
                S, Q = api.sat_build(img, squares=True, ws=ws)
                api.workspace_check(ws)
                assert np.array_equal(to_host(S), ref_S), name
                assert np.array_equal(to_host(Q), ref_Q), name
            else:
                with pytest.raises(SatError) as e:
                    api.sat_build(img, squares=True, ws=ws)
                assert e.value.status == SAT_ERR_ARG
            for im in img8s:
                S8 = api.sat_build(im, ws=ws)
                assert np.array_equal(to_host(S8), ref8_S), name
                if name in u8_sq:
                    S8, Q8 = api.sat_build(im, squares=True, ws=ws)
                    api.workspace_check(ws)
                    assert np.array_equal(to_host(S8), ref8_S), name
                    assert np.array_equal(to_host(Q8), ref8_Q), name
    finally:
        api.force_variant(0, -1)


def test_every_gather_variant_bit_exact():
    rng = np.random.default_rng(10)
    img_np = rng.integers(0, 256, (700, 3000)).astype(np.uint8)
    S = api.sat_build(to_device(img_np))
    ref_S = oracle.sat(img_np)
    try:
        for v, name in enumerate(api.variants(1)):
            print("case: gather variant", name, flush=True)
            api.force_variant(1, v)
            for (h, w, s) in [(100, 100, 1), (250, 31, 2), (3, 2999, 1)]:
                out = api.window_sum(S, h, w, s, pixel_type="u8")
                assert np.array_equal(to_host(out).astype(np.uint64), oracle.window_sum_sat(ref_S, h, w, s)), name
    finally:
        api.force_variant(1, -1)


def test_lookback_repeated_builds_many_strips():
    """Many short strips (deep lookback chains), rebuilt repeatedly into the same workspace."""
    rng = np.random.default_rng(11)
    img_np = rng.integers(0, 256, (4099, 777)).astype(np.uint8)
    ref_S = oracle.sat(img_np)
    img = to_device(img_np)
    ws = torch.empty(api.build_workspace_bytes(4099, 777, 1, False), dtype=torch.uint8, device="cuda:0")
    try:
        api.force_variant(0, api.variants(0).index("lookback_px4_rw8_nw4"))   # 32-row strips: 129 strips
        for it in range(20):
            S = api.sat_build(img, ws=ws)
            api.workspace_check(ws)
            assert np.array_equal(to_host(S), ref_S), it
    finally:
        api.force_variant(0, -1)


def test_multi_window_matches_single():
    rng = np.random.default_rng(12)
    img_np = (rng.random((900, 1300)) < 0.01).astype(np.uint8)
    S = api.sat_build(to_device(img_np))
    ref_S = oracle.sat(img_np)
    wins = [(100, 100), (250, 250), (500, 500), (7, 300)]
    for s in (1, 3):
        outs = api.window_sum_multi(S, wins, s, pixel_type="u8")
        for (h, w), o in zip(wins, outs):
            assert np.array_equal(to_host(o).astype(np.uint64), oracle.window_sum_sat(ref_S, h, w, s)), (h, w, s)


def test_batched_build_and_mean_std():
    from paper_2410_16291_amd import batch
    imgs_np = synth.uneven_batch(9, lo=70, hi=900, seed=13)
    imgs = [to_device(i) for i in imgs_np]
    tables = batch.build_batched(imgs, squares=True)
    outs = batch.mean_std_batched(tables, 64, 64, 4)
    torch.cuda.synchronize()
    for i, img_np in enumerate(imgs_np):
        ref_S, ref_Q = oracle.sat(img_np, squares=True)
        assert np.array_equal(to_host(tables[i][0]), ref_S), i
        assert np.array_equal(to_host(tables[i][1]), ref_Q), i
        sums = oracle.window_sum_sat(ref_S, 64, 64, 4)
        ref_mean, ref_std = oracle.mean_std(sums, oracle.window_sum_sat(ref_Q, 64, 64, 4), 64 * 64)
        s1, mean, std = outs[i]
        assert np.array_equal(to_host(s1), sums), i
        assert np.array_equal(to_host(mean), ref_mean), i
        check_std(to_host(std), ref_std)


def test_balanced_strip_heights_tall_image():
    """More strips than resident workgroups: adaptive variants shorten the strips so they fill
    whole rounds; every variant must stay bit-exact, including a ragged last strip."""
    rng = np.random.default_rng(14)
    for dtype, hi in [(np.uint8, 256), (np.uint16, 65536)]:
        img_np = rng.integers(0, hi, (33001, 523)).astype(dtype)
        ref_S = oracle.sat(img_np)
        img = to_device(img_np)
        names = api.variants(0)
        try:
            for name in api.variants(0, "u8" if dtype == np.uint8 else "u16"):
                print("case: tall image", np.dtype(dtype).name, name, flush=True)
                api.force_variant(0, names.index(name))
                ws = torch.empty(api.build_workspace_bytes(33001, 523, 1 if dtype == np.uint8 else 2, False),
                                 dtype=torch.uint8, device="cuda:0")
                S = api.sat_build(img, ws=ws)
                api.workspace_check(ws)
                assert np.array_equal(to_host(S), ref_S), name
        finally:
            api.force_variant(0, -1)


# ------------------------------------------------------------------ chain gathers

CHAIN_CASES = [(1, 1, 1), (2, 5, 1), (301, 1111, 1), (64, 64, 4), (12, 7, 3), (300, 2, 1), (5, 517, 5),
               (100, 100, 1), (5, 1500, 1), (7, 2500, 1), (1, 3111, 1),
               (7, 300, 3)]      # the last: height not a multiple of the stride (row pairs)


@pytest.mark.parametrize("out64", [False, True])
def test_chain_gather_every_variant(out64):
    rng = np.random.default_rng(15)
    img_np = rng.integers(0, 65536, (301, 3111)).astype(np.uint16)
    S = api.sat_build(to_device(img_np))
    ref_S = oracle.sat(img_np)
    odt = torch.uint64 if out64 else torch.uint32
    try:
        for v, name in enumerate(api.variants(1)):
            if not name.startswith("chain"):
                continue
            api.force_variant(1, v)
            for (h, w, s) in CHAIN_CASES:
                if not out64 and h * w * 65535 > 0xFFFFFFFF:
                    continue
                print("case: chain", name, h, w, s, "u64" if out64 else "u32", flush=True)
                out = api.window_sum(S, h, w, s, pixel_type="u16", out_dtype=odt)
                assert np.array_equal(to_host(out).astype(np.uint64), oracle.window_sum_sat(ref_S, h, w, s)), \
                    (name, h, w, s)
    finally:
        api.force_variant(1, -1)


def test_chain_segments_tall_narrow():
    """Short windows on a tall image: chains are cut into many segments per residue."""
    rng = np.random.default_rng(16)
    img_np = rng.integers(0, 256, (20000, 200)).astype(np.uint8)
    S = api.sat_build(to_device(img_np))
    ref_S = oracle.sat(img_np)
    for (h, w, s) in [(3, 2, 1), (1, 200, 1), (10, 10, 2), (40, 3, 4)]:
        print("case: chain tall", h, w, s, flush=True)
        out = api.window_sum(S, h, w, s, pixel_type="u8")
        assert np.array_equal(to_host(out).astype(np.uint64), oracle.window_sum_sat(ref_S, h, w, s)), (h, w, s)
    wins = [(10, 5), (20, 20), (30, 1)]            # one lattice: q = 10, lags 1, 2, 3
    outs = api.window_sum_multi(S, wins, 1, pixel_type="u8")
    for (h, w), o in zip(wins, outs):
        assert np.array_equal(to_host(o).astype(np.uint64), oracle.window_sum_sat(ref_S, h, w, 1)), (h, w)


@pytest.mark.parametrize("out64", [False, True])
def test_chain_multi_window_groups(out64):
    rng = np.random.default_rng(17)
    img_np = (rng.random((1500, 1700)) < 0.02).astype(np.uint8)
    S = api.sat_build(to_device(img_np))
    ref_S = oracle.sat(img_np)
    odt = torch.uint64 if out64 else torch.uint32
    sets = [
        ([(100, 100), (250, 250), (500, 500)], 1),                  # one lattice, lags 2, 5, 10
        ([(6, 4), (9, 5), (15, 2)], 3),                             # q = 1 in stride units
        ([(97, 5), (101, 7), (103, 9), (107, 3), (109, 11), (113, 13), (127, 2), (131, 1)], 1),  # rings too big
        ([(100, 100), (7, 300), (250, 31), (12, 12)], 3),           # mixed: chains and row pairs
        ([(1500, 1700)], 1),                                        # the whole image
    ]
    try:
        for v, name in enumerate(api.variants(1)):
            if name not in ("chain_auto", "chain_v1", "chain_v2", "chain_v4", "rowpair_v4_banded"):
                continue
            api.force_variant(1, v)
            for wins, s in sets:
                print("case: multi", name, wins, s, flush=True)
                outs = api.window_sum_multi(S, wins, s, pixel_type="u8", out_dtype=odt)
                for (h, w), o in zip(wins, outs):
                    ref = oracle.window_sum_sat(ref_S, h, w, s)
                    assert np.array_equal(to_host(o).astype(np.uint64), ref), (name, h, w, s)
    finally:
        api.force_variant(1, -1)


def test_mean_std_chain_and_rowpair():
    img_np = synth.lognormal_u16(700, 900, seed=18)
    S, Q = api.sat_build(to_device(img_np), squares=True)
    ref_S, ref_Q = oracle.sat(img_np, squares=True)
    try:
        for v, name in enumerate(api.variants(1)):
            if name not in ("chain_v1", "chain_v2", "chain_v4", "rowpair_v4_banded"):
                continue
            api.force_variant(1, v)
            for (h, w, s) in [(64, 64, 1), (64, 64, 4), (3, 700, 1), (50, 9, 5), (7, 11, 3), (700, 900, 1)]:
                print("case: mean/std", name, h, w, s, flush=True)
                s1, mean, std = api.window_mean_std(S, Q, h, w, s)
                sums = oracle.window_sum_sat(ref_S, h, w, s)
                ref_mean, ref_std = oracle.mean_std(sums, oracle.window_sum_sat(ref_Q, h, w, s), h * w)
                assert np.array_equal(to_host(s1), sums), (name, h, w, s)
                assert np.array_equal(to_host(mean), ref_mean), (name, h, w, s)
                check_std(to_host(std), ref_std)
    finally:
        api.force_variant(1, -1)


def test_batched_mean_std_every_gather_family():
    from paper_2410_16291_amd import batch
    imgs_np = synth.uneven_batch(7, lo=64, hi=700, seed=19)
    imgs = [to_device(i) for i in imgs_np]
    tables = batch.build_batched(imgs, squares=True)
    refs = [oracle.sat(i, squares=True) for i in imgs_np]
    try:
        for v, name in enumerate(api.variants(1)):
            if name not in ("chain_v1", "chain_v2", "chain_v4", "rowpair_v4_banded"):
                continue
            api.force_variant(1, v)
            for (h, w, s) in [(64, 64, 4), (30, 20, 7)]:
                print("case: batched mean/std", name, h, w, s, flush=True)
                outs = batch.mean_std_batched(tables, h, w, s)
                torch.cuda.synchronize()
                for i, (ref_S, ref_Q) in enumerate(refs):
                    sums = oracle.window_sum_sat(ref_S, h, w, s)
                    ref_mean, ref_std = oracle.mean_std(sums, oracle.window_sum_sat(ref_Q, h, w, s), h * w)
                    s1, mean, std = outs[i]
                    assert np.array_equal(to_host(s1), sums), (name, i)
                    assert np.array_equal(to_host(mean), ref_mean), (name, i)
                    check_std(to_host(std), ref_std)
    finally:
        api.force_variant(1, -1)


# ------------------------------------------------------------------ autotuned batches

def test_autotuned_batch_matches_oracle(tmp_path):
    from paper_2410_16291_amd import autotune, batch
    imgs_np = synth.uneven_batch(5, lo=100, hi=700, seed=20)
    imgs = [to_device(i) for i in imgs_np]
    tuner = autotune.Tuner(path=str(tmp_path / "tune.json"), reps=1)
    choice = tuner.tune_batch(imgs, squares=True, win=(32, 48), stride=2)
    print("case: autotune choice", choice["build"], choice["gather"], flush=True)
    assert choice["build"] in api.variants(0) and choice["gather"] in api.variants(1)
    assert set(choice["build_ms"]) == set(api.variants(0, "u16", True))
    again = autotune.Tuner(path=str(tmp_path / "tune.json")).tune_batch(imgs, squares=True, win=(32, 48), stride=2)
    assert again["build"] == choice["build"] and again["gather_ms"] == choice["gather_ms"]    # from the cache
    assert choice["strip_h"] is None or 8 <= choice["strip_h"] < autotune.strip_height(choice["build"])
    assert set(choice["fused_ms"]) == {"one_launch", "two_launches"}
    tables = batch.alloc_tables(imgs, True)
    outs = batch.alloc_stats(tables, 32, 48, 2)
    autotune.Tuner.run_batch(choice, imgs, True, (32, 48), 2, tables, outs)
    torch.cuda.synchronize()
    for i, img_np in enumerate(imgs_np):
        ref_S, ref_Q = oracle.sat(img_np, squares=True)
        assert np.array_equal(to_host(tables[i][0]), ref_S), i
        assert np.array_equal(to_host(tables[i][1]), ref_Q), i
        sums = oracle.window_sum_sat(ref_S, 32, 48, 2)
        ref_mean, ref_std = oracle.mean_std(sums, oracle.window_sum_sat(ref_Q, 32, 48, 2), 32 * 48)
        assert np.array_equal(to_host(outs[i][0]), sums), i
        assert np.array_equal(to_host(outs[i][1]), ref_mean), i
        check_std(to_host(outs[i][2]), ref_std)


def fused_check(imgs_np, tables, outs, h, w, s, what):
    for i, img_np in enumerate(imgs_np):
        ref_S, ref_Q = oracle.sat(img_np, squares=True)
        assert np.array_equal(to_host(tables[i][0]), ref_S), (what, i, "S")
        assert np.array_equal(to_host(tables[i][1]), ref_Q), (what, i, "Q")
        sums = oracle.window_sum_sat(ref_S, h, w, s)
        ref_mean, ref_std = oracle.mean_std(sums, oracle.window_sum_sat(ref_Q, h, w, s), h * w)
        if outs[i][0] is not None:
            assert np.array_equal(to_host(outs[i][0]), sums), (what, i, "sum")
        assert np.array_equal(to_host(outs[i][1]), ref_mean), (what, i, "mean")
        check_std(to_host(outs[i][2]), ref_std)


@pytest.mark.parametrize("dtype", ["u16", "u8"])
def test_fused_build_and_stats_every_variant(dtype):
    """sat_build_stats_batched (tables and window statistics in one launch) against the oracle, for
    every build variant of the fused kernel and every chain gather variant, then a window whose
    height is not a multiple of the stride (the two-launch path), then a second call on the same
    tables with other images (no result may come from the first call)."""
    from paper_2410_16291_amd import batch
    imgs_np = synth.uneven_batch(7, lo=70, hi=700, seed=31)
    if dtype == "u8":
        imgs_np = [(i % 256).astype(np.uint8) for i in imgs_np]
    imgs = [to_device(i) for i in imgs_np]
    fused = ["lookback_nt_px4_rw16_nw4", "lookback_px4_rw16_nw4", "lookback_px4_rw8_nw4"]
    chains = [g for g in api.variants(1) if g.startswith("chain_v")]
    assert chains
    for bv in fused:
        for gv in chains:
            print("case: fused", dtype, bv, gv, flush=True)
            tables, outs = batch.build_stats_batched(imgs, 32, 48, 4, build_variant=bv, gather_variant=gv)
            torch.cuda.synchronize()
            fused_check(imgs_np, tables, outs, 32, 48, 4, (bv, gv))
    print("case: fused, row-pair window 30x20 stride 4", flush=True)
    tables, outs = batch.build_stats_batched(imgs, 30, 20, 4)
    torch.cuda.synchronize()
    fused_check(imgs_np, tables, outs, 30, 20, 4, "row-pair")
    print("case: fused, second call on the same tables", flush=True)
    other_np = [np.ascontiguousarray(np.flipud(i)) for i in imgs_np]
    tables2, outs2 = batch.build_stats_batched([to_device(i) for i in other_np], 32, 48, 4, tables=tables,
                                               with_sum=False)
    torch.cuda.synchronize()
    fused_check(other_np, tables2, outs2, 32, 48, 4, "second call")


def test_batched_build_forced_strip_heights():
    """Batched builds at strip heights the tuner may set (sat_force_variant kind 2), including
    heights that leave waves with partial or no rows."""
    from paper_2410_16291_amd import autotune, batch
    imgs_np = synth.uneven_batch(5, lo=60, hi=500, seed=33)
    imgs = [to_device(i) for i in imgs_np]
    refs = [oracle.sat(i, squares=True) for i in imgs_np]
    for name in ("lookback_nt_px4_rw16_nw4", "lookback_px4_rw8_nw4"):
        for rows in (48, 32, 13, 5, 1):
            print("case: strip height", name, rows, flush=True)
            with autotune.forced(0, name), autotune.forced_strip(rows):
                tables = batch.build_batched(imgs, True)
            torch.cuda.synchronize()
            for i, (ref_S, ref_Q) in enumerate(refs):
                assert np.array_equal(to_host(tables[i][0]), ref_S), (name, rows, i)
                assert np.array_equal(to_host(tables[i][1]), ref_Q), (name, rows, i)


def test_device_generator_through_the_path():
    """The device-side log-normal generator's image, built and gathered, matches the oracle run
    on the same image copied to the host."""
    img = synth.lognormal_u16_device(777, 1033, 21, "cuda:0")
    img_np = to_host(img)
    assert img_np.dtype == np.uint16 and 300 < np.median(img_np) < 520
    S, Q = api.sat_build(img, squares=True)
    ref_S, ref_Q = oracle.sat(img_np, squares=True)
    assert np.array_equal(to_host(S), ref_S)
    s1, mean, std = api.window_mean_std(S, Q, 64, 64, 4)
    sums = oracle.window_sum_sat(ref_S, 64, 64, 4)
    ref_mean, ref_std = oracle.mean_std(sums, oracle.window_sum_sat(ref_Q, 64, 64, 4), 64 * 64)
    assert np.array_equal(to_host(s1), sums)
    assert np.array_equal(to_host(mean), ref_mean)
    check_std(to_host(std), ref_std)


# ------------------------------------------------------------------ serving

def check_served_against_oracle(srv, label):
    """Every query answered in the mix equals the same query run alone on a fresh table and the
    oracle's result for it: sums bit-exact, mean bit-exact, std within 1e-12 (the masks are 0/1,
    so the table of squares is the table itself)."""
    from paper_2410_16291_amd import serve
    gpu_tables, ref_tables = {}, {}
    n_sum = n_stats = 0
    for j in srv.done:
        if j.req.kind != "query":
            continue
        iid = serve.image_id(j.req)
        b = srv.builds[iid]
        if iid not in gpu_tables:
            gpu_tables[iid] = api.sat_build(synth.thomas_mask_device(b.H, b.W, b.image_seed, "cuda:0"))
            ref_tables[iid] = oracle.sat(synth.thomas_mask(b.H, b.W, seed=b.image_seed))
        S, ref_S = gpu_tables[iid], ref_tables[iid]
        h, w, st = min(j.req.win_h, b.H), min(j.req.win_w, b.W), j.req.stride
        sums = oracle.window_sum_sat(ref_S, h, w, st)
        if j.req.op == "sum":
            alone = api.window_sum(S, h, w, st, pixel_type="u8")
            got = to_host(j.result)
            assert np.array_equal(to_host(alone), got), (label, j.idx)
            assert np.array_equal(got.astype(np.uint64), sums), (label, j.idx)
            n_sum += 1
        else:
            alone = api.window_mean_std(S, S, h, w, st)
            for a, g in zip(alone, j.result):
                assert np.array_equal(to_host(a), to_host(g)), (label, j.idx)
            ref_mean, ref_std = oracle.mean_std(sums, sums, h * w)
            g_sum, g_mean, g_std = (to_host(t) for t in j.result)
            assert np.array_equal(g_sum, sums), (label, j.idx)
            assert np.array_equal(g_mean, ref_mean), (label, j.idx)
            check_std(g_std, ref_std)
            n_stats += 1
    return n_sum, n_stats


def test_serving_results_same_alone_and_in_mix():
    """Requests served concurrently (4 streams, evictions under a tight budget) give exactly the
    results of the same requests run alone, one at a time, and the oracle's, for every query."""
    import time
    from paper_2410_16291_amd import serve
    reqs = synth.request_stream(rate=300.0, duration=0.5, seed=22, side_lo=200, side_hi=1200,
                                win_lo=8, win_hi=120, stride_hi=4)
    ex = serve.GpuExecutor("cuda:0", slots=4)
    srv = serve.Server(ex, budget_bytes=40e6, slots=4, keep_results=True)
    rep = srv.run(reqs, idle=lambda: time.sleep(2e-5))
    torch.cuda.synchronize()
    ex.close()
    print("case: serving", rep.as_dict(), flush=True)
    assert rep.n == len(reqs) and rep.max_in_flight > 1 and rep.peak_bytes <= 40e6
    n_sum, n_stats = check_served_against_oracle(srv, "small")
    assert n_sum > 10 and n_stats > 3


@pytest.mark.slow
def test_serving_full_size_images_every_query():
    """The serving workload's own sizes: 8-bit cluster masks with sides on 2000..16000 (builds on
    128-byte row lines, taking the helper-wave plans), windows 16..512 at strides 1..8, a quarter
    of them mean/std, under a budget that forces evictions and rebuilds.  Every query in the mix is
    compared with the same query alone and with the oracle."""
    import time
    from paper_2410_16291_amd import serve
    reqs = synth.request_stream(rate=60.0, duration=0.6, seed=31)
    builds = [r for r in reqs if r.kind == "build"]
    assert max(max(r.H, r.W) for r in builds) > 14000 and min(min(r.H, r.W) for r in builds) < 2500
    ex = serve.GpuExecutor("cuda:0", slots=4)
    srv = serve.Server(ex, budget_bytes=3e9, slots=4, keep_results=True)
    rep = srv.run(reqs, idle=lambda: time.sleep(2e-5))
    torch.cuda.synchronize()
    ex.close()
    print("case: serving full size", rep.as_dict(), flush=True)
    assert rep.device_ms["h2d"]["n"] == rep.device_ms["build"]["n"] >= len(builds)
    assert rep.n == len(reqs) and rep.max_in_flight > 1 and rep.peak_bytes <= 3e9
    assert rep.evictions > 0
    n_sum, n_stats = check_served_against_oracle(srv, "full size")
    assert n_sum + n_stats == len(reqs) - len(builds) and n_stats >= 5


# ------------------------------------------------------------------ full size

@pytest.mark.slow
def test_full_scale_70000x85000_every_output(capsys):
    """The bench workload in the bench's launch configuration (one build, one fused 100/250/500
    gather, then the mean/std of every 250x250 window), compared with the oracle element by element
    over the whole output: every table row, every output row of all three windows and every
    mean/std row, band by band (the oracle streamed from the start of each part of the rows, in
    parallel parts).  Then random windows by direct summation of the image."""
    import banded_compare
    H, W = 70000, 85000
    dev = torch.device("cuda:0")

    def say(msg):
        with capsys.disabled():
            print("full scale: " + msg, flush=True)

    say("host mask")
    img_np = synth.thomas_mask(H, W, seed=2)
    img = api.empty_image(H, W, torch.uint8, dev)          # the bench's layout: rows on 128-byte lines
    img.copy_(torch.from_numpy(img_np))
    S = api.empty_table(H, W, dev)
    ws = torch.empty(api.build_workspace_bytes(H, W, 1, False), dtype=torch.uint8, device=dev)
    api.sat_build(img, sat=S, ws=ws)
    api.workspace_check(ws)
    del img, ws
    wins = [(100, 100), (250, 250), (500, 500)]
    outs = [api.empty_out(*api.out_shape(H, W, h, w, 1), torch.uint32, dev) for h, w in wins]
    api.window_sum_multi(S, wins, 1, pixel_type="u8", outs=outs)
    oh, ow = api.out_shape(H, W, 250, 250, 1)
    mean, std = api.empty_out(oh, ow, torch.float64, dev), api.empty_out(oh, ow, torch.float64, dev)
    # a 0/1 mask is its own table of squares
    api.window_mean_std(S, S, 250, 250, 1, with_sum=False, outs=(None, mean, std))
    torch.cuda.synchronize()
    say("GPU done; comparing every row with the streamed oracle")
    counts = banded_compare.compare(
        img_np, wins, 1, table=lambda a, b: to_host(S[a:b]), out=lambda i, k0, k1: to_host(outs[i][k0:k1]),
        stats=lambda k0, k1: (to_host(mean[k0:k1]), to_host(std[k0:k1])), stats_window=1, progress=say)
    say("compared %s" % counts)
    assert counts["table_rows"] == H and counts["stat_rows"] == oh
    assert int(to_host(S[H - 1])[W - 1]) == int(img_np.sum(dtype=np.uint64))
    say("random windows by direct summation")
    rng = np.random.default_rng(23)
    for _ in range(300):
        i = int(rng.integers(0, 3))
        h, w = wins[i]
        k, l = int(rng.integers(0, H - h + 1)), int(rng.integers(0, W - w + 1))
        got = int(to_host(outs[i][k, l:l + 1])[0])
        assert got == int(img_np[k:k + h, l:l + w].sum(dtype=np.int64)), (h, k, l)


# ------------------------------------------------------------------ banded (out-of-core) window sums

@pytest.mark.parametrize("band_rows", [1, 50, 333, 5000])
def test_banded_window_sums_match_oracle(band_rows):
    from paper_2410_16291_amd import banded
    rng = np.random.default_rng(24)
    img_np = rng.integers(0, 256, (1001, 700)).astype(np.uint8)
    ref_S = oracle.sat(img_np)
    wins = [(7, 5), (64, 64), (100, 300)]
    for s in (1, 3):
        print("case: banded", band_rows, s, flush=True)
        outs = banded.banded_window_sums(lambda r0, r1: img_np[r0:r1], 1001, 700, wins, s, pixel_type="u8",
                                         band_rows=band_rows)
        for (h, w), o in zip(wins, outs):
            assert np.array_equal(o.astype(np.uint64), oracle.window_sum_sat(ref_S, h, w, s)), (band_rows, h, w, s)


def test_banded_u16_from_device_rows():
    from paper_2410_16291_amd import banded
    img = synth.lognormal_u16_device(3000, 257, 25, "cuda:0")
    img_np = to_host(img)
    wins = [(16, 16), (120, 7)]
    outs = banded.banded_window_sums(lambda r0, r1: img[r0:r1], 3000, 257, wins, 2, pixel_type="u16",
                                     band_rows=512)
    ref_S = oracle.sat(img_np)
    for (h, w), o in zip(wins, outs):
        assert np.array_equal(o.astype(np.uint64), oracle.window_sum_sat(ref_S, h, w, 2)), (h, w)


def test_batched_build_every_variant_with_squares():
    """Every build variant, squared table included, over one batch (the split variants run a
    second pass from a second descriptor table)."""
    from paper_2410_16291_amd import batch
    imgs_np = synth.uneven_batch(6, lo=60, hi=900, seed=26)
    imgs = [to_device(i) for i in imgs_np]
    refs = [oracle.sat(i, squares=True) for i in imgs_np]
    for name in api.variants(0, "u16", True):
        print("case: batched build", name, flush=True)
        tables = batch.build_batched(imgs, True, variant=name)
        torch.cuda.synchronize()
        for i, (ref_S, ref_Q) in enumerate(refs):
            assert np.array_equal(to_host(tables[i][0]), ref_S), (name, i)
            assert np.array_equal(to_host(tables[i][1]), ref_Q), (name, i)
