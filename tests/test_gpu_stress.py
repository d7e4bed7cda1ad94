"""The column lookback under perturbed timing: with a stress seed set (sat_force_variant kind 3),
every build sleeps a pseudo-random time before each lookback publication (and each fused ready
count), so strips publish their aggregates and prefixes, and finish, in an order that differs
from the unperturbed run and between seeds.  Every table must still be bit-exact against the
oracle and no wait may hit its bound (sat_workspace_check).  Covers the single-image build plans,
a tall image built in several rounds of strips, band builds seeded with carries, batches, the
fused batched tables and statistics, and the tables of pixel powers."""
import numpy as np
import pytest
import torch

import oracle
from paper_2410_16291_amd import api, batch, synth
from gpu_util import to_device, to_host

pytestmark = pytest.mark.gpu

SEEDS = [0x5eed1, 0x2b3c4d]


@pytest.fixture
def stress(request):
    def set_seed(seed):
        api.force_variant(3, seed)
    yield set_seed
    api.force_variant(3, 0)


def image(H, W, dtype, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 256 if dtype == np.uint8 else 65536, (H, W)).astype(dtype)


def aligned(img_np):
    H, W = img_np.shape
    tdt = torch.uint8 if img_np.dtype == np.uint8 else torch.uint16
    img = api.empty_image(H, W, tdt, "cuda:0")
    img.copy_(to_device(img_np))
    return img


@pytest.mark.parametrize("seed", SEEDS)
@pytest.mark.parametrize("H,W,dtype,squares", [(16000, 4096, np.uint8, False), (2000, 4096, np.uint8, False),
                                               (12000, 1000, np.uint16, True), (300, 40000, np.uint8, False),
                                               (33001, 3000, np.uint8, False), (9001, 777, np.uint16, True)])
def test_stressed_single_builds(stress, seed, H, W, dtype, squares):
    print("case: stressed build", H, W, np.dtype(dtype).name, squares, hex(seed), flush=True)
    img_np = image(H, W, dtype, seed ^ H)
    stress(seed)
    for img in (aligned(img_np), to_device(img_np)):          # helper plans, and the packed-row plans
        ws = torch.empty(api.build_workspace_bytes(H, W, np.dtype(dtype).itemsize, squares), dtype=torch.uint8,
                         device="cuda:0")
        res = api.sat_build(img, squares=squares, ws=ws)
        api.workspace_check(ws)
        ref = oracle.sat(img_np, squares=squares)
        got = res if squares else (res,)
        for g, r in zip(got, ref if squares else (ref,)):
            assert np.array_equal(to_host(g), r), (H, W, seed)


@pytest.mark.parametrize("seed", SEEDS)
def test_stressed_band_builds(stress, seed):
    print("case: stressed band builds", hex(seed), flush=True)
    img_np = image(5000, 2500, np.uint16, seed)
    img = to_device(img_np)
    ref_S, ref_Q = oracle.sat(img_np, squares=True)
    stress(seed)
    carry = carry_q = None
    for r0, r1 in ((0, 1700), (1700, 1701), (1701, 5000)):
        S, Q, T, TQ = api.sat_build_band(img[r0:r1], squares=True, carry=carry, carry_sq=carry_q, rows_above=r0)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(S), ref_S[r0:r1]) and np.array_equal(to_host(Q), ref_Q[r0:r1]), (r0, r1)
        carry, carry_q = T, TQ


@pytest.mark.parametrize("seed", SEEDS)
def test_stressed_batches_and_fused(stress, seed):
    print("case: stressed batches", hex(seed), flush=True)
    imgs_np = synth.uneven_batch(9, lo=50, hi=1500, seed=seed & 0xffff)
    imgs = [to_device(i) for i in imgs_np]
    stress(seed)
    tables = batch.build_batched(imgs, True)
    api.workspace_check(api.workspace(0, imgs[0].device))
    tables2, outs = batch.build_stats_batched(imgs, 40, 40, 4)
    api.workspace_check(api.workspace(0, imgs[0].device))
    for i, img_np in enumerate(imgs_np):
        ref_S, ref_Q = oracle.sat(img_np, squares=True)
        for S, Q in (tables[i], tables2[i]):
            assert np.array_equal(to_host(S), ref_S) and np.array_equal(to_host(Q), ref_Q), (seed, i)
        sums = oracle.window_sum_sat(ref_S, 40, 40, 4)
        ref_mean, _ = oracle.mean_std(sums, oracle.window_sum_sat(ref_Q, 40, 40, 4), 1600)
        assert np.array_equal(to_host(outs[i][0]), sums) and np.array_equal(to_host(outs[i][1]), ref_mean), (seed, i)


@pytest.mark.parametrize("seed", SEEDS)
def test_stressed_power_tables(stress, seed):
    print("case: stressed power tables", hex(seed), flush=True)
    img_np = image(3000, 2100, np.uint8, seed)
    stress(seed)
    tabs = api.sat_build_powers(to_device(img_np), 4)
    torch.cuda.synchronize()
    for p, t in enumerate(tabs, start=1):
        assert np.array_equal(to_host(t), oracle.sat_power(img_np, p)), (seed, p)


def test_stress_seed_reaches_the_kernels(stress):
    """The delays are real: a stressed build takes clearly longer than the same build without."""
    from paper_2410_16291_amd import autotune
    img = aligned(image(16000, 4096, np.uint8, 7))
    ws = torch.empty(api.build_workspace_bytes(16000, 4096, 1, False), dtype=torch.uint8, device="cuda:0")
    S = api.empty_table(16000, 4096, "cuda:0")
    plain = autotune.time_ms(lambda: api.sat_build(img, sat=S, ws=ws), reps=5)
    stress(SEEDS[0])
    slow = autotune.time_ms(lambda: api.sat_build(img, sat=S, ws=ws), reps=5)
    print("case: stress timing, plain %.3f ms, stressed %.3f ms" % (plain, slow), flush=True)
    assert slow > 1.3 * plain
