"""Builds that keep their lookback state in 32-bit words (no squared table, every column total
below 2^30) against the oracle's tables: batches of 8- and 16-bit images over every build
variant, the largest column totals the 32-bit words may hold and the first that may not (16-bit
images of 16383 and 16385 rows of 65535), a batch with one image too tall for them (every image
then keeps 64-bit words), and band builds whose carries approach the bound.  Also under the
lookback stress seed (pseudo-random delays before every publication).  Tables must be bit-exact
and every fault word clear."""
import numpy as np
import pytest
import torch

import oracle
from paper_2410_16291_amd import api, batch, synth
from gpu_util import to_device, to_host

pytestmark = pytest.mark.gpu


def batch_images(dtype, seed):
    imgs = synth.uneven_batch(7, lo=50, hi=1500, seed=seed)
    return [i if dtype == np.uint16 else (i & 0xff).astype(np.uint8) for i in imgs]


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_batched_without_squares_every_variant(dtype):
    imgs_np = batch_images(dtype, 41)
    imgs = [to_device(i) for i in imgs_np]
    refs = [oracle.sat(i) for i in imgs_np]
    for name in api.variants(0, "u8" if dtype == np.uint8 else "u16", False):
        print("case: batched S-only build", np.dtype(dtype).name, name, flush=True)
        tables = batch.build_batched(imgs, False, variant=name)
        api.workspace_check(api.workspace(0, imgs[0].device))
        for i, ((S, _), ref) in enumerate(zip(tables, refs)):
            assert np.array_equal(to_host(S), ref), (name, i)


@pytest.mark.parametrize("H", [16383, 16385])
def test_column_totals_at_the_32_bit_bound(H):
    """A column of 65535s: 16383 rows total 2^30 - 65537 (32-bit words), 16385 rows exceed 2^30
    (64-bit words).  Both tables exact, on the helper plan and on the packed-row plan."""
    W = 700
    img_np = np.random.default_rng(H).integers(0, 65536, (H, W)).astype(np.uint16)
    img_np[:, 5] = 65535
    img_np[:, W - 1] = 65535
    ref = oracle.sat(img_np)
    for img in (to_device(img_np), None):
        if img is None:
            img = api.empty_image(H, W, torch.uint16, "cuda:0")
            img.copy_(to_device(img_np))
        print("case: 32-bit bound", H, img.stride(0), flush=True)
        ws = torch.empty(api.build_workspace_bytes(H, W, 2, False), dtype=torch.uint8, device="cuda:0")
        S = api.sat_build(img, ws=ws)
        api.workspace_check(ws)
        assert np.array_equal(to_host(S), ref), H


def test_batch_with_one_image_too_tall_for_32_bit_words():
    imgs_np = batch_images(np.uint16, 43)[:4]
    tall = np.random.default_rng(3).integers(60000, 65536, (17000, 90)).astype(np.uint16)
    imgs_np.insert(2, tall)
    imgs = [to_device(i) for i in imgs_np]
    tables = batch.build_batched(imgs, False)
    api.workspace_check(api.workspace(0, imgs[0].device))
    for i, ((S, _), img_np) in enumerate(zip(tables, imgs_np)):
        assert np.array_equal(to_host(S), oracle.sat(img_np)), i


@pytest.mark.parametrize("stress", [0, 0x5eed7])
def test_band_builds_without_squares(stress):
    """8-bit bands (32-bit words throughout) and 16-bit bands whose rows above pass 16384 (32-bit
    words for the first bands, 64-bit after), each seeded with the carried totals."""
    try:
        api.force_variant(3, stress)
        for dtype, H, W, cuts in ((np.uint8, 6000, 2600, (0, 1500, 1501, 6000)),
                                  (np.uint16, 20000, 900, (0, 8000, 16000, 20000))):
            img_np = np.random.default_rng(H).integers(0, 256 if dtype == np.uint8 else 65536, (H, W)).astype(dtype)
            img = to_device(img_np)
            ref = oracle.sat(img_np)
            carry = None
            for r0, r1 in zip(cuts, cuts[1:]):
                print("case: S-only band", np.dtype(dtype).name, r0, r1, hex(stress), flush=True)
                ws = torch.empty(api.build_workspace_bytes(r1 - r0, W, np.dtype(dtype).itemsize, False),
                                 dtype=torch.uint8, device="cuda:0")
                S, T = api.sat_build_band(img[r0:r1], carry=carry, rows_above=r0, ws=ws)
                api.workspace_check(ws)
                assert np.array_equal(to_host(S), ref[r0:r1]), (r0, r1)
                carry = T
            assert np.array_equal(to_host(carry), oracle.column_totals(img_np))
    finally:
        api.force_variant(3, 0)


def test_stressed_batch_without_squares():
    imgs_np = batch_images(np.uint8, 47)
    imgs = [to_device(i) for i in imgs_np]
    try:
        api.force_variant(3, 0x2b3c5)
        tables = batch.build_batched(imgs, False)
        api.workspace_check(api.workspace(0, imgs[0].device))
    finally:
        api.force_variant(3, 0)
    for i, ((S, _), img_np) in enumerate(zip(tables, imgs_np)):
        assert np.array_equal(to_host(S), oracle.sat(img_np)), i
