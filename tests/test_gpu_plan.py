"""Every branch of the built-in build plan for one image with 16-byte aligned rows, against the
oracle's tables (needs an MI355X with 256 compute units, the device the plan is measured on).

The plan picks the helper-wave variant and its strip height from the image shape: eight pixels
per lane at 48-row strips split into column segments for images of at most 4096 rows, in one
round of the shortest strips that fit on the CUs (24 to 48 rows) above that, or in heights
balanced over rounds for taller images; four pixels per lane at one 64-row strip per CU; and four
pixels per lane at 32, 48 or 64 rows (or balanced heights) for narrow images and 16-bit images
with squares.  Above 4096 rows, strips at their least height (half a tile) are split into three
column segments.  Images take the three-stage
helper pipeline where its three tile buffers fit the LDS, except images wider than 32768 pixels
with more than two rounds of 48-row strips; those, and 16-bit images at eight pixels per lane, take
the two-stage one.  Each case below lands in one branch; widths that are not a multiple of the block
width end in a ragged block.  Tables must be bit-exact.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2410_16291_amd import api
from gpu_util import to_host

pytestmark = pytest.mark.gpu

CASES = [
    # (H, W, pixel dtype, squares, branch)
    (2000, 4096, np.uint8, False, "8 px/lane, 24-row strips (few strips)"),
    (3200, 4100, np.uint8, True, "8 px/lane, 48-row strips split into column segments, ragged last block, with squares"),
    (5000, 4200, np.uint8, False, "8 px/lane, one round of the shortest strips: 24 rows in 3 column segments, ragged"),
    (9000, 4096, np.uint8, False, "8 px/lane, one round of the shortest strips: 36 rows"),
    (16000, 4096, np.uint8, False, "4 px/lane, one 64-row strip per CU"),
    (20000, 4352, np.uint8, False, "8 px/lane, more 48-row strips than CUs: heights balanced over two rounds"),
    (30000, 4096, np.uint8, False, "8 px/lane, heights balanced over three rounds"),
    (9000, 2000, np.uint8, False, "narrow: 4 px/lane, 48-row strips"),
    (7000, 3001, np.uint8, False, "narrow: 4 px/lane, 32-row strips, ragged"),
    (12000, 1000, np.uint16, True, "16-bit with squares: 4 px/lane, 48-row strips"),
    (6000, 1500, np.uint16, True, "16-bit with squares above 4096 rows at 32-row strips: 3 column segments, ragged"),
    (20000, 1000, np.uint16, True, "16-bit with squares: balanced heights"),
    (6000, 5000, np.uint16, False, "16-bit without squares: two-stage helper, 8 px/lane, 48-row strips"),
    (1, 4096, np.uint8, True, "one row: 8 px/lane, one strip"),
    (5, 8200, np.uint16, True, "five rows, 16-bit with squares, ragged"),
    (1, 1, np.uint8, False, "one pixel: narrow, 4 px/lane"),
    (47, 4096, np.uint16, False, "one strip just short of 48 rows"),
    (300, 40000, np.uint8, False, "wider than 32768: three-stage helper, 8 px/lane, 24-row strips"),
    (100, 33000, np.uint16, True, "wider than 32768, 16-bit with squares: three-stage helper, 4 px/lane, ragged"),
    (24700, 33000, np.uint8, False, "wider than 32768, more than two rounds of strips: two-stage helper, balanced heights"),
]


@pytest.mark.parametrize("H,W,dtype,squares,branch", CASES,
                         ids=["%dx%d-%s%s" % (c[0], c[1], np.dtype(c[2]).name, "-sq" if c[3] else "") for c in CASES])
def test_plan_branch_matches_oracle(H, W, dtype, squares, branch):
    print("case: build plan", H, W, np.dtype(dtype).name, "squares" if squares else "", branch, flush=True)
    rng = np.random.default_rng(H + W)
    hi = 256 if dtype == np.uint8 else 65536
    img_np = rng.integers(0, hi, (H, W)).astype(dtype)
    tdt = torch.uint8 if dtype == np.uint8 else torch.uint16
    img = api.empty_image(H, W, tdt, "cuda:0")                 # rows on 128-byte lines
    src = torch.from_numpy(img_np if dtype == np.uint8 else img_np.view(np.int16)).to("cuda:0")
    img.copy_(src if dtype == np.uint8 else src.view(torch.uint16))
    del src
    ws = torch.empty(api.build_workspace_bytes(H, W, np.dtype(dtype).itemsize, squares), dtype=torch.uint8,
                     device="cuda:0")
    res = api.sat_build(img, squares=squares, ws=ws)
    api.workspace_check(ws)
    ref = oracle.sat(img_np, squares=squares)
    if squares:
        assert np.array_equal(to_host(res[0]), ref[0])
        assert np.array_equal(to_host(res[1]), ref[1])
    else:
        assert np.array_equal(to_host(res), ref)
