"""libsat.so driven through its C ABI alone: a host program (tests/c_abi/capi_check.cpp, built by
__graft_entry__.build()) allocates with the HIP runtime, calls sat_build, window_sum,
window_sum_multi and window_mean_std from include/sat.h on an image with unaligned rows, then
builds the same table in two bands (sat_column_totals, sat_build_band), and writes the results;
they must match the oracle (integers bit-exact, the mean bit-exact, the std within 1e-12
relative)."""
import os
import subprocess

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "capi_check")


def image(H, W):
    y = np.arange(H, dtype=np.int64)[:, None]
    x = np.arange(W, dtype=np.int64)[None, :]
    return ((y * 131 + x * 71 + (x * y) % 17) % 256).astype(np.uint8)


def test_c_abi_program_matches_oracle(tmp_path):
    if not os.path.exists(EXE):
        pytest.fail("tests/c_abi/capi_check is not built: run __graft_entry__.build()")
    H, W = 157, 211
    out = tmp_path / "capi.bin"
    print("case: C-ABI program", H, W, flush=True)
    r = subprocess.run([EXE, str(H), str(W), str(out)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    raw = out.read_bytes()
    img = image(H, W)
    S, Q = oracle.sat(img, squares=True)
    ref_sum = oracle.window_sum_sat(S, 7, 5, 2)
    ref_m = [oracle.window_sum_sat(S, h, h, 1) for h in (3, 9)]
    ref_s1 = oracle.window_sum_sat(S, 4, 6, 3)
    ref_mean, ref_std = oracle.mean_std(ref_s1, oracle.window_sum_sat(Q, 4, 6, 3), 24)
    pos = 0

    def take(dtype, shape):
        nonlocal pos
        n = int(np.prod(shape)) * np.dtype(dtype).itemsize
        a = np.frombuffer(raw, dtype, count=int(np.prod(shape)), offset=pos).reshape(shape)
        pos += n
        return a

    assert np.array_equal(take(np.uint64, S.shape), S)
    assert np.array_equal(take(np.uint64, Q.shape), Q)
    assert np.array_equal(take(np.uint32, ref_sum.shape).astype(np.uint64), ref_sum)
    for ref in ref_m:
        assert np.array_equal(take(np.uint32, ref.shape).astype(np.uint64), ref)
    assert np.array_equal(take(np.uint64, ref_s1.shape), ref_s1)
    assert np.array_equal(take(np.float64, ref_mean.shape), ref_mean)
    std = take(np.float64, ref_std.shape)
    nz = ref_std > 0
    assert np.all(std[~nz] == 0.0)
    assert np.max(np.abs(std[nz] - ref_std[nz]) / ref_std[nz]) <= 1e-12
    h1 = H // 2
    assert np.array_equal(take(np.uint64, S.shape), S)                        # table from two bands
    upper = oracle.column_totals(img[:h1])
    assert np.array_equal(take(np.uint64, (W,)), upper)                       # upper band's totals output
    assert np.array_equal(take(np.uint64, (W,)), upper)                       # sat_column_totals
    assert np.array_equal(take(np.uint64, (W,)), oracle.column_totals(img))   # advanced in place
    assert pos == len(raw)
