"""The multi-core CPU baseline of the benchmark against the oracle (bit-exact tables and sums)."""
import numpy as np
import pytest

import cpu_baseline
import oracle
from paper_2410_16291_amd import synth


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_omp_table_and_windows_match_oracle(threads):
    img = synth.thomas_mask(701, 1333, seed=5, parent_density=2e-5, children=80, sigma=12.0)
    img[::37, ::11] = 255
    S, n = cpu_baseline.sat_u8(img, threads)
    assert n == threads
    ref = oracle.sat(img)
    assert np.array_equal(S, ref)
    for h, w, s in ((1, 1, 1), (100, 100, 1), (250, 17, 3), (701, 1333, 1)):
        out, _ = cpu_baseline.window_sum_u32(S, h, w, s, threads)
        assert np.array_equal(out.astype(np.uint64), oracle.window_sum_sat(ref, h, w, s)), (h, w, s)


def test_omp_more_threads_than_rows_and_padded_rows():
    rng = np.random.default_rng(6)
    buf = rng.integers(0, 256, (5, 300)).astype(np.uint8)
    img = buf[:, 7:290]
    S, n = cpu_baseline.sat_u8(img, 16)
    assert n == 5
    assert np.array_equal(S, oracle.sat(np.ascontiguousarray(img)))
