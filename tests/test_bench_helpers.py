"""bench.py's byte accounting and its reading of the committed traffic summary (CPU only)."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def touched_entries(H, W, hs):
    """Distinct table entries the four-corner lookups of all square windows (stride 1) read."""
    seen = np.zeros((H, W), bool)
    for h in hs:
        oh, ow = H - h + 1, W - h + 1
        for y0 in range(oh):
            for x0 in range(ow):
                y1, x1 = y0 + h - 1, x0 + h - 1
                for y, x in ((y1, x1), (y0 - 1, x1), (y1, x0 - 1), (y0 - 1, x0 - 1)):
                    if y >= 0 and x >= 0:
                        seen[y, x] = True
    return int(seen.sum())


@pytest.mark.parametrize("H,W,hs", [(9, 7, (1,)), (9, 7, (3,)), (9, 7, (7, 5)), (12, 15, (2, 5)), (6, 6, (6,)),
                                    (20, 11, (4, 10))])
def test_window_bytes_count_every_touched_entry_once(H, W, hs):
    outs = sum((H - h + 1) * (W - h + 1) for h in hs)
    assert bench.alg_bytes_windows(H, W, hs) == touched_entries(H, W, hs) * 8 + outs * 4


def test_build_bytes():
    assert bench.alg_bytes_build(70000, 85000) == 70000 * 85000 * 9


def test_traffic_only_for_the_profiled_source(tmp_path, monkeypatch):
    digest = bench.source_digest(bench.GATHER_SRC)
    f = tmp_path / "t.md"
    f.write_text("kernel_source_sha256: %s\ntraffic_bytes_per_launch: 1.5e+11\nworkload_rows_cols: 70000x85000\n"
                 % digest)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.committed_traffic(70000, 85000) == 1.5e11
    assert bench.committed_traffic(1000, 1000) is None                     # another workload
    f.write_text("kernel_source_sha256: %s\ntraffic_bytes_per_launch: 1.5e+11\nworkload_rows_cols: 70000x85000\n"
                 % ("0" * 64))
    assert bench.committed_traffic(70000, 85000) is None                   # kernel changed since


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
