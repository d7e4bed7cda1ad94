"""sat_upload: host-to-device copies by a kernel reading pinned host memory, byte for byte."""
import numpy as np
import pytest
import torch

from paper_2410_16291_amd import _lib, api
from paper_2410_16291_amd._lib import SAT_ERR_ARG

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [1, 15, 16, 17, 4095, 4096 * 256 + 7, (64 << 20) + 3, 16000 * 16000])
def test_upload_is_exact(nbytes):
    print("case: upload", nbytes, flush=True)
    rng = np.random.default_rng(nbytes)
    host = torch.empty(nbytes + 64, dtype=torch.uint8, pin_memory=True)
    host.numpy()[:] = rng.integers(0, 256, nbytes + 64, dtype=np.uint8)
    dst = torch.full((nbytes + 64,), 0xA5, dtype=torch.uint8, device="cuda:0")
    s = torch.cuda.Stream()
    api.upload(host[16:16 + nbytes], dst[32:32 + nbytes], stream=s)
    s.synchronize()
    got = dst.cpu().numpy()
    assert np.array_equal(got[32:32 + nbytes], host.numpy()[16:16 + nbytes])
    assert np.all(got[:32] == 0xA5) and np.all(got[32 + nbytes:] == 0xA5)      # nothing outside dst


def test_uploads_on_several_streams_at_once():
    n = 48 << 20
    hosts = [torch.randint(0, 256, (n,), dtype=torch.uint8).pin_memory() for _ in range(4)]
    dsts = [torch.empty(n, dtype=torch.uint8, device="cuda:0") for _ in range(4)]
    streams = [torch.cuda.Stream() for _ in range(4)]
    for h, d, s in zip(hosts, dsts, streams):
        api.upload(h, d, stream=s)
    torch.cuda.synchronize()
    for h, d in zip(hosts, dsts):
        assert torch.equal(d.cpu(), h)


def test_pageable_host_memory_is_refused_and_leaves_no_error():
    host = torch.zeros(4096, dtype=torch.uint8)                 # not pinned
    dst = torch.empty(4096, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(ValueError):
        api.upload(host, dst)
    st = _lib.load().sat_upload(host.data_ptr(), dst.data_ptr(), 4096, None)
    assert st == SAT_ERR_ARG and "pinned" in _lib.load().sat_last_error().decode()
    x = torch.arange(1000, device="cuda:0").sum()               # the runtime is still healthy
    torch.cuda.synchronize()
    assert int(x) == 499500
