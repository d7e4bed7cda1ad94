"""The Python binding's per-stream workspace cache (CPU only: torch's allocator and streams are
replaced by recording fakes).  A buffer is allocated on the stream its builds run on, and a
buffer replaced by a larger one is recorded on that stream before it is dropped, so the
allocator cannot hand its memory out while launches that use it are still queued."""
import types

from paper_2410_16291_amd import api


class FakeTensor:
    def __init__(self, n):
        self.n = n
        self.recorded = []

    def numel(self):
        return self.n

    def record_stream(self, s):
        self.recorded.append(s)


def test_workspace_allocates_on_its_stream_and_records_replaced_buffers(monkeypatch):
    current, allocs = [], []

    class StreamCtx:
        def __init__(self, s):
            self.s = s

        def __enter__(self):
            current.append(self.s)

        def __exit__(self, *exc):
            current.pop()

    def fake_empty(n, dtype=None, device=None):
        allocs.append(list(current))
        return FakeTensor(n)

    monkeypatch.setattr(api, "_workspaces", {})
    monkeypatch.setattr(api.torch.cuda, "stream", StreamCtx)
    monkeypatch.setattr(api.torch, "empty", fake_empty)
    dev = types.SimpleNamespace(index=0)
    s1 = types.SimpleNamespace(cuda_stream=11)
    s2 = types.SimpleNamespace(cuda_stream=22)
    a = api.workspace(1000, dev, s1)
    assert api.workspace(500, dev, s1) is a              # cached: large enough
    b = api.workspace(5000, dev, s1)                     # replaced
    assert b is not a and a.recorded == [s1] and b.numel() == 5000
    c = api.workspace(100, dev, s2)                      # another stream: its own buffer
    assert c is not b and c.recorded == [] and b.recorded == []
    assert allocs == [[s1], [s1], [s2]]                  # each allocated inside its stream's context
