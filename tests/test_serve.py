"""Scheduling of the serving loop, driven on the CPU by a simulated executor and clock."""
import math

import pytest

from paper_2410_16291_amd import synth
from paper_2410_16291_amd.serve import Arena, Server, image_id, percentile


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def idle(self):
        self.t += 2e-4


class FakeExecutor:
    """Builds take 4 ms per Mpx, queries 1 ms per Mpx of table; slots run concurrently.  Checks
    that the arena blocks the server hands out lie inside the reserved region and that no two
    blocks in use overlap."""

    def __init__(self, clock):
        self.clock = clock
        self.tables = {}
        self.log = []            # (event, image id, request index or None)
        self.waited = 0
        self.freed = []
        self.size = None
        self.blocks = {}         # offset -> (end, owner) of the blocks in use

    def reserve(self, nbytes):
        self.size = nbytes

    def _take(self, off, n, owner):
        assert self.size is not None and 0 <= off and off + n <= self.size and off % Arena.ALIGN == 0
        for o, (e, _) in self.blocks.items():
            assert off + n <= o or e <= off, "blocks overlap"
        self.blocks[off] = (off + n, owner)

    def _give(self, owner):
        for o in [o for o, (_, w) in self.blocks.items() if w == owner]:
            del self.blocks[o]

    def table_bytes(self, H, W):
        return H * W * 8

    def prefetch(self, reqs):
        self.prefetched = getattr(self, "prefetched", []) + [image_id(r) for r in reqs]

    def image_ready(self, req):
        return image_id(req) in getattr(self, "prefetched", [])

    def build_transient_bytes(self, H, W):
        return H * W

    def query_transient_bytes(self, req, r):
        h, w = min(req.win_h, r.H), min(req.win_w, r.W)
        return ((r.H - h) // req.stride + 1) * ((r.W - w) // req.stride + 1) * 4

    def start_build(self, req, r, slot, block):
        end = self.clock() + 4e-3 * req.H * req.W / 1e6
        r.tables = ("table", image_id(req))
        self._take(r.offset, self.table_bytes(req.H, req.W), ("table", image_id(req)))
        h = {"end": end, "req": req}
        self._take(block, self.build_transient_bytes(req.H, req.W), id(h))
        self.log.append(("build", image_id(req), self.clock()))
        return h

    def finish_build(self, h):
        self._give(id(h))

    def start_query(self, req, r, slot, after, block):
        assert r.tables == ("table", image_id(req)), "query started on a table that is not there"
        start = self.clock()
        if after is not None:
            self.waited += 1
            start = max(start, after["end"])
        end = start + 1e-3 * r.H * r.W / 1e6
        self.log.append(("query", image_id(req), self.clock()))
        h = {"end": end, "req": req, "after": after}
        self._take(block, self.query_transient_bytes(req, r), id(h))
        return h

    def is_done(self, h):
        return self.clock() >= h["end"] - 1e-12

    def finish_query(self, h, keep):
        self._give(id(h))
        req = h["req"]
        return (image_id(req), req.win_h, req.win_w, req.stride, req.op) if keep else None

    def free(self, r):
        self.freed.append(r.image_id)
        self._give(("table", r.image_id))
        r.tables = None


def stream(rate=400.0, duration=1.0, seed=5, lo=200, hi=1500):
    return synth.request_stream(rate=rate, duration=duration, seed=seed, side_lo=lo, side_hi=hi, win_lo=8, win_hi=64)


def serve(reqs, budget=200e9, slots=4, keep=False):
    clock = Clock()
    ex = FakeExecutor(clock)
    srv = Server(ex, budget_bytes=budget, slots=slots, keep_results=keep)
    rep = srv.run(reqs, clock=clock, idle=clock.idle)
    return srv, ex, rep


def test_percentile():
    assert percentile([3.0, 1.0, 2.0], 0.5) == 2.0
    assert percentile([1.0, 2.0], 0.99) == pytest.approx(1.99)
    assert math.isnan(percentile([], 0.5))


def test_every_request_completes_with_sane_latency():
    reqs = stream()
    srv, ex, rep = serve(reqs, keep=True)
    assert rep.n == len(reqs)
    assert sorted(j.idx for j in srv.done) == list(range(len(reqs)))
    for j in srv.done:
        assert j.t_done >= j.t_arrival and j.t_admit >= j.t_arrival
        if j.req.kind == "query":
            assert j.result[0] == image_id(j.req)
    lat = rep.latency_ms
    assert lat["all"]["n"] == len(reqs)
    assert lat["query"]["p99"] >= lat["query"]["p50"] > 0
    assert rep.misses == 0 and rep.evictions == 0


def test_builds_are_admitted_in_arrival_order():
    reqs = stream(rate=2000.0, duration=0.3)
    srv, ex, rep = serve(reqs, budget=40e6, slots=3)
    admits = sorted((j.t_admit, j.idx) for j in srv.done if j.req.kind == "build")
    idxs = [i for _, i in admits]
    assert idxs == sorted(idxs)


def test_budget_is_respected_with_evictions_and_rebuilds():
    reqs = stream(rate=800.0, duration=1.0)
    budget = 60e6
    srv, ex, rep = serve(reqs, budget=budget, slots=4)
    assert rep.n == len(reqs)
    assert rep.peak_bytes <= budget
    assert rep.evictions > 0 and rep.misses > 0
    assert set(ex.freed) <= {image_id(r) for r in reqs if r.kind == "build"}


def test_query_overlaps_the_build_of_its_image():
    reqs = [synth.Request(0.0, "build", image_seed=1000, H=1000, W=1000),
            synth.Request(0.0, "query", image_seed=0, win_h=10, win_w=10, stride=1)]
    srv, ex, rep = serve(reqs)
    assert ex.waited == 1                                  # admitted while the build was in flight
    b = next(j for j in srv.done if j.req.kind == "build")
    q = next(j for j in srv.done if j.req.kind == "query")
    assert q.t_admit <= b.t_done and q.t_done >= b.t_done


def test_slots_bound_concurrency():
    reqs = [synth.Request(0.0, "build", image_seed=1000 + k, H=500, W=500) for k in range(10)]
    srv, ex, rep = serve(reqs, slots=3)
    assert rep.max_in_flight == 3
    srv, ex, rep = serve(reqs, slots=1)
    assert rep.max_in_flight == 1


def test_tight_budget_does_not_deadlock():
    # room for one table at a time: every query behind another image's build forces an eviction
    reqs = []
    for k in range(4):
        reqs.append(synth.Request(0.001 * k, "build", image_seed=1000 + k, H=1000, W=1000))
    for k in range(4):
        reqs.append(synth.Request(0.01 + 0.001 * k, "query", image_seed=3 - k, win_h=5, win_w=5, stride=1))
    srv, ex, rep = serve(reqs, budget=1000 * 1000 * 8 + 1000 * 1000 + 4 * 1000 * 1000, slots=2)
    assert rep.n == len(reqs)
    assert rep.peak_bytes <= 1000 * 1000 * 8 + 1000 * 1000 + 4 * 1000 * 1000
    assert rep.misses == 2           # images 1 and 0 were evicted; image 3 waits for its own build


def test_oversized_image_is_refused():
    reqs = [synth.Request(0.0, "build", image_seed=1000, H=2000, W=2000)]
    with pytest.raises(ValueError):
        serve(reqs, budget=1e6)


def test_builds_wait_for_their_images_and_prefetch_covers_the_stream():
    """A build is admitted only once its image is ready (host data prepared ahead), in arrival
    order; rebuilds after eviction ask for their image again; executor calls are timed."""
    clock = Clock()
    ex = FakeExecutor(clock)
    reqs = synth.request_stream(rate=200.0, duration=0.5, seed=9, side_lo=100, side_hi=400)
    srv = Server(ex, budget_bytes=4e6, slots=2)
    rep = srv.run(reqs, clock=clock, idle=clock.idle)
    builds = [image_id(r) for r in reqs if r.kind == "build"]
    assert ex.prefetched[:len(builds)] == builds                 # the whole stream, in arrival order
    assert len(ex.prefetched) == len(builds) + rep.misses        # one more per rebuild
    assert set(rep.host_call_ms) >= {"image_ready", "start_build", "is_done"}


def test_builds_wait_for_late_images_without_a_budget_error():
    """Images that become ready only after several scheduler passes (a slow producer) delay their
    builds; the loop keeps idling instead of reporting a memory deadlock."""
    clock = Clock()

    class SlowImages(FakeExecutor):
        def image_ready(self, req):
            self.asked = getattr(self, "asked", {})
            self.asked[image_id(req)] = self.asked.get(image_id(req), 0) + 1
            return super().image_ready(req) and self.asked[image_id(req)] > 5

    ex = SlowImages(clock)
    reqs = synth.request_stream(rate=100.0, duration=0.3, seed=10, side_lo=100, side_hi=300)
    rep = Server(ex, budget_bytes=50e6, slots=2).run(reqs, clock=clock, idle=clock.idle)
    assert rep.n == len(reqs)


def test_arena_placement_against_a_byte_map():
    """Random placements and releases: every block lies inside the region, no two live blocks
    overlap, free runs are merged (their count never exceeds live blocks + 1) and the free bytes
    add up; fits() agrees with what alloc() then does."""
    import random
    rnd = random.Random(7)
    size = 1 << 20
    a = Arena(size)
    used = bytearray(size // Arena.ALIGN)
    live = {}
    for step in range(4000):
        if live and (rnd.random() < 0.45 or a.largest_free < Arena.ALIGN):
            off = rnd.choice(sorted(live))
            n = live.pop(off)
            a.release(off)
            for k in range(off // Arena.ALIGN, (off + n) // Arena.ALIGN):
                assert used[k] == 1
                used[k] = 0
        else:
            want = rnd.choice([1, 255, 256, 257, 3000, 20000, 65536, 200000])
            ok = a.fits([want])
            off = a.alloc(want)
            assert ok == (off is not None)
            if off is None:
                assert a.largest_free < Arena.rounded(want)
                continue
            n = Arena.rounded(want)
            assert off % Arena.ALIGN == 0 and off + n <= size
            for k in range(off // Arena.ALIGN, (off + n) // Arena.ALIGN):
                assert used[k] == 0, "blocks overlap"
                used[k] = 1
            live[off] = n
        assert a.free_bytes == (len(used) - sum(used)) * Arena.ALIGN
        assert len(a.starts) <= len(live) + 1
        for i in range(len(a.starts) - 1):
            assert a.starts[i] + a.lens[i] < a.starts[i + 1]     # sorted, disjoint, never adjacent
    for off in list(live):
        a.release(off)
    assert a.starts == [0] and a.lens == [size]


def test_arena_fits_places_several_blocks_in_order():
    a = Arena(10 * 256)
    x = a.alloc(3 * 256)
    a.alloc(256)
    a.release(x)                                   # free runs: 3 blocks at 0, 6 blocks at 4
    assert a.fits([3 * 256, 6 * 256])
    assert not a.fits([4 * 256, 4 * 256])
    assert a.alloc(2 * 256) == 0                   # best fit: the smaller run
    assert a.alloc(5 * 256) == 4 * 256


def test_no_allocation_when_served_through_the_arena():
    """Under a budget that forces evictions, every table and transient block the executor is handed
    lies in the reserved region and none overlaps another in use (FakeExecutor checks both)."""
    reqs = stream(rate=800.0, duration=1.0, seed=11)
    srv, ex, rep = serve(reqs, budget=50e6, slots=4)
    assert rep.n == len(reqs) and rep.evictions > 0
    assert ex.size == srv.arena.size
    assert rep.peak_bytes <= srv.arena.size


def test_a_query_never_evicts_its_own_table():
    """A query whose outputs cannot be placed beside its own table makes room from other tables
    only (the table it reads stays); one whose outputs could never fit beside it is refused."""
    build = synth.Request(0.0, "build", image_seed=1000, H=1000, W=1000)
    other = synth.Request(0.0, "build", image_seed=1001, H=300, W=300)
    small = synth.Request(0.05, "query", image_seed=0, win_h=990, win_w=990, stride=1)
    big = synth.Request(0.06, "query", image_seed=0, win_h=2, win_w=2, stride=1)
    budget = 1000 * 1000 * 8 + 1000 * 1000 + 300 * 300 * 8 + 4096
    srv, ex, rep = serve([build, other, small], budget=budget, slots=2)
    assert rep.n == 3 and rep.misses == 0
    with pytest.raises(ValueError, match="do not fit"):
        serve([build, other, small, big], budget=budget, slots=2)


def test_a_table_that_splits_the_free_space_is_rebuilt_for_its_query():
    """The only resident table sits between two free runs, neither of which holds the query's
    outputs: with nothing in flight the table is given up and rebuilt (a miss), and the query is
    then served from the rebuilt table."""
    clock = Clock()
    ex = FakeExecutor(clock)
    a = synth.Request(0.0, "build", image_seed=1000, H=1000, W=1000)
    q = synth.Request(0.5, "query", image_seed=0, win_h=2, win_w=2, stride=1)
    budget = 8_000_000 + 3_000_000 + 3_500_000
    srv = Server(ex, budget_bytes=budget, slots=1)
    srv.builds[0] = a
    from paper_2410_16291_amd.serve import Resident
    # place the table in the middle by hand: 3 MB free below it, 3.5 MB above
    off = srv.arena.alloc(3_000_000)
    r = Resident(0, 1000, 1000, Arena.rounded(8_000_000), offset=srv.arena.alloc(8_000_000), state="resident")
    srv.arena.release(off)
    ex.reserve(srv.arena.size)
    ex._take(r.offset, 8_000_000, ("table", 0))
    r.tables = ("table", 0)
    srv.res[0] = r
    srv.used = r.nbytes
    assert not srv.arena.fits([ex.query_transient_bytes(q, r)])
    rep = srv.run([q], clock=clock, idle=clock.idle)
    assert rep.n == 1 and rep.misses == 1 and rep.evictions == 1


def test_cyclic_gc_is_paused_and_switch_interval_shortened_during_the_loop():
    import gc
    import sys
    seen = []

    class Watch(FakeExecutor):
        def is_done(self, h):
            seen.append((gc.isenabled(), sys.getswitchinterval()))
            return super().is_done(h)

    clock = Clock()
    assert gc.isenabled()
    before = sys.getswitchinterval()
    Server(Watch(clock), budget_bytes=200e9, slots=2).run(stream(duration=0.2), clock=clock, idle=clock.idle)
    assert seen and not any(on for on, _ in seen)
    assert all(abs(iv - Server.SWITCH_INTERVAL) < 1e-9 for _, iv in seen)
    assert gc.isenabled() and sys.getswitchinterval() == before


def test_arena_cuts_long_lived_blocks_from_the_top():
    """Tables (top=True) pack towards the region's end and transients towards its start, so the
    free space between them stays in one piece."""
    a = Arena(64 * 256)
    t1 = a.alloc(8 * 256, top=True)
    x = a.alloc(4 * 256)
    t2 = a.alloc(8 * 256, top=True)
    assert t1 == 56 * 256 and t2 == 48 * 256 and x == 0
    a.release(x)
    assert a.largest_free == 48 * 256                  # one run below the two tables
    a.release(t1)
    assert a.starts == [0, 56 * 256] and a.lens == [48 * 256, 8 * 256]
    a.release(t2)
    assert a.starts == [0] and a.lens == [64 * 256]
