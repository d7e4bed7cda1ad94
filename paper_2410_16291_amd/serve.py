"""Serving: a request loop over integral images kept resident in HBM.

Requests (synth.Request) are either a build -- a new image whose table is built and kept
resident (the images are 0/1 centroid masks, so the table also serves as the table of squares for
mean/std) -- or a query: the sums, or sums, means and standard deviations, of every window of
one size and stride over a resident image, O(1) per output from its table.

Scheduling is continuous batching, not a queue alone:
  * up to `slots` requests are in flight on the device at once, each on a stream of its own
    (default priority), so their kernels overlap;
  * whenever a slot or memory frees up, waiting requests are admitted in arrival order.  A build
    that cannot be admitted yet (its table does not fit) does not block the queries behind it,
    but no later build overtakes it;
  * admission is by placement in an arena of `budget_bytes`, one device allocation made before
    the stream starts: every resident table, and the transient image, workspace and output bytes
    of each request in flight, is a block of it (Arena).  A request is admitted once its blocks
    can be placed; to make room, the least recently used resident tables that no in-flight or
    imminent query reads are evicted.  No request allocates or frees device memory, so no
    allocator call (and none of the device synchronisation a caching allocator falls back on
    near the memory's end) lands on the scheduler thread;
  * a query may be admitted while its image is still being built: its stream waits for the
    build's completion event on the device, not on the host;
  * a query whose table was evicted rebuilds it first (the image is regenerated from its seed)
    and counts as a miss.

Images arrive as host data: a producer thread (ImageSource) draws each build request's image into
a buffer of a pinned host pool ahead of its arrival, as a client upload would have it ready; the
scheduler admits a build only once its image is ready and copies it to the device asynchronously
on the request's stream, by a kernel that reads the pinned pages (the H2D copy is timed
separately from the build).  No request does host
work on the scheduler thread beyond launching; the longest scheduler-side executor call is
reported.  Python's cyclic garbage collector is paused while the loop runs (after one collection
and a freeze of everything allocated before the stream): a full collection walks every object the
process holds, torch's included, and stopped all threads for tens of milliseconds; the loop's own
objects form no reference cycles and are freed by reference counting.  The interpreter's switch
interval is shortened to 0.2 ms for the loop, so that the producer threads give the lock back to
the scheduler promptly.

Latency runs from a request's arrival to the moment the host observes its completion event.
Results stay on the device; copying them to the host is not part of the latency.

The scheduling logic does not touch the GPU: `Server` drives an executor (GpuExecutor below;
the CPU tests drive a simulated one).
"""
from __future__ import annotations

import bisect
import collections
import dataclasses
import gc
import math
import sys
import threading
import time
from typing import Callable, Dict, List, Optional

from .synth import Request


def image_id(req: Request) -> int:
    """Build requests carry the seed 1000 + k of the k-th image; queries name k directly."""
    return req.image_seed - 1000 if req.kind == "build" else req.image_seed


@dataclasses.dataclass
class Resident:
    image_id: int
    H: int
    W: int
    nbytes: int
    offset: int = -1                   # the table's block in the arena
    state: str = "building"            # "building" or "resident"
    tables: object = None              # executor-owned (device tensors)
    build_job: Optional["Job"] = None
    pins: int = 0                      # in-flight queries reading the table
    last_used: float = 0.0


@dataclasses.dataclass
class Job:
    idx: int                           # position in the request stream (-1: a rebuild after eviction)
    req: Request
    t_arrival: float
    t_admit: float = math.nan
    t_done: float = math.nan
    slot: int = -1
    handle: object = None
    transient: int = 0                 # bytes held while in flight
    block: int = -1                    # their block in the arena
    result: object = None
    miss: bool = False
    waiting_on: Optional["Job"] = None  # a query behind the (re)build of its image


def percentile(xs: List[float], q: float) -> float:
    if not xs:
        return math.nan
    s = sorted(xs)
    k = (len(s) - 1) * q
    lo, hi = int(math.floor(k)), int(math.ceil(k))
    return s[lo] + (s[hi] - s[lo]) * (k - lo)


@dataclasses.dataclass
class Report:
    n: int
    wall_s: float
    latency_ms: Dict[str, Dict[str, float]]
    build_gpix: float                  # image pixels built
    query_gpix: float                  # image pixels covered by the answered queries
    outputs_g: float                   # window outputs produced
    misses: int
    evictions: int
    peak_bytes: int
    max_in_flight: int
    host_call_ms: Dict[str, float] = dataclasses.field(default_factory=dict)   # longest executor call, by kind
    device_ms: Dict[str, Dict[str, float]] = dataclasses.field(default_factory=dict)   # H2D / build split

    def as_dict(self) -> dict:
        w = max(self.wall_s, 1e-9)
        return {"requests": self.n, "wall_s": round(self.wall_s, 3), "latency_ms": self.latency_ms,
                "max_host_call_ms": self.host_call_ms, "build_device_ms": self.device_ms,
                "build_gpix_s": round(self.build_gpix / w, 3),
                "served_gpix_s": round((self.build_gpix + self.query_gpix) / w, 3),
                "window_outputs_g_s": round(self.outputs_g / w, 3),
                "misses": self.misses, "evictions": self.evictions,
                "peak_GB": round(self.peak_bytes / 1e9, 3), "max_in_flight": self.max_in_flight}


class Arena:
    """Placement of blocks in one fixed device region of `size` bytes, by offset: best fit (the
    smallest free run that holds the block, lowest offset among equals), a released block merged
    with free neighbours.  The server places every table and every in-flight request's transient
    block here, so the device memory of the stream is one allocation made before it starts and
    no request allocates or frees device memory.  Long-lived blocks (tables) are cut from the top
    of their run and short-lived ones (transients) from the bottom, so that tables pack towards
    the region's end and the space the transients come and go in stays in one piece."""

    ALIGN = 256

    def __init__(self, size: int):
        self.size = int(size) // self.ALIGN * self.ALIGN
        self.starts: List[int] = [0] if self.size else []      # free runs, sorted by offset
        self.lens: List[int] = [self.size] if self.size else []
        self.live: Dict[int, int] = {}                          # placed block offset -> rounded length

    @classmethod
    def rounded(cls, n: int) -> int:
        return (max(int(n), 1) + cls.ALIGN - 1) // cls.ALIGN * cls.ALIGN

    @staticmethod
    def _best(lens: List[int], n: int) -> int:
        best = -1
        for i, ln in enumerate(lens):
            if ln >= n and (best < 0 or ln < lens[best]):
                best = i
        return best

    def fits(self, sizes) -> bool:
        """Whether blocks of `sizes` bytes can all be placed now (in that order, as alloc would)."""
        lens = list(self.lens)
        for n in sizes:
            n = self.rounded(n)
            i = self._best(lens, n)
            if i < 0:
                return False
            lens[i] -= n
        return True

    def alloc(self, n: int, top: bool = False) -> Optional[int]:
        """Offset of a new block of n bytes (cut from the top of its run with `top`), or None if
        no free run holds it."""
        n = self.rounded(n)
        i = self._best(self.lens, n)
        if i < 0:
            return None
        off = self.starts[i] + (self.lens[i] - n if top else 0)
        if self.lens[i] == n:
            del self.starts[i]
            del self.lens[i]
        else:
            if not top:
                self.starts[i] += n
            self.lens[i] -= n
        self.live[off] = n
        return off

    def release(self, off: int) -> None:
        n = self.live.pop(off)
        i = bisect.bisect_left(self.starts, off)
        # merge with the free run that ends at `off` and with the one that starts where it ends
        if i > 0 and self.starts[i - 1] + self.lens[i - 1] == off:
            i -= 1
            self.lens[i] += n
        else:
            self.starts.insert(i, off)
            self.lens.insert(i, n)
        if i + 1 < len(self.starts) and self.starts[i] + self.lens[i] == self.starts[i + 1]:
            self.lens[i] += self.lens.pop(i + 1)
            del self.starts[i + 1]

    @property
    def free_bytes(self) -> int:
        return sum(self.lens)

    @property
    def largest_free(self) -> int:
        return max(self.lens, default=0)


class Server:
    # While the loop runs, a thread holding the interpreter lock is asked to hand it over after
    # this long (Python's default is 5 ms): the image producers' bookkeeping then delays a
    # scheduler call by at most about this much.
    SWITCH_INTERVAL = 2e-4

    def __init__(self, executor, budget_bytes: float = 200e9, slots: int = 4, keep_results: bool = False):
        if slots < 1:
            raise ValueError("need at least one slot")
        self.ex = executor
        self.budget = int(budget_bytes)
        self.arena = Arena(self.budget)
        self.keep = keep_results
        self.res: "collections.OrderedDict[int, Resident]" = collections.OrderedDict()   # LRU first
        self.builds: Dict[int, Request] = {}      # image id -> its build request (for rebuilds)
        self.queued_build: Dict[int, Job] = {}    # image id -> build job still in the queue
        self.queue: List[Job] = []
        self.flight: List[Job] = []
        self.free_slots = list(range(slots))[::-1]
        self.used = 0
        self.peak = 0
        self.evictions = 0
        self.max_flight = 0
        self.done: List[Job] = []
        self.protect = True                       # keep tables that queued queries are about to read
        self.host_max: Dict[str, float] = collections.defaultdict(float)
        self.image_wait = False

    def _call(self, kind: str, fn, *args):
        """An executor call from the scheduler, its duration kept per kind (the longest)."""
        t = time.perf_counter()
        out = fn(*args)
        dt = (time.perf_counter() - t) * 1e3
        if dt > self.host_max[kind]:
            self.host_max[kind] = dt
        return out

    # -------------------------------------------------------------- memory
    def _make_room(self, sizes: List[int], reads: Optional[int] = None) -> bool:
        """Evict least recently used tables until blocks of `sizes` can be placed in the arena
        (never the table `reads`, which the request being admitted reads)."""
        if self.arena.fits(sizes):
            return True
        soon = {image_id(j.req) for j in self.queue[:64] if j.req.kind == "query"} if self.protect else set()
        for iid in list(self.res.keys()):
            r = self.res[iid]
            if r.state != "resident" or r.pins > 0 or iid in soon or iid == reads:
                continue
            self._evict(r)
            if self.arena.fits(sizes):
                return True
        return False

    def _evict(self, r: Resident) -> None:
        self.ex.free(r)
        del self.res[r.image_id]
        self.arena.release(r.offset)
        self.used -= r.nbytes
        self.evictions += 1

    # -------------------------------------------------------------- admission
    def _start(self, job: Job, now: float, transient: int) -> None:
        job.slot = self.free_slots.pop()
        job.t_admit = now
        job.transient = Arena.rounded(transient)
        job.block = self.arena.alloc(transient)
        self.used += job.transient
        self.flight.append(job)

    def _admit_build(self, job: Job, now: float) -> bool:
        req = job.req
        iid = image_id(req)
        nbytes = Arena.rounded(self.ex.table_bytes(req.H, req.W))
        trans = self.ex.build_transient_bytes(req.H, req.W)
        if nbytes + Arena.rounded(trans) > self.arena.size:
            raise ValueError("image %d (%dx%d) cannot fit the %d-byte budget" % (iid, req.H, req.W, self.budget))
        if not self._call("image_ready", self.ex.image_ready, req):
            self.image_wait = True
            return False
        if not self._make_room([nbytes, trans]):
            return False
        r = Resident(iid, req.H, req.W, nbytes, offset=self.arena.alloc(nbytes, top=True), last_used=now)
        self.res[iid] = r
        self.used += nbytes
        self._start(job, now, trans)
        r.build_job = job
        job.handle = self._call("start_build", self.ex.start_build, req, r, job.slot, job.block)
        return True

    def _admit_query(self, job: Job, r: Resident, now: float) -> bool:
        trans = self.ex.query_transient_bytes(job.req, r)
        if r.nbytes + Arena.rounded(trans) > self.arena.size:
            raise ValueError("the outputs of query %d do not fit the %d-byte budget beside their table"
                             % (job.idx, self.budget))
        if not self._make_room([trans], reads=r.image_id):
            if not self.protect and not self.flight and r.state == "resident" and r.pins == 0:
                # the table itself splits the free space: give it up too and rebuild it (a miss)
                self._evict(r)
            return False
        self._start(job, now, trans)
        after = r.build_job.handle if r.state == "building" else None
        r.pins += 1
        r.last_used = now
        self.res.move_to_end(r.image_id)
        job.handle = self._call("start_query", self.ex.start_query, job.req, r, job.slot, after, job.block)
        return True

    def _schedule(self, now: float) -> None:
        build_blocked = False
        self.image_wait = False                   # a build waits for its image (not for memory)
        i = 0
        while i < len(self.queue) and self.free_slots:
            job = self.queue[i]
            iid = image_id(job.req)
            if job.req.kind == "build":
                if not build_blocked and self._admit_build(job, now):
                    self.queue.pop(i)
                    self.queued_build.pop(iid, None)
                    continue
                build_blocked = True
                i += 1
                continue
            r = self.res.get(iid)
            if r is None:
                if iid not in self.queued_build:          # evicted: rebuild it ahead of this query
                    rb = Job(-1, self.builds[iid], now)
                    self.queued_build[iid] = rb
                    job.miss = True
                    self.queue.insert(i, rb)
                    self._call("prefetch", self.ex.prefetch, [rb.req])
                    continue
                i += 1                                    # its build has not been admitted yet
                continue
            if self._admit_query(job, r, now):
                self.queue.pop(i)
                continue
            i += 1
        self.peak = max(self.peak, self.used)
        self.max_flight = max(self.max_flight, len(self.flight))

    def _retire(self, now: float) -> int:
        still, n = [], 0
        for job in self.flight:
            if not self._call("is_done", self.ex.is_done, job.handle):
                still.append(job)
                continue
            n += 1
            job.t_done = now
            self.used -= job.transient
            self.arena.release(job.block)
            job.block = -1
            self.free_slots.append(job.slot)
            r = self.res.get(image_id(job.req))
            if job.req.kind == "build":
                if r is not None and r.build_job is job:
                    r.state = "resident"
                    r.build_job = None
                self._call("finish_build", self.ex.finish_build, job.handle)
            else:
                if r is not None:
                    r.pins -= 1
                    r.last_used = now
                job.result = self._call("finish_query", self.ex.finish_query, job.handle, self.keep)
            job.handle = None if not self.keep else job.handle
            if job.idx >= 0:
                self.done.append(job)
        self.flight = still
        return n

    # -------------------------------------------------------------- loop
    def run(self, requests: List[Request], clock: Callable[[], float] = time.perf_counter,
            idle: Callable[[], None] = lambda: None) -> Report:
        """Serve `requests` (arrival times in seconds from the start) and report latencies."""
        for req in requests:
            if req.kind == "build":
                self.builds[image_id(req)] = req
        order = sorted(range(len(requests)), key=lambda k: requests[k].t_arrival)
        self.ex.reserve(self.arena.size)        # the arena's device memory, before the clock starts
        # the images the stream will upload, in arrival order, prepared ahead by the executor
        self.ex.prefetch([requests[k] for k in order if requests[k].kind == "build"])
        gc_was_on = gc.isenabled()
        gc.collect()
        gc.freeze()
        gc.disable()
        switch = sys.getswitchinterval()
        sys.setswitchinterval(self.SWITCH_INTERVAL)
        try:
            return self._loop(requests, order, clock, idle)
        finally:
            sys.setswitchinterval(switch)
            gc.unfreeze()
            if gc_was_on:
                gc.enable()

    def _loop(self, requests: List[Request], order: List[int], clock: Callable[[], float],
              idle: Callable[[], None]) -> Report:
        t0 = clock()
        nxt = 0
        while nxt < len(order) or self.queue or self.flight:
            now = clock() - t0
            while nxt < len(order) and requests[order[nxt]].t_arrival <= now:
                k = order[nxt]
                job = Job(k, requests[k], requests[k].t_arrival)
                if job.req.kind == "build":
                    self.queued_build[image_id(job.req)] = job
                self.queue.append(job)
                nxt += 1
            retired = self._retire(now)
            n_before = len(self.flight)
            self._schedule(now)
            if not self.flight and self.queue and not self.image_wait:
                # nothing in flight will free memory: let eviction take protected tables too
                ev = self.evictions
                self.protect = False
                self._schedule(now)
                self.protect = True
                if not self.flight and not self.image_wait and self.evictions == ev:
                    raise RuntimeError("no queued request fits the memory budget")
            if not retired and len(self.flight) == n_before:
                idle()
        return self._report(clock() - t0)

    def _report(self, wall: float) -> Report:
        lat = {}
        for kind in ("build", "query", "all"):
            xs = [(j.t_done - j.t_arrival) * 1e3 for j in self.done if kind == "all" or j.req.kind == kind]
            lat[kind] = {"n": len(xs), "p50": round(percentile(xs, 0.5), 3), "p99": round(percentile(xs, 0.99), 3)}
        bpx = sum(j.req.H * j.req.W for j in self.done if j.req.kind == "build") / 1e9
        qpx = opx = 0.0
        for j in self.done:
            if j.req.kind == "query":
                b = self.builds[image_id(j.req)]
                qpx += b.H * b.W / 1e9
                h, w = min(j.req.win_h, b.H), min(j.req.win_w, b.W)
                opx += ((b.H - h) // j.req.stride + 1) * ((b.W - w) // j.req.stride + 1) / 1e9
        dev = {}
        split = getattr(self.ex, "build_split_ms", None)
        if split:
            for part in ("h2d", "build"):
                xs = [x[part] for x in split]
                dev[part] = {"n": len(xs), "p50": round(percentile(xs, 0.5), 3), "p99": round(percentile(xs, 0.99), 3),
                             "max": round(max(xs), 3)}
        return Report(len(self.done), wall, lat, bpx, qpx, opx, sum(1 for j in self.done if j.miss),
                      self.evictions, self.peak, self.max_flight,
                      {k: round(v, 3) for k, v in sorted(self.host_max.items())}, dev)


class ImageSource:
    """Producer threads that prepare the images of build requests as host data ahead of their
    arrival, the way a client's upload would be waiting in host memory: the 8-bit cluster mask of
    each request (synth.thomas_points, seeded by the request) drawn into a pinned buffer of a
    fixed pool, on rows of image_pitch(W) bytes.  Requests are taken in the order given; an
    image asked for again (a rebuild after eviction) draws from one buffer kept apart for that, so
    that buffers held by images waiting for admission can never block it.  The drawing (numpy's
    generator, torch's fill and scatter on CPU tensors) runs outside the GIL for all but the
    bookkeeping."""

    def __init__(self, torch, pool: int = 4, max_pixels: int = 16000 * 16064, workers: int = 2):
        self.torch = torch
        self.cv = threading.Condition()
        self.free = [torch.empty(max_pixels, dtype=torch.uint8, pin_memory=True) for _ in range(pool)]
        self.spare = [torch.empty(max_pixels, dtype=torch.uint8, pin_memory=True)]
        self.max_pixels = max_pixels
        self.todo: "collections.deque" = collections.deque()
        self.seen = set()
        self.ready: Dict[int, tuple] = {}
        self.closed = False
        self.threads = [threading.Thread(target=self._work, name="image-source-%d" % i, daemon=True)
                        for i in range(workers)]
        for t in self.threads:
            t.start()

    def request(self, reqs) -> None:
        with self.cv:
            for r in reqs:
                iid = image_id(r)
                again = iid in self.seen
                self.seen.add(iid)
                self.todo.append((r, again))
            self.cv.notify_all()

    def is_ready(self, iid: int) -> bool:
        with self.cv:
            return iid in self.ready

    def take(self, iid: int):
        """(buffer, H, W, pitch, spare) of a ready image, now owned by the caller."""
        with self.cv:
            return self.ready.pop(iid)

    def give_back(self, buf, spare: bool) -> None:
        with self.cv:
            (self.spare if spare else self.free).append(buf)
            self.cv.notify_all()

    def close(self) -> None:
        with self.cv:
            self.closed = True
            self.cv.notify_all()
        for t in self.threads:
            t.join()

    def _work(self) -> None:
        from .api import image_pitch
        from .synth import thomas_points
        torch = self.torch
        while True:
            with self.cv:
                while True:
                    if self.closed:
                        return
                    # the first request a buffer is free for (a rebuild waits only for the spare)
                    k = next((i for i, (_, again) in enumerate(self.todo) if (self.spare if again else self.free)),
                             None)
                    if k is not None:
                        break
                    self.cv.wait()
                req, again = self.todo[k]
                del self.todo[k]
                buf = (self.spare if again else self.free).pop()
            H, W = req.H, req.W
            pitch = image_pitch(W, torch.uint8)
            if H * pitch > self.max_pixels:
                raise ValueError("image %dx%d exceeds the source's buffers" % (H, W))
            ys, xs = thomas_points(H, W, seed=req.image_seed)
            view = buf[:H * pitch]
            view.zero_()
            view[torch.from_numpy(ys * pitch + xs)] = 1
            with self.cv:
                self.ready[image_id(req)] = (buf, H, W, pitch, again)


class GpuExecutor:
    """Runs the requests on one GPU through the library, one stream per slot, in the device memory
    of one arena allocation (reserve) carved by the server's block offsets.  Build requests copy
    their image from the ImageSource's pinned buffer into their transient block on their stream
    (api.upload: a kernel reading the pinned pages, whose enqueue never waits for other copies
    in flight as a DMA copy's can), then build into their table's block with the workspace that
    follows the image; the upload and the build are timed apart with events (build_split_ms).
    Query outputs are views of their transient block, given back when the query retires; with
    keep=True a result is copied out before that."""

    def __init__(self, device, slots: int, pool: int = 4):
        import torch
        self.torch = torch
        self.dev = torch.device(device)
        self.streams = [torch.cuda.Stream(self.dev) for _ in range(slots)]
        self.src = ImageSource(torch, pool)
        self.build_split_ms: List[dict] = []
        self.mem = None

    def reserve(self, nbytes: int) -> None:
        """The arena's device memory (kept across runs of the same size), then the executor's
        start-up: one upload from pinned host memory, one table build and one gather of each kind on
        every slot's stream, with timing events, on a small image in the still empty arena.  The
        HIP runtime sets up its copy path, events and code objects on first use (tens of
        milliseconds of host time); start-up takes that before the server accepts requests."""
        torch = self.torch
        if self.mem is not None and self.mem.numel() == nbytes:
            return
        self.mem = None
        self.mem = torch.empty(nbytes, dtype=torch.uint8, device=self.dev)
        from . import api
        H, W = 96, 200
        pitch = api.image_pitch(W, torch.uint8)
        need = H * pitch + api.build_workspace_bytes(H, W, 1, False) + 2 * H * api.table_pitch(W) * 8 + 4 * 65536
        if need > nbytes:
            torch.cuda.synchronize(self.dev)
            return
        host = torch.ones(H * pitch, dtype=torch.uint8, pin_memory=True)
        img = self.mem[:H * pitch].view(H, pitch)
        ws_off = (H * pitch + 255) // 256 * 256
        ws_n = api.build_workspace_bytes(H, W, 1, False)
        t_off = (ws_off + ws_n + 255) // 256 * 256
        tp = api.table_pitch(W)
        S = self._view(t_off, H, tp, W, torch.uint64)
        o_off = (t_off + H * tp * 8 + 255) // 256 * 256
        for s in self.streams:
            with torch.cuda.stream(s):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(s)
                api.upload(host, self.mem[:H * pitch], stream=s)
                api.sat_build(img[:, :W], sat=S, ws=self.mem[ws_off:ws_off + ws_n], stream=s)
                for h, w, dt in ((8, 8, torch.uint32), (90, 190, torch.uint64)):
                    oh, ow = api.out_shape(H, W, h, w, 1)
                    op = api.out_pitch(ow, dt)
                    api.window_sum(S, h, w, 1, pixel_type="u8", stream=s, out=self._view(o_off, oh, op, ow, dt))
                oh, ow = api.out_shape(H, W, 16, 16, 2)
                op = api.out_pitch(ow, torch.float64)
                part = oh * op * 8
                outs = (self._view(o_off, oh, op, ow, torch.uint64), self._view(o_off + part, oh, op, ow, torch.float64),
                        self._view(o_off + 2 * part, oh, op, ow, torch.float64))
                api.window_mean_std(S, S, 16, 16, 2, outs=outs, stream=s)
                e1.record(s)
            e1.synchronize()
            e0.elapsed_time(e1)
        torch.cuda.synchronize(self.dev)

    def close(self) -> None:
        self.src.close()
        self.mem = None

    def prefetch(self, reqs) -> None:
        self.src.request(reqs)

    def image_ready(self, req: Request) -> bool:
        return self.src.is_ready(image_id(req))

    def _view(self, off: int, rows: int, pitch: int, cols: int, dtype):
        n = rows * pitch * dtype.itemsize
        return self.mem[off:off + n].view(dtype).view(rows, pitch)[:, :cols]

    @staticmethod
    def _image_bytes(H: int, W: int) -> int:
        from .api import image_pitch
        import torch
        return (H * image_pitch(W, torch.uint8) + 255) // 256 * 256

    def table_bytes(self, H: int, W: int) -> int:
        from .api import table_pitch
        return H * table_pitch(W) * 8

    def build_transient_bytes(self, H: int, W: int) -> int:
        from .api import build_workspace_bytes
        return self._image_bytes(H, W) + build_workspace_bytes(H, W, 1, False)

    def _out_layout(self, req: Request, r: Resident):
        import torch
        from .api import out_pitch
        h, w = min(req.win_h, r.H), min(req.win_w, r.W)
        oh, ow = (r.H - h) // req.stride + 1, (r.W - w) // req.stride + 1
        if req.op == "sum":
            dt = torch.uint32 if h * w * 255 <= 0xFFFFFFFF else torch.uint64
            return h, w, oh, ow, dt, out_pitch(ow, dt), 1
        return h, w, oh, ow, torch.float64, out_pitch(ow, torch.float64), 3

    def query_transient_bytes(self, req: Request, r: Resident) -> int:
        _, _, oh, _, dt, pitch, n = self._out_layout(req, r)
        return n * oh * pitch * dt.itemsize

    def start_build(self, req: Request, r: Resident, slot: int, block: int):
        from . import api
        torch = self.torch
        s = self.streams[slot]
        buf, H, W, pitch, spare = self.src.take(image_id(req))
        tp = api.table_pitch(W)
        S = self._view(r.offset, H, tp, W, torch.uint64)
        base = self._view(block, H, pitch, pitch, torch.uint8)
        ws_off = block + self._image_bytes(H, W)
        ws = self.mem[ws_off:ws_off + api.build_workspace_bytes(H, W, 1, False)]
        with torch.cuda.stream(s):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            ev = torch.cuda.Event(enable_timing=True)
            e0.record(s)
            api.upload(buf[:H * pitch], self.mem[block:block + H * pitch], stream=s)
            e1.record(s)
            img = base[:, :W]                    # rows on 128-byte lines: the helper-wave plans
            r.tables = api.sat_build(img, sat=S, ws=ws, stream=s)
            ev.record(s)
        return {"ev": ev, "e0": e0, "e1": e1, "buf": buf, "spare": spare}

    def finish_build(self, handle) -> None:
        self.build_split_ms.append({"h2d": handle["e0"].elapsed_time(handle["e1"]),
                                    "build": handle["e1"].elapsed_time(handle["ev"])})
        self.src.give_back(handle["buf"], handle["spare"])
        handle["buf"] = None

    def start_query(self, req: Request, r: Resident, slot: int, after, block: int):
        from . import api
        torch = self.torch
        s = self.streams[slot]
        if after is not None:
            s.wait_event(after["ev"])
        h, w, oh, ow, dt, pitch, n = self._out_layout(req, r)
        S = r.tables
        part = oh * pitch * dt.itemsize
        with torch.cuda.stream(s):
            if req.op == "sum":
                out = api.window_sum(S, h, w, req.stride, pixel_type="u8", stream=s,
                                     out=self._view(block, oh, pitch, ow, dt))
            else:
                outs = (self._view(block, oh, pitch, ow, torch.uint64),
                        self._view(block + part, oh, pitch, ow, dt), self._view(block + 2 * part, oh, pitch, ow, dt))
                out = api.window_mean_std(S, S, h, w, req.stride, outs=outs, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        return {"ev": ev, "out": out, "stream": s}

    def is_done(self, handle) -> bool:
        return handle["ev"].query()

    def finish_query(self, handle, keep: bool):
        """The result (copied out of the arena block, which is given back next) with keep=True."""
        if not keep:
            return None
        torch = self.torch
        out = handle["out"]
        with torch.cuda.stream(handle["stream"]):
            res = out.clone() if isinstance(out, torch.Tensor) else tuple(o.clone() for o in out)
        handle["stream"].synchronize()
        return res

    def free(self, r: Resident) -> None:
        r.tables = None
