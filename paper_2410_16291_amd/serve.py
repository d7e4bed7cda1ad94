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
  * admission is by memory footprint under `budget_bytes`: resident tables plus the transient
    image, workspace and output bytes of the requests in flight.  To make room, the least
    recently used resident tables that no in-flight or imminent query reads are evicted;
  * a query may be admitted while its image is still being built: its stream waits for the
    build's completion event on the device, not on the host;
  * a query whose table was evicted rebuilds it first (the image is regenerated from its seed)
    and counts as a miss.

Images arrive as host data: a producer thread (ImageSource) draws each build request's image into
a buffer of a pinned host pool ahead of its arrival, as a client upload would have it ready; the
scheduler admits a build only once its image is ready and copies it to the device asynchronously
on the request's stream (the H2D copy is timed separately from the build).  No request does host
work on the scheduler thread beyond launching; the longest scheduler-side executor call is
reported.

Latency runs from a request's arrival to the moment the host observes its completion event.
Results stay on the device; copying them to the host is not part of the latency.

The scheduling logic does not touch the GPU: `Server` drives an executor (GpuExecutor below;
the CPU tests drive a simulated one).
"""
from __future__ import annotations

import collections
import dataclasses
import math
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


class Server:
    def __init__(self, executor, budget_bytes: float = 200e9, slots: int = 4, keep_results: bool = False):
        if slots < 1:
            raise ValueError("need at least one slot")
        self.ex = executor
        self.budget = int(budget_bytes)
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
    def _make_room(self, need: int) -> bool:
        if self.used + need <= self.budget:
            return True
        soon = {image_id(j.req) for j in self.queue[:64] if j.req.kind == "query"} if self.protect else set()
        for iid in list(self.res.keys()):
            r = self.res[iid]
            if r.state != "resident" or r.pins > 0 or iid in soon:
                continue
            self.ex.free(r)
            del self.res[iid]
            self.used -= r.nbytes
            self.evictions += 1
            if self.used + need <= self.budget:
                return True
        return False

    # -------------------------------------------------------------- admission
    def _start(self, job: Job, now: float, transient: int) -> None:
        job.slot = self.free_slots.pop()
        job.t_admit = now
        job.transient = transient
        self.used += transient
        self.flight.append(job)

    def _admit_build(self, job: Job, now: float) -> bool:
        req = job.req
        iid = image_id(req)
        nbytes = self.ex.table_bytes(req.H, req.W)
        trans = self.ex.build_transient_bytes(req.H, req.W)
        if nbytes + trans > self.budget:
            raise ValueError("image %d (%dx%d) cannot fit the %d-byte budget" % (iid, req.H, req.W, self.budget))
        if not self._call("image_ready", self.ex.image_ready, req):
            self.image_wait = True
            return False
        if not self._make_room(nbytes + trans):
            return False
        r = Resident(iid, req.H, req.W, nbytes, last_used=now)
        self.res[iid] = r
        self.used += nbytes
        self._start(job, now, trans)
        r.build_job = job
        job.handle = self._call("start_build", self.ex.start_build, req, r, job.slot)
        return True

    def _admit_query(self, job: Job, r: Resident, now: float) -> bool:
        trans = self.ex.query_transient_bytes(job.req, r)
        if not self._make_room(trans):
            return False
        self._start(job, now, trans)
        after = r.build_job.handle if r.state == "building" else None
        r.pins += 1
        r.last_used = now
        self.res.move_to_end(r.image_id)
        job.handle = self._call("start_query", self.ex.start_query, job.req, r, job.slot, after)
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
        # the images the stream will upload, in arrival order, prepared ahead by the executor
        self.ex.prefetch([requests[k] for k in order if requests[k].kind == "build"])
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
                self.protect = False
                self._schedule(now)
                self.protect = True
                if not self.flight and not self.image_wait:
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
    """Runs the requests on one GPU through the library, one stream per slot.  Build requests
    copy their image from the ImageSource's pinned buffer to the device on their stream, then
    build; the H2D copy and the build are timed apart with events (build_split_ms)."""

    def __init__(self, device, slots: int, pool: int = 4):
        import torch
        self.torch = torch
        self.dev = torch.device(device)
        self.streams = [torch.cuda.Stream(self.dev) for _ in range(slots)]
        self.src = ImageSource(torch, pool)
        self.build_split_ms: List[dict] = []

    def close(self) -> None:
        self.src.close()

    def prefetch(self, reqs) -> None:
        self.src.request(reqs)

    def image_ready(self, req: Request) -> bool:
        return self.src.is_ready(image_id(req))

    def table_bytes(self, H: int, W: int) -> int:
        from .api import table_pitch
        return H * table_pitch(W) * 8

    def build_transient_bytes(self, H: int, W: int) -> int:
        from .api import build_workspace_bytes, image_pitch
        return H * image_pitch(W, self.torch.uint8) + build_workspace_bytes(H, W, 1, False)

    def query_transient_bytes(self, req: Request, r: Resident) -> int:
        import torch
        from .api import out_pitch
        h, w = min(req.win_h, r.H), min(req.win_w, r.W)
        oh, ow = (r.H - h) // req.stride + 1, (r.W - w) // req.stride + 1
        if req.op == "sum":
            dt = torch.uint32 if h * w * 255 <= 0xFFFFFFFF else torch.uint64
            return oh * out_pitch(ow, dt) * dt.itemsize
        return 3 * oh * out_pitch(ow, torch.float64) * 8

    def start_build(self, req: Request, r: Resident, slot: int):
        from . import api
        torch = self.torch
        s = self.streams[slot]
        buf, H, W, pitch, spare = self.src.take(image_id(req))
        with torch.cuda.stream(s):
            base = torch.empty((H, pitch), dtype=torch.uint8, device=self.dev)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            ev = torch.cuda.Event(enable_timing=True)
            e0.record(s)
            base.copy_(buf[:H * pitch].view(H, pitch), non_blocking=True)
            e1.record(s)
            img = base[:, :W]                    # rows on 128-byte lines: the helper-wave plans
            r.tables = api.sat_build(img, stream=s)
            ev.record(s)
        return {"ev": ev, "e0": e0, "e1": e1, "img": img, "buf": buf, "spare": spare}

    def finish_build(self, handle) -> None:
        self.build_split_ms.append({"h2d": handle["e0"].elapsed_time(handle["e1"]),
                                    "build": handle["e1"].elapsed_time(handle["ev"])})
        self.src.give_back(handle["buf"], handle["spare"])
        handle["img"] = None
        handle["buf"] = None

    def start_query(self, req: Request, r: Resident, slot: int, after):
        from . import api
        torch = self.torch
        s = self.streams[slot]
        if after is not None:
            s.wait_event(after["ev"])
        h, w = min(req.win_h, r.H), min(req.win_w, r.W)
        S = r.tables
        with torch.cuda.stream(s):
            if req.op == "sum":
                out = api.window_sum(S, h, w, req.stride, pixel_type="u8", stream=s)
            else:
                out = api.window_mean_std(S, S, h, w, req.stride, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        S.record_stream(s)
        return {"ev": ev, "out": out}

    def is_done(self, handle) -> bool:
        return handle["ev"].query()

    def finish_query(self, handle, keep: bool):
        return handle["out"] if keep else None

    def free(self, r: Resident) -> None:
        r.tables = None
