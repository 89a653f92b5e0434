"""Continuous-batching CDEF server.

Requests are frames either already resident in device memory (as when
CDEF runs inside a GPU codec pipeline: the reconstruction is produced on the
device and the source was uploaded once) or arriving in pinned host memory,
each asking either for the encoder's strength search or for the direction
search + filter at given per-filter-block strengths.  The scheduler

* validates each request on its own at submission (a bad request fails
  alone and never joins a batch),
* admits requests first-in first-out while the device bytes they need fit a
  budget (by default 90 % of the free device memory): their outputs, and for
  a host frame not yet on the device its planes, which are uploaded on a
  copy stream at admission and then stay resident (a later request on the
  same frame -- the filter after the search, say -- finds them there) until
  the budget needs room and no running request uses them (least recently
  used first),
* launches every admitted request not yet running as one batch
  (cdef_batch_prepare + cdef_batch_launch) on the next free stream of a
  small pool, without waiting for earlier batches, so requests that arrive
  while others run join the next batch and batches overlap on the device,
* retires batches by polling their completion events and releases their
  budget.

The same scheduler drives the plain path (one request per launch through the
per-frame entry points, in arrival order on one stream) for comparison, and
a test executor with no GPU.  Results are bit-identical whichever path or
batch a request takes.
"""
from __future__ import annotations

import collections
import dataclasses
import json
import sys
import time
from typing import Callable, Deque, Dict, List, Optional

import numpy as np

from . import cdef

SEARCH = cdef.MODE_SEARCH
FILTER = cdef.MODE_FILTER


@dataclasses.dataclass
class Request:
    rid: int
    mode: int
    recon: "cdef.Frame"
    src: Optional["cdef.Frame"] = None  # search
    strengths: object = None            # filter: uint8 [fbr][fbc][4] device tensor
    skip: object = None
    damping: int = 3
    host: Optional["HostFrame"] = None  # frame in pinned host memory (recon/src/skip set
                                        # to its device copies at admission)
    host_strengths: object = None       # filter, host frame: pinned uint8 [fbr][fbc][4]
    arrival: float = 0.0                # host clock, seconds
    # filled in by the server
    status: int = 0
    outputs: tuple = ()
    out_bytes: int = 0
    in_bytes: int = 0                   # device bytes of frame planes this request uploaded
    ready: object = None                # event after its uploads (None: nothing to wait for)
    admitted: float = -1.0
    done: float = -1.0
    job: object = None
    batch_id: int = -1

    @property
    def luma_px(self) -> int:
        f = self.host if self.host is not None else self.recon
        return f.width * f.height


def output_bytes(req: Request) -> int:
    """Device bytes a request's outputs occupy while it is in flight."""
    f = req.recon
    fbr, fbc = f.fb_shape
    br, bc = f.block_shape
    dv = br * bc * 5
    if req.mode == SEARCH:
        return f.nplanes * fbr * fbc * 64 * 8 + dv
    w, h = f.width, f.height
    px = w * h + (2 * ((w + 1) // 2) * ((h + 1) // 2) if f.nplanes == 3 else 0)
    return 2 * px + dv


@dataclasses.dataclass
class HostFrame:
    """A frame in pinned host memory.  `key` names the frame: requests with the
    same key share one device copy while it stays resident."""

    key: object
    recon: List            # pinned CPU tensors, 2-D, int16 storage
    src: Optional[List]    # searches
    skip: object           # pinned uint8 [ceil(h/8)][ceil(w/8)] or None
    width: int
    height: int
    bitdepth: int
    layout: int

    def plane_bytes(self, planes) -> int:
        return sum(t.numel() * t.element_size() for t in planes)


class ResidentFrames:
    """Device copies of host frames.  Uploads run on `stream`; an entry stays
    after its requests finish and is evicted least recently used first when
    room is needed and no request holds it."""

    def __init__(self, stream):
        self.stream = stream
        self.entries: "collections.OrderedDict" = collections.OrderedDict()

    def bytes_needed(self, host: HostFrame, need_src: bool) -> int:
        e = self.entries.get(host.key)
        if e is None:
            n = host.plane_bytes(host.recon)
            if host.skip is not None:
                n += host.skip.numel()
            return n + (host.plane_bytes(host.src) if need_src else 0)
        return host.plane_bytes(host.src) if need_src and e["src"] is None else 0

    def _upload(self, planes):
        import torch
        out = []
        with torch.cuda.stream(self.stream):
            for t in planes:
                d = torch.empty(t.shape, dtype=t.dtype, device="cuda")
                d.copy_(t, non_blocking=True)
                out.append(d)
        return out

    def _record(self):
        """An event after the uploads enqueued so far."""
        import torch
        ev = torch.cuda.Event()
        ev.record(self.stream)
        return ev

    @staticmethod
    def _done(ev) -> bool:
        return ev.query()

    def acquire(self, host: HostFrame, need_src: bool):
        """The device entry of `host` (uploading what is missing), held until
        release(); returns (entry, bytes newly resident, event or None)."""
        e = self.entries.get(host.key)
        added = self.bytes_needed(host, need_src)
        fresh = False
        if e is None:
            rec = self._upload(host.recon)
            skip = self._upload([host.skip])[0] if host.skip is not None else None
            e = {"recon": cdef.Frame(rec, host.width, host.height, host.bitdepth, host.layout),
                 "src": None, "skip": skip, "bytes": 0, "refs": 0, "event": None}
            self.entries[host.key] = e
            fresh = True
        if need_src and e["src"] is None:
            e["src"] = cdef.Frame(self._upload(host.src), host.width, host.height,
                                  host.bitdepth, host.layout)
            fresh = True
        if fresh:
            e["event"] = self._record()
        e["bytes"] += added
        e["refs"] += 1
        self.entries.move_to_end(host.key)
        ev = e["event"]
        if ev is not None and self._done(ev):
            e["event"] = ev = None
        return e, added, ev

    def release(self, key) -> None:
        e = self.entries.get(key)
        if e is not None:
            e["refs"] -= 1

    def evict(self, nbytes: int, keep=None) -> int:
        """Drop idle entries other than `keep`, least recently used first,
        until `nbytes` are freed or none is idle; returns the bytes freed."""
        freed = 0
        for key in list(self.entries):
            if freed >= nbytes:
                break
            e = self.entries[key]
            if e["refs"] == 0 and key != keep:
                freed += e["bytes"]
                del self.entries[key]
        return freed

    @property
    def resident_bytes(self) -> int:
        return sum(e["bytes"] for e in self.entries.values())


def _attach_host(frames: ResidentFrames, req: Request) -> None:
    """Point a host request at the device copies of its frame (uploading
    what is missing) and upload its strengths."""
    e, added, ev = frames.acquire(req.host, req.mode == SEARCH)
    req.recon, req.skip = e["recon"], e["skip"]
    req.src = e["src"] if req.mode == SEARCH else None
    req.in_bytes = added
    req.ready = ev
    if req.mode == FILTER and req.host_strengths is not None:
        req.strengths = frames._upload([req.host_strengths])[0]
        req.ready = frames._record()


class DeviceClock:
    """Maps completion-event times to the host clock.

    The offset is calibrated once per process and shared by every executor,
    so latencies of different executors are comparable.  Each calibration
    event k is recorded right after host time a_k; it is stamped on the
    device lat_k >= 0 later, so the host time of event 0 is at least
    a_k - elapsed(0, k) for every k, and the largest such bound is the
    tightest (it is reached for the smallest submission delay)."""

    _shared = None

    def __init__(self, rounds: int = 64):
        import torch
        s = torch.cuda.current_stream()
        torch.cuda.synchronize()
        self.ref = torch.cuda.Event(enable_timing=True)
        self.ref.record(s)
        torch.cuda.synchronize()
        best = -1e30
        for _ in range(rounds):
            ev = torch.cuda.Event(enable_timing=True)
            a = time.perf_counter()
            ev.record(s)
            ev.synchronize()
            best = max(best, a - self.ref.elapsed_time(ev) / 1e3)
        self.t0_host = best

    @classmethod
    def shared(cls) -> "DeviceClock":
        if cls._shared is None:
            cls._shared = cls()
        return cls._shared

    def host_time(self, ev) -> float:
        return self.t0_host + self.ref.elapsed_time(ev) / 1e3


# Device work of one filter block in units of a filter-mode filter block: a
# strength-search filter block costs about four (0.159 against 0.043 ms per
# 4K 10-bit frame in a batch).
SEARCH_WORK = 4


def request_work(req: Request, search_work: int = SEARCH_WORK) -> int:
    """Device work of a request: its filter blocks (workgroups), each weighted
    by its mode's cost."""
    fbr, fbc = req.recon.fb_shape
    return fbr * fbc * (search_work if req.mode == SEARCH else 1)


def choose_stream(inflight: List[List[int]], work: int, depth: int, heavy_work: int,
                  fifo_heavy: bool) -> int:
    """Stream for a new batch of `work` units, given the work of the batches
    in flight on each stream (oldest first); -1 when every stream holds
    `depth` batches.  A heavy batch goes behind a heavy one in flight
    (fifo_heavy), else to an idle stream, else to the stream with the least
    work in flight."""
    room = [i for i, q in enumerate(inflight) if len(q) < depth]
    if not room:
        return -1
    if fifo_heavy and work > heavy_work:
        behind = [i for i in room if any(n > heavy_work for n in inflight[i])]
        if behind:
            return min(behind, key=lambda i: len(inflight[i]))
    idle = [i for i in room if not inflight[i]]
    if idle:
        return idle[0]
    return min(room, key=lambda i: sum(inflight[i]))


class GpuBatchExecutor:
    """Batches of requests through cdef_batch_prepare / cdef_batch_launch on a
    pool of streams (default priority).  Each stream runs one batch and may
    hold `depth - 1` more queued behind it, so a batch formed while every
    stream is busy is already on the device when the running one ends.

    Stream choice: a light batch (at most `heavy_work` units of
    request_work, by default one round of search workgroups over the chip,
    768 x SEARCH_WORK) runs beside whatever is running, on an idle stream if
    there is one, and fills the CUs that a running batch's last workgroups
    leave idle.  A heavy batch is queued behind a heavy batch already in
    flight when `fifo_heavy` is set: two heavy batches sharing the chip
    would both finish late, while in order the first finishes as early as
    it would alone.  search_work = 1 counts filter blocks alone."""

    def __init__(self, n_streams: int = 4, variant: Optional[int] = None, max_batch: int = 256,
                 depth: int = 2, heavy_work: int = 768 * SEARCH_WORK, fifo_heavy: bool = True,
                 search_work: int = SEARCH_WORK):
        import torch
        self.torch = torch
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.depth = depth
        self.heavy_work = heavy_work
        self.fifo_heavy = fifo_heavy
        self.search_work = search_work
        # per stream: the slots (Batch objects) of its in-flight batches
        self.slots = [[cdef.Batch() for _ in range(depth)] for _ in range(n_streams)]
        for row in self.slots:
            for b in row:
                b.reserve(max_batch)
        self.inflight: List[collections.deque] = [collections.deque() for _ in range(n_streams)]
        self.handles: Dict[int, tuple] = {}  # handle -> (stream index, event)
        self.next = 0
        self.variant = variant
        self.clock = None
        self.frames = ResidentFrames(torch.cuda.Stream())

    def set_epoch(self):
        self.clock = DeviceClock.shared()

    def input_bytes(self, req: Request) -> int:
        return 0 if req.host is None else self.frames.bytes_needed(req.host, req.mode == SEARCH)

    def evict(self, nbytes: int, req: Optional[Request] = None) -> int:
        keep = req.host.key if req is not None and req.host is not None else None
        return self.frames.evict(nbytes, keep)

    def release(self, req: Request) -> None:
        if req.host is not None:
            self.frames.release(req.host.key)

    def allocate(self, req: Request):
        torch = self.torch
        if req.host is not None:
            _attach_host(self.frames, req)
        f = req.recon
        br, bc = f.block_shape
        d = torch.empty((br, bc), dtype=torch.uint8, device="cuda")
        v = torch.empty((br, bc), dtype=torch.int32, device="cuda")
        if req.mode == SEARCH:
            fbr, fbc = f.fb_shape
            sse = torch.empty((f.nplanes, fbr, fbc, 16, 4), dtype=torch.int64, device="cuda")
            req.outputs = (sse, d, v)
            req.job = cdef.make_search_job(f, req.src, req.skip, req.damping, sse, d, v)
        else:
            outs = [torch.empty_like(p) for p in f.planes[:f.nplanes]]
            req.outputs = (outs, d, v)
            req.job = cdef.make_filter_job(f, outs, req.skip, req.damping, req.strengths, d, v)

    def validate(self, req: Request) -> int:
        return cdef.validate_job(req.job)

    def free_slot(self) -> int:
        """A stream with room for another batch (an idle one first), else -1."""
        best, load = -1, self.depth
        for i, q in enumerate(self.inflight):
            if len(q) < load:
                best, load = i, len(q)
        return best

    def launch(self, reqs: List[Request]):
        work = sum(request_work(r, self.search_work) for r in reqs)
        i = choose_stream([[n for _, _, n in q] for q in self.inflight], work, self.depth,
                          self.heavy_work, self.fifo_heavy)
        assert i >= 0
        used = {id(b) for b, _, _ in self.inflight[i]}
        b = next(x for x in self.slots[i] if id(x) not in used)
        b.jobs, b._keep = [], []
        for r in reqs:
            b.add_job(r.job, (r.recon, r.src, r.skip, r.strengths, r.outputs))
        s = self.streams[i]
        for r in reqs:  # frames uploaded on the copy stream
            if r.ready is not None:
                s.wait_event(r.ready)
        b.prepare(s)
        if self.variant is not None:
            b.plan.variant = self.variant
        b.launch(s)
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record(s)
        self.inflight[i].append((b, ev, work))
        h = self.next
        self.next += 1
        self.handles[h] = (i, ev)
        return h

    def poll(self, handle) -> Optional[float]:
        """Completion time (host clock) of a finished launch, else None."""
        i, ev = self.handles[handle]
        if not ev.query():
            return None
        del self.handles[handle]
        q = self.inflight[i]
        for k, (_, e, _) in enumerate(q):
            if e is ev:  # it and the batches before it on its stream are done
                for _ in range(k + 1):
                    q.popleft()
                break
        return self.clock.host_time(ev)

    @property
    def capacity(self) -> int:
        return len(self.streams) * self.depth


class GpuPlainExecutor:
    """One request per launch through the per-frame entry points, in order,
    on one stream."""

    in_order = True

    def __init__(self):
        import torch
        self.torch = torch
        self.stream = torch.cuda.Stream()
        self.pending: Dict[int, object] = {}
        self.next = 0
        self.clock = None
        self.frames = ResidentFrames(self.stream)  # uploads in order on the one stream

    set_epoch = GpuBatchExecutor.set_epoch
    allocate = GpuBatchExecutor.allocate
    validate = GpuBatchExecutor.validate
    input_bytes = GpuBatchExecutor.input_bytes
    evict = GpuBatchExecutor.evict
    release = GpuBatchExecutor.release

    def launch(self, reqs: List[Request]):
        assert len(reqs) == 1
        r = reqs[0]
        s = self.stream
        if r.mode == SEARCH:
            sse, d, v = r.outputs
            cdef.cdef_search_strengths(r.recon, r.src, r.skip, r.damping, sse, d, v, s)
        else:
            outs, d, v = r.outputs
            cdef.cdef_find_dir(r.recon, d, v, s)
            cdef.cdef_filter_frame(r.recon, outs, d, v, r.skip, r.damping, r.strengths, s)
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record(s)
        h = self.next
        self.next += 1
        self.pending[h] = ev
        return h

    def poll(self, handle) -> Optional[float]:
        ev = self.pending.get(handle)
        if ev is None or not ev.query():
            return None
        del self.pending[handle]
        return self.clock.host_time(ev)

    @property
    def capacity(self) -> int:
        return 1 << 30  # launches queue on the stream in order


class Scheduler:
    """Admission by device bytes, continuous batching, completion polling.
    Executor-agnostic: it needs allocate / validate / launch / poll /
    capacity, and for host frames input_bytes / evict / release (bytes a
    request would upload, freeing idle resident frames, dropping a request's
    hold on its frame)."""

    def __init__(self, executor, budget_bytes: int, max_batch: int = 256,
                 batching: bool = True, clock: Callable[[], float] = time.perf_counter,
                 release_outputs: bool = False, split_modes: bool = True):
        self.ex = executor
        # one mode per batch: a batch of filter jobs only runs on the leaner
        # filter-only kernels, a mixed one runs its filter jobs inside the
        # search kernel
        self.split_modes = split_modes
        # drop each finished request's output tensors (a consumer that only
        # needs timings), so the caching allocator reuses their memory
        self.release_outputs = release_outputs
        self.budget = budget_bytes
        self.in_use = 0
        self.max_batch = max_batch if batching else 1
        self.queue: Deque[Request] = collections.deque()   # submitted, not admitted
        self.ready: List[Request] = []                       # admitted, not launched
        self.running: Dict[object, List[Request]] = {}
        self.finished: List[Request] = []
        self.rejected: List[Request] = []
        self.clock = clock
        self.nbatches = 0

    def submit(self, req: Request) -> None:
        self.queue.append(req)

    def cancel(self, rid: int) -> bool:
        """Withdraw a request that has not been admitted yet."""
        for r in list(self.queue):
            if r.rid == rid:
                self.queue.remove(r)
                return True
        return False

    def _input_bytes(self, r: Request) -> int:
        f = getattr(self.ex, "input_bytes", None)
        return f(r) if f else 0

    def _admit(self, now: float) -> None:
        while self.queue:
            r = self.queue[0]
            out = output_bytes(r)
            need = out + self._input_bytes(r)
            if need > self.budget:  # can never fit: reject rather than block the queue
                self.queue.popleft()
                r.status = cdef.CDEF_E_NOMEM
                self.rejected.append(r)
                continue
            if self.in_use + need > self.budget:
                evict = getattr(self.ex, "evict", None)
                if evict:  # idle resident frames, never the one `r` is about to use
                    self.in_use -= evict(self.in_use + need - self.budget, r)
                if self.in_use + need > self.budget:
                    return
            self.queue.popleft()
            self.ex.allocate(r)
            # frame planes it uploaded stay resident (and charged) until evicted
            self.in_use += r.in_bytes
            st = self.ex.validate(r)
            if st != cdef.CDEF_OK:
                r.status = st
                r.outputs, r.job = (), None
                self._release(r)
                self.rejected.append(r)
                continue
            r.out_bytes = out
            r.admitted = now
            self.in_use += out
            self.ready.append(r)

    def _release(self, r: Request) -> None:
        f = getattr(self.ex, "release", None)
        if f:
            f(r)

    def _retire(self) -> List[Request]:
        done = []
        in_order = getattr(self.ex, "in_order", False)
        for h in list(self.running):
            t = self.ex.poll(h)
            if t is None:
                if in_order:  # launches on one stream finish in order
                    break
                continue
            for r in self.running.pop(h):
                r.done = t
                self.in_use -= r.out_bytes
                self._release(r)
                if self.release_outputs:
                    r.outputs, r.job = (), None
                    if r.host is not None:  # the device frame belongs to the residency
                        r.recon = r.src = r.skip = r.strengths = None
                done.append(r)
        self.finished.extend(done)
        return done

    def step(self) -> List[Request]:
        """One scheduling round; returns the requests completed in it."""
        done = self._retire()
        self._admit(self.clock())
        while self.ready and len(self.running) < self.ex.capacity:
            if getattr(self.ex, "free_slot", None) and self.ex.free_slot() < 0:
                break
            if self.split_modes and self.max_batch > 1:
                # the oldest ready request's mode, its requests in arrival order
                mode = self.ready[0].mode
                take, rest = [], []
                for r in self.ready:
                    (take if r.mode == mode and len(take) < self.max_batch else rest).append(r)
                self.ready = rest
            else:
                take, self.ready = self.ready[:self.max_batch], self.ready[self.max_batch:]
            h = self.ex.launch(take)
            for r in take:
                r.batch_id = self.nbatches
            self.nbatches += 1
            self.running[h] = take
        return done

    @property
    def idle(self) -> bool:
        return not (self.queue or self.ready or self.running)


def run_trace(sched: Scheduler, requests: List[Request], offsets: np.ndarray,
              spin: float = 20e-6) -> float:
    """Submit request k at start + offsets[k] (host clock) and run the
    scheduler until all complete.  Returns the wall time.  Python's cyclic
    garbage collector is paused meanwhile (a collection would stall the
    loop for milliseconds)."""
    import gc
    gc.collect()
    was = gc.isenabled()
    gc.disable()
    try:
        return _run_trace(sched, requests, offsets, spin)
    finally:
        if was:
            gc.enable()


def _run_trace(sched, requests, offsets, spin):
    start = time.perf_counter()
    k = 0
    n = len(requests)
    while k < n or not sched.idle:
        now = time.perf_counter()
        while k < n and start + offsets[k] <= now:
            requests[k].arrival = start + offsets[k]
            sched.submit(requests[k])
            k += 1
        sched.step()
        if k < n and sched.idle:
            time.sleep(max(0.0, min(spin, start + offsets[k] - time.perf_counter())))
    return time.perf_counter() - start


# ---- benchmark (bench.py --workload serve) ---------------------------------

def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_request_pool(n_frames: int = 20, seed: int = 4):
    """Device-resident frames of the mixed resolution / bit-depth set."""
    import torch
    from . import synth
    rng = np.random.default_rng(seed)
    pool = []
    params = synth.mixed_frame_params(n_frames, 4)
    for i, (w, h, bd, D) in enumerate(params):
        fr = synth.make_frame(w, h, bd, synth.LAYOUT_420, synth.workload_seed(synth.WL_SERVE, i), damping=D)
        rec = cdef.Frame.from_numpy(fr.recon, w, h, bd, fr.layout)
        src = cdef.Frame.from_numpy(fr.src, w, h, bd, fr.layout)
        st = torch.from_numpy(synth.random_strengths(fr, 70 + i)).cuda()
        pool.append((fr, rec, src, st))
    del rng
    return pool


def make_host_pool(n_frames: int = 20, seed: int = 4):
    """The request frames of make_request_pool in pinned host memory: per
    frame (synth frame, recon planes, source planes, skip map, strengths)."""
    import torch
    from . import synth

    def pin(a):
        t = torch.from_numpy(a.view("int16") if a.dtype.name == "uint16" else a)
        return t.pin_memory()

    pool = []
    for i, (w, h, bd, D) in enumerate(synth.mixed_frame_params(n_frames, 4)):
        fr = synth.make_frame(w, h, bd, synth.LAYOUT_420, synth.workload_seed(synth.WL_SERVE, i),
                              damping=D)
        pool.append((fr, [pin(p) for p in fr.recon], [pin(p) for p in fr.src], None,
                     pin(synth.random_strengths(fr, 70 + i))))
    return pool


def make_host_requests(pool, n_frames: int, seed: int, key0: int = 0):
    """Frames arriving from host memory, each asking for the strength search
    and then the filter (an encoder's two passes over one frame): 2 n_frames
    requests; every frame is new (its own key), so each is uploaded once and
    its filter request finds it resident."""
    rng = np.random.default_rng(seed)
    reqs = []
    for k in range(n_frames):
        fr, rec, src, skip, st = pool[int(rng.integers(0, len(pool)))]
        host = HostFrame(key0 + k, rec, src, skip, fr.width, fr.height, fr.bitdepth, fr.layout)
        stub = cdef.Frame([None] * 3, fr.width, fr.height, fr.bitdepth, fr.layout)
        reqs.append(Request(rid=2 * k, mode=SEARCH, recon=stub, host=host, damping=fr.damping))
        reqs.append(Request(rid=2 * k + 1, mode=FILTER, recon=stub, host=host,
                            host_strengths=st, damping=fr.damping))
    return reqs


def make_requests(pool, n: int, seed: int) -> List[Request]:
    rng = np.random.default_rng(seed)
    reqs = []
    for k in range(n):
        fr, rec, src, st = pool[int(rng.integers(0, len(pool)))]
        mode = SEARCH if rng.random() < 0.5 else FILTER
        reqs.append(Request(rid=k, mode=mode, recon=rec, src=src if mode == SEARCH else None,
                            strengths=st if mode == FILTER else None, damping=fr.damping))
    return reqs


def _stats(reqs: List[Request], wall: float) -> dict:
    lat = np.array([(r.done - r.arrival) * 1e3 for r in reqs])
    px = sum(r.luma_px for r in reqs)
    worst = np.argsort(lat)[-3:][::-1]
    t0 = min(r.arrival for r in reqs)
    return {"p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "max_ms": round(float(lat.max()), 3),
            "mean_ms": round(float(lat.mean()), 3),
            "mpixel_s": round(float(px / wall / 1e6), 1),
            "requests": len(reqs),
            "worst": [{"rid": reqs[i].rid, "ms": round(float(lat[i]), 3),
                       "at_s": round(reqs[i].arrival - t0, 4),
                       "admit_wait_ms": round((reqs[i].admitted - reqs[i].arrival) * 1e3, 3)}
                      for i in worst]}


def capacity(pool, batching: bool, n_req: int, budget: int, seed: int = 2) -> float:
    """Requests per second of one path with every request submitted at once."""
    ex = GpuBatchExecutor() if batching else GpuPlainExecutor()
    ex.set_epoch()
    sch = Scheduler(ex, budget, batching=batching, release_outputs=True)
    reqs = make_requests(pool, n_req, seed)
    wall = run_trace(sch, reqs, np.zeros(len(reqs)))
    return n_req / wall


def rate_trace(pool, rate: float, n_req: int, warm: int, budget: int, seed: int) -> dict:
    """Both paths on the same Poisson arrivals at `rate` requests/s: latency
    percentiles and throughput of the n_req requests after `warm`."""
    rng = np.random.default_rng(seed)
    offs = np.cumsum(rng.exponential(1.0 / rate, n_req + warm))
    res = {"rate_req_s": round(rate, 1)}
    for name, mk, batching in (("plain", GpuPlainExecutor, False),
                               ("batched", GpuBatchExecutor, True)):
        ex = mk()
        ex.set_epoch()
        sch = Scheduler(ex, budget, batching=batching, release_outputs=True)
        reqs = make_requests(pool, n_req + warm, 3)
        run_trace(sch, reqs, offs)
        kept = sorted(sch.finished, key=lambda r: r.rid)[warm:]
        span = max(r.done for r in kept) - min(r.arrival for r in kept)
        st = _stats(kept, span)
        st["batches"] = sch.nbatches
        res[name] = st
        _log(f"rate {rate:.0f}/s {name}: p50 {st['p50_ms']} p99 {st['p99_ms']} ms")
    res["p99_gain"] = round(res["plain"]["p99_ms"] / res["batched"]["p99_ms"], 3)
    res["p50_gain"] = round(res["plain"]["p50_ms"] / res["batched"]["p50_ms"], 3)
    return res


def host_capacity(pool, batching: bool, n_frames: int, budget: int, seed: int = 2) -> float:
    """Frames per second of one path with every host frame submitted at once."""
    ex = GpuBatchExecutor() if batching else GpuPlainExecutor()
    ex.set_epoch()
    sch = Scheduler(ex, budget, batching=batching, release_outputs=True)
    reqs = make_host_requests(pool, n_frames, seed, key0=10 ** 9 * (1 + seed))
    wall = run_trace(sch, reqs, np.zeros(len(reqs)))
    return n_frames / wall


def host_rate_trace(pool, rate: float, n_frames: int, warm: int, budget: int, seed: int) -> dict:
    """Both paths on the same Poisson arrivals of host frames (`rate` frames/s,
    each a search request then a filter request): latency of each request
    from the frame's arrival, over the frames after `warm`."""
    rng = np.random.default_rng(seed)
    offs = np.repeat(np.cumsum(rng.exponential(1.0 / rate, n_frames + warm)), 2)
    res = {"rate_frames_s": round(rate, 1)}
    for name, mk, batching in (("plain", GpuPlainExecutor, False),
                               ("batched", GpuBatchExecutor, True)):
        ex = mk()
        ex.set_epoch()
        sch = Scheduler(ex, budget, batching=batching, release_outputs=True)
        reqs = make_host_requests(pool, n_frames + warm, 3, key0=10 ** 6 * (1 + seed))
        run_trace(sch, reqs, offs)
        kept = sorted(sch.finished, key=lambda r: r.rid)[2 * warm:]
        span = max(r.done for r in kept) - min(r.arrival for r in kept)
        st = _stats(kept, span)
        st["batches"] = sch.nbatches
        res[name] = st
        _log(f"host frames {rate:.0f}/s {name}: p50 {st['p50_ms']} p99 {st['p99_ms']} ms")
    res["p99_gain"] = round(res["plain"]["p99_ms"] / res["batched"]["p99_ms"], 3)
    res["p50_gain"] = round(res["plain"]["p50_ms"] / res["batched"]["p50_ms"], 3)
    return res


HOST_WORKLOAD = ("Poisson arrivals of frames in pinned host memory (resolutions uniform over "
                 "426x240..3840x2160, 8/10-bit, 4:2:0), each uploaded on admission and kept "
                 "resident, asking for the strength search and then the filter at random "
                 "per-filter-block strengths")


def host_latency_summary(n_frames: int = 500, warm: int = 50, frac: float = 0.7,
                         pool_frames: int = 20) -> dict:
    """Host arrivals: the plain path's capacity, then both paths at `frac` of it."""
    import torch
    _log("serving from host memory: building the pinned pool")
    pool = make_host_pool(pool_frames)
    budget = int(torch.cuda.mem_get_info()[0] * 0.9)
    host_capacity(pool, False, min(warm, n_frames), budget, seed=1)  # warm-up
    plain = host_capacity(pool, False, n_frames, budget)
    _log(f"serving from host memory: plain path capacity {plain:.0f} frames/s")
    res = host_rate_trace(pool, frac * plain, n_frames, warm, budget, int(frac * 100))
    res.update({"workload": HOST_WORKLOAD, "rate_fraction_of_plain": frac,
                "plain_capacity_frames_s": round(plain, 1)})
    return res


WORKLOAD = ("Poisson arrivals of device-resident frames, resolutions uniform over "
            "426x240..3840x2160, 8/10-bit, 4:2:0, 50% strength search / 50% "
            "direction search + filter at random per-filter-block strengths")


def latency_summary(n_req: int = 2000, warm: int = 200, frac: float = 0.7,
                    pool_frames: int = 20) -> dict:
    """The serving trace of the benchmark's headline line: the plain path's
    capacity, then both paths at `frac` of it."""
    import torch
    _log("serving: building the request pool")
    pool = make_request_pool(pool_frames)
    budget = int(torch.cuda.mem_get_info()[0] * 0.9)
    capacity(pool, False, min(warm, n_req), budget, seed=1)  # warm-up
    plain_rate = capacity(pool, False, n_req, budget)
    _log(f"serving: plain path capacity {plain_rate:.0f} requests/s")
    res = rate_trace(pool, frac * plain_rate, n_req, warm, budget, int(frac * 100))
    res.update({"workload": WORKLOAD, "rate_fraction_of_plain": frac,
                "plain_capacity_req_s": round(plain_rate, 1)})
    return res


def bench_main(args) -> None:
    import torch
    n_req = 4000
    warm = 200
    _log("building the request pool")
    pool = make_request_pool()
    budget = int(torch.cuda.mem_get_info()[0] * 0.9)
    capacity(pool, False, warm, budget, seed=1)  # warm-up
    plain_rate = capacity(pool, False, n_req, budget)
    _log(f"plain path back-to-back: {plain_rate:.0f} requests/s")
    batched_rate = capacity(pool, True, n_req, budget)
    _log(f"batched path back-to-back: {batched_rate:.0f} requests/s")
    out = {"workload": WORKLOAD,
           "plain_capacity_req_s": round(plain_rate, 1),
           "batched_capacity_req_s": round(batched_rate, 1), "rates": []}
    for frac in (0.7, 0.3, 0.9, 1.2, 1.6):
        res = rate_trace(pool, frac * plain_rate, n_req, warm, budget, int(frac * 100))
        res["rate_fraction_of_plain"] = frac
        out["rates"].append(res)
    # frames arriving in host memory
    hpool = make_host_pool()
    n_fr = n_req // 4
    host_capacity(hpool, False, warm, budget, seed=1)  # warm-up
    hplain = host_capacity(hpool, False, n_fr, budget)
    hbatch = host_capacity(hpool, True, n_fr, budget)
    out["host"] = {"workload": HOST_WORKLOAD, "plain_capacity_frames_s": round(hplain, 1),
                   "batched_capacity_frames_s": round(hbatch, 1), "rates": []}
    for frac in (0.7, 1.2):
        res = host_rate_trace(hpool, frac * hplain, n_fr, warm // 4, budget, int(frac * 100))
        res["rate_fraction_of_plain"] = frac
        out["host"]["rates"].append(res)
    print(json.dumps(out), flush=True)
