"""Continuous-batching CDEF server.

Requests are frames that are already resident in device memory (as when
CDEF runs inside a GPU codec pipeline: the reconstruction is produced on the
device and the source was uploaded once), each asking either for the
encoder's strength search or for the direction search + filter at given
per-filter-block strengths.  The scheduler

* validates each request on its own at submission (a bad request fails
  alone and never joins a batch),
* admits requests first-in first-out while the device bytes of their
  outputs fit a budget (by default 90 % of the free device memory),
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
    arrival: float = 0.0                # host clock, seconds
    # filled in by the server
    status: int = 0
    outputs: tuple = ()
    out_bytes: int = 0
    admitted: float = -1.0
    done: float = -1.0
    job: object = None
    batch_id: int = -1

    @property
    def luma_px(self) -> int:
        return self.recon.width * self.recon.height


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

    def set_epoch(self):
        self.clock = DeviceClock.shared()

    def allocate(self, req: Request):
        torch = self.torch
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

    set_epoch = GpuBatchExecutor.set_epoch
    allocate = GpuBatchExecutor.allocate
    validate = GpuBatchExecutor.validate

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
    """Admission by output bytes, continuous batching, completion polling.
    Executor-agnostic: it needs allocate / validate / launch / poll /
    capacity."""

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

    def _admit(self, now: float) -> None:
        while self.queue:
            r = self.queue[0]
            need = output_bytes(r)
            if need > self.budget:  # can never fit: reject rather than block the queue
                self.queue.popleft()
                r.status = cdef.CDEF_E_NOMEM
                self.rejected.append(r)
                continue
            if self.in_use + need > self.budget:
                return
            self.queue.popleft()
            self.ex.allocate(r)
            st = self.ex.validate(r)
            if st != cdef.CDEF_OK:
                r.status = st
                r.outputs, r.job = (), None
                self.rejected.append(r)
                continue
            r.out_bytes = need
            r.admitted = now
            self.in_use += need
            self.ready.append(r)

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
                if self.release_outputs:
                    r.outputs, r.job = (), None
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
    print(json.dumps(out), flush=True)
