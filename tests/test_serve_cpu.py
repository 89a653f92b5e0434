"""Scheduler logic of the serving loop, on the CPU with a fake executor and
a virtual clock: admission by byte budget, first-in first-out order,
rejection of bad or oversized requests without disturbing the others,
cancellation, and batching of requests that arrive while others run."""
import pytest

from paper_1602_05975_amd import cdef, serve


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Completes a launch `cost` seconds after it starts, two at a time."""

    capacity = 2

    def __init__(self, clock, cost_per_px=1e-9):
        self.clock, self.cost = clock, cost_per_px
        self.running = {}
        self.launches = []
        self.n = 0

    def allocate(self, req):
        req.outputs = ("out",)
        req.job = object()

    def validate(self, req):
        return cdef.CDEF_OK if 3 <= req.damping <= 6 else cdef.CDEF_E_INVAL

    def free_slot(self):
        return 0 if len(self.running) < self.capacity else -1

    def launch(self, reqs):
        h = self.n
        self.n += 1
        self.launches.append([r.rid for r in reqs])
        self.running[h] = self.clock() + self.cost * sum(r.luma_px for r in reqs)
        return h

    def poll(self, h):
        t = self.running.get(h)
        if t is None or self.clock() < t:
            return None
        del self.running[h]
        return t


def _req(rid, w=64, h=64, mode=serve.SEARCH, damping=3):
    f = cdef.Frame([None, None, None], w, h, 10, cdef.LAYOUT_420)
    return serve.Request(rid=rid, mode=mode, recon=f, damping=damping)


def _run(sched, clock, reqs, arrivals, dt=1e-6, limit=10.0):
    k = 0
    peak = 0
    while k < len(reqs) or not sched.idle:
        while k < len(reqs) and arrivals[k] <= clock.t:
            reqs[k].arrival = arrivals[k]
            sched.submit(reqs[k])
            k += 1
        sched.step()
        peak = max(peak, sched.in_use)
        assert sched.in_use <= sched.budget
        clock.t += dt
        assert clock.t < limit
    return peak


def test_budget_fifo_and_completion():
    clock = Clock()
    ex = FakeExecutor(clock)
    need = serve.output_bytes(_req(0))
    sched = serve.Scheduler(ex, budget_bytes=3 * need, clock=clock)
    reqs = [_req(i) for i in range(20)]
    peak = _run(sched, clock, reqs, [0.0] * 20)
    assert peak <= 3 * need and peak > need
    assert sorted(r.rid for r in sched.finished) == list(range(20))
    order = [r.admitted for r in sorted(sched.finished, key=lambda r: r.rid)]
    assert order == sorted(order)  # admitted first-in first-out
    assert all(r.done >= r.arrival for r in sched.finished)


def test_oversized_and_invalid_requests_fail_alone():
    clock = Clock()
    ex = FakeExecutor(clock)
    small = serve.output_bytes(_req(0))
    sched = serve.Scheduler(ex, budget_bytes=4 * small, clock=clock)
    reqs = [_req(0), _req(1, w=4000, h=4000), _req(2, damping=9), _req(3), _req(4)]
    _run(sched, clock, reqs, [0.0] * 5)
    assert sorted(r.rid for r in sched.finished) == [0, 3, 4]
    rej = {r.rid: r.status for r in sched.rejected}
    assert rej == {1: cdef.CDEF_E_NOMEM, 2: cdef.CDEF_E_INVAL}
    for launch in ex.launches:
        assert 1 not in launch and 2 not in launch


def test_cancel_before_admission():
    clock = Clock()
    ex = FakeExecutor(clock)
    need = serve.output_bytes(_req(0))
    sched = serve.Scheduler(ex, budget_bytes=need, clock=clock)
    for i in range(4):
        sched.submit(_req(i))
    sched.step()  # admits and launches request 0 only (budget of one)
    assert sched.cancel(2) and not sched.cancel(0)
    while not sched.idle:
        clock.t += 1e-5
        sched.step()
    assert sorted(r.rid for r in sched.finished) == [0, 1, 3]


def test_requests_arriving_during_a_launch_join_the_next_batch():
    clock = Clock()
    ex = FakeExecutor(clock, cost_per_px=1e-7)  # a 64x64 request takes 0.4 ms
    sched = serve.Scheduler(ex, budget_bytes=1 << 30, clock=clock)
    reqs = [_req(i) for i in range(12)]
    arrivals = [0.0] + [1e-4 * i for i in range(1, 12)]
    _run(sched, clock, reqs, arrivals, dt=5e-6)
    sizes = [len(b) for b in ex.launches]
    assert sizes[0] == 1 and max(sizes) > 1 and sum(sizes) == 12
    flat = [rid for b in ex.launches for rid in b]
    assert flat == sorted(flat)  # batches keep arrival order


def test_plain_mode_is_one_request_per_launch():
    clock = Clock()
    ex = FakeExecutor(clock)
    sched = serve.Scheduler(ex, budget_bytes=1 << 30, batching=False, clock=clock)
    _run(sched, clock, [_req(i) for i in range(6)], [0.0] * 6)
    assert all(len(b) == 1 for b in ex.launches) and len(ex.launches) == 6


def test_release_outputs_drops_finished_results():
    clock = Clock()
    ex = FakeExecutor(clock)
    sched = serve.Scheduler(ex, budget_bytes=1 << 30, clock=clock, release_outputs=True)
    _run(sched, clock, [_req(i) for i in range(5)], [0.0] * 5)
    assert len(sched.finished) == 5
    assert all(r.outputs == () and r.job is None and r.done >= r.arrival for r in sched.finished)


def test_request_work():
    f = cdef.Frame([None, None, None], 3840, 2160, 10, cdef.LAYOUT_420)
    search = serve.Request(rid=0, mode=serve.SEARCH, recon=f)
    filt = serve.Request(rid=1, mode=serve.FILTER, recon=f)
    assert serve.request_work(filt) == 60 * 34
    assert serve.request_work(search) == 60 * 34 * serve.SEARCH_WORK
    assert serve.request_work(search, 1) == 60 * 34


def test_stream_choice():
    H = 768
    # idle stream first; no room anywhere -> -1
    assert serve.choose_stream([[], []], 10, 2, H, True) == 0
    assert serve.choose_stream([[5], []], 10, 2, H, True) == 1
    assert serve.choose_stream([[5, 5], [9, 9]], 10, 2, H, True) == -1
    # light batch with every stream busy: least work in flight
    assert serve.choose_stream([[2000], [30]], 10, 2, H, True) == 1
    # heavy batch behind a heavy one in flight, even when a stream is idle
    assert serve.choose_stream([[30], [2040], []], 2040, 2, H, True) == 1
    assert serve.choose_stream([[30], [2040], []], 2040, 2, H, False) == 2
    # the heavy stream is full: an idle stream takes it
    assert serve.choose_stream([[2040, 2040], []], 2040, 2, H, True) == 1
    # depth 1 never queues behind
    assert serve.choose_stream([[2040], []], 2040, 1, H, True) == 1


def test_batches_hold_one_mode_in_arrival_order():
    clock = Clock()
    ex = FakeExecutor(clock, cost_per_px=1e-7)
    sched = serve.Scheduler(ex, budget_bytes=1 << 30, clock=clock)
    modes = [serve.SEARCH, serve.FILTER, serve.SEARCH, serve.FILTER, serve.FILTER, serve.SEARCH]
    reqs = [_req(i, mode=m) for i, m in enumerate(modes)]
    _run(sched, clock, reqs, [0.0] * len(reqs), dt=5e-6)
    mode_of = {r.rid: r.mode for r in reqs}
    assert sorted(rid for b in ex.launches for rid in b) == list(range(len(reqs)))
    for b in ex.launches:
        assert len({mode_of[rid] for rid in b}) == 1 and b == sorted(b)
    # the first batch takes the oldest request's mode; the other mode follows
    assert ex.launches[0] == [0, 2, 5] and ex.launches[1] == [1, 3, 4]
    # without splitting, one batch takes everything that is ready
    ex2 = FakeExecutor(Clock(), cost_per_px=1e-7)
    sched2 = serve.Scheduler(ex2, budget_bytes=1 << 30, clock=ex2.clock, split_modes=False)
    _run(sched2, ex2.clock, [_req(i, mode=m) for i, m in enumerate(modes)], [0.0] * 6, dt=5e-6)
    assert ex2.launches[0] == list(range(6))


class FakeResident(serve.ResidentFrames):
    """Residency without a device: uploads are recorded, events are done."""

    def __init__(self):
        super().__init__(stream=None)
        self.uploads = []

    def _upload(self, planes):
        self.uploads.append(sum(t.numel() * t.element_size() for t in planes))
        return [t for t in planes]

    def _record(self):
        return "event"

    @staticmethod
    def _done(ev):
        return False


class HostExecutor(FakeExecutor):
    """FakeExecutor with host frames kept resident as the GPU executors do."""

    def __init__(self, clock, cost_per_px=1e-9):
        super().__init__(clock, cost_per_px)
        self.frames = FakeResident()

    def input_bytes(self, req):
        return 0 if req.host is None else self.frames.bytes_needed(req.host, req.mode == serve.SEARCH)

    def evict(self, nbytes, req=None):
        keep = req.host.key if req is not None and req.host is not None else None
        return self.frames.evict(nbytes, keep)

    def release(self, req):
        if req.host is not None:
            self.frames.release(req.host.key)

    def allocate(self, req):
        if req.host is not None:
            serve._attach_host(self.frames, req)
        super().allocate(req)


def _host(key, w=64, h=64):
    import torch
    rec = [torch.zeros((h, w), dtype=torch.int16), torch.zeros((h // 2, w // 2), dtype=torch.int16),
           torch.zeros((h // 2, w // 2), dtype=torch.int16)]
    src = [torch.zeros_like(t) for t in rec]
    return serve.HostFrame(key, rec, src, None, w, h, 10, cdef.LAYOUT_420)


def _hreq(rid, host, mode=serve.SEARCH):
    return serve.Request(rid=rid, mode=mode, recon=cdef.Frame([None] * 3, host.width, host.height,
                                                              10, cdef.LAYOUT_420),
                         host=host, damping=3)


def test_host_frames_are_charged_uploaded_once_and_evicted_when_idle():
    clock = Clock()
    ex = HostExecutor(clock)
    a, b, c = _host("a"), _host("b"), _host("c")
    planes = a.plane_bytes(a.recon)
    out = serve.output_bytes(_hreq(0, a))
    # room for two frames with sources and the outputs of two requests
    budget = 2 * (2 * planes) + 2 * out
    sched = serve.Scheduler(ex, budget_bytes=budget, clock=clock)
    reqs = [_hreq(0, a), _hreq(1, a, serve.FILTER), _hreq(2, b), _hreq(3, c), _hreq(4, a)]
    _run(sched, clock, reqs, [0.0, 1e-3, 2e-3, 3e-3, 4e-3], dt=1e-5)
    assert sorted(r.rid for r in sched.finished) == [0, 1, 2, 3, 4] and not sched.rejected
    # a: recon+src once for requests 0 and 1; b; c (evicting a, idle); a again
    assert ex.frames.uploads.count(planes) == 2 * 4
    assert [r.in_bytes for r in sorted(sched.finished, key=lambda r: r.rid)] == \
        [2 * planes, 0, 2 * planes, 2 * planes, 2 * planes]
    assert set(ex.frames.entries) <= {"a", "b", "c"} and len(ex.frames.entries) <= 2
    assert sched.in_use == ex.frames.resident_bytes  # only resident frames stay charged
    assert all(r.recon is not None and r.src is not None for r in sched.finished
               if r.mode == serve.SEARCH)


def test_a_frame_in_use_is_never_evicted():
    clock = Clock()
    ex = HostExecutor(clock, cost_per_px=1e-6)  # each request runs 4 ms
    a, b = _host("a"), _host("b")
    planes = a.plane_bytes(a.recon)
    out = serve.output_bytes(_hreq(0, a))
    sched = serve.Scheduler(ex, budget_bytes=2 * planes + 2 * out + 8, clock=clock)
    # b cannot be admitted until a's request finishes and a can be evicted
    reqs = [_hreq(0, a), _hreq(1, b)]
    _run(sched, clock, reqs, [0.0, 1e-4], dt=1e-5)
    r0, r1 = sorted(sched.finished, key=lambda r: r.rid)
    assert r1.admitted >= r0.done
    assert list(ex.frames.entries) == ["b"]
