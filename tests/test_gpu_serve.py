"""The continuous-batching server on the GPU: every request's result is
bit-identical to the same request computed alone through the per-frame
entry points, whichever batch it joined, and a bad request fails alone."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_05975_amd import cdef
    cdef.load()


def _pool():
    import torch
    from paper_1602_05975_amd import cdef, synth
    pool = []
    for i, (w, h, bd, D) in enumerate([(426, 240, 8, 3), (200, 136, 10, 4), (131, 67, 10, 6),
                                       (640, 360, 10, 3), (96, 70, 8, 5)]):
        fr = synth.make_frame(w, h, bd, synth.LAYOUT_420, 77000 + i, skip_prob=0.2, damping=D)
        rec = cdef.Frame.from_numpy(fr.recon, w, h, bd, fr.layout)
        src = cdef.Frame.from_numpy(fr.src, w, h, bd, fr.layout)
        st = torch.from_numpy(synth.random_strengths(fr, 90 + i)).cuda()
        skip = torch.from_numpy(fr.skip).cuda()
        pool.append((fr, rec, src, st, skip))
    return pool


def _requests(pool, n, seed):
    from paper_1602_05975_amd import serve
    rng = np.random.default_rng(seed)
    reqs = []
    for k in range(n):
        fr, rec, src, st, skip = pool[int(rng.integers(0, len(pool)))]
        mode = serve.SEARCH if rng.random() < 0.5 else serve.FILTER
        reqs.append(serve.Request(rid=k, mode=mode, recon=rec,
                                  src=src if mode == serve.SEARCH else None,
                                  strengths=st if mode == serve.FILTER else None,
                                  skip=skip, damping=fr.damping))
    return reqs


def _alone(req):
    from paper_1602_05975_amd import cdef, serve
    if req.mode == serve.SEARCH:
        return cdef.search_strengths(req.recon, req.src, req.skip, req.damping)
    d, v = cdef.find_dir(req.recon)
    return cdef.filter_frame(req.recon, d, v, req.skip, req.damping, req.strengths)


# heavy_work 64: searches above 16 filter blocks (and filters above 64)
# count as heavy, so the small test frames exercise the policy that queues
# heavy batches behind each other
@pytest.mark.parametrize("batching,streams,depth,heavy", [
    (True, 2, 1, 3072), (True, 1, 2, 3072), (True, 2, 2, 3072), (True, 2, 2, 64), (True, 3, 2, 64),
    (False, 1, 1, 0)])
def test_served_results_equal_alone(batching, streams, depth, heavy):
    import torch
    from paper_1602_05975_amd import serve
    pool = _pool()
    reqs = _requests(pool, 120, 5)
    if batching:
        ex = serve.GpuBatchExecutor(n_streams=streams, depth=depth, heavy_work=heavy)
    else:
        ex = serve.GpuPlainExecutor()
    ex.set_epoch()
    sched = serve.Scheduler(ex, budget_bytes=64 << 20, batching=batching)
    offs = np.cumsum(np.random.default_rng(6).exponential(1.0 / 4000.0, len(reqs)))
    print(f"serving {len(reqs)} requests, batching={batching}, {streams} streams, "
          f"depth {depth}, heavy above {heavy} work units", flush=True)
    serve.run_trace(sched, reqs, offs)
    torch.cuda.synchronize()
    assert len(sched.finished) == len(reqs) and not sched.rejected
    if batching:
        assert sched.nbatches < len(reqs)
    for r in sched.finished:
        assert r.done >= r.arrival
        ref = _alone(r)
        torch.cuda.synchronize()
        if r.mode == serve.SEARCH:
            assert torch.equal(r.outputs[0], ref), r.rid
        else:
            for a, b in zip(r.outputs[0], ref):
                assert torch.equal(a, b), r.rid


def test_bad_request_fails_alone():
    import torch
    from paper_1602_05975_amd import serve
    pool = _pool()
    reqs = _requests(pool, 10, 8)
    reqs[4].damping = 9  # invalid
    ex = serve.GpuBatchExecutor()
    ex.set_epoch()
    sched = serve.Scheduler(ex, budget_bytes=64 << 20)
    serve.run_trace(sched, reqs, np.zeros(len(reqs)))
    torch.cuda.synchronize()
    assert [r.rid for r in sched.rejected] == [4]
    assert sorted(r.rid for r in sched.finished) == [0, 1, 2, 3, 5, 6, 7, 8, 9]
    for r in sched.finished:
        ref = _alone(r)
        torch.cuda.synchronize()
        got = r.outputs[0]
        if r.mode == serve.SEARCH:
            assert torch.equal(got, ref)
        else:
            assert all(torch.equal(a, b) for a, b in zip(got, ref))


def _host_pool():
    import torch
    from paper_1602_05975_amd import synth

    def pin(a):
        return torch.from_numpy(a.view(np.int16) if a.dtype == np.uint16 else a).pin_memory()

    pool = []
    for i, (w, h, bd, D) in enumerate([(426, 240, 8, 3), (200, 136, 10, 4), (131, 67, 10, 6),
                                       (640, 360, 10, 3), (96, 70, 8, 5)]):
        fr = synth.make_frame(w, h, bd, synth.LAYOUT_420, 78000 + i, skip_prob=0.2, damping=D)
        st = synth.random_strengths(fr, 95 + i)
        pool.append((fr, [pin(p) for p in fr.recon], [pin(p) for p in fr.src], pin(fr.skip),
                     pin(st), st))
    return pool


@pytest.mark.parametrize("batching", [True, False])
def test_host_arrivals_equal_alone(batching):
    # Frames arrive in pinned host memory; each is uploaded on admission,
    # kept resident for its later requests and evicted when idle and the
    # budget (a few frames) needs room.  Every result equals the request
    # computed alone on device copies made independently of the server.
    import torch
    from helpers import gpu_frame
    from paper_1602_05975_amd import cdef, serve
    pool = _host_pool()
    rng = np.random.default_rng(12)
    reqs, refs = [], []
    keys = [int(k) for k in rng.integers(0, 9, size=40)]  # repeated keys: residency hits
    for k, key in enumerate(keys):
        fr, rec, src, skip, st, st_np = pool[key % len(pool)]
        host = serve.HostFrame(key, rec, src, skip, fr.width, fr.height, fr.bitdepth, fr.layout)
        stub = cdef.Frame([None] * 3, fr.width, fr.height, fr.bitdepth, fr.layout)
        mode = serve.SEARCH if rng.random() < 0.5 else serve.FILTER
        reqs.append(serve.Request(rid=k, mode=mode, recon=stub, host=host, damping=fr.damping,
                                  host_strengths=st if mode == serve.FILTER else None))
        refs.append((fr, st_np))
    big = max(sum(p.nbytes for p in fr.recon + fr.src) + fr.skip.nbytes for fr, *_ in pool)
    out = max(serve.output_bytes(r) for r in reqs)
    budget = 3 * (big + out)
    ex = serve.GpuBatchExecutor(n_streams=2) if batching else serve.GpuPlainExecutor()
    ex.set_epoch()
    sched = serve.Scheduler(ex, budget_bytes=budget, batching=batching)
    offs = np.cumsum(np.random.default_rng(13).exponential(1.0 / 3000.0, len(reqs)))
    print(f"serving {len(reqs)} host-memory requests, batching={batching}", flush=True)
    serve.run_trace(sched, reqs, offs)
    torch.cuda.synchronize()
    assert len(sched.finished) == len(reqs) and not sched.rejected
    assert sum(r.in_bytes > 0 for r in sched.finished) < len(reqs)  # some found their frame
    assert sched.in_use == ex.frames.resident_bytes <= budget
    for r in sched.finished:
        fr, st_np = refs[r.rid]
        rec, src = gpu_frame(fr.recon, fr), gpu_frame(fr.src, fr)
        sk = torch.from_numpy(fr.skip).cuda()
        if r.mode == serve.SEARCH:
            want = cdef.search_strengths(rec, src, sk, fr.damping)
            torch.cuda.synchronize()
            assert torch.equal(r.outputs[0], want), r.rid
        else:
            d, v = cdef.find_dir(rec)
            want = cdef.filter_frame(rec, d, v, sk, fr.damping, torch.from_numpy(st_np).cuda())
            torch.cuda.synchronize()
            for a, b in zip(r.outputs[0], want):
                assert torch.equal(a, b), r.rid
