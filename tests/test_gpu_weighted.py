"""The contrast-weighted search (Section 5, Eq. 14) on the GPU against the
oracle.

Tolerance: both sides sum the same integer pixels; the GPU forms each unit's
weight from exact integer moments (n sum x^2 - (sum x)^2) and the oracle from
the textbook two-pass variance, both in double precision.  Each unit's value
then differs by a few units in the last place (relative ~1e-15), and a
filter block's sum of at most 128 units by less than 1e-13 relative; the
tests allow 1e-10.
"""
import numpy as np
import pytest

from helpers import ORACLE_THREADS, gpu_frame

pytestmark = pytest.mark.gpu

RTOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_05975_amd import cdef
    cdef.load()


def _synth():
    from paper_1602_05975_amd import synth
    return synth


def _gpu_weighted(fr, skip=True):
    import torch
    from paper_1602_05975_amd import cdef
    rec, src = gpu_frame(fr.recon, fr), gpu_frame(fr.src, fr)
    sk = torch.from_numpy(fr.skip).cuda() if skip else None
    dist, d, v = cdef.search_strengths(rec, src, sk, fr.damping, want_dir=True, weighted=True)
    torch.cuda.synchronize()
    return dist.cpu().numpy(), d.cpu().numpy(), v.cpu().numpy()


def _compare(oracle, fr, skip=True, fbs=None):
    dist, d, v = _gpu_weighted(fr, skip)
    od, ov = oracle.find_dir(fr.recon[0], fr.bitdepth)
    assert (d == od).all() and (v == ov).all()
    if fbs is None:
        fbs = [(by, bx) for by in range(fr.fb_rows) for bx in range(fr.fb_cols)]
    ref = oracle.search_fbs_weighted(fr.recon, fr.src, fr.width, fr.height, fr.bitdepth, od, ov,
                                     fr.skip if skip else None, fr.damping, fbs,
                                     threads=ORACLE_THREADS)
    for k, (by, bx) in enumerate(fbs):
        got = dist[:, by, bx]
        if not np.allclose(got, ref[k], rtol=RTOL, atol=1e-9):
            bad = np.argwhere(~np.isclose(got, ref[k], rtol=RTOL, atol=1e-9))
            p, sp, si = bad[0]
            raise AssertionError(f"FB ({by},{bx}) plane {p} pri {sp} sec#{si}: gpu "
                                 f"{got[p, sp, si]!r} oracle {ref[k][p, sp, si]!r}")
    return dist


@pytest.mark.parametrize("w,h,bd,D", [(200, 136, 10, 3), (200, 136, 8, 4), (131, 67, 10, 5),
                                      (136, 72, 10, 6), (426, 240, 10, 3), (426, 240, 8, 6)])
def test_weighted_small_frames(oracle, w, h, bd, D):
    s = _synth()
    fr = s.make_frame(w, h, bd, s.LAYOUT_420, 61000 + w + D, skip_prob=0.3, damping=D)
    if fr.fb_cols > 1:
        fr.skip[0:8, 8:16] = 1
    print(f"weighted {w}x{h} {bd}-bit D={D}", flush=True)
    _compare(oracle, fr)


def test_weighted_tiny_luma_only_unskipped(oracle):
    s = _synth()
    for (w, h) in [(1, 1), (7, 5), (65, 65), (130, 9)]:
        fr = s.make_frame(w, h, 10, s.LAYOUT_420, 62000 + w, skip_prob=0.3, damping=3)
        print(f"weighted tiny {w}x{h}", flush=True)
        _compare(oracle, fr)
    fr = s.make_frame(150, 70, 8, s.LAYOUT_400, 62077, skip_prob=0.3, damping=4)
    print("weighted luma only", flush=True)
    _compare(oracle, fr)
    fr = s.make_frame(150, 70, 10, s.LAYOUT_420, 62078, damping=5)
    print("weighted without skip map", flush=True)
    _compare(oracle, fr, skip=False)


def test_weighted_all_skipped(oracle):
    s = _synth()
    fr = s.make_frame(128, 64, 10, s.LAYOUT_420, 63000, damping=3)
    fr.skip[:] = 1
    dist = _compare(oracle, fr)
    for p in range(3):
        assert (dist[p] == dist[p, :, :, :1, :1]).all()


def test_weighted_1080p_sampled(oracle):
    s = _synth()
    base = s.hd1080_frame()
    fr = s.make_frame(base.width, base.height, 10, s.LAYOUT_420, base.seed, skip_prob=0.3,
                      damping=3)
    rng = np.random.default_rng(64000)
    fbs = {(0, 0), (0, 29), (16, 0), (16, 29), (8, 15)}
    while len(fbs) < 40:
        fbs.add((int(rng.integers(0, 17)), int(rng.integers(0, 30))))
    print("weighted 1920x1080 sampled", flush=True)
    _compare(oracle, fr, fbs=sorted(fbs))


def test_weighted_in_batch_equals_per_frame():
    import torch
    from paper_1602_05975_amd import cdef
    s = _synth()
    b = cdef.Batch()
    jobs = []
    for i, (w, h, bd, D, mode) in enumerate([(200, 136, 10, 3, "weighted"),
                                             (131, 67, 8, 5, "search"),
                                             (64, 64, 10, 4, "weighted"),
                                             (150, 70, 10, 6, "search128")]):
        fr = s.make_frame(w, h, bd, s.LAYOUT_420, 65000 + i, skip_prob=0.3, damping=D)
        rec, src = gpu_frame(fr.recon, fr), gpu_frame(fr.src, fr)
        skip = torch.from_numpy(fr.skip).cuda()
        full, weighted = mode == "search128", mode == "weighted"
        shape = (3, fr.fb_rows, fr.fb_cols) + ((2, 16, 4) if full else (16, 4))
        out = torch.full(shape, -1, dtype=torch.float64 if weighted else torch.int64,
                         device="cuda")
        b.add_search(rec, src, skip, D, out, full=full, weighted=weighted)
        jobs.append((rec, src, skip, D, full, weighted, out))
    b.prepare()
    # 4:2:0 weighted searches run on the base kernels (three waves per SIMD)
    assert not (b.plan.flags & 1)
    print(f"batch of {len(jobs)} jobs with weighted searches", flush=True)
    for variant in range(cdef.BATCH_VARIANTS):
        b.plan.variant = variant
        for j in jobs:
            j[-1].fill_(-1)
        b.launch()
        torch.cuda.synchronize()
        for rec, src, skip, D, full, weighted, out in jobs:
            want = cdef.search_strengths(rec, src, skip, D, full=full, weighted=weighted)
            torch.cuda.synchronize()
            assert torch.equal(out, want), (variant, full, weighted)


def test_weighted_420_in_extended_batch_equals_per_frame():
    # a 4:4:4 job puts the whole batch on the extended kernels; the 4:2:0
    # and 4:0:0 weighted jobs in it run the same moment code there, so their
    # tables equal the per-frame (base kernel) ones bit for bit
    import torch
    from paper_1602_05975_amd import cdef
    s = _synth()
    b = cdef.Batch()
    jobs = []
    for i, (w, h, bd, layout, mode) in enumerate([(200, 136, 10, s.LAYOUT_420, "weighted"),
                                                  (136, 72, 10, s.LAYOUT_444, "search"),
                                                  (131, 67, 12, s.LAYOUT_420, "weighted"),
                                                  (72, 40, 8, s.LAYOUT_400, "weighted")]):
        fr = s.make_frame(w, h, bd, layout, 65500 + i, skip_prob=0.3, damping=3 + i)
        rec, src = gpu_frame(fr.recon, fr), gpu_frame(fr.src, fr)
        skip = torch.from_numpy(fr.skip).cuda()
        weighted = mode == "weighted"
        shape = (fr.search_planes, fr.fb_rows, fr.fb_cols, 16, 4)
        out = torch.full(shape, -1, dtype=torch.float64 if weighted else torch.int64,
                         device="cuda")
        b.add_search(rec, src, skip, fr.damping, out, weighted=weighted)
        jobs.append((rec, src, skip, fr.damping, weighted, out))
    b.prepare()
    assert b.plan.flags & 1
    print(f"extended batch of {len(jobs)} jobs", flush=True)
    for variant in range(cdef.BATCH_VARIANTS):
        b.plan.variant = variant
        for j in jobs:
            j[-1].fill_(-1)
        b.launch()
        torch.cuda.synchronize()
        for rec, src, skip, D, weighted, out in jobs:
            want = cdef.search_strengths(rec, src, skip, D, weighted=weighted)
            torch.cuda.synchronize()
            assert torch.equal(out, want), (variant, weighted)
