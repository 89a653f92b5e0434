"""The skip condition bit and the (19, 7) preset on the GPU (Section 4), the
128-combination search and preset selection over it (Section 5), all
bit-exact against the oracle."""
import numpy as np
import pytest

from helpers import gpu_frame, gpu_search, oracle_search, to_np_u16

pytestmark = pytest.mark.gpu


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


def _frame(w, h, bd, D, seed, layout=None, skip_prob=0.3):
    s = _synth()
    layout = s.LAYOUT_420 if layout is None else layout
    fr = s.make_frame(w, h, bd, layout, seed, skip_prob=skip_prob, damping=D)
    if fr.fb_cols > 1:
        fr.skip[0:8, 8:16] = 1      # filter block (0, 1): every block skipped
    if fr.fb_rows > 1:
        fr.skip[8:16, 0:8] = 0      # filter block (1, 0): none skipped
    return fr


# ---- filter with presets ------------------------------------------------------

FILTER_CASES = [(426, 240, 10, 3), (200, 136, 8, 4), (131, 67, 10, 5), (136, 72, 10, 6),
                (5, 3, 8, 3)]


@pytest.mark.parametrize("w,h,bd,D", FILTER_CASES)
def test_filter_presets_match_oracle(oracle, w, h, bd, D):
    import torch
    from paper_1602_05975_amd import cdef
    s = _synth()
    fr = _frame(w, h, bd, D, 41000 + w + D)
    st = s.random_presets(fr, 42000 + h)
    print(f"filter presets {w}x{h} {bd}-bit D={D}", flush=True)
    f = gpu_frame(fr.recon, fr)
    d, v = cdef.find_dir(f)
    sk = torch.from_numpy(fr.skip).cuda()
    stg = torch.from_numpy(st).cuda()
    plain = cdef.filter_frame(f, d, v, sk, fr.damping, stg)
    # the fused filter (batch job) too
    b = cdef.Batch()
    fused = [torch.full_like(p, -1) for p in f.planes[:fr.nplanes]]
    b.add_filter(f, fused, sk, fr.damping, stg)
    b.prepare()
    b.launch()
    torch.cuda.synchronize()
    od, ov = oracle.find_dir(fr.recon[0], fr.bitdepth)
    ref = oracle.filter_frame(fr.recon, fr.width, fr.height, fr.bitdepth, od, ov, fr.skip,
                              fr.damping, st)
    for p in range(fr.nplanes):
        for name, got in (("plain", to_np_u16(plain[p])), ("fused", to_np_u16(fused[p]))):
            bad = np.argwhere(got != ref[p])
            assert bad.size == 0, (name, p, bad[:5])


# ---- 128-combination search -----------------------------------------------------

def _compare_full(oracle, fr, skip=True, fbs=None):
    sse, d, v = gpu_search(fr, skip=skip, full=True)
    ref, od, ov, fbs = oracle_search(oracle, fr, skip=skip, fbs=fbs, full=True)
    assert (d == od).all() and (v == ov).all()
    assert sse.shape == (fr.nplanes, fr.fb_rows, fr.fb_cols, 2, 16, 4)
    for k, (by, bx) in enumerate(fbs):
        got = sse[:, by, bx]
        if not (got == ref[k]).all():
            bad = np.argwhere(got != ref[k])
            p, kk, sp, si = bad[0]
            raise AssertionError(f"FB ({by},{bx}) plane {p} bit {kk} pri {sp} sec#{si}: "
                                 f"gpu {got[p, kk, sp, si]} oracle {ref[k][p, kk, sp, si]} "
                                 f"({len(bad)} mismatches)")
    return sse


@pytest.mark.parametrize("w,h,bd,D", [(200, 136, 10, 3), (200, 136, 8, 4), (131, 67, 10, 5),
                                      (136, 72, 10, 6), (426, 240, 10, 3), (426, 240, 8, 6)])
def test_search128_small_frames(oracle, w, h, bd, D):
    fr = _frame(w, h, bd, D, 43000 + w + D)
    print(f"search128 {w}x{h} {bd}-bit D={D}", flush=True)
    sse = _compare_full(oracle, fr)
    # the half without the bit is the 64-combination search
    half, _, _ = gpu_search(fr)
    assert (sse[:, :, :, 0] == half).all()


def test_search128_tiny_luma_only_unskipped(oracle):
    s = _synth()
    for (w, h) in [(1, 1), (7, 5), (65, 65), (130, 9)]:
        fr = s.make_frame(w, h, 10, s.LAYOUT_420, 44000 + w, skip_prob=0.3, damping=3)
        print(f"search128 tiny {w}x{h}", flush=True)
        _compare_full(oracle, fr)
    fr = s.make_frame(150, 70, 8, s.LAYOUT_400, 44077, skip_prob=0.3, damping=4)
    print("search128 luma only", flush=True)
    _compare_full(oracle, fr)
    fr = s.make_frame(150, 70, 10, s.LAYOUT_420, 44078, damping=5)
    print("search128 without skip map", flush=True)
    _compare_full(oracle, fr, skip=False)


def test_search128_all_skipped(oracle):
    s = _synth()
    fr = s.make_frame(128, 64, 10, s.LAYOUT_420, 45000, damping=3)
    fr.skip[:] = 1
    sse = _compare_full(oracle, fr)
    for p in range(3):
        for bx in range(2):
            assert (sse[p, 0, bx] == sse[p, 0, bx, 0, 0, 0]).all()


def test_search128_1080p_sampled(oracle):
    # 1920x1080 10-bit 4:2:0 with 30% skipped blocks: 40 of the 510 filter
    # blocks (edges, corners and a spread of interior ones) checked entry by
    # entry, the rest through the half that equals the 64-combination search.
    s = _synth()
    base = s.hd1080_frame()
    fr = s.make_frame(base.width, base.height, 10, s.LAYOUT_420, base.seed, skip_prob=0.3,
                      damping=3)
    rng = np.random.default_rng(46000)
    fbs = {(0, 0), (0, 29), (16, 0), (16, 29), (8, 15)}
    while len(fbs) < 40:
        fbs.add((int(rng.integers(0, 17)), int(rng.integers(0, 30))))
    print("search128 1920x1080 sampled", flush=True)
    sse = _compare_full(oracle, fr, fbs=sorted(fbs))
    half, _, _ = gpu_search(fr)
    assert (sse[:, :, :, 0] == half).all()


# ---- batches with every job mode ------------------------------------------------

def test_batch_with_all_modes(oracle):
    import torch
    from paper_1602_05975_amd import cdef
    s = _synth()
    specs = [(200, 136, 10, 3, "search128"), (131, 67, 8, 5, "filter"),
             (136, 72, 10, 6, "search"), (64, 64, 8, 4, "search128"),
             (150, 70, 10, 4, "filter")]
    b = cdef.Batch()
    jobs = []
    for i, (w, h, bd, D, mode) in enumerate(specs):
        fr = _frame(w, h, bd, D, 47000 + i)
        rec = gpu_frame(fr.recon, fr)
        skip = torch.from_numpy(fr.skip).cuda()
        if mode.startswith("search"):
            full = mode == "search128"
            src = gpu_frame(fr.src, fr)
            shape = (fr.nplanes, fr.fb_rows, fr.fb_cols) + ((2, 16, 4) if full else (16, 4))
            sse = torch.full(shape, -1, dtype=torch.int64, device="cuda")
            b.add_search(rec, src, skip, D, sse, full=full)
            jobs.append((fr, mode, sse, (rec, src, skip)))
        else:
            st = torch.from_numpy(s.random_presets(fr, 48000 + i)).cuda()
            o = [torch.full_like(p, -1) for p in rec.planes[:fr.nplanes]]
            b.add_filter(rec, o, skip, D, st)
            jobs.append((fr, mode, o, (rec, st, skip)))
    b.prepare()
    print(f"batch of {len(jobs)} jobs, {b.nitems} filter blocks", flush=True)
    b.launch()
    torch.cuda.synchronize()
    for fr, mode, res, inp in jobs:
        if mode.startswith("search"):
            rec, src, skip = inp
            want = cdef.search_strengths(rec, src, skip, fr.damping, full=mode == "search128")
            torch.cuda.synchronize()
            assert torch.equal(res, want), mode
        else:
            rec, st, skip = inp
            d, v = cdef.find_dir(rec)
            want = cdef.filter_frame(rec, d, v, skip, fr.damping, st)
            torch.cuda.synchronize()
            for p in range(fr.nplanes):
                assert torch.equal(res[p], want[p]), (mode, p)


# ---- preset selection over 128 candidates ---------------------------------------

KEYS = ("n", "luma", "chroma", "dist", "cost", "fb_luma", "fb_chroma")


def _compare_select(oracle, sse_np, lam, refine):
    import torch
    from paper_1602_05975_amd import cdef
    print(f"select_presets shape={sse_np.shape} lambda={lam} refine={refine}", flush=True)
    g = cdef.select_presets(torch.from_numpy(sse_np.view(np.int64)).cuda(), lam, refine)
    o = oracle.select_presets(sse_np, lam, refine)
    for k in KEYS:
        assert np.array_equal(np.asarray(g[k]), np.asarray(o[k])), k
    return g


@pytest.mark.parametrize("nplanes,fbr,fbc,ties", [
    (3, 1, 1, False), (1, 5, 9, True), (3, 17, 30, False), (3, 34, 60, True),
    (3, 68, 120, False)])
def test_select_presets_128_random(oracle, nplanes, fbr, fbc, ties):
    # 48 blocks per workgroup at 128 candidates: 34 x 60 blocks (a 4K frame)
    # use 43 workgroups per group; 68 x 120 no longer fit in LDS
    rng = np.random.default_rng(nplanes * 100 + fbr + fbc)
    top = 5 if ties else 1 << 30
    sse = rng.integers(0, top, size=(nplanes, fbr, fbc, 2, 16, 4)).astype(np.uint64)
    for lam, refine in ((0.0, 0), (float(top) / 64, 2), (float(top) / 4, 16)):
        _compare_select(oracle, sse, lam, refine)


def test_select_presets_128_on_searched_frame(oracle):
    s = _synth()
    fr = _frame(426, 240, 10, 3, 49000)
    sse, _, _ = gpu_search(fr, full=True)
    for lam in (0.0, 2e3, 2e5):
        for refine in (0, 4):
            r = _compare_select(oracle, sse, lam, refine)
            assert r["n"] in (1, 2, 4, 8)
