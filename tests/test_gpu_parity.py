"""Bit-exact parity of the HIP path (through the C ABI) with the CPU oracle.

Every comparison is exact: directions, contrasts, filtered pixels and SSE
values are integers with a single correct value.
"""
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


# ---- direction search -------------------------------------------------------

@pytest.mark.parametrize("w,h,bd", [(352, 288, 8), (426, 240, 10), (67, 33, 8), (1, 1, 10),
                                    (9, 17, 10), (1920, 1080, 10)])
def test_find_dir_matches_oracle(oracle, w, h, bd):
    import torch
    from paper_1602_05975_amd import cdef
    s = _synth()
    fr = s.make_frame(w, h, bd, s.LAYOUT_400, 5000 + w + h)
    print(f"find_dir {w}x{h} {bd}-bit", flush=True)
    d, v = cdef.find_dir(gpu_frame(fr.recon, fr))
    torch.cuda.synchronize()
    od, ov = oracle.find_dir(fr.recon[0], bd)
    assert (d.cpu().numpy() == od).all()
    assert (v.cpu().numpy() == ov).all()


# ---- plain filter -----------------------------------------------------------

def _filter_case(oracle, fr, strengths, skip):
    import torch
    from paper_1602_05975_amd import cdef
    f = gpu_frame(fr.recon, fr)
    d, v = cdef.find_dir(f)
    sk = torch.from_numpy(skip).cuda() if skip is not None else None
    st = torch.from_numpy(np.ascontiguousarray(strengths)).cuda()
    outs = cdef.filter_frame(f, d, v, sk, fr.damping, st)
    torch.cuda.synchronize()
    od, ov = oracle.find_dir(fr.recon[0], fr.bitdepth)
    ref = oracle.filter_frame(fr.recon, fr.width, fr.height, fr.bitdepth, od, ov, skip,
                              fr.damping, strengths)
    for p in range(fr.nplanes):
        got = to_np_u16(outs[p])
        bad = np.argwhere(got != ref[p])
        assert bad.size == 0, (p, bad[:5], got[tuple(bad[0])], ref[p][tuple(bad[0])])


def test_filter_cif_luma(oracle):
    # 352x288 8-bit luma, every filter block at (pri 4, sec 2), damping 5.
    s = _synth()
    fr = s.cif_luma()
    st = np.zeros(fr.skip.shape[:0] + (fr.fb_rows, fr.fb_cols, 4), np.uint8)
    st[..., 0], st[..., 1] = 4, 2
    print("filter 352x288 luma", flush=True)
    _filter_case(oracle, fr, st, None)


@pytest.mark.parametrize("w,h,bd,D", [(426, 240, 10, 3), (200, 136, 8, 4), (131, 67, 10, 5),
                                      (64, 64, 10, 6), (5, 3, 8, 3)])
def test_filter_random_strengths_skip(oracle, w, h, bd, D):
    s = _synth()
    fr = s.make_frame(w, h, bd, s.LAYOUT_420, 7000 + w, skip_prob=0.25, damping=D)
    st = s.random_strengths(fr, 9000 + h)
    print(f"filter {w}x{h} {bd}-bit D={D}", flush=True)
    _filter_case(oracle, fr, st, fr.skip)


# ---- fused search -----------------------------------------------------------

def _compare_search(oracle, fr, skip=True, fbs=None):
    sse, d, v = gpu_search(fr, skip=skip)
    ref, od, ov, fbs = oracle_search(oracle, fr, skip=skip, fbs=fbs)
    assert (d == od).all() and (v == ov).all()
    for k, (by, bx) in enumerate(fbs):
        got = sse[:, by, bx]
        if not (got == ref[k]).all():
            bad = np.argwhere(got != ref[k])
            p, sp, si = bad[0]
            raise AssertionError(f"FB ({by},{bx}) plane {p} pri {sp} sec#{si}: "
                                 f"gpu {got[p, sp, si]} oracle {ref[k][p, sp, si]} "
                                 f"({len(bad)} mismatches)")


@pytest.mark.parametrize("w,h,bd,D", [(200, 136, 10, 3), (200, 136, 8, 4), (131, 67, 10, 5),
                                      (96, 70, 8, 6), (426, 240, 10, 3), (426, 240, 8, 6)])
def test_search_small_frames(oracle, w, h, bd, D):
    s = _synth()
    fr = s.make_frame(w, h, bd, s.LAYOUT_420, 8000 + w + D, skip_prob=0.3, damping=D)
    print(f"search {w}x{h} {bd}-bit D={D}", flush=True)
    _compare_search(oracle, fr)


def test_search_luma_only_and_tiny(oracle):
    s = _synth()
    for (w, h) in [(1, 1), (7, 5), (65, 65), (130, 9)]:
        fr = s.make_frame(w, h, 10, s.LAYOUT_420, 100 + w, skip_prob=0.2, damping=3)
        print(f"search tiny {w}x{h}", flush=True)
        _compare_search(oracle, fr)
    fr = s.make_frame(150, 70, 8, s.LAYOUT_400, 77, skip_prob=0.2, damping=4)
    _compare_search(oracle, fr)


def test_search_all_skipped(oracle):
    s = _synth()
    fr = s.make_frame(128, 64, 10, s.LAYOUT_420, 55, damping=3)
    fr.skip[:] = 1
    sse, _, _ = gpu_search(fr)
    r = [p.astype(np.int64) - q.astype(np.int64) for p, q in zip(fr.recon, fr.src)]
    for p in range(3):
        fs = 64 if p == 0 else 32
        for bx in range(2):
            want = (r[p][:, bx * fs:(bx + 1) * fs] ** 2).sum()
            assert (sse[p, 0, bx] == want).all()
    _compare_search(oracle, fr)


def test_search_1080p_full(oracle):
    # 1920x1080 10-bit 4:2:0, damping 3, no skip: all 97,920 SSEs.
    s = _synth()
    fr = s.hd1080_frame()
    print("search 1920x1080", flush=True)
    _compare_search(oracle, fr, skip=False)


@pytest.fixture(scope="module")
def uhd_batch():
    """The benchmarked launch: the eight 3840x2160 10-bit 4:2:0 frames (30 %
    of blocks skipped, damping 3) in one batch with the default plan; every
    entry also equals the frame's own cdef_search_strengths launch."""
    import torch
    from paper_1602_05975_amd import cdef
    s = _synth()
    frames = s.uhd4k_frames(8)
    b = cdef.Batch()
    outs = []
    for fr in frames:
        rec, src = gpu_frame(fr.recon, fr), gpu_frame(fr.src, fr)
        sk = torch.from_numpy(fr.skip).cuda()
        t = torch.empty((3, fr.fb_rows, fr.fb_cols, 16, 4), dtype=torch.int64, device="cuda")
        d = torch.empty((fr.blk_rows, fr.blk_cols), dtype=torch.uint8, device="cuda")
        v = torch.empty((fr.blk_rows, fr.blk_cols), dtype=torch.int32, device="cuda")
        b.add_search(rec, src, sk, fr.damping, t, d, v)
        outs.append((rec, src, sk, t, d, v))
    b.prepare()
    assert b.plan.variant == 0 and not (b.plan.flags & 1)
    print("search 8 x 3840x2160 in one batched launch", flush=True)
    b.launch()
    torch.cuda.synchronize()
    res = []
    for fr, (rec, src, sk, t, d, v) in zip(frames, outs):
        one, d1, v1 = cdef.search_strengths(rec, src, sk, fr.damping, want_dir=True)
        torch.cuda.synchronize()
        assert torch.equal(one, t) and torch.equal(d1, d) and torch.equal(v1, v)
        res.append((t.cpu().numpy().view(np.uint64), d.cpu().numpy(), v.cpu().numpy()))
    return frames, res


@pytest.mark.timeout(600)
@pytest.mark.parametrize("k", range(8))
def test_search_4k_batched_every_block(oracle, uhd_batch, k):
    # every direction, contrast and SSE of frame k of the benchmarked batch
    # (2,040 filter blocks x 3 planes x 64 pairs) against the oracle, which
    # runs on all host threads
    from helpers import ORACLE_THREADS
    frames, res = uhd_batch
    fr = frames[k]
    got, d, v = res[k]
    print(f"oracle on every filter block of 3840x2160 frame {k} (seed {fr.seed})", flush=True)
    ref, od, ov = oracle.search(fr.recon, fr.src, fr.width, fr.height, fr.bitdepth, fr.skip,
                                fr.damping, threads=ORACLE_THREADS)
    assert (d == od).all() and (v == ov).all()
    if not np.array_equal(got, ref):
        bad = np.argwhere(got != ref)
        raise AssertionError(f"{len(bad)} SSEs differ, first {tuple(bad[0])}: "
                             f"gpu {got[tuple(bad[0])]} oracle {ref[tuple(bad[0])]}")


@pytest.mark.parametrize("w,h", [(65536, 72), (24, 65536)])
def test_maximum_frame_sizes(oracle, w, h):
    # The largest width and height the library takes (2^16): the search on
    # sampled filter blocks (every one along the long edge's ends and a seeded
    # set) and the whole filtered frame, against the oracle.
    import torch
    from helpers import ORACLE_THREADS
    from paper_1602_05975_amd import cdef
    s = _synth()
    fr = s.make_frame(w, h, 10, s.LAYOUT_420, 23000 + w, skip_prob=0.3, damping=4)
    print(f"maximum size {w}x{h}", flush=True)
    rec, src = gpu_frame(fr.recon, fr), gpu_frame(fr.src, fr)
    sk = torch.from_numpy(fr.skip).cuda()
    sse, d, v = cdef.search_strengths(rec, src, sk, fr.damping, want_dir=True)
    st = s.random_presets(fr, 23100 + w)
    outs = cdef.filter_frame(rec, d, v, sk, fr.damping, torch.from_numpy(st).cuda())
    torch.cuda.synchronize()
    od, ov = oracle.find_dir(fr.recon[0], 10)
    assert (d.cpu().numpy() == od).all() and (v.cpu().numpy() == ov).all()
    fbr, fbc = fr.fb_rows, fr.fb_cols
    rng = np.random.default_rng(23)
    fbs = {(by, bx) for by in range(fbr) for bx in range(fbc)
           if min(by, fbr - 1 - by) < 2 and min(bx, fbc - 1 - bx) < 2}
    fbs |= {(int(rng.integers(0, fbr)), int(rng.integers(0, fbc))) for _ in range(12)}
    fbs = sorted(fbs)
    ref = oracle.search_fbs(fr.recon, fr.src, w, h, 10, od, ov, fr.skip, fr.damping, fbs,
                            threads=ORACLE_THREADS)
    got = sse.cpu().numpy().view(np.uint64)
    for k, (by, bx) in enumerate(fbs):
        assert (got[:, by, bx] == ref[k]).all(), (by, bx)
    want = oracle.filter_frame(fr.recon, w, h, 10, od, ov, fr.skip, fr.damping, st)
    for p in range(3):
        assert (to_np_u16(outs[p]) == want[p]).all(), p


@pytest.mark.parametrize("w,h,bd,layout", [(200, 136, 10, 1), (131, 67, 8, 0), (136, 72, 12, 3),
                                           (67, 33, 10, 2), (426, 240, 12, 1)])
def test_filter_frame_uses_caller_directions(oracle, w, h, bd, layout):
    # cdef_filter_frame filters with the directions and contrasts it is given
    # (a direction is taken modulo 8), not with ones it finds itself
    import torch
    from paper_1602_05975_amd import cdef
    s = _synth()
    fr = s.make_frame(w, h, bd, layout, 24000 + w + bd, skip_prob=0.3, damping=4)
    rng = np.random.default_rng(24 + w)
    d = rng.integers(0, 16, size=(fr.blk_rows, fr.blk_cols)).astype(np.uint8)
    v = rng.integers(-5, 1 << 27, size=(fr.blk_rows, fr.blk_cols)).astype(np.int32)
    v[rng.random(v.shape) < 0.2] = 0
    st = s.random_presets(fr, 24100 + h)
    print(f"filter with caller directions {w}x{h} {bd}-bit layout {layout}", flush=True)
    f = gpu_frame(fr.recon, fr)
    outs = cdef.filter_frame(f, torch.from_numpy(d).cuda(), torch.from_numpy(v).cuda(),
                             torch.from_numpy(fr.skip).cuda(), fr.damping,
                             torch.from_numpy(st).cuda())
    torch.cuda.synchronize()
    want = oracle.filter_frame(fr.recon, w, h, bd, d & 7, v, fr.skip, fr.damping, st,
                               layout=layout)
    for p in range(fr.nplanes):
        got = to_np_u16(outs[p])
        bad = np.argwhere(got != want[p])
        assert bad.size == 0, (p, bad[:5])


@pytest.mark.parametrize("w,h,bd,layout", [(336, 200, 10, 1), (336, 200, 12, 3), (320, 136, 8, 0),
                                           (384, 72, 10, 2)])
def test_filter_aligned_outputs(oracle, w, h, bd, layout):
    # Output rows 16-byte aligned (every plane's pitch a multiple of 8
    # samples): the filter copies block rows out whole, except in the
    # right-hand partial filter blocks; plain and batched against the oracle.
    import torch
    from paper_1602_05975_amd import cdef
    s = _synth()
    fr = s.make_frame(w, h, bd, layout, 25000 + w + bd, skip_prob=0.3, damping=5)
    st = s.random_presets(fr, 25100 + h)
    print(f"filter aligned {w}x{h} {bd}-bit layout {layout}", flush=True)
    f = gpu_frame(fr.recon, fr)
    assert all(p.stride(0) % 8 == 0 for p in f.planes[:fr.nplanes])
    sk = torch.from_numpy(fr.skip).cuda()
    stg = torch.from_numpy(st).cuda()
    d, v = cdef.find_dir(f)
    plain = cdef.filter_frame(f, d, v, sk, fr.damping, stg)
    b = cdef.Batch()
    fused = [torch.full_like(p, -1) for p in f.planes[:fr.nplanes]]
    b.add_filter(f, fused, sk, fr.damping, stg)
    b.prepare()
    b.launch()
    torch.cuda.synchronize()
    od, ov = oracle.find_dir(fr.recon[0], bd)
    want = oracle.filter_frame(fr.recon, w, h, bd, od, ov, fr.skip, fr.damping, st, layout=layout)
    for p in range(fr.nplanes):
        for name, got in (("plain", to_np_u16(plain[p])), ("batched", to_np_u16(fused[p]))):
            bad = np.argwhere(got != want[p])
            assert bad.size == 0, (name, p, bad[:5])
