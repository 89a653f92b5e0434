"""Degenerate inputs of the method and arithmetic limits of the kernels, on
the GPU against the oracle, at 8, 10 and 12 bits:

* flat planes (every line cost equal: d = 0 by the strict comparison, v = 0,
  every tap difference 0);
* the largest |recon - source| in both signs (at 12 bits a whole 64x64
  filter block of 4095-sample errors: the widest per-lane sums of the SSE
  reduction; at 10 bits the extreme of the folded rounding offset);
* two-level stripes and checkerboards (several directions with equal cost);
* blocks constant along the lines of each direction (Section 2);
* blocks whose contrast v is exactly at a threshold of Eq. (13);
* full-range noise and two-level full-range noise (largest tap differences,
  the clamp of Eq. 9-12 active).

Each frame runs the 64-pair, 128-combination and weighted searches and the
filter (random presets with the skip condition bit and the (19, 7) preset),
one frame per call and as batch jobs.  Integers are compared exactly, the
weighted table to the relative 1e-10 of its test module.
"""
import os

import numpy as np
import pytest

from helpers import ORACLE_THREADS, gpu_frame, to_np_u16

pytestmark = pytest.mark.gpu

W, H = 136, 72  # 3 x 2 filter blocks, the last column and row cut to 8 samples
RTOL = 1e-10
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "threshold_blocks.txt")


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


def threshold_blocks():
    """[(v, 8x8 int deviation block)] from the golden file."""
    out = []
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            blk = np.zeros((8, 8), np.int64)
            for t in parts[1:]:
                i, j, d = (int(x) for x in t.split(","))
                blk[i, j] = d
            out.append((int(parts[0]), blk))
    return out


def _directional_luma(oracle, bd, rng):
    """Every 8x8 block constant along the lines of one direction (block k
    takes direction k mod 8), line values drawn over the whole range."""
    maxv = (1 << bd) - 1
    key = [np.array([[oracle.line_number(d, i, j) for j in range(8)] for i in range(8)])
           for d in range(8)]
    luma = np.zeros((H, W), np.int64)
    k = 0
    for by in range(0, H, 8):
        for bx in range(0, W, 8):
            d = k % 8
            k += 1
            lines = key[d] - key[d].min()
            vals = rng.integers(0, maxv + 1, size=int(lines.max()) + 1)
            blk = vals[lines]
            h, w = min(8, H - by), min(8, W - bx)
            luma[by:by + h, bx:bx + w] = blk[:h, :w]
    return luma


def _threshold_luma(bd, rng):
    """Mid-grey with the threshold blocks in every whole 8x8 block (cycled);
    above 8 bits the dropped low bits are random."""
    c = bd - 8
    blocks = threshold_blocks()
    luma = np.full((H, W), 128, np.int64)
    k = 0
    for by in range(0, H - 7, 8):
        for bx in range(0, W - 7, 8):
            luma[by:by + 8, bx:bx + 8] += blocks[k % len(blocks)][1]
            k += 1
    return (luma << c) | rng.integers(0, 1 << c, size=luma.shape)


def make_case(oracle, kind, bd, layout):
    s = _synth()
    seed = 71000 + 100 * bd + 10 * layout + (s.EDGE_KINDS + ("directional", "thresholds")).index(kind)
    damping = 3 + seed % 4
    base = "noise" if kind in ("directional", "thresholds") else kind
    fr = s.edge_frame(base, W, H, bd, layout, seed, damping=damping)
    rng = np.random.default_rng(seed)
    if kind == "directional":
        fr.recon[0] = np.ascontiguousarray(_directional_luma(oracle, bd, rng).astype(np.uint16))
    elif kind == "thresholds":
        fr.recon[0] = np.ascontiguousarray(_threshold_luma(bd, rng).astype(np.uint16))
    return fr


KINDS = ("constant", "extreme_hi", "extreme_lo", "stripes", "checker", "noise", "binary",
         "directional", "thresholds")
CASES = ([(k, bd, 1) for k in KINDS for bd in (8, 10, 12)]
         + [("extreme_hi", 12, 3), ("noise", 10, 3), ("binary", 8, 0), ("checker", 12, 2),
            ("extreme_lo", 10, 3)])


def _oracle_all(oracle, fr, presets):
    od, ov = oracle.find_dir(fr.recon[0], fr.bitdepth)
    fbs = [(by, bx) for by in range(fr.fb_rows) for bx in range(fr.fb_cols)]
    kw = dict(threads=ORACLE_THREADS, layout=fr.layout)
    sse = oracle.search_fbs(fr.recon, fr.src, W, H, fr.bitdepth, od, ov, fr.skip, fr.damping,
                            fbs, **kw)
    full = oracle.search_fbs(fr.recon, fr.src, W, H, fr.bitdepth, od, ov, fr.skip, fr.damping,
                             fbs, full=True, **kw)
    wtd = oracle.search_fbs_weighted(fr.recon, fr.src, W, H, fr.bitdepth, od, ov, fr.skip,
                                     fr.damping, fbs, **kw)
    filt = oracle.filter_frame(fr.recon, W, H, fr.bitdepth, od, ov, fr.skip, fr.damping,
                               presets, layout=fr.layout)

    def table(t):  # [fbs][planes][..] -> [planes][fbr][fbc][..]
        t = t.reshape((fr.fb_rows, fr.fb_cols) + t.shape[1:])
        return np.ascontiguousarray(np.moveaxis(t, 2, 0))

    return od, ov, table(sse), table(full), table(wtd), filt


def _assert_table(name, got, want):
    if np.array_equal(got, want):
        return
    bad = np.argwhere(got != want)
    raise AssertionError(f"{name}: {len(bad)} entries differ, first at {tuple(bad[0])}: "
                         f"gpu {got[tuple(bad[0])]} oracle {want[tuple(bad[0])]}")


def _assert_weighted(got, want):
    ok = np.isclose(got, want, rtol=RTOL, atol=1e-9)
    if not ok.all():
        bad = np.argwhere(~ok)
        raise AssertionError(f"weighted: {len(bad)} entries differ, first at {tuple(bad[0])}: "
                             f"gpu {got[tuple(bad[0])]!r} oracle {want[tuple(bad[0])]!r}")


@pytest.mark.parametrize("kind,bd,layout", CASES)
def test_edge_case_all_modes(oracle, kind, bd, layout):
    import torch
    from paper_1602_05975_amd import cdef
    s = _synth()
    fr = make_case(oracle, kind, bd, layout)
    presets = s.random_presets(fr, 72000 + bd + layout)
    print(f"edge case {kind} {bd}-bit layout {layout} D={fr.damping}", flush=True)
    od, ov, w_sse, w_full, w_wtd, w_filt = _oracle_all(oracle, fr, presets)

    rec, src = gpu_frame(fr.recon, fr), gpu_frame(fr.src, fr)
    sk = torch.from_numpy(fr.skip).cuda()
    st = torch.from_numpy(presets).cuda()
    sse, d, v = cdef.search_strengths(rec, src, sk, fr.damping, want_dir=True)
    full = cdef.search_strengths(rec, src, sk, fr.damping, full=True)
    wtd = cdef.search_strengths(rec, src, sk, fr.damping, weighted=True)
    outs = cdef.filter_frame(rec, d, v, sk, fr.damping, st)
    torch.cuda.synchronize()
    assert (d.cpu().numpy() == od).all(), "directions"
    assert (v.cpu().numpy() == ov).all(), "contrasts"
    if kind == "constant":
        assert (od == 0).all() and (ov == 0).all()
    if kind == "thresholds":
        wanted = {t for t, _ in threshold_blocks()}
        assert wanted <= set(np.unique(ov).tolist())
    _assert_table("search", sse.cpu().numpy().view(np.uint64), w_sse)
    _assert_table("search128", full.cpu().numpy().view(np.uint64), w_full)
    _assert_weighted(wtd.cpu().numpy(), w_wtd)
    for p in range(fr.nplanes):
        _assert_table(f"filter plane {p}", to_np_u16(outs[p]), w_filt[p])

    # the same four as batch jobs: one batch of the search, search128 and
    # filter jobs, and one of the weighted search
    res = {}
    base = cdef.Batch()
    for name, kw in (("search", {}), ("search128", {"full": True})):
        shape = (fr.search_planes, fr.fb_rows, fr.fb_cols) + ((2, 16, 4) if kw else (16, 4))
        res[name] = torch.full(shape, -1, dtype=torch.int64, device="cuda")
        base.add_search(rec, src, sk, fr.damping, res[name], **kw)
    res["filter"] = [torch.full_like(p, -1) for p in rec.planes[:fr.nplanes]]
    base.add_filter(rec, res["filter"], sk, fr.damping, st)
    base.prepare()
    base.launch()
    ext = cdef.Batch()
    res["weighted"] = torch.full(wtd.shape, -1.0, dtype=torch.float64, device="cuda")
    ext.add_search(rec, src, sk, fr.damping, res["weighted"], weighted=True)
    ext.prepare()
    ext.launch()
    torch.cuda.synchronize()
    assert torch.equal(res["search"], sse) and torch.equal(res["search128"], full)
    assert torch.equal(res["weighted"], wtd)
    for p in range(fr.nplanes):
        assert torch.equal(res["filter"][p], outs[p]), p


def test_filter_at_threshold_contrasts(oracle):
    # cdef_filter_frame with caller contrasts exactly at and around the
    # thresholds of Eq. (13), and at its extremes, for every direction
    import torch
    from paper_1602_05975_amd import cdef
    s = _synth()
    values = [0, 1, 1023, 1024, 1025, 65535, 65536, 131071, 131072, (1 << 28) - 1, 1 << 28,
              880803840]
    for bd in (8, 10, 12):
        fr = s.edge_frame("noise", 200, 136, bd, s.LAYOUT_420, 73000 + bd, damping=3 + bd % 4)
        rng = np.random.default_rng(73000 + bd)
        v = np.array(values, np.int32)[rng.integers(0, len(values),
                                                    size=(fr.blk_rows, fr.blk_cols))]
        d = rng.integers(0, 8, size=v.shape).astype(np.uint8)
        st = s.random_presets(fr, 73100 + bd)
        print(f"filter at threshold contrasts {bd}-bit", flush=True)
        f = gpu_frame(fr.recon, fr)
        outs = cdef.filter_frame(f, torch.from_numpy(d).cuda(), torch.from_numpy(v).cuda(),
                                 torch.from_numpy(fr.skip).cuda(), fr.damping,
                                 torch.from_numpy(st).cuda())
        torch.cuda.synchronize()
        want = oracle.filter_frame(fr.recon, fr.width, fr.height, bd, d, v, fr.skip, fr.damping,
                                   st)
        for p in range(3):
            _assert_table(f"{bd}-bit plane {p}", to_np_u16(outs[p]), want[p])
