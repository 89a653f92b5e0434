"""Preset subsets on the GPU (Section 5, low-complexity search): the subset
search, as a call and as a batch job, and preset selection restricted to a
subset, all bit-exact against the oracle."""
import numpy as np
import pytest

from helpers import ORACLE_THREADS, gpu_frame

pytestmark = pytest.mark.gpu

ALL_ONES = np.uint64(2**64 - 1)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_05975_amd import cdef
    cdef.load()


def _frame(w, h, bd, D, seed, layout=None):
    from paper_1602_05975_amd import synth
    layout = synth.LAYOUT_420 if layout is None else layout
    fr = synth.make_frame(w, h, bd, layout, seed, skip_prob=0.3, damping=D)
    if fr.fb_cols > 1:
        fr.skip[0:8, 8:16] = 1      # filter block (0, 1): every block skipped
    if fr.fb_rows > 1:
        fr.skip[8:16, 0:8] = 0      # filter block (1, 0): none skipped
    return fr


def _word(pri, sec, skb):
    from paper_1602_05975_amd import cdef
    return cdef.subset(pri=pri, sec_index=sec, skip_bits=skb)


SUBSETS = [
    # (S^(p) set, S^(s) index set, skip bits)
    ((0, 1, 2, 3, 4, 6, 8, 12), (0, 1, 3), (0,)),
    ((0, 5, 10, 15), (0, 2), (0, 1)),
    ((2, 3, 7, 8, 9), (1, 2, 3), (1,)),
    ((0,), (0, 1, 2, 3), (0, 1)),
    ((15,), (3,), (0,)),
    (tuple(range(16)), (0, 1, 2, 3), (0, 1)),
]

CASES = [(136, 72, 10, 3, None), (200, 136, 8, 4, None), (131, 67, 10, 5, None),
         (136, 72, 10, 6, 0), (67, 45, 8, 3, 2), (72, 72, 10, 4, 3), (136, 72, 12, 5, None)]


@pytest.mark.parametrize("w,h,bd,D,layout", CASES)
@pytest.mark.parametrize("si", range(len(SUBSETS)))
def test_subset_search_matches_oracle(oracle, w, h, bd, D, layout, si):
    import torch
    from paper_1602_05975_amd import cdef
    fr = _frame(w, h, bd, D, 61000 + w + 7 * si, layout)
    pri, sec, skb = SUBSETS[si]
    cand = _word(pri, sec, skb)
    full = 1 in skb
    print(f"subset search {w}x{h} {bd}-bit D={D} layout={fr.layout} cand={cand:#x}", flush=True)
    rec, src = gpu_frame(fr.recon, fr), gpu_frame(fr.src, fr)
    sk = torch.from_numpy(fr.skip).cuda()
    sse = cdef.search_subset(rec, src, sk, D, cand)
    torch.cuda.synchronize()
    got = sse.cpu().numpy().view(np.uint64)
    ref, _, _ = oracle.search(fr.recon, fr.src, w, h, bd, fr.skip, D, threads=ORACLE_THREADS,
                              full=full, layout=fr.layout, cand=cand)
    assert got.shape == ref.shape
    bad = np.argwhere(got != ref)
    assert bad.size == 0, bad[:5]
    nc = 128 if full else 64
    flat = got.reshape(got.shape[0], -1, nc)
    inside = np.zeros(nc, bool)
    m = cdef.candidate_mask(cand)
    for i in range(nc):
        inside[i] = (m[i >> 6] >> (i & 63)) & 1
    assert (flat[:, :, ~inside] == ALL_ONES).all()
    assert (flat[:, :, inside] != ALL_ONES).all()


def test_subset_batch_jobs_match_calls(oracle):
    # one batch holding a subset job, the full search and a 128 subset job
    import torch
    from paper_1602_05975_amd import cdef
    fr = _frame(200, 136, 10, 4, 62000)
    rec, src = gpu_frame(fr.recon, fr), gpu_frame(fr.src, fr)
    sk = torch.from_numpy(fr.skip).cuda()
    fbr, fbc = fr.fb_rows, fr.fb_cols
    c64 = _word((0, 1, 3, 7, 11), (0, 2, 3), (0,))
    c128 = _word((0, 2, 4, 6, 8), (0, 1), (0, 1))
    t64 = torch.empty((3, fbr, fbc, 16, 4), dtype=torch.int64, device="cuda")
    tall = torch.empty_like(t64)
    t128 = torch.empty((3, fbr, fbc, 2, 16, 4), dtype=torch.int64, device="cuda")
    b = cdef.Batch()
    b.add_search(rec, src, sk, 4, t64, candidates=c64)
    b.add_search(rec, src, sk, 4, tall)
    b.add_search(rec, src, sk, 4, t128, full=True, candidates=c128)
    b.prepare()
    b.launch()
    torch.cuda.synchronize()
    for t, full, cand in ((t64, False, c64), (tall, False, 0), (t128, True, c128)):
        ref, _, _ = oracle.search(fr.recon, fr.src, fr.width, fr.height, 10, fr.skip, 4,
                                  threads=ORACLE_THREADS, full=full, cand=cand)
        assert np.array_equal(t.cpu().numpy().view(np.uint64), ref), (full, cand)


def test_batch_rejects_bad_subsets():
    import torch
    from paper_1602_05975_amd import cdef
    fr = _frame(64, 64, 10, 3, 62100)
    rec, src = gpu_frame(fr.recon, fr), gpu_frame(fr.src, fr)
    t = torch.empty((3, 1, 1, 16, 4), dtype=torch.int64, device="cuda")
    for cand, kw in ((_word((0,), (0,), (1,)), {}),                 # skip bit in a 64 search
                     (_word((0, 1), (0,), (0,)), {"weighted": True}),
                     (0xFFFF | (1 << 20), {})):                      # no S^(s)
        b = cdef.Batch()
        b.add_search(rec, src, None, 3, t, candidates=cand, **kw)
        with pytest.raises(RuntimeError):
            b.prepare()


@pytest.mark.parametrize("nc,si,lam,refine", [(64, 0, 1e3, 0), (64, 1, 5e2, 2), (128, 1, 2e3, 3),
                                              (128, 2, 1e4, 1), (64, 4, 1e3, 2)])
def test_selection_with_subset_matches_oracle(oracle, nc, si, lam, refine):
    # the search of a subset feeds the selection restricted to the same subset
    import torch
    from paper_1602_05975_amd import cdef
    pri, sec, skb = SUBSETS[si]
    if nc == 64:
        skb = (0,)
    cand = _word(pri, sec, skb)
    mask = cdef.candidate_mask(cand)
    if nc == 64:
        mask[1] = 0
    if sum(bin(w).count("1") for w in mask) < 8:
        # too few presets for N = 8: the call refuses the mask
        sse = torch.zeros((3, 2, 2, 16, 4), dtype=torch.int64, device="cuda")
        with pytest.raises(RuntimeError):
            cdef.select_presets(sse, lam, refine, cand_mask=mask)
        return
    fr = _frame(426, 240, 10, 3, 63000 + nc + si)
    rec, src = gpu_frame(fr.recon, fr), gpu_frame(fr.src, fr)
    sk = torch.from_numpy(fr.skip).cuda()
    sse = cdef.search_subset(rec, src, sk, 3, cand)
    r = cdef.select_presets(sse, lam, refine, cand_mask=mask)
    torch.cuda.synchronize()
    table = sse.cpu().numpy().view(np.uint64)
    o = oracle.select_presets(table, lam, refine, cand_mask=mask)
    for key in ("n", "luma", "chroma", "dist", "cost", "fb_luma", "fb_chroma"):
        assert np.array_equal(np.asarray(r[key]), np.asarray(o[key])), key
    allowed = {i for i in range(nc) if (mask[i >> 6] >> (i & 63)) & 1}
    for row, n in zip(r["luma"], (1, 2, 4, 8)):
        assert set(row[:n].tolist()) <= allowed
