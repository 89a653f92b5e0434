"""Pins of the oracle's chroma layouts beyond 4:2:0 (Section 4): 4:2:2,
whose chroma is never filtered, and 4:4:4, whose 8x8 chroma blocks follow
the co-located luma blocks.  Each is stated another way: 4:2:2 luma equals a
luma-only frame and its chroma is copied; a 4:4:4 chroma plane equals that
plane filtered as luma with the chroma rules substituted (the luma block's
direction, an Eq. 13 contrast large enough to leave the strength as is, and
the chroma damping max(D - 1, floor(log2 S))).
"""
import numpy as np
import pytest

SEC = (0, 1, 2, 4)


def _synth():
    from paper_1602_05975_amd import synth
    return synth


def _uniform(fr, pre):
    return np.tile(np.array(pre, np.uint8), (fr.fb_rows, fr.fb_cols, 1))


@pytest.mark.parametrize("w,h,bd", [(136, 72, 10), (67, 33, 8)])
def test_422_chroma_is_copied_and_luma_is_unchanged(oracle, w, h, bd):
    s = _synth()
    fr = s.make_frame(w, h, bd, s.LAYOUT_422, 70 + w, skip_prob=0.3, damping=4)
    assert fr.recon[1].shape == (h, (w + 1) // 2)
    d, v = oracle.find_dir(fr.recon[0], bd)
    st = s.random_presets(fr, 71)
    out = oracle.filter_frame(fr.recon, w, h, bd, d, v, fr.skip, 4, st, layout=s.LAYOUT_422)
    for p in (1, 2):
        assert np.array_equal(out[p], fr.recon[p])
    luma_only = oracle.filter_frame([fr.recon[0]], w, h, bd, d, v, fr.skip, 4, st)
    assert np.array_equal(out[0], luma_only[0])
    # the search covers luma only, and equals the 4:0:0 search
    t, _, _ = oracle.search(fr.recon, fr.src, w, h, bd, fr.skip, 4, threads=4,
                            layout=s.LAYOUT_422)
    t0, _, _ = oracle.search([fr.recon[0]], [fr.src[0]], w, h, bd, fr.skip, 4, threads=4)
    assert t.shape[0] == 1 and np.array_equal(t, t0)


@pytest.mark.parametrize("w,h,bd,D", [(136, 72, 10, 4), (67, 45, 8, 5), (64, 64, 10, 6)])
def test_444_chroma_is_luma_filter_with_chroma_rules(oracle, w, h, bd, D):
    s = _synth()
    fr = s.make_frame(w, h, bd, s.LAYOUT_444, 80 + w, skip_prob=0.3, damping=D)
    assert fr.recon[1].shape == (h, w)
    d, v = oracle.find_dir(fr.recon[0], bd)
    big = np.full_like(v, 1 << 30)  # Eq. (13) with i = 12: (16 S + 8) / 16 = S
    for pri, si in ((0, 2), (5, 1), (8, 3), (15, 0), (3, 3)):
        sec = SEC[si]
        st = _uniform(fr, (0, 0, pri, sec))
        out = oracle.filter_frame(fr.recon, w, h, bd, d, v, fr.skip, D, st, layout=s.LAYOUT_444)
        Dc = max(D - 1, int(np.floor(np.log2(pri)))) if pri else D - 1
        for p in (1, 2):
            ref = oracle.filter_frame([fr.recon[p]], w, h, bd, d, big, fr.skip, Dc,
                                      _uniform(fr, (pri, sec, 0, 0)))[0]
            assert np.array_equal(out[p], ref), (pri, sec, p)


def test_444_search_against_frame_filter(oracle):
    s = _synth()
    fr = s.make_frame(136, 72, 10, s.LAYOUT_444, 90, skip_prob=0.3, damping=3)
    t, d, v = oracle.search(fr.recon, fr.src, 136, 72, 10, fr.skip, 3, threads=4,
                            layout=s.LAYOUT_444)
    assert t.shape == (3, fr.fb_rows, fr.fb_cols, 16, 4)
    for pri, si in ((0, 0), (6, 2), (15, 3)):
        st = _uniform(fr, (pri, SEC[si], pri, SEC[si]))
        out = oracle.filter_frame(fr.recon, 136, 72, 10, d, v, fr.skip, 3, st,
                                  layout=s.LAYOUT_444)
        for p in range(3):
            for by in range(fr.fb_rows):
                for bx in range(fr.fb_cols):
                    a = out[p][64 * by:64 * by + 64, 64 * bx:64 * bx + 64].astype(np.int64)
                    b = fr.src[p][64 * by:64 * by + 64, 64 * bx:64 * bx + 64].astype(np.int64)
                    assert t[p, by, bx, pri, si] == ((a - b) ** 2).sum()


def test_12bit_search_identity_pair_and_downscaled_direction(oracle):
    # 12 bits: the direction search sees x >> 4 (R3); pair (0, 0) is the
    # unfiltered SSE; the table stays exact far above 2^32 per block.
    s = _synth()
    fr = s.make_frame(136, 72, 12, s.LAYOUT_420, 91, skip_prob=0.3, damping=5)
    t, d, v = oracle.search(fr.recon, fr.src, 136, 72, 12, fr.skip, 5, threads=4)
    d8, v8 = oracle.find_dir((fr.recon[0] >> 4).astype(np.uint16), 8)
    assert np.array_equal(d, d8) and np.array_equal(v, v8)
    for p in range(3):
        fs = 64 if p == 0 else 32
        for by in range(fr.fb_rows):
            for bx in range(fr.fb_cols):
                a = fr.recon[p][fs * by:fs * by + fs, fs * bx:fs * bx + fs].astype(np.int64)
                b = fr.src[p][fs * by:fs * by + fs, fs * bx:fs * bx + fs].astype(np.int64)
                assert t[p, by, bx, 0, 0] == ((a - b) ** 2).sum()
    flat = np.full((64, 64), 4095, np.uint16)
    zero = np.zeros((64, 64), np.uint16)
    t, _, _ = oracle.search([flat], [zero], 64, 64, 12, None, 3)
    assert t[0, 0, 0, 0, 0] == 64 * 64 * 4095 ** 2 > 1 << 32
