"""The algorithmic operation counts bench.py prices its roofline with, on a
small 4:2:0 frame counted by hand: blocks cut by the frame edge, a skipped
block, tap groups at strength 0 and the Eq. 13 adjustment of the luma
primary strength."""
import numpy as np

import bench
from paper_1602_05975_amd import synth

# 13x10 luma: 8x8 blocks of 64, 40 (8 x 5), 16 (2 x 8) and 10 (2 x 5)
# samples; 4:2:0 chroma planes 7x5: blocks of 16, 12, 4 and 3 samples.
SKIP = np.array([[0, 0], [1, 0]], np.uint8)


def _frame():
    return synth.Frame(width=13, height=10, bitdepth=10, layout=synth.LAYOUT_420, src=[],
                       recon=[], skip=SKIP.copy())


def test_filter_ops_per_sample_table():
    t, f = True, False
    assert bench.filter_ops_per_sample(t, t) == 127
    assert bench.filter_ops_per_sample(t, f) == 36
    assert bench.filter_ops_per_sample(f, t) == 68
    assert bench.filter_ops_per_sample(f, f) == 0


def test_adjusted_luma_strength_eq13():
    # (strength, variance) -> (S (4 + i) + 8) >> 4 with i = min(floor(log2(v >> 16)), 12),
    # 0 below v = 1024 and i = 0 while v < 2^16
    cases = [(15, 1023, 0), (15, 1024, 4), (1, 60000, 0), (2, 70000, 1), (15, 8 << 16, 7),
             (15, 1 << 40, 15), (4, 3 << 16, 1), (0, 1 << 30, 0)]
    for s, v, want in cases:
        assert int(bench.adjusted_luma_strength(s, v)) == want, (s, v)


def test_filter_work_by_hand():
    fr = _frame()
    st = np.array([[[2, 1, 0, 4]]], np.uint8)
    var = np.array([[70000, 500], [4 << 16, 5000]], np.int32)
    ops, ny, nc = bench.filter_work(fr, st, var)
    # luma: block (0,0) both groups (adjusted 1, secondary 1): 127 x 64; (0,1)
    # adjusted to 0 (v < 1024): secondary only, 68 x 40; (1,0) skipped; (1,1)
    # v = 5000 adjusts 2 to 1: both, 127 x 10
    luma = 127 * 64 + 68 * 40 + 127 * 10
    # chroma: primary 0, secondary 4 -> 68 per sample of the live blocks, both planes
    chroma = 68 * 2 * (16 + 12 + 3)
    assert ops == luma + chroma + 10 * 13 * 10
    assert ny == 64 + 40 + 10 and nc == 2 * (16 + 12 + 3)


def test_search_work_by_hand():
    fr = _frame()
    ops, _ = bench.frame_work(fr)
    filtered = (130 - 16) + 2 * (35 - 4)
    skipped = 16 + 2 * 4
    assert ops == 1064 * filtered + 3 * skipped + 10 * 130
