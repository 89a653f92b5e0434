"""The edge-case inputs of the GPU parity tests: ranges of the generated
frames, and the golden blocks' contrasts sitting on the thresholds of
Eq. (13) (Section 3.2) as the oracle computes them."""
import numpy as np
import pytest

from test_gpu_edge_cases import CASES, H, W, make_case, threshold_blocks


def test_threshold_blocks_hit_eq13_thresholds(oracle):
    blocks = threshold_blocks()
    assert [t for t, _ in blocks] == [1023, 1024, 65535, 65536, 131071, 131072]
    for t, dev in blocks:
        c = oracle.direction_costs((128 + dev).astype(np.uint16), 8)
        best = 0
        for d in range(1, 8):
            if c[d] > c[best]:
                best = d
        assert c[best] - c[(best + 4) & 7] == t
    # the adjustment changes across each pair (S = 15): v < 2^10 disables the
    # primary filter, the log term starts at v >> 16 = 2
    adj = {t: oracle.adjust_strength(15, t) for t, _ in blocks}
    assert adj[1023] == 0 and adj[1024] == adj[65535] == adj[65536] == adj[131071] == 4
    assert adj[131072] == 5


@pytest.mark.parametrize("kind,bd,layout", CASES)
def test_edge_frames_in_range(oracle, kind, bd, layout):
    fr = make_case(oracle, kind, bd, layout)
    assert (fr.width, fr.height) == (W, H)
    for p in range(fr.nplanes):
        for a in (fr.recon[p], fr.src[p]):
            assert a.dtype == np.uint16 and a.flags.c_contiguous
            assert a.shape == fr.plane_dims(p)[::-1]
            assert int(a.max()) < (1 << bd)
    if kind == "extreme_hi":
        assert (fr.recon[0] == (1 << bd) - 1).all() and (fr.src[0] == 0).all()
    if kind == "thresholds":
        d, v = oracle.find_dir(fr.recon[0], bd)
        assert {t for t, _ in threshold_blocks()} <= set(np.unique(v).tolist())
    assert fr.skip[0:8, 8:16].all() and not fr.skip[8:9, 0:8].any()
