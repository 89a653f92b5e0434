"""Pins of the oracle's preset subsets (Section 5, low-complexity search):
a subset search equals the full search on its presets and marks the rest;
the selection never chooses an excluded preset, and what it chooses does
not depend on the excluded entries' values."""
import numpy as np
import pytest


def _mask_of(cand, ncand):
    """Candidate indices of a (S^(p), S^(s), skip bit) product mask."""
    pri, sec, skb = cand & 0xFFFF, (cand >> 16) & 15, (cand >> 20) & 3
    idx = []
    for k in range(ncand // 64):
        for p in range(16):
            for si in range(4):
                if (pri >> p) & 1 and (sec >> si) & 1 and (skb >> k) & 1:
                    idx.append(64 * k + 4 * p + si)
    return idx


def _words(idx):
    w = [0, 0]
    for i in idx:
        w[i >> 6] |= 1 << (i & 63)
    return w


@pytest.mark.parametrize("full", [False, True])
def test_subset_search_matches_full_search(oracle, full):
    from paper_1602_05975_amd import synth
    fr = synth.make_frame(136, 72, 10, synth.LAYOUT_420, 95, skip_prob=0.3, damping=4)
    fr.skip[0:8, 8:16] = 1
    cand = 0b0101000100010011 | (0b1011 << 16) | ((0b11 if full else 0b01) << 20)
    t, _, _ = oracle.search(fr.recon, fr.src, 136, 72, 10, fr.skip, 4, threads=4, full=full)
    u, _, _ = oracle.search(fr.recon, fr.src, 136, 72, 10, fr.skip, 4, threads=4, full=full,
                            cand=cand)
    nc = 128 if full else 64
    tf, uf = t.reshape(3, -1, nc), u.reshape(3, -1, nc)
    inside = np.zeros(nc, bool)
    inside[_mask_of(cand, nc)] = True
    assert np.array_equal(uf[:, :, inside], tf[:, :, inside])
    assert (uf[:, :, ~inside] == np.uint64(2**64 - 1)).all()


def test_selection_respects_subset(oracle):
    rng = np.random.default_rng(96)
    sse = rng.integers(0, 1 << 24, size=(3, 4, 9, 2, 16, 4)).astype(np.uint64)
    cand = 0b1100110000110001 | (0b0110 << 16) | (0b10 << 20)
    idx = _mask_of(cand, 128)
    words = _words(idx)
    r = oracle.select_presets(sse, 1e3, 3, cand_mask=words)
    for key in ("luma", "chroma"):
        for k, n in enumerate((1, 2, 4, 8)):
            assert set(r[key][k][:n]) <= set(idx)
    # N = 1: the allowed candidate with the smallest column sum
    D = sse.reshape(3, -1, 128).astype(np.int64)[0]
    sums = D.sum(axis=0)
    assert r["luma"][0][0] == idx[int(np.argmin(sums[idx]))]
    # excluded entries do not matter: overwrite them with the all-ones marker
    marked = sse.reshape(3, -1, 128).copy()
    out = np.setdiff1d(np.arange(128), idx)
    marked[:, :, out] = np.uint64(2**64 - 1)
    r2 = oracle.select_presets(marked.reshape(sse.shape), 1e3, 3, cand_mask=words)
    for key in ("n", "luma", "chroma", "dist", "cost", "fb_luma", "fb_chroma"):
        assert np.array_equal(np.asarray(r[key]), np.asarray(r2[key])), key
    # the full mask is the unrestricted selection
    r3 = oracle.select_presets(sse, 1e3, 3, cand_mask=[2**64 - 1, 2**64 - 1])
    r4 = oracle.select_presets(sse, 1e3, 3)
    for key in ("n", "luma", "chroma", "dist", "cost"):
        assert np.array_equal(np.asarray(r3[key]), np.asarray(r4[key])), key
