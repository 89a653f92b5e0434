"""Pins of the oracle's preset selection (Section 5, Eq. 15).

The selection is a heuristic (greedy growth, then slot-by-slot refinement), so
it has no closed form; these tests fix it from outside: a small table worked by
hand, brute force over candidate sets and single-slot swaps, the special
cases of the rate term (lambda = 0, a rate that dwarfs every distortion), the
definitions of the distortion sums and of the per-block preset, and planted
cluster structure that any correct greedy search must recover.
"""
import itertools

import numpy as np
import pytest

NS = (1, 2, 4, 8)


def _table(luma, chroma1=None, chroma2=None):
    """sse [nplanes][1][nfb][16][4] from [nfb][64] distortion arrays."""
    planes = [luma] if chroma1 is None else [luma, chroma1, chroma2]
    t = np.stack([np.asarray(p, dtype=np.uint64) for p in planes])
    nfb = t.shape[1]
    return t.reshape(len(planes), 1, nfb, 16, 4)


def _flat(sse):
    n = sse.shape[0]
    return sse.reshape(n, -1, 64).astype(np.int64)


def _groups(sse):
    f = _flat(sse)
    luma = f[0]
    chroma = f[1] + f[2] if f.shape[0] == 3 else np.zeros_like(luma)
    return luma, chroma


def _set_dist(D, s):
    return int(D[:, list(s)].min(axis=1).sum())


def _hand_table():
    # Two blocks; candidates 0, 1, 2 are special, every other costs 100.
    #   block 0: D = 4, 0, 10     block 1: D = 4, 10, 0
    D = np.full((2, 64), 100, dtype=np.uint64)
    D[0, :3] = (4, 0, 10)
    D[1, :3] = (4, 10, 0)
    return _table(D)


def test_hand_worked_greedy(oracle):
    # Greedy, worked by hand: the single best is 0 (sum 8 against 10, 10);
    # given {0}, adding 1 or 2 both reach 4, the lower index wins; given
    # {0, 1} (mins 0, 4) only 2 reaches 0; after that every candidate ties at
    # 0 and the lowest unused indices 3, 4, ... follow.
    r = oracle.select_presets(_hand_table(), 0.0, 0)
    assert list(r["luma"][0]) == [0] + [-1] * 7
    assert list(r["luma"][1]) == [0, 1] + [-1] * 6
    assert list(r["luma"][2]) == [0, 1, 2, 3] + [-1] * 4
    assert list(r["luma"][3]) == list(range(8))
    assert list(r["dist"][0]) == [8, 4, 0, 0]
    assert list(r["dist"][1]) == [0, 0, 0, 0]          # luma only: no chroma term
    assert list(r["chroma"][0]) == [0] + [-1] * 7       # all-zero chroma: lowest indices
    # lambda = 0: J = D, and N = 4 is the smallest N that reaches 0
    assert r["n"] == 4 and list(r["cost"]) == [8.0, 4.0, 0.0, 0.0]
    assert list(r["fb_luma"].ravel()) == [1, 2]


def test_hand_worked_refinement(oracle):
    # One refinement pass on N = 2: slot 0 (candidate 0) is re-chosen given
    # slot 1 = candidate 1 (mins 0, 10): candidate 2 gives 0 < 4, so the set
    # becomes {2, 1}; slot 1 given {2} (mins 10, 0): candidate 1 gives 0, not
    # strictly better than the current 0, so it stays.  Larger N are already 0.
    r = oracle.select_presets(_hand_table(), 1.0, 1)
    assert list(r["luma"][1]) == [2, 1] + [-1] * 6
    assert list(r["dist"][0]) == [8, 0, 0, 0]
    # J = lambda * B * log2 N + D with B = 2 blocks: 8, 2, 4, 6 -> N = 2
    assert list(r["cost"]) == [8.0, 2.0, 4.0, 6.0] and r["n"] == 2
    assert list(r["fb_luma"].ravel()) == [1, 0]   # block 0 -> candidate 1, block 1 -> 2
    # without refinement: 8, 6, 4, 6 -> N = 4
    r0 = oracle.select_presets(_hand_table(), 1.0, 0)
    assert list(r0["cost"]) == [8.0, 6.0, 4.0, 6.0] and r0["n"] == 4
    # a rate of 3 per block and doubling: 8, 10, 12, 18 -> N = 1
    r3 = oracle.select_presets(_hand_table(), 3.0, 0)
    assert list(r3["cost"]) == [8.0, 10.0, 12.0, 18.0] and r3["n"] == 1
    assert list(r3["fb_luma"].ravel()) == [0, 0]


def _random_sse(seed, nfb, nplanes=3, hi=1 << 20, ties=False):
    rng = np.random.default_rng(seed)
    top = 6 if ties else hi
    return rng.integers(0, top, size=(nplanes, 1, nfb, 16, 4)).astype(np.uint64)


@pytest.mark.parametrize("seed,nplanes,ties", [(1, 3, False), (2, 1, False), (3, 3, True)])
def test_n1_is_exhaustive_optimum(oracle, seed, nplanes, ties):
    sse = _random_sse(seed, 37, nplanes, ties=ties)
    r = oracle.select_presets(sse, 0.0, 0)
    for g, D in enumerate(_groups(sse)):
        sums = D.sum(axis=0)
        key = "luma" if g == 0 else "chroma"
        assert r[key][0][0] == int(np.argmin(sums))          # first minimum
        assert int(r["dist"][g][0]) == int(sums.min())


@pytest.mark.parametrize("seed", [4, 5])
def test_greedy_steps_by_brute_force(oracle, seed):
    # Without refinement the N = 8 set is the greedy sequence; each element is
    # the first candidate minimizing the set distortion given the previous ones.
    sse = _random_sse(seed, 23)
    r = oracle.select_presets(sse, 0.0, 0)
    for g, D in enumerate(_groups(sse)):
        seq = list((r["luma"] if g == 0 else r["chroma"])[3])
        for step in range(8):
            cand = [p for p in range(64) if p not in seq[:step]]
            vals = [_set_dist(D, seq[:step] + [p]) for p in cand]
            assert seq[step] == cand[int(np.argmin(vals))]
        for k, n in enumerate(NS):
            assert list((r["luma"] if g == 0 else r["chroma"])[k][:n]) == seq[:n]


@pytest.mark.parametrize("seed,ties", [(6, False), (7, True)])
def test_refined_sets_are_swap_optimal(oracle, seed, ties):
    # With enough passes every refined set is a local optimum: no single slot
    # can be replaced by an unused candidate with a strictly smaller distortion.
    sse = _random_sse(seed, 41, ties=ties)
    r = oracle.select_presets(sse, 0.0, 16)
    r0 = oracle.select_presets(sse, 0.0, 0)
    for g, D in enumerate(_groups(sse)):
        key = "luma" if g == 0 else "chroma"
        for k, n in enumerate(NS):
            s = list(r[key][k][:n])
            assert len(set(s)) == n and all(0 <= p < 64 for p in s)
            assert all(p == -1 for p in r[key][k][n:])
            cur = _set_dist(D, s)
            assert cur == int(r["dist"][g][k])
            assert cur <= int(r0["dist"][g][k])       # refinement never hurts
            for i in range(n):
                for p in range(64):
                    if p in s:
                        continue
                    t = s[:i] + [p] + s[i + 1:]
                    assert _set_dist(D, t) >= cur


def test_n2_against_exhaustive_pairs(oracle):
    # Brute force over all 2016 pairs: the refined pair is never worse than the
    # greedy one and never better than the exhaustive optimum.
    sse = _random_sse(8, 29)
    r = oracle.select_presets(sse, 0.0, 16)
    r0 = oracle.select_presets(sse, 0.0, 0)
    for g, D in enumerate(_groups(sse)):
        best = min(_set_dist(D, s) for s in itertools.combinations(range(64), 2))
        assert best <= int(r["dist"][g][1]) <= int(r0["dist"][g][1])


def test_cost_and_choice(oracle):
    # J(N) = lambda * B * log2 N + D^luma(N) + D^chroma(N) (Eq. 15); B = number
    # of filter blocks; the smallest N of minimal J is chosen.
    sse = _random_sse(9, 53)
    nfb = 53
    for lam in (0.0, 0.5, 1e3, 1e5, 1e7):
        r = oracle.select_presets(sse, lam, 2)
        tot = r["dist"][0].astype(np.int64) + r["dist"][1].astype(np.int64)
        want = [lam * nfb * k + float(tot[k]) for k in range(4)]
        assert list(r["cost"]) == want
        assert r["n"] == NS[int(np.argmin(want))]
    # a rate that dwarfs every distortion forces one preset
    assert oracle.select_presets(sse, 1e30, 2)["n"] == 1


def test_zero_rate_picks_smallest_minimal_distortion(oracle):
    # all-equal distortions: every N costs the same at lambda = 0 -> N = 1
    D = np.full((5, 64), 7, dtype=np.uint64)
    r = oracle.select_presets(_table(D, D, D), 0.0, 3)
    assert r["n"] == 1
    for key in ("luma", "chroma"):
        assert list(r[key][3]) == list(range(8))
    assert list(r["dist"][0]) == [35] * 4 and list(r["dist"][1]) == [70] * 4
    assert (r["fb_luma"] == 0).all() and (r["fb_chroma"] == 0).all()


def test_planted_clusters(oracle):
    # Blocks fall into 4 clusters; the luma distortion is 0 for the cluster's
    # own candidate and at least 1000 elsewhere, chroma is flat.  Four presets
    # reach zero, so the greedy search must find exactly the four cluster
    # candidates; at a rate of 1 per block and doubling, J = 128 for N = 4
    # beats 192 for N = 8 and the >= 1000 left over by N = 1 or 2; every block
    # is mapped to the slot holding its cluster's candidate.
    rng = np.random.default_rng(10)
    nfb, own = 64, [9, 33, 50, 17]
    cl = rng.integers(0, 4, size=nfb)
    cl[:4] = np.arange(4)
    D = rng.integers(1000, 5000, size=(nfb, 64)).astype(np.uint64)
    for b in range(nfb):
        D[b, own[cl[b]]] = 0
    Z = np.zeros_like(D)
    r = oracle.select_presets(_table(D, Z, Z), 1.0, 4)
    assert sorted(r["luma"][2][:4]) == sorted(own)
    assert int(r["dist"][0][2]) == 0 and int(r["dist"][0][3]) == 0
    assert r["n"] == 4 and r["cost"][2] == 128.0
    s = list(r["luma"][2][:4])
    for b in range(nfb):
        assert s[r["fb_luma"].ravel()[b]] == own[cl[b]]


@pytest.mark.parametrize("lam", [0.0, 1e4])
def test_per_block_presets_are_first_minima(oracle, lam):
    sse = _random_sse(11, 31, ties=True)
    r = oracle.select_presets(sse, lam, 1)
    k = NS.index(r["n"])
    for g, D in enumerate(_groups(sse)):
        key, fbk = ("luma", "fb_luma") if g == 0 else ("chroma", "fb_chroma")
        s = list(r[key][k][:r["n"]])
        ids = r[fbk].ravel()
        for b in range(D.shape[0]):
            vals = [int(D[b, p]) for p in s]
            assert ids[b] == int(np.argmin(vals))


def test_chroma_is_sum_of_planes(oracle):
    # D^chroma = D^Cb + D^Cr: swapping the two chroma planes, or moving all of
    # the chroma distortion into one of them, changes nothing.
    rng = np.random.default_rng(12)
    L = rng.integers(0, 1000, size=(19, 64)).astype(np.uint64)
    a = rng.integers(0, 1000, size=(19, 64)).astype(np.uint64)
    b = rng.integers(0, 1000, size=(19, 64)).astype(np.uint64)
    r1 = oracle.select_presets(_table(L, a, b), 50.0, 2)
    r2 = oracle.select_presets(_table(L, b, a), 50.0, 2)
    r3 = oracle.select_presets(_table(L, a + b, np.zeros_like(a)), 50.0, 2)
    for r in (r2, r3):
        for key in ("n", "luma", "chroma", "dist", "cost", "fb_luma", "fb_chroma"):
            assert np.array_equal(np.asarray(r1[key]), np.asarray(r[key])), key
