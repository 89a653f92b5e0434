"""Seeded random configurations against the oracle, and one large batch of
many small jobs.

Each configuration draws a frame size (1 to 300 samples a side, so blocks
and filter blocks are cut at every offset), a bit depth, a layout, a
damping, a skip probability, a frame kind (the coded-video recipe or one
of the edge-case kinds) and a mode (64-pair, 128-combination, weighted or
subset search, or the filter at random presets); the result must equal
the oracle's.  The batch test puts 240 such jobs into one launch, in every
launch variant, and compares each job with its own one-frame call."""
import numpy as np
import pytest

from helpers import ORACLE_THREADS, gpu_frame, to_np_u16

pytestmark = pytest.mark.gpu

MODES = ("search", "search128", "weighted", "subset", "filter")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_05975_amd import cdef
    cdef.load()


def _config(seed):
    from paper_1602_05975_amd import synth
    rng = np.random.default_rng(seed)
    w, h = (int(v) for v in rng.integers(1, 301, 2))
    bd = int(rng.choice([8, 10, 12]))
    layout = int(rng.integers(0, 4))
    D = int(rng.integers(3, 7))
    skip = float(rng.choice([0.0, 0.3, 0.9]))
    kind = str(rng.choice(["coded", "coded"] + list(synth.EDGE_KINDS)))
    mode = MODES[int(rng.integers(0, len(MODES)))]
    if kind == "coded":
        fr = synth.make_frame(w, h, bd, layout, seed, skip_prob=skip, damping=D)
    else:
        fr = synth.edge_frame(kind, w, h, bd, layout, seed, damping=D, skip_prob=skip)
    cand = 0
    if mode == "subset":
        pri = [p for p in range(16) if rng.random() < 0.5] or [0]
        sec = [i for i in range(4) if rng.random() < 0.6] or [1]
        skb = [0] if rng.random() < 0.5 else [0, 1]
        cand = sum(1 << p for p in pri) | sum(1 << (16 + i) for i in sec) | \
            sum(1 << (20 + k) for k in skb)
    return fr, kind, mode, cand


def _gpu_result(fr, mode, cand, presets):
    import torch
    from paper_1602_05975_amd import cdef
    rec = gpu_frame(fr.recon, fr)
    sk = torch.from_numpy(fr.skip).cuda()
    if mode == "filter":
        d, v = cdef.find_dir(rec)
        outs = cdef.filter_frame(rec, d, v, sk, fr.damping, torch.from_numpy(presets).cuda())
        torch.cuda.synchronize()
        return [to_np_u16(o) for o in outs]
    src = gpu_frame(fr.src, fr)
    if mode == "subset":
        t = cdef.search_subset(rec, src, sk, fr.damping, cand)
    else:
        t = cdef.search_strengths(rec, src, sk, fr.damping, full=mode == "search128",
                                  weighted=mode == "weighted")
    torch.cuda.synchronize()
    t = t.cpu().numpy()
    return t if mode == "weighted" else t.view(np.uint64)


def _oracle_result(oracle, fr, mode, cand, presets):
    kw = dict(threads=ORACLE_THREADS, layout=fr.layout)
    if mode == "filter":
        d, v = oracle.find_dir(fr.recon[0], fr.bitdepth)
        return oracle.filter_frame(fr.recon, fr.width, fr.height, fr.bitdepth, d, v, fr.skip,
                                   fr.damping, presets, layout=fr.layout)
    if mode == "weighted":
        d, v = oracle.find_dir(fr.recon[0], fr.bitdepth)
        fbs = [(by, bx) for by in range(fr.fb_rows) for bx in range(fr.fb_cols)]
        t = oracle.search_fbs_weighted(fr.recon, fr.src, fr.width, fr.height, fr.bitdepth, d, v,
                                       fr.skip, fr.damping, fbs, **kw)
        return np.moveaxis(t.reshape((fr.fb_rows, fr.fb_cols) + t.shape[1:]), 2, 0)
    full = mode == "search128" or (mode == "subset" and (cand >> 21) & 1)
    t, _, _ = oracle.search(fr.recon, fr.src, fr.width, fr.height, fr.bitdepth, fr.skip,
                            fr.damping, full=bool(full), cand=cand, **kw)
    return t


@pytest.mark.parametrize("seed", range(120))
def test_random_configuration_matches_oracle(oracle, seed):
    from paper_1602_05975_amd import synth
    fr, kind, mode, cand = _config(92000 + seed)
    presets = synth.random_presets(fr, 93000 + seed)
    print(f"random {seed}: {fr.width}x{fr.height} {fr.bitdepth}-bit layout {fr.layout} "
          f"D={fr.damping} {kind} {mode} cand={cand:#x}", flush=True)
    got = _gpu_result(fr, mode, cand, presets)
    want = _oracle_result(oracle, fr, mode, cand, presets)
    if mode == "filter":
        for p in range(fr.nplanes):
            assert np.array_equal(got[p], want[p]), p
    elif mode == "weighted":
        assert np.allclose(got, want, rtol=1e-10, atol=1e-9)
    else:
        assert got.shape == want.shape and np.array_equal(got, want)


def test_many_small_jobs_in_one_batch():
    # 240 jobs of random sizes (1x1 to 96x96 luma), formats and modes: the
    # job lookup over many descriptors, in every launch variant, against
    # each job's one-frame call
    import torch
    from paper_1602_05975_amd import cdef, synth
    rng = np.random.default_rng(94000)
    outs, refs = [], []
    b = cdef.Batch()
    for k in range(240):
        w, h = (int(v) for v in rng.integers(1, 97, 2))
        bd, layout = int(rng.choice([8, 10, 12])), int(rng.choice([0, 1, 2]))
        D = int(rng.integers(3, 7))
        fr = synth.make_frame(w, h, bd, layout, 94100 + k, skip_prob=0.3, damping=D)
        rec, src = gpu_frame(fr.recon, fr), gpu_frame(fr.src, fr)
        sk = torch.from_numpy(fr.skip).cuda()
        mode = ("search", "search128", "filter")[k % 3]
        if mode == "filter":
            st = torch.from_numpy(synth.random_presets(fr, 94500 + k)).cuda()
            o = [torch.full_like(p, -1) for p in rec.planes[:fr.nplanes]]
            b.add_filter(rec, o, sk, D, st)
            d, v = cdef.find_dir(rec)
            refs.append(cdef.filter_frame(rec, d, v, sk, D, st))
            outs.append(o)
        else:
            full = mode == "search128"
            ref = cdef.search_strengths(rec, src, sk, D, full=full)
            t = torch.full_like(ref, -1)
            b.add_search(rec, src, sk, D, t, full=full)
            refs.append([ref])
            outs.append([t])
    b.prepare()
    torch.cuda.synchronize()
    print(f"{len(outs)} jobs, {b.nitems} filter blocks in one batch", flush=True)
    for variant in range(cdef.BATCH_VARIANTS):
        b.plan.variant = variant
        for o in outs:
            for t in o:
                t.fill_(-1)
        b.launch()
        torch.cuda.synchronize()
        for k, (o, r) in enumerate(zip(outs, refs)):
            for a, c in zip(o, r):
                assert torch.equal(a, c), (variant, k)
