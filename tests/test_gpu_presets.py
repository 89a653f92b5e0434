"""Preset selection on the GPU (Section 5, Eq. 15) against the oracle.

Both sides take every decision on the same uint64 sums and compute J(N) in
double precision with the same operations, so every output is compared
exactly: candidate sets, distortion sums, costs, the chosen N and the
per-block preset slots.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

KEYS = ("n", "luma", "chroma", "dist", "cost", "fb_luma", "fb_chroma")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_05975_amd import cdef
    cdef.load()


def _gpu_select(sse_np, lam, refine):
    import torch
    from paper_1602_05975_amd import cdef
    t = torch.from_numpy(sse_np.view(np.int64)).cuda()
    return cdef.select_presets(t, lam, refine)


def _compare(sse_np, lam, refine, oracle):
    print(f"select_presets shape={sse_np.shape} lambda={lam} refine={refine}", flush=True)
    g = _gpu_select(sse_np, lam, refine)
    o = oracle.select_presets(sse_np, lam, refine)
    for k in KEYS:
        assert np.array_equal(np.asarray(g[k]), np.asarray(o[k])), k
    return g


def test_hand_table(oracle):
    D = np.full((2, 64), 100, dtype=np.uint64)
    D[0, :3] = (4, 0, 10)
    D[1, :3] = (4, 10, 0)
    sse = D.reshape(1, 1, 2, 16, 4)
    for lam, refine, n in ((0.0, 0, 4), (1.0, 1, 2), (1.0, 0, 4), (3.0, 0, 1)):
        assert _compare(sse, lam, refine, oracle)["n"] == n


@pytest.mark.parametrize("nplanes,fbr,fbc,ties", [
    (3, 1, 1, False), (1, 3, 7, False), (3, 5, 9, True), (3, 17, 30, False),
    (1, 64, 70, True), (3, 65, 70, False), (3, 68, 120, False), (3, 96, 100, True)])
def test_random_tables(oracle, nplanes, fbr, fbc, ties):
    # up to 64 blocks per workgroup, 128 workgroups per group: 68 x 120 blocks
    # (an 8K frame) fill every slice; 96 x 100 blocks no longer fit in LDS
    rng = np.random.default_rng(nplanes * 1000 + fbr * 37 + fbc)
    top = 5 if ties else 1 << 30
    sse = rng.integers(0, top, size=(nplanes, fbr, fbc, 16, 4)).astype(np.uint64)
    for lam, refine in ((0.0, 0), (float(top) / 64, 2), (float(top) / 4, 16), (1e30, 1)):
        _compare(sse, lam, refine, oracle)


def test_on_searched_frame(oracle):
    # the table the strength search produces for a 1080p 10-bit 4:2:0 frame
    from helpers import gpu_search
    from paper_1602_05975_amd import synth
    sse, _, _ = gpu_search(synth.hd1080_frame())
    for lam in (0.0, 2e3, 2e4, 2e5):
        for refine in (0, 4):
            _compare(sse, lam, refine, oracle)


def test_device_outputs_stay_on_device():
    import torch
    from paper_1602_05975_amd import cdef
    rng = np.random.default_rng(3)
    sse = torch.from_numpy(rng.integers(0, 1 << 20, size=(3, 2, 3, 16, 4))).cuda()
    res = torch.zeros(360, dtype=torch.uint8, device="cuda")
    fl = torch.full((2, 3), 255, dtype=torch.uint8, device="cuda")
    fc = torch.full((2, 3), 255, dtype=torch.uint8, device="cuda")
    ws = cdef.preset_workspace()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        cdef.cdef_select_presets(sse, 1e3, 2, res, fl, fc, ws, s)
    s.synchronize()
    n = int(res[:4].cpu().numpy().view(np.int32)[0])
    assert n in (1, 2, 4, 8)
    assert int(fl.max()) < n and int(fc.max()) < n
