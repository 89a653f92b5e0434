"""cdef_select_presets_noalloc (the selection on the library's own per-device
workspace) gives exactly the results of cdef_select_presets with a caller
workspace, on consecutive calls whose second table is smaller than the
first (the scratch keeps the first call's contents and must not leak
them)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_05975_amd import cdef
    cdef.load()


def _run(fn, sse, lam, refine, mask):
    import torch
    from paper_1602_05975_amd import cdef
    fbr, fbc = sse.shape[1], sse.shape[2]
    res = torch.full((cdef.C.sizeof(cdef.CdefPresetResult),), 0xAB, dtype=torch.uint8,
                     device="cuda")
    fl = torch.full((fbr, fbc), 0xEE, dtype=torch.uint8, device="cuda")
    fc = torch.full((fbr, fbc), 0xEE, dtype=torch.uint8, device="cuda")
    if fn == "noalloc":
        cdef.cdef_select_presets_noalloc(sse, lam, refine, res, fl, fc, cand_mask=mask)
    else:
        ws = cdef.preset_workspace()
        cdef.cdef_select_presets(sse, lam, refine, res, fl, fc, ws, cand_mask=mask)
    torch.cuda.synchronize()
    return res.cpu().numpy(), fl.cpu().numpy(), fc.cpu().numpy()


def _table(nplanes, fbr, fbc, ncand, seed):
    import torch
    rng = np.random.default_rng(seed)
    shape = (nplanes, fbr, fbc) + ((2, 16, 4) if ncand == 128 else (16, 4))
    t = rng.integers(0, 1 << 40, size=shape, dtype=np.int64)
    return torch.from_numpy(t).cuda()


@pytest.mark.parametrize("first,second", [((3, 34, 60, 64, 0), (3, 5, 7, 64, 2)),
                                          ((3, 40, 70, 128, 1), (1, 2, 3, 128, 0)),
                                          ((1, 17, 30, 64, 2), (3, 1, 1, 128, 1))])
def test_noalloc_matches_workspace_entry_point(oracle, first, second):
    from paper_1602_05975_amd import cdef
    for k, (npl, fbr, fbc, nc, refine) in enumerate((first, second)):
        sse = _table(npl, fbr, fbc, nc, 900 + 10 * k + nc + fbr)
        mask = None if k == 0 else cdef.candidate_mask(
            cdef.subset(pri=range(0, 16, 2), skip_bits=(0, 1) if nc == 128 else (0,)))
        lam = 3.0e6 * (k + 1)
        print(f"noalloc selection call {k}: {npl}x{fbr}x{fbc}, {nc} candidates", flush=True)
        a = _run("noalloc", sse, lam, refine, mask)
        b = _run("workspace", sse, lam, refine, mask)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
        r = cdef.CdefPresetResult.from_buffer_copy(a[0].tobytes())
        assert r.n in (1, 2, 4, 8)
        ref = oracle.select_presets(sse.cpu().numpy().view(np.uint64), lam, refine, mask)
        assert r.n == ref["n"]
        assert np.array_equal(np.array(r.luma), ref["luma"])
        assert np.array_equal(a[1], ref["fb_luma"]) and np.array_equal(a[2], ref["fb_chroma"])
