"""The C-ABI library loads without a GPU, exports every declared symbol, and
rejects bad host-side arguments before touching the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "cdef.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cdef_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1602_05975_amd import cdef
    return cdef.load()


def test_every_declared_symbol_is_exported(lib):
    from paper_1602_05975_amd import cdef
    names = _declared_symbols()
    assert "cdef_search_strengths" in names and "cdef_find_dir" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(cdef.EXPORTS)
    assert lib.cdef_abi_version() == 1


def test_status_strings(lib):
    from paper_1602_05975_amd import cdef
    for s in (0, -1, -2, -3, -4, -5, 7):
        assert isinstance(cdef.status_str(s), str) and cdef.status_str(s)
    assert len({cdef.status_str(s) for s in (0, -1, -2, -3, -4, -5, 7)}) == 7


def test_select_presets_incomplete_result_raises(lib, monkeypatch):
    # A result with n == 0 (the cooperative selection gave up waiting for its
    # workgroups) must surface as a CdefError carrying CDEF_E_TIMEOUT.  The
    # device call is replaced by a no-op, so the zero-filled result buffer
    # reaches the result handling unchanged; host tensors stand in for device
    # ones.
    import torch
    from paper_1602_05975_amd import cdef
    calls = []
    monkeypatch.setattr(cdef, "cdef_select_presets", lambda *a, **k: calls.append(a))
    monkeypatch.setattr(cdef, "preset_workspace", lambda device="cuda": torch.empty(16, dtype=torch.uint8))
    sse = torch.zeros((3, 2, 2, 16, 4), dtype=torch.int64)
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: calls.append("sync"))
    with pytest.raises(cdef.CdefError) as e:
        cdef.select_presets(sse, 1.0, 0)
    assert e.value.status == cdef.CDEF_E_TIMEOUT
    assert "did not complete" in str(e.value)
    # one retry after the device has drained, then the error
    assert len(calls) == 3 and calls[1] == "sync"
    calls.clear()
    with pytest.raises(cdef.CdefError):
        cdef.select_presets(sse, 1.0, 0, retries=0)
    assert len(calls) == 1


def _frame(w=64, h=64, bd=10, layout=1, stride=None, ptr=0x10000):
    from paper_1602_05975_amd import cdef
    f = cdef.CdefFrame()
    f.width, f.height, f.bitdepth, f.layout = w, h, bd, layout
    np_ = 1 if layout == 0 else 3
    for p in range(np_):
        pw = w if p == 0 or layout == 3 else (w + 1) // 2
        f.plane[p] = ptr + p * 0x100000
        f.stride[p] = pw if stride is None else stride if isinstance(stride, int) else stride[p]
    return f


def test_find_dir_argument_checks(lib):
    P = 0x20000
    assert lib.cdef_find_dir(None, P, P, None) == -1
    assert lib.cdef_find_dir(C.byref(_frame()), None, P, None) == -1
    assert lib.cdef_find_dir(C.byref(_frame(stride=3)), P, P, None) == -1
    assert lib.cdef_find_dir(C.byref(_frame(w=0)), P, P, None) == -1
    assert lib.cdef_find_dir(C.byref(_frame(bd=9)), P, P, None) == -1
    assert lib.cdef_find_dir(C.byref(_frame(bd=16)), P, P, None) == -1
    assert lib.cdef_find_dir(C.byref(_frame(layout=4)), P, P, None) == -1
    assert lib.cdef_find_dir(C.byref(_frame(layout=-1)), P, P, None) == -1
    assert lib.cdef_find_dir(C.byref(_frame(w=70000)), P, P, None) == -2
    # 4:2:2 and 4:4:4 chroma planes: the stride must cover their width
    f = _frame(w=64, layout=3, stride=(64, 32, 64))
    assert lib.cdef_find_dir(C.byref(f), P, P, None) == -1
    f = _frame()
    f.plane[1] = None
    assert lib.cdef_find_dir(C.byref(f), P, P, None) == -1


@pytest.mark.parametrize("name", ["cdef_search_strengths", "cdef_search_strengths128",
                                  "cdef_search_weighted"])
def test_search_argument_checks(lib, name):
    f = getattr(lib, name)
    P = 0x20000
    r, s = _frame(), _frame(ptr=0x900000)
    assert f(C.byref(r), C.byref(s), None, 2, P, None, None, None) == -1
    assert f(C.byref(r), C.byref(s), None, 7, P, None, None, None) == -1
    assert f(C.byref(r), C.byref(s), None, 3, None, None, None, None) == -1
    assert f(C.byref(r), C.byref(s), None, 3, P, P, None, None) == -1
    s2 = _frame(w=66, ptr=0x900000)
    assert f(C.byref(r), C.byref(s2), None, 3, P, None, None, None) == -1
    assert f(None, C.byref(s), None, 3, P, None, None, None) == -1


def test_filter_argument_checks(lib):
    from paper_1602_05975_amd import cdef
    P = 0x20000
    f = _frame()
    o = cdef.CdefFrameOut()
    for p in range(3):
        o.plane[p] = 0x4000000 + p * 0x100000
        o.stride[p] = 64
    assert lib.cdef_filter_frame(C.byref(f), C.byref(o), P, P, None, 2, P, None) == -1
    assert lib.cdef_filter_frame(C.byref(f), None, P, P, None, 3, P, None) == -1
    assert lib.cdef_filter_frame(C.byref(f), C.byref(o), P, P, None, 3, None, None) == -1
    alias = cdef.CdefFrameOut()
    for p in range(3):
        alias.plane[p] = f.plane[p]
        alias.stride[p] = f.stride[p]
    assert lib.cdef_filter_frame(C.byref(f), C.byref(alias), P, P, None, 3, P, None) == -1


def test_batch_argument_checks(lib):
    from paper_1602_05975_amd import cdef
    assert lib.cdef_batch_workspace_bytes(0) == 0
    per = lib.cdef_batch_workspace_bytes(1)
    # the job table (descriptors, padded to 256 bytes) and the work-queue counters
    five = lib.cdef_batch_workspace_bytes(5)
    assert per > 0 and five > per and (five - per) % 256 == 0 and five < 5 * per
    plan = cdef.CdefBatchPlan()
    j = cdef.CdefJob()
    j.recon = _frame()
    j.src = _frame(ptr=0x900000)
    j.sse = 0x5000000
    j.damping = 3
    j.mode = 0
    jobs = (cdef.CdefJob * 1)(j)
    W = 0x7000000
    assert lib.cdef_batch_prepare(None, 1, None, W, per, C.byref(plan), None) == -1
    assert lib.cdef_batch_prepare(jobs, 0, None, W, per, C.byref(plan), None) == -1
    assert lib.cdef_batch_prepare(jobs, 1, None, W, per - 1, C.byref(plan), None) == -4
    for field, bad in (("damping", 9), ("mode", 5), ("sse", None)):
        jb = cdef.CdefJob.from_buffer_copy(j)
        setattr(jb, field, bad)
        assert lib.cdef_batch_prepare((cdef.CdefJob * 1)(jb), 1, None, W, per, C.byref(plan),
                                      None) == -1, field
    jf = cdef.CdefJob.from_buffer_copy(j)
    jf.mode = 1  # filter without strengths or outputs
    assert lib.cdef_batch_prepare((cdef.CdefJob * 1)(jf), 1, None, W, per, C.byref(plan),
                                  None) == -1
    empty = cdef.CdefBatchPlan()
    assert lib.cdef_batch_launch(C.byref(empty), None) == -1
    assert lib.cdef_batch_launch(None, None) == -1


def test_select_presets_argument_checks(lib):
    P = C.c_void_p(0x10000)
    W = C.c_void_p(0x20000)
    n = lib.cdef_select_presets_workspace_bytes()
    assert 0 < n < (1 << 20)
    f = lib.cdef_select_presets

    def call(sse=P, npl=3, fbr=2, fbc=2, nc=64, lam=1.0, ref=0, res=P, fl=P, fc=P, ws=W, wsb=n,
             mask=None):
        return f(sse, npl, fbr, fbc, nc, mask, lam, ref, res, fl, fc, ws, wsb, None)

    assert call(sse=None) == -1
    assert call(res=None) == -1
    assert call(fl=None) == -1
    assert call(fc=None) == -1
    assert call(ws=None) == -1
    assert call(wsb=n - 1) == -1
    assert call(ws=C.c_void_p(0x20008)) == -1
    assert call(npl=2) == -1
    assert call(nc=0) == -1 and call(nc=65) == -1 and call(nc=256) == -1
    assert call(fbr=0) == -1
    assert call(fbc=-1) == -1
    assert call(lam=-1.0) == -1
    assert call(lam=float("nan")) == -1
    assert call(lam=float("inf")) == -1
    assert call(ref=-1) == -1
    assert call(ref=17) == -1
    assert call(npl=1, fbr=4097, fbc=4097) == -2
    assert call(npl=1, fbr=4097, fbc=4097, nc=128) == -2
    # fewer than 8 allowed candidates (the second word does not count at 64)
    seven = (C.c_uint64 * 2)(0x7F, 0)
    assert call(mask=C.addressof(seven)) == -1
    hi = (C.c_uint64 * 2)(0, 0xFF)
    assert call(mask=C.addressof(hi)) == -1
    assert call(nc=128, mask=C.addressof(hi), npl=1, fbr=4097, fbc=4097) == -2


def test_subset_masks(lib):
    from paper_1602_05975_amd import cdef
    w = cdef.subset(pri=(0, 3, 15), sec_index=(1, 2), skip_bits=(0, 1))
    m = cdef.candidate_mask(w)
    want = [0, 0]
    for k in (0, 1):
        for p in (0, 3, 15):
            for i in (1, 2):
                want[k] |= 1 << (4 * p + i)
    assert m == want
    assert cdef.candidate_mask(0) == [2**64 - 1, 2**64 - 1]
    P = 0x20000
    r, s = _frame(), _frame(ptr=0x900000)
    f = lib.cdef_search_subset
    assert f(C.byref(r), C.byref(s), None, 3, 0, P, None, None, None) == -1
    assert f(C.byref(r), C.byref(s), None, 3, 1 << 22, P, None, None, None) == -1
    assert f(C.byref(r), C.byref(s), None, 3, 0xFFFF | (1 << 20), P, None, None, None) == -1
    assert f(C.byref(r), C.byref(s), None, 3, 0xF0000 | (1 << 20), P, None, None, None) == -1
    assert f(C.byref(r), C.byref(s), None, 3, 0xFFFF | 0xF0000, P, None, None, None) == -1
    assert f(C.byref(r), C.byref(s), None, 7, w, P, None, None, None) == -1


def test_select_presets_noalloc_argument_checks(lib):
    # every host-side check runs before the library looks up its scratch, so
    # a bad argument never reaches the device
    P = C.c_void_p(0x10000)
    f = lib.cdef_select_presets_noalloc

    def call(sse=P, npl=3, fbr=2, fbc=2, nc=64, lam=1.0, ref=0, res=P, fl=P, fc=P, mask=None):
        return f(sse, npl, fbr, fbc, nc, mask, lam, ref, res, fl, fc, None)

    assert call(sse=None) == -1 and call(res=None) == -1
    assert call(fl=None) == -1 and call(fc=None) == -1
    assert call(npl=2) == -1 and call(nc=65) == -1
    assert call(fbr=0) == -1 and call(fbc=-1) == -1
    assert call(lam=-1.0) == -1 and call(lam=float("nan")) == -1
    assert call(ref=17) == -1
    assert call(npl=1, fbr=4097, fbc=4097) == -2
    seven = (C.c_uint64 * 2)(0x7F, 0)
    assert call(mask=C.addressof(seven)) == -1
    assert lib.cdef_select_presets_workspace_bytes() <= 20480


def test_tuning_to_variant(lib):
    from paper_1602_05975_amd import cdef, tune
    for v, (wg, order, pers) in tune.VARIANT_TUNING.items():
        assert cdef.tuning_variant(cdef.tuning(wg, order, pers)) == v
    assert cdef.tuning_variant(cdef.tuning()) == 0
    t = cdef.tuning()
    t.tile_w = t.tile_h = 64
    t.cand_group = 64
    assert cdef.tuning_variant(t) == 0
    v = C.c_int32()
    for field, value, status in (("tile_w", 32, -2), ("tile_h", 128, -2), ("cand_group", 16, -2),
                                 ("wg_per_cu", 4, -2), ("order", 2, -1), ("persistent", 3, -1)):
        t = cdef.tuning()
        setattr(t, field, value)
        assert lib.cdef_tuning_variant(C.byref(t), C.byref(v)) == status, field
    assert lib.cdef_tuning_variant(C.byref(cdef.tuning(3, 1, 1)), C.byref(v)) == -2
    assert lib.cdef_tuning_variant(None, C.byref(v)) == -1
    assert set(tune.VARIANT_NAMES) == set(range(cdef.BATCH_VARIANTS))


def test_search_batch_rejects_before_enqueue(lib):
    # bad jobs, tunings and workspaces fail on the host (no GPU here)
    from paper_1602_05975_amd import cdef
    P = 0x20000
    j = cdef.CdefJob()
    j.recon = _frame()
    j.src = _frame(ptr=0x900000)
    j.sse = P
    j.damping = 3
    arr = (cdef.CdefJob * 1)(j)
    n = lib.cdef_batch_workspace_bytes(1)
    assert n >= C.sizeof(cdef.CdefJob)
    assert lib.cdef_search_batch(arr, 1, C.byref(cdef.tuning(wg_per_cu=5)), C.c_void_p(P), n,
                                 None) == -2
    assert lib.cdef_search_batch(arr, 0, None, C.c_void_p(P), n, None) == -1
    assert lib.cdef_search_batch(arr, 1, None, None, n, None) == -1
    assert lib.cdef_search_batch(arr, 1, None, C.c_void_p(P), n - 1, None) == -4
    j.damping = 9
    arr = (cdef.CdefJob * 1)(j)
    assert lib.cdef_search_batch(arr, 1, None, C.c_void_p(P), n, None) == -1
