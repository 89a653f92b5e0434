"""Python binding of the gfx950 CDEF library (libcdef_hip.so).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in include/cdef.h.  PyTorch provides the
device memory and the stream.  There is no CPU fallback: when the library is
missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcdef_hip.so")

CDEF_OK = 0
CDEF_E_INVAL = -1
CDEF_E_UNSUPPORTED = -2
CDEF_E_HIP = -3
CDEF_E_NOMEM = -4
CDEF_E_TIMEOUT = -5
LAYOUT_400 = 0
LAYOUT_420 = 1
LAYOUT_422 = 2
LAYOUT_444 = 3

# Exported symbols of include/cdef.h (the tests check that each one exists).
EXPORTS = (
    "cdef_find_dir",
    "cdef_filter_frame",
    "cdef_search_strengths",
    "cdef_search_strengths128",
    "cdef_search_subset",
    "cdef_candidate_mask",
    "cdef_search_weighted",
    "cdef_batch_workspace_bytes",
    "cdef_batch_prepare",
    "cdef_batch_launch",
    "cdef_tuning_variant",
    "cdef_search_batch",
    "cdef_job_validate",
    "cdef_select_presets",
    "cdef_select_presets_workspace_bytes",
    "cdef_select_presets_noalloc",
    "cdef_status_str",
    "cdef_abi_version",
)
MODE_SEARCH = 0
MODE_FILTER = 1
MODE_SEARCH128 = 2
MODE_SEARCH_WEIGHTED = 3
SKIP_CONDITION = 0x80  # bit 7 of a secondary-strength byte


class CdefFrame(C.Structure):
    _fields_ = [
        ("plane", C.c_void_p * 3),
        ("stride", C.c_int64 * 3),
        ("width", C.c_int32),
        ("height", C.c_int32),
        ("bitdepth", C.c_int32),
        ("layout", C.c_int32),
    ]


class CdefFrameOut(C.Structure):
    _fields_ = [("plane", C.c_void_p * 3), ("stride", C.c_int64 * 3)]


class CdefJob(C.Structure):
    _fields_ = [
        ("recon", CdefFrame),
        ("src", CdefFrame),
        ("out", CdefFrameOut),
        ("skip8x8", C.c_void_p),
        ("fb", C.c_void_p),
        ("sse", C.c_void_p),
        ("dir", C.c_void_p),
        ("var", C.c_void_p),
        ("damping", C.c_int32),
        ("mode", C.c_int32),
        ("candidates", C.c_uint32),
        ("reserved", C.c_int32),
    ]


class CdefBatchPlan(C.Structure):
    _fields_ = [
        ("table", C.c_void_p),
        ("njobs", C.c_int32),
        ("nitems", C.c_int32),
        ("variant", C.c_int32),
        ("flags", C.c_int32),
    ]


class CdefTuning(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("wg_per_cu", C.c_int32),
                ("cand_group", C.c_int32), ("order", C.c_int32), ("persistent", C.c_int32)]


BATCH_VARIANTS = 6


class CdefPresetResult(C.Structure):
    _fields_ = [
        ("n", C.c_int32),
        ("reserved", C.c_int32),
        ("luma", (C.c_int32 * 8) * 4),
        ("chroma", (C.c_int32 * 8) * 4),
        ("dist_luma", C.c_uint64 * 4),
        ("dist_chroma", C.c_uint64 * 4),
        ("cost", C.c_double * 4),
    ]


class CdefError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {status_str(status)} ({status})")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libcdef_hip.so once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "(hipcc --offload-arch=gfx950); there is no CPU fallback")
    L = C.CDLL(path)
    P = C.c_void_p
    L.cdef_find_dir.argtypes = [C.POINTER(CdefFrame), P, P, P]
    L.cdef_find_dir.restype = C.c_int
    L.cdef_filter_frame.argtypes = [C.POINTER(CdefFrame), C.POINTER(CdefFrameOut), P, P, P,
                                    C.c_int32, P, P]
    L.cdef_filter_frame.restype = C.c_int
    L.cdef_search_strengths.argtypes = [C.POINTER(CdefFrame), C.POINTER(CdefFrame), P,
                                        C.c_int32, P, P, P, P]
    L.cdef_search_strengths.restype = C.c_int
    L.cdef_search_strengths128.argtypes = L.cdef_search_strengths.argtypes
    L.cdef_search_strengths128.restype = C.c_int
    L.cdef_search_weighted.argtypes = L.cdef_search_strengths.argtypes
    L.cdef_search_weighted.restype = C.c_int
    L.cdef_search_subset.argtypes = [C.POINTER(CdefFrame), C.POINTER(CdefFrame), P, C.c_int32,
                                     C.c_uint32, P, P, P, P]
    L.cdef_search_subset.restype = C.c_int
    L.cdef_candidate_mask.argtypes = [C.c_uint32, C.POINTER(C.c_uint64 * 2)]
    L.cdef_candidate_mask.restype = None
    L.cdef_batch_workspace_bytes.argtypes = [C.c_int32]
    L.cdef_batch_workspace_bytes.restype = C.c_size_t
    L.cdef_batch_prepare.argtypes = [C.POINTER(CdefJob), C.c_int32, P, P, C.c_size_t,
                                     C.POINTER(CdefBatchPlan), P]
    L.cdef_batch_prepare.restype = C.c_int
    L.cdef_batch_launch.argtypes = [C.POINTER(CdefBatchPlan), P]
    L.cdef_batch_launch.restype = C.c_int
    L.cdef_tuning_variant.argtypes = [C.POINTER(CdefTuning), C.POINTER(C.c_int32)]
    L.cdef_tuning_variant.restype = C.c_int
    L.cdef_search_batch.argtypes = [C.POINTER(CdefJob), C.c_int32, C.POINTER(CdefTuning), P,
                                    C.c_size_t, P]
    L.cdef_search_batch.restype = C.c_int
    L.cdef_job_validate.argtypes = [C.POINTER(CdefJob)]
    L.cdef_job_validate.restype = C.c_int
    L.cdef_select_presets.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, P,
                                      C.c_double, C.c_int32, P, P, P, P, C.c_size_t, P]
    L.cdef_select_presets_workspace_bytes.argtypes = []
    L.cdef_select_presets_workspace_bytes.restype = C.c_size_t
    L.cdef_select_presets.restype = C.c_int
    L.cdef_select_presets_noalloc.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, P,
                                              C.c_double, C.c_int32, P, P, P, P]
    L.cdef_select_presets_noalloc.restype = C.c_int
    L.cdef_status_str.argtypes = [C.c_int]
    L.cdef_status_str.restype = C.c_char_p
    L.cdef_abi_version.argtypes = []
    L.cdef_abi_version.restype = C.c_int32
    _lib = L
    return L


def status_str(status: int) -> str:
    return load().cdef_status_str(status).decode()


def _check(status: int, where: str):
    if status != CDEF_OK:
        raise CdefError(status, where)


@dataclasses.dataclass
class Frame:
    """Device-resident frame: 2-D uint16 (or int16) planes, row-major."""

    planes: List  # torch tensors
    width: int
    height: int
    bitdepth: int
    layout: int

    @property
    def nplanes(self) -> int:
        return 1 if self.layout == LAYOUT_400 else 3

    @property
    def search_planes(self) -> int:
        """Planes the searches write (4:2:2 chroma is never filtered)."""
        return 3 if self.layout in (LAYOUT_420, LAYOUT_444) else 1

    @property
    def block_shape(self):
        return ((self.height + 7) // 8, (self.width + 7) // 8)

    @property
    def fb_shape(self):
        return ((self.height + 63) // 64, (self.width + 63) // 64)

    def c_struct(self) -> CdefFrame:
        """The cdef_frame of this frame.  Built once and reused while the
        planes' addresses and row strides and the geometry stay the same (the
        struct holds nothing else; a serving loop calls this per request);
        the callers copy it by value or only read it."""
        key = (tuple(None if t is None else (t.data_ptr(), t.stride(0)) for t in self.planes[:3]),
               self.width, self.height, self.bitdepth, self.layout)
        cached = self.__dict__.get("_cstruct")
        if cached is not None and cached[0] == key:
            return cached[1]
        f = CdefFrame()
        for p, t in enumerate(self.planes[:3]):
            if t is None:
                continue
            assert t.dim() == 2 and t.stride(1) == 1 and t.element_size() == 2
            f.plane[p] = t.data_ptr()
            f.stride[p] = t.stride(0)
        f.width, f.height, f.bitdepth, f.layout = self.width, self.height, self.bitdepth, self.layout
        self.__dict__["_cstruct"] = (key, f)
        return f

    @staticmethod
    def from_numpy(planes: Sequence, width: int, height: int, bitdepth: int, layout: int,
                   device="cuda") -> "Frame":
        import torch
        ts = [torch.from_numpy(p.view("int16") if p.dtype.name == "uint16" else p).to(device)
              for p in planes]
        return Frame(ts, width, height, bitdepth, layout)


def _stream_handle(stream) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


# ---- the C ABI, one function per entry point --------------------------------

def cdef_find_dir(frame: Frame, dir, var, stream=None) -> None:
    st = load().cdef_find_dir(C.byref(frame.c_struct()), _ptr(dir), _ptr(var),
                              _stream_handle(stream))
    _check(st, "cdef_find_dir")


def cdef_filter_frame(frame: Frame, out_planes: Sequence, dir, var, skip, damping: int, fb,
                      stream=None) -> None:
    o = CdefFrameOut()
    for p, t in enumerate(out_planes[:3]):
        if t is not None:
            o.plane[p] = t.data_ptr()
            o.stride[p] = t.stride(0)
    st = load().cdef_filter_frame(C.byref(frame.c_struct()), C.byref(o), _ptr(dir), _ptr(var),
                                  _ptr(skip), damping, _ptr(fb), _stream_handle(stream))
    _check(st, "cdef_filter_frame")


def cdef_search_strengths(recon: Frame, src: Frame, skip, damping: int, sse, dir=None, var=None,
                          stream=None) -> None:
    st = load().cdef_search_strengths(C.byref(recon.c_struct()), C.byref(src.c_struct()),
                                      _ptr(skip), damping, _ptr(sse), _ptr(dir), _ptr(var),
                                      _stream_handle(stream))
    _check(st, "cdef_search_strengths")


def cdef_search_strengths128(recon: Frame, src: Frame, skip, damping: int, sse, dir=None,
                             var=None, stream=None) -> None:
    st = load().cdef_search_strengths128(C.byref(recon.c_struct()), C.byref(src.c_struct()),
                                         _ptr(skip), damping, _ptr(sse), _ptr(dir), _ptr(var),
                                         _stream_handle(stream))
    _check(st, "cdef_search_strengths128")


def subset(pri=range(16), sec_index=range(4), skip_bits=(0,)) -> int:
    """Preset subset word: the S^(p) values, S^(s) indices (0..3 for 0, 1,
    2, 4) and skip condition bits to evaluate."""
    w = 0
    for p in pri:
        w |= 1 << p
    for i in sec_index:
        w |= 1 << (16 + i)
    for k in skip_bits:
        w |= 1 << (20 + k)
    return w


def candidate_mask(candidates: int):
    """The two 64-bit candidate words of a subset (cdef_candidate_mask)."""
    m = (C.c_uint64 * 2)()
    load().cdef_candidate_mask(candidates, C.byref(m))
    return [int(m[0]), int(m[1])]


def cdef_search_subset(recon: Frame, src: Frame, skip, damping: int, candidates: int, sse,
                       dir=None, var=None, stream=None) -> None:
    st = load().cdef_search_subset(C.byref(recon.c_struct()), C.byref(src.c_struct()),
                                   _ptr(skip), damping, candidates, _ptr(sse), _ptr(dir),
                                   _ptr(var), _stream_handle(stream))
    _check(st, "cdef_search_subset")


def search_subset(recon: Frame, src: Frame, skip, damping: int, candidates: int, stream=None):
    """The subset search's table (128-combination layout when the subset has
    the skip condition bit set, else 64); presets outside: 2^64 - 1."""
    import torch
    fbr, fbc = recon.fb_shape
    full = bool((candidates >> 21) & 1)
    shape = (recon.search_planes, fbr, fbc) + ((2, 16, 4) if full else (16, 4))
    sse = torch.empty(shape, dtype=torch.int64, device=recon.planes[0].device)
    cdef_search_subset(recon, src, skip, damping, candidates, sse, stream=stream)
    return sse


def cdef_search_weighted(recon: Frame, src: Frame, skip, damping: int, dist, dir=None, var=None,
                         stream=None) -> None:
    st = load().cdef_search_weighted(C.byref(recon.c_struct()), C.byref(src.c_struct()),
                                     _ptr(skip), damping, _ptr(dist), _ptr(dir), _ptr(var),
                                     _stream_handle(stream))
    _check(st, "cdef_search_weighted")


# ---- allocating conveniences -------------------------------------------------

def find_dir(frame: Frame, stream=None):
    import torch
    dev = frame.planes[0].device
    d = torch.empty(frame.block_shape, dtype=torch.uint8, device=dev)
    v = torch.empty(frame.block_shape, dtype=torch.int32, device=dev)
    cdef_find_dir(frame, d, v, stream)
    return d, v


def filter_frame(frame: Frame, dir, var, skip, damping: int, fb, stream=None):
    import torch
    outs = [torch.empty_like(p) for p in frame.planes[:frame.nplanes]]
    cdef_filter_frame(frame, outs, dir, var, skip, damping, fb, stream)
    return outs


def search_strengths(recon: Frame, src: Frame, skip, damping: int, want_dir=False, stream=None,
                     full=False, weighted=False):
    """SSE table [nplanes][fbr][fbc][16][4], or with full=True the 128
    combinations [nplanes][fbr][fbc][2][16][4] (skip condition bit 0, 1), or
    with weighted=True the Eq. (14) distortion as float64 [..][16][4]."""
    import torch
    dev = recon.planes[0].device
    fbr, fbc = recon.fb_shape
    shape = (recon.search_planes, fbr, fbc) + ((2, 16, 4) if full else (16, 4))
    sse = torch.empty(shape, dtype=torch.float64 if weighted else torch.int64, device=dev)
    d = v = None
    if want_dir:
        d = torch.empty(recon.block_shape, dtype=torch.uint8, device=dev)
        v = torch.empty(recon.block_shape, dtype=torch.int32, device=dev)
    assert not (full and weighted), "the weighted search covers the 64 pairs"
    fn = (cdef_search_weighted if weighted else
          cdef_search_strengths128 if full else cdef_search_strengths)
    fn(recon, src, skip, damping, sse, d, v, stream)
    return (sse, d, v) if want_dir else sse


# ---- batches ------------------------------------------------------------------

def _out_struct(out_planes) -> CdefFrameOut:
    o = CdefFrameOut()
    for p, t in enumerate(out_planes[:3]):
        if t is not None:
            o.plane[p] = t.data_ptr()
            o.stride[p] = t.stride(0)
    return o


def make_search_job(recon: Frame, src: Frame, skip, damping: int, sse, dir=None,
                    var=None, full=False, weighted=False, candidates=0) -> CdefJob:
    j = CdefJob()
    j.recon, j.src = recon.c_struct(), src.c_struct()
    j.skip8x8, j.sse = _ptr(skip), _ptr(sse)
    j.dir, j.var = _ptr(dir), _ptr(var)
    j.damping = damping
    j.mode = MODE_SEARCH_WEIGHTED if weighted else MODE_SEARCH128 if full else MODE_SEARCH
    j.candidates = candidates
    return j


def make_filter_job(recon: Frame, out_planes, skip, damping: int, fb, dir=None,
                    var=None) -> CdefJob:
    j = CdefJob()
    j.recon = recon.c_struct()
    j.out = _out_struct(out_planes)
    j.skip8x8, j.fb = _ptr(skip), _ptr(fb)
    j.dir, j.var = _ptr(dir), _ptr(var)
    j.damping, j.mode = damping, MODE_FILTER
    return j


def validate_job(job: CdefJob) -> int:
    """Status of the host-side checks of one job (no GPU work)."""
    return load().cdef_job_validate(C.byref(job))


class Batch:
    """A prepared set of jobs launched together (cdef_batch_prepare /
    cdef_batch_launch).  Jobs keep references to their tensors; the device
    workspace and pinned staging buffer live as long as the batch."""

    def __init__(self):
        self.jobs: list = []
        self._keep: list = []
        self.plan = CdefBatchPlan()
        self.workspace = None
        self.staging = None

    def add_search(self, recon: Frame, src: Frame, skip, damping: int, sse, dir=None, var=None,
                   full=False, weighted=False, candidates=0):
        return self.add_job(make_search_job(recon, src, skip, damping, sse, dir, var, full,
                                            weighted, candidates),
                            (recon, src, skip, sse, dir, var))

    def add_filter(self, recon: Frame, out_planes, skip, damping: int, fb, dir=None, var=None):
        return self.add_job(make_filter_job(recon, out_planes, skip, damping, fb, dir, var),
                            (recon, out_planes, skip, fb, dir, var))

    def add_job(self, job: "CdefJob", keep) -> int:
        """Add a ready job; `keep` holds the tensors it points to."""
        self.jobs.append(job)
        self._keep.append(keep)
        return len(self.jobs) - 1

    def reserve(self, njobs: int) -> None:
        """Size the workspace and pinned staging for up to njobs jobs now, so
        later prepares never allocate (pinned allocation blocks the host)."""
        import torch
        nbytes = load().cdef_batch_workspace_bytes(max(1, njobs))
        if self.workspace is None or self.workspace.numel() < nbytes:
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            self.staging = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)

    def prepare(self, stream=None) -> None:
        L = load()
        n = len(self.jobs)
        self.reserve(n)
        arr = (CdefJob * n)(*self.jobs)
        st = L.cdef_batch_prepare(arr, n, self.staging.data_ptr(), self.workspace.data_ptr(),
                                  self.workspace.numel(), C.byref(self.plan),
                                  _stream_handle(stream))
        _check(st, "cdef_batch_prepare")

    def launch(self, stream=None) -> None:
        _check(load().cdef_batch_launch(C.byref(self.plan), _stream_handle(stream)),
               "cdef_batch_launch")

    @property
    def nitems(self) -> int:
        return self.plan.nitems


def tuning(wg_per_cu=0, order=0, persistent=0) -> CdefTuning:
    t = CdefTuning()
    t.wg_per_cu, t.order, t.persistent = wg_per_cu, order, persistent
    return t


def tuning_variant(t: CdefTuning) -> int:
    v = C.c_int32()
    _check(load().cdef_tuning_variant(C.byref(t), C.byref(v)), "cdef_tuning_variant")
    return v.value


def cdef_search_batch(jobs: Sequence[CdefJob], t: Optional[CdefTuning], workspace,
                      stream=None) -> None:
    """Validate, upload and launch a batch in one call (the caller keeps the
    jobs' tensors and the workspace alive until the stream has passed it)."""
    n = len(jobs)
    arr = (CdefJob * n)(*jobs)
    st = load().cdef_search_batch(arr, n, None if t is None else C.byref(t), _ptr(workspace),
                                  workspace.numel() * workspace.element_size(),
                                  _stream_handle(stream))
    _check(st, "cdef_search_batch")


def batch_workspace(njobs: int, device="cuda"):
    import torch
    return torch.empty(load().cdef_batch_workspace_bytes(max(1, njobs)), dtype=torch.uint8,
                       device=device)


# ---- preset selection (Section 5, Eq. 15) -------------------------------------

def cdef_select_presets(sse, lam: float, refine_passes: int, result, fb_luma, fb_chroma,
                        workspace, stream=None, cand_mask=None) -> None:
    """sse: [nplanes][fbr][fbc][16][4] (64 candidates) or [..][2][16][4] (128);
    cand_mask: two 64-bit words of allowed candidates (None: all)."""
    nplanes, fbr, fbc = sse.shape[0], sse.shape[1], sse.shape[2]
    ncand = 1
    for n in sse.shape[3:]:
        ncand *= n
    cm = None if cand_mask is None else (C.c_uint64 * 2)(*cand_mask)
    st = load().cdef_select_presets(_ptr(sse), nplanes, fbr, fbc, ncand,
                                    None if cm is None else C.addressof(cm), float(lam),
                                    refine_passes,
                                    _ptr(result), _ptr(fb_luma), _ptr(fb_chroma),
                                    _ptr(workspace), workspace.numel() * workspace.element_size(),
                                    _stream_handle(stream))
    _check(st, "cdef_select_presets")


def cdef_select_presets_noalloc(sse, lam: float, refine_passes: int, result, fb_luma, fb_chroma,
                                stream=None, cand_mask=None) -> None:
    """cdef_select_presets on the library's own per-device workspace (no
    allocation anywhere; calls that may overlap on one device race)."""
    nplanes, fbr, fbc = sse.shape[0], sse.shape[1], sse.shape[2]
    ncand = 1
    for n in sse.shape[3:]:
        ncand *= n
    cm = None if cand_mask is None else (C.c_uint64 * 2)(*cand_mask)
    st = load().cdef_select_presets_noalloc(_ptr(sse), nplanes, fbr, fbc, ncand,
                                            None if cm is None else C.addressof(cm), float(lam),
                                            refine_passes, _ptr(result), _ptr(fb_luma),
                                            _ptr(fb_chroma), _stream_handle(stream))
    _check(st, "cdef_select_presets_noalloc")


def preset_workspace(device="cuda"):
    import torch
    n = load().cdef_select_presets_workspace_bytes()
    return torch.empty(n, dtype=torch.uint8, device=device)


def select_presets(sse, lam: float, refine_passes: int = 0, stream=None, workspace=None,
                   cand_mask=None, retries: int = 1) -> dict:
    """Run the preset selection on a device SSE table and return the result
    (this reads the result back, so it synchronizes the stream).  A selection
    that could not complete (its workgroups were not all resident within the
    kernels' bounded wait, behind other work on the device) is run again,
    after every stream of the device has finished, up to `retries` times."""
    import numpy as np
    import torch
    dev = sse.device
    fbr, fbc = sse.shape[1], sse.shape[2]
    res = torch.zeros(C.sizeof(CdefPresetResult), dtype=torch.uint8, device=dev)
    fl = torch.empty((fbr, fbc), dtype=torch.uint8, device=dev)
    fc = torch.empty((fbr, fbc), dtype=torch.uint8, device=dev)
    ws = preset_workspace(dev) if workspace is None else workspace
    for attempt in range(retries + 1):
        cdef_select_presets(sse, lam, refine_passes, res, fl, fc, ws, stream, cand_mask)
        r = CdefPresetResult.from_buffer_copy(res.cpu().numpy().tobytes())
        if r.n != 0:
            break
        if attempt < retries:
            torch.cuda.synchronize(dev)  # let the competing work drain first
    if r.n == 0:
        # the cooperative selection kernel gave up waiting for its workgroups
        # (all of them must be resident at once; see cdef_select_presets)
        raise CdefError(CDEF_E_TIMEOUT, "cdef_select_presets: the selection did not complete")
    return {"n": r.n, "luma": np.array(r.luma, dtype=np.int32),
            "chroma": np.array(r.chroma, dtype=np.int32),
            "dist": np.array([list(r.dist_luma), list(r.dist_chroma)], dtype=np.uint64),
            "cost": np.array(list(r.cost)), "fb_luma": fl.cpu().numpy(),
            "fb_chroma": fc.cpu().numpy()}
