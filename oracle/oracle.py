"""ctypes access to the CPU oracle (TEST INFRASTRUCTURE ONLY).

Only tests, the smoke check and the benchmark's CPU-baseline leg import this
module.  Arrays are numpy; the oracle works on host memory only.
"""
from __future__ import annotations

import ctypes as C
import os
from concurrent.futures import ThreadPoolExecutor
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# CDEF_ORACLE_LIB selects another build of the same source (the sanitizer
# run of the CPU tests loads an instrumented copy this way).
LIB_PATH = os.environ.get("CDEF_ORACLE_LIB") or os.path.join(HERE, "libcdef_oracle.so")


class OracleFrame(C.Structure):
    _fields_ = [
        ("plane", C.c_void_p * 3),
        ("stride", C.c_int64 * 3),
        ("width", C.c_int32),
        ("height", C.c_int32),
        ("bitdepth", C.c_int32),
        ("nplanes", C.c_int32),
        ("layout", C.c_int32),
    ]


LAYOUT_400, LAYOUT_420, LAYOUT_422, LAYOUT_444 = 0, 1, 2, 3


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.cdef_oracle_line_number.argtypes = [C.c_int, C.c_int, C.c_int]
        L.cdef_oracle_line_number.restype = C.c_int
        L.cdef_oracle_direction_costs.argtypes = [P, C.c_int64, C.c_int, C.c_int, C.c_int, P]
        L.cdef_oracle_direction_costs.restype = None
        L.cdef_oracle_find_dir.argtypes = [P, C.c_int64, C.c_int, C.c_int, C.c_int, P, P]
        L.cdef_oracle_find_dir.restype = None
        L.cdef_oracle_constrain.argtypes = [C.c_int, C.c_int, C.c_int]
        L.cdef_oracle_constrain.restype = C.c_int
        L.cdef_oracle_adjust_strength.argtypes = [C.c_int, C.c_int32]
        L.cdef_oracle_adjust_strength.restype = C.c_int
        L.cdef_oracle_chroma_damping.argtypes = [C.c_int, C.c_int]
        L.cdef_oracle_chroma_damping.restype = C.c_int
        L.cdef_oracle_filter_pixel.argtypes = [P, C.c_int64, C.c_int, C.c_int, C.c_int, C.c_int,
                                               C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                               C.c_int, C.c_int]
        L.cdef_oracle_filter_pixel.restype = C.c_int
        L.cdef_oracle_filter_frame.argtypes = [C.POINTER(OracleFrame), P, P, P, P, P, C.c_int, P]
        L.cdef_oracle_filter_frame.restype = None
        L.cdef_oracle_search_fb.argtypes = [C.POINTER(OracleFrame), C.POINTER(OracleFrame), P, P,
                                            P, C.c_int, C.c_int, C.c_int, P]
        L.cdef_oracle_search_fb.restype = None
        L.cdef_oracle_search.argtypes = [C.POINTER(OracleFrame), C.POINTER(OracleFrame), P,
                                         C.c_int, P, P, P]
        L.cdef_oracle_search.restype = None
        L.cdef_oracle_search_fb2.argtypes = [C.POINTER(OracleFrame), C.POINTER(OracleFrame), P,
                                             P, P, C.c_int, C.c_int, C.c_int, C.c_int, P]
        L.cdef_oracle_search_fb2.restype = None
        L.cdef_oracle_search_fb3.argtypes = [C.POINTER(OracleFrame), C.POINTER(OracleFrame), P,
                                             P, P, C.c_int, C.c_int, C.c_uint32, C.c_int,
                                             C.c_int, P]
        L.cdef_oracle_search_fb3.restype = None
        L.cdef_oracle_search_fb_weighted.argtypes = [C.POINTER(OracleFrame),
                                                     C.POINTER(OracleFrame), P, P, P, C.c_int,
                                                     C.c_int, C.c_int, P]
        L.cdef_oracle_search_fb_weighted.restype = None
        L.cdef_oracle_select_presets.argtypes = [P, C.c_int, C.c_int, C.c_int, P, C.c_double,
                                                 C.c_int, P, P, P, P, P, P, P]
        L.cdef_oracle_select_presets.restype = None
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def infer_layout(planes: Sequence[np.ndarray], width: int, height: int) -> int:
    """Layout from the plane shapes (4:2:0 when shapes do not tell apart)."""
    if len(planes) == 1:
        return LAYOUT_400
    h, w = planes[1].shape
    if (h, w) == ((height + 1) // 2, (width + 1) // 2):
        return LAYOUT_420
    if (h, w) == (height, (width + 1) // 2):
        return LAYOUT_422
    assert (h, w) == (height, width), "chroma planes match no layout"
    return LAYOUT_444


def _frame(planes: Sequence[np.ndarray], width: int, height: int, bitdepth: int,
           layout: Optional[int] = None) -> OracleFrame:
    f = OracleFrame()
    for p, a in enumerate(planes):
        assert a.dtype == np.uint16 and a.flags.c_contiguous
        f.plane[p] = a.ctypes.data
        f.stride[p] = a.shape[1]
    f.width, f.height, f.bitdepth, f.nplanes = width, height, bitdepth, len(planes)
    f.layout = infer_layout(planes, width, height) if layout is None else layout
    return f


def search_planes(nplanes: int, layout: int) -> int:
    """Planes a search covers: luma only at 4:0:0 and 4:2:2."""
    return 3 if nplanes == 3 and layout != LAYOUT_422 else 1


def line_number(d: int, i: int, j: int) -> int:
    return lib().cdef_oracle_line_number(d, i, j)


def direction_costs(block: np.ndarray, bitdepth: int) -> np.ndarray:
    """Algorithm 1's 840-scaled s[d] for a (bh, bw) block, bh, bw <= 8."""
    b = np.ascontiguousarray(block, dtype=np.uint16)
    cost = np.zeros(8, dtype=np.int64)
    lib().cdef_oracle_direction_costs(b.ctypes.data, b.shape[1], b.shape[1], b.shape[0],
                                      bitdepth, cost.ctypes.data)
    return cost


def find_dir(luma: np.ndarray, bitdepth: int):
    luma = np.ascontiguousarray(luma, dtype=np.uint16)
    h, w = luma.shape
    shape = ((h + 7) // 8, (w + 7) // 8)
    d = np.zeros(shape, dtype=np.uint8)
    v = np.zeros(shape, dtype=np.int32)
    lib().cdef_oracle_find_dir(luma.ctypes.data, w, w, h, bitdepth, d.ctypes.data, v.ctypes.data)
    return d, v


def constrain(diff: int, strength: int, damping: int) -> int:
    return lib().cdef_oracle_constrain(diff, strength, damping)


def adjust_strength(strength: int, var: int) -> int:
    return lib().cdef_oracle_adjust_strength(strength, var)


def chroma_damping(damping: int, pri: int) -> int:
    return lib().cdef_oracle_chroma_damping(damping, pri)


def filter_pixel(plane: np.ndarray, i: int, j: int, d: int, pri_s: int, pri_d: int, w1: int,
                 w2: int, sec_s: int, sec_d: int) -> int:
    plane = np.ascontiguousarray(plane, dtype=np.uint16)
    h, w = plane.shape
    return lib().cdef_oracle_filter_pixel(plane.ctypes.data, w, w, h, i, j, d, pri_s, pri_d,
                                          w1, w2, sec_s, sec_d)


def filter_frame(planes: Sequence[np.ndarray], width: int, height: int, bitdepth: int,
                 dir: np.ndarray, var: np.ndarray, skip: Optional[np.ndarray], damping: int,
                 strengths: np.ndarray, layout: Optional[int] = None):
    planes = [np.ascontiguousarray(p, dtype=np.uint16) for p in planes]
    f = _frame(planes, width, height, bitdepth, layout)
    outs = [np.zeros_like(p) for p in planes]
    outp = (C.c_void_p * 3)(*([o.ctypes.data for o in outs] + [None] * (3 - len(outs))))
    outs_stride = (C.c_int64 * 3)(*([o.shape[1] for o in outs] + [0] * (3 - len(outs))))
    dir = np.ascontiguousarray(dir, dtype=np.uint8)
    var = np.ascontiguousarray(var, dtype=np.int32)
    st = np.ascontiguousarray(strengths, dtype=np.uint8)
    sk = None if skip is None else np.ascontiguousarray(skip, dtype=np.uint8)
    lib().cdef_oracle_filter_frame(C.byref(f), outp, outs_stride, dir.ctypes.data,
                                   var.ctypes.data, _ptr(sk), damping, st.ctypes.data)
    return outs


def search_fbs(recon: Sequence[np.ndarray], src: Sequence[np.ndarray], width: int, height: int,
               bitdepth: int, dir: np.ndarray, var: np.ndarray, skip: Optional[np.ndarray],
               damping: int, fbs, threads: int = 1, full: bool = False,
               layout: Optional[int] = None, cand: int = 0) -> np.ndarray:
    """SSE tables [len(fbs)][nplanes][16][4] for the listed (fby, fbx) blocks,
    or [len(fbs)][nplanes][2][16][4] with full=True (skip condition bit 0, 1).
    cand: preset subset (S^(p) mask | S^(s) index mask << 16 | skip bit mask
    << 20, 0 = all); entries outside it are 2^64 - 1.

    dir/var must come from find_dir (the oracle's own).  ctypes releases the
    GIL during the call, so a thread pool runs filter blocks in parallel."""
    recon = [np.ascontiguousarray(p, dtype=np.uint16) for p in recon]
    src = [np.ascontiguousarray(p, dtype=np.uint16) for p in src]
    fr = _frame(recon, width, height, bitdepth, layout)
    fs = _frame(src, width, height, bitdepth, fr.layout)
    dir = np.ascontiguousarray(dir, dtype=np.uint8)
    var = np.ascontiguousarray(var, dtype=np.int32)
    sk = None if skip is None else np.ascontiguousarray(skip, dtype=np.uint8)
    fbs = list(fbs)
    nskip = 2 if full else 1
    out = np.zeros((len(fbs), search_planes(len(recon), fr.layout), nskip, 16, 4),
                   dtype=np.uint64)
    L = lib()

    def one(k):
        by, bx = fbs[k]
        L.cdef_oracle_search_fb3(C.byref(fr), C.byref(fs), dir.ctypes.data, var.ctypes.data,
                                 _ptr(sk), damping, nskip, cand, by, bx, out[k].ctypes.data)

    if threads <= 1:
        for k in range(len(fbs)):
            one(k)
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(one, range(len(fbs))))
    return out if full else out[:, :, 0]


def search(recon: Sequence[np.ndarray], src: Sequence[np.ndarray], width: int, height: int,
           bitdepth: int, skip: Optional[np.ndarray], damping: int, threads: int = 1,
           full: bool = False, layout: Optional[int] = None, cand: int = 0):
    """Whole-frame search: (sse, dir, var); sse is [nplanes][fbr][fbc][16][4],
    or [nplanes][fbr][fbc][2][16][4] with full=True (nplanes: the planes the
    search covers)."""
    d, v = find_dir(recon[0], bitdepth)
    fbr, fbc = (height + 63) // 64, (width + 63) // 64
    fbs = [(by, bx) for by in range(fbr) for bx in range(fbc)]
    t = search_fbs(recon, src, width, height, bitdepth, d, v, skip, damping, fbs, threads, full,
                   layout, cand)
    t = t.reshape((fbr, fbc, t.shape[1]) + t.shape[2:])
    sse = np.moveaxis(t, 2, 0)
    return np.ascontiguousarray(sse), d, v


def search_fbs_weighted(recon: Sequence[np.ndarray], src: Sequence[np.ndarray], width: int,
                        height: int, bitdepth: int, dir: np.ndarray, var: np.ndarray,
                        skip: Optional[np.ndarray], damping: int, fbs,
                        threads: int = 1, layout: Optional[int] = None) -> np.ndarray:
    """Eq. (14) distortion tables, float64 [len(fbs)][nplanes][16][4]."""
    recon = [np.ascontiguousarray(p, dtype=np.uint16) for p in recon]
    src = [np.ascontiguousarray(p, dtype=np.uint16) for p in src]
    fr = _frame(recon, width, height, bitdepth, layout)
    fs = _frame(src, width, height, bitdepth, fr.layout)
    dir = np.ascontiguousarray(dir, dtype=np.uint8)
    var = np.ascontiguousarray(var, dtype=np.int32)
    sk = None if skip is None else np.ascontiguousarray(skip, dtype=np.uint8)
    fbs = list(fbs)
    out = np.zeros((len(fbs), search_planes(len(recon), fr.layout), 16, 4), dtype=np.float64)
    L = lib()

    def one(k):
        by, bx = fbs[k]
        L.cdef_oracle_search_fb_weighted(C.byref(fr), C.byref(fs), dir.ctypes.data,
                                         var.ctypes.data, _ptr(sk), damping, by, bx,
                                         out[k].ctypes.data)

    if threads <= 1:
        for k in range(len(fbs)):
            one(k)
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(one, range(len(fbs))))
    return out


def select_presets(sse: np.ndarray, lam: float, refine_passes: int = 0,
                   cand_mask: Optional[Sequence[int]] = None) -> dict:
    """Eq. (15) preset selection on an SSE table [nplanes][fbr][fbc][16][4]
    (64 candidates) or [nplanes][fbr][fbc][2][16][4] (128 candidates);
    cand_mask: two 64-bit words of allowed candidates (None: all)."""
    sse = np.ascontiguousarray(sse, dtype=np.uint64)
    nplanes = sse.shape[0]
    nfb = int(np.prod(sse.shape[1:3]))
    ncand = int(np.prod(sse.shape[3:]))
    assert ncand in (64, 128)
    n = np.zeros(1, np.int32)
    sl = np.zeros((4, 8), np.int32)
    sc = np.zeros((4, 8), np.int32)
    dist = np.zeros((2, 4), np.uint64)
    cost = np.zeros(4, np.float64)
    fl = np.zeros(nfb, np.uint8)
    fc = np.zeros(nfb, np.uint8)
    cm = None if cand_mask is None else np.array(cand_mask, dtype=np.uint64)
    lib().cdef_oracle_select_presets(sse.ctypes.data, nplanes, nfb, ncand, _ptr(cm), float(lam),
                                     refine_passes, n.ctypes.data, sl.ctypes.data, sc.ctypes.data,
                                     dist.ctypes.data, cost.ctypes.data, fl.ctypes.data,
                                     fc.ctypes.data)
    shape = sse.shape[1:3]
    return {"n": int(n[0]), "luma": sl, "chroma": sc, "dist": dist, "cost": cost,
            "fb_luma": fl.reshape(shape), "fb_chroma": fc.reshape(shape)}
