"""Shared test helpers: moving synthetic frames to the GPU and running the
oracle on the same arrays."""
from __future__ import annotations

import os

import numpy as np

ORACLE_THREADS = max(1, min(16, os.cpu_count() or 1))


def gpu_frame(planes, fr):
    from paper_1602_05975_amd import cdef
    return cdef.Frame.from_numpy(planes, fr.width, fr.height, fr.bitdepth, fr.layout)


def to_np_u16(t):
    return t.cpu().numpy().view(np.uint16)


def gpu_search(fr, skip=True, damping=None, full=False):
    """GPU SSE table ([nplanes][fbr][fbc][16][4], or [..][2][16][4] with
    full=True), dir and var, as numpy arrays."""
    import torch
    from paper_1602_05975_amd import cdef
    rec = gpu_frame(fr.recon, fr)
    src = gpu_frame(fr.src, fr)
    sk = torch.from_numpy(fr.skip).cuda() if skip else None
    sse, d, v = cdef.search_strengths(rec, src, sk, fr.damping if damping is None else damping,
                                      want_dir=True, full=full)
    torch.cuda.synchronize()
    return sse.cpu().numpy().view(np.uint64), d.cpu().numpy(), v.cpu().numpy()


def oracle_search(oracle, fr, skip=True, damping=None, fbs=None, full=False):
    """Oracle SSE tables [len(fbs)][nplanes][(2,)16][4].  fbs: list of
    (fby, fbx) (default all)."""
    sk = fr.skip if skip else None
    D = fr.damping if damping is None else damping
    d, v = oracle.find_dir(fr.recon[0], fr.bitdepth)
    fbr, fbc = (fr.height + 63) // 64, (fr.width + 63) // 64
    if fbs is None:
        fbs = [(by, bx) for by in range(fbr) for bx in range(fbc)]
    t = oracle.search_fbs(fr.recon, fr.src, fr.width, fr.height, fr.bitdepth, d, v, sk, D, fbs,
                          threads=ORACLE_THREADS, full=full, layout=fr.layout)
    return t, d, v, fbs
