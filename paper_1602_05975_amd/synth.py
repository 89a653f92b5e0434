"""Seeded synthetic CDEF workloads.

This module holds no CDEF arithmetic. It only makes frames that look like
coded video: a source image and a "reconstruction" that carries quantization
ringing, which is what CDEF is designed to remove (Section 1 and Section 2 of
the paper: the filter runs on deblocked reconstructed pixels, and the encoder
search scores filtered pixels against the uncoded source, Section 5).

Recipe, per plane (chroma planes at chroma resolution, with independent
random streams), for every R x R region (R = 64 luma, 32 chroma at 4:2:0):

* a sinusoidal grating A * sin(2 pi (x cos t + y sin t) / P + phi) with
  t ~ U[0, pi), P ~ U[3, 16] px, phi ~ U[0, 2 pi), A ~ U[16, 96] (8-bit units);
* plus a linear gradient g * (x cos psi + y sin psi), g ~ U[-1, 1] per px,
  psi ~ U[0, 2 pi);
* plus 128, times 2^(bitdepth - 8), rounded half-to-even and clipped to the
  sample range.  That is the source.

The reconstruction pads the source to a multiple of 8 by edge replication,
applies the orthonormal 8x8 DCT-II to every block, quantizes every
coefficient to q * round(c / q), inverts, rounds, clips and crops.  The step q
is 24 for 8-bit and 64 for 10-bit content.

Both the oracle-based tests and the GPU path consume the arrays produced
here; nothing else is shared between them.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

SEED_BASE = 1602059750

LAYOUT_400 = 0
LAYOUT_420 = 1
LAYOUT_422 = 2
LAYOUT_444 = 3


def chroma_shift(layout: int):
    """(horizontal, vertical) chroma subsampling shifts."""
    return {LAYOUT_420: (1, 1), LAYOUT_422: (1, 0), LAYOUT_444: (0, 0)}.get(layout, (0, 0))

# Configurations of the synthetic workloads: (width, height) choices of the
# mixed batch and serving requests.
MIXED_RESOLUTIONS = [(426, 240), (640, 360), (1280, 720), (1920, 1080), (3840, 2160)]


# Seed streams of the synthetic workloads.
WL_CIF, WL_1080P, WL_4K, WL_MIXED, WL_SERVE = 0, 1, 2, 3, 4


def workload_seed(workload: int, frame: int) -> int:
    return SEED_BASE + 1000 * workload + frame


@dataclasses.dataclass
class Frame:
    """One frame: planes are uint16 2-D arrays (rows, cols), C-contiguous."""

    width: int
    height: int
    bitdepth: int
    layout: int
    src: List[np.ndarray]
    recon: List[np.ndarray]
    skip: np.ndarray  # uint8 [ceil(h/8)][ceil(w/8)], 1 = block has no residual
    damping: int = 3
    seed: int = 0

    @property
    def nplanes(self) -> int:
        return 1 if self.layout == LAYOUT_400 else 3

    @property
    def search_planes(self) -> int:
        """Planes the searches cover (4:2:2 chroma is never filtered)."""
        return 3 if self.layout in (LAYOUT_420, LAYOUT_444) else 1

    def plane_dims(self, p: int):
        if p == 0:
            return self.width, self.height
        sx, sy = chroma_shift(self.layout)
        return (self.width + sx) >> sx, (self.height + sy) >> sy

    @property
    def luma_pixels(self) -> int:
        return self.width * self.height

    @property
    def fb_cols(self) -> int:
        return (self.width + 63) // 64

    @property
    def fb_rows(self) -> int:
        return (self.height + 63) // 64

    @property
    def blk_cols(self) -> int:
        return (self.width + 7) // 8

    @property
    def blk_rows(self) -> int:
        return (self.height + 7) // 8


def _dct_matrix() -> np.ndarray:
    n = np.arange(8)
    k = n[:, None]
    c = np.cos(np.pi * (2 * n[None, :] + 1) * k / 16.0)
    c[0, :] *= math.sqrt(1.0 / 8.0)
    c[1:, :] *= math.sqrt(2.0 / 8.0)
    return c


_DCT = _dct_matrix()


def _grating_plane(rng: np.random.Generator, w: int, h: int, region: int, bitdepth: int) -> np.ndarray:
    nrx = (w + region - 1) // region
    nry = (h + region - 1) // region
    nreg = nrx * nry
    theta = rng.uniform(0.0, math.pi, nreg)
    period = rng.uniform(3.0, 16.0, nreg)
    phase = rng.uniform(0.0, 2 * math.pi, nreg)
    amp = rng.uniform(16.0, 96.0, nreg)
    grad = rng.uniform(-1.0, 1.0, nreg)
    psi = rng.uniform(0.0, 2 * math.pi, nreg)

    def grid(a):
        return a.reshape(nry, 1, nrx, 1)

    yy = np.arange(region, dtype=np.float64).reshape(1, region, 1, 1)
    xx = np.arange(region, dtype=np.float64).reshape(1, 1, 1, region)
    th, pe, ph, am = grid(theta), grid(period), grid(phase), grid(amp)
    gr, ps = grid(grad), grid(psi)
    val = am * np.sin(2 * np.pi * (xx * np.cos(th) + yy * np.sin(th)) / pe + ph)
    val = val + gr * (xx * np.cos(ps) + yy * np.sin(ps)) + 128.0
    val = val.reshape(nry * region, nrx * region)[:h, :w]
    val = val * float(1 << (bitdepth - 8))
    return np.clip(np.rint(val), 0, (1 << bitdepth) - 1)


def _code_plane(src: np.ndarray, q: float, bitdepth: int) -> np.ndarray:
    h, w = src.shape
    ph = (h + 7) // 8 * 8
    pw = (w + 7) // 8 * 8
    x = np.pad(src.astype(np.float64), ((0, ph - h), (0, pw - w)), mode="edge")
    b = x.reshape(ph // 8, 8, pw // 8, 8).transpose(0, 2, 1, 3)
    coef = _DCT @ b @ _DCT.T
    coef = q * np.rint(coef / q)
    rec = _DCT.T @ coef @ _DCT
    rec = rec.transpose(0, 2, 1, 3).reshape(ph, pw)[:h, :w]
    return np.clip(np.rint(rec), 0, (1 << bitdepth) - 1)


def make_frame(width: int, height: int, bitdepth: int, layout: int, seed: int,
               skip_prob: float = 0.0, damping: int = 3, q: Optional[float] = None) -> Frame:
    """Build one seeded frame (source, ringing reconstruction, skip map)."""
    if q is None:
        q = 24.0 if bitdepth == 8 else 64.0 * (1 << max(0, bitdepth - 10))
    nplanes = 1 if layout == LAYOUT_400 else 3
    sx, sy = chroma_shift(layout)
    src, recon = [], []
    for p in range(nplanes):
        rng = np.random.Generator(np.random.PCG64([seed, p]))
        if p == 0:
            w, h, region = width, height, 64
        else:
            w, h, region = (width + sx) >> sx, (height + sy) >> sy, 64 >> max(sx, sy)
        s = _grating_plane(rng, w, h, region, bitdepth)
        r = _code_plane(s, q, bitdepth)
        src.append(np.ascontiguousarray(s.astype(np.uint16)))
        recon.append(np.ascontiguousarray(r.astype(np.uint16)))
    brows, bcols = (height + 7) // 8, (width + 7) // 8
    rng = np.random.Generator(np.random.PCG64([seed, 7]))
    if skip_prob > 0:
        skip = (rng.random((brows, bcols)) < skip_prob).astype(np.uint8)
    else:
        skip = np.zeros((brows, bcols), dtype=np.uint8)
    return Frame(width, height, bitdepth, layout, src, recon, skip, damping, seed)


def random_strengths(frame: Frame, seed: int) -> np.ndarray:
    """Per-FB strengths (pri_y, sec_y, pri_uv, sec_uv), uint8 [fb_rows][fb_cols][4]."""
    rng = np.random.Generator(np.random.PCG64([seed, 11]))
    shape = (frame.fb_rows, frame.fb_cols)
    sec_vals = np.array([0, 1, 2, 4], dtype=np.uint8)
    out = np.zeros(shape + (4,), dtype=np.uint8)
    out[..., 0] = rng.integers(0, 16, shape)
    out[..., 1] = sec_vals[rng.integers(0, 4, shape)]
    out[..., 2] = rng.integers(0, 16, shape)
    out[..., 3] = sec_vals[rng.integers(0, 4, shape)]
    return out


def random_presets(frame: Frame, seed: int, p_skipcond: float = 0.5,
                   p_special: float = 0.15) -> np.ndarray:
    """Per-FB presets as random_strengths, with the skip condition bit (bit 7
    of each secondary byte) set with probability p_skipcond and, per plane
    group, the (0, 0)-with-bit preset (strengths 19, 7) with p_special."""
    out = random_strengths(frame, seed)
    rng = np.random.Generator(np.random.PCG64([seed, 13]))
    shape = (frame.fb_rows, frame.fb_cols)
    for pri, sec in ((0, 1), (2, 3)):
        bit = rng.random(shape) < p_skipcond
        special = rng.random(shape) < p_special
        out[..., pri][special] = 0
        out[..., sec][special] = 0
        out[..., sec] |= ((bit | special).astype(np.uint8) << 7)
    return out


# Inputs that reach the method's degenerate cases and the arithmetic limits
# of a fixed-width implementation: flat planes, the largest possible
# |recon - source| in both signs, two-level stripes and checkerboards (equal
# line costs for several directions), and full-range noise.
EDGE_KINDS = ("constant", "extreme_hi", "extreme_lo", "stripes", "checker", "noise", "binary")


def _edge_plane(kind: str, rng: np.random.Generator, w: int, h: int, maxv: int):
    """(recon, source) of one plane for an edge-case kind."""
    def noise():
        return rng.integers(0, maxv + 1, size=(h, w))

    if kind == "constant":
        a, b = (int(x) for x in rng.integers(0, maxv + 1, 2))
        return np.full((h, w), a), np.full((h, w), b)
    if kind == "extreme_hi":
        return np.full((h, w), maxv), np.zeros((h, w), np.int64)
    if kind == "extreme_lo":
        return np.zeros((h, w), np.int64), np.full((h, w), maxv)
    if kind == "noise":
        return noise(), noise()
    if kind == "binary":
        return maxv * rng.integers(0, 2, size=(h, w)), noise()
    # two-level patterns per 8x8 region of the plane
    yy, xx = np.mgrid[0:h, 0:w]
    rec = np.zeros((h, w), np.int64)
    for ry in range(0, h, 8):
        for rx in range(0, w, 8):
            y = yy[ry:ry + 8, rx:rx + 8]
            x = xx[ry:ry + 8, rx:rx + 8]
            lo, hi = (int(v) for v in rng.integers(0, maxv + 1, 2))
            if kind == "stripes":
                period = int(rng.integers(1, 5))
                orient = int(rng.integers(0, 4))
                coord = (y, x, x + y, x - y + 64)[orient]
                on = (coord // period) % 2
            else:  # checker
                cell = int((1, 2, 4)[rng.integers(0, 3)])
                on = (y // cell + x // cell) % 2
            rec[ry:ry + 8, rx:rx + 8] = np.where(on == 1, hi, lo)
    src = noise() if kind == "stripes" else np.full((h, w), (maxv + 1) // 2)
    return rec, src


def edge_frame(kind: str, width: int, height: int, bitdepth: int, layout: int, seed: int,
               damping: int = 3, skip_prob: float = 0.3) -> Frame:
    """A seeded frame of one of EDGE_KINDS.  The skip map is Bernoulli
    (skip_prob) per 8x8 block, with every block of filter block (0, 1)
    skipped and none of filter block (1, 0), where those exist."""
    assert kind in EDGE_KINDS, kind
    nplanes = 1 if layout == LAYOUT_400 else 3
    sx, sy = chroma_shift(layout)
    maxv = (1 << bitdepth) - 1
    src, recon = [], []
    for p in range(nplanes):
        rng = np.random.Generator(np.random.PCG64([seed, p, 17]))
        w, h = (width, height) if p == 0 else ((width + sx) >> sx, (height + sy) >> sy)
        r, s = _edge_plane(kind, rng, w, h, maxv)
        recon.append(np.ascontiguousarray(r.astype(np.uint16)))
        src.append(np.ascontiguousarray(s.astype(np.uint16)))
    brows, bcols = (height + 7) // 8, (width + 7) // 8
    rng = np.random.Generator(np.random.PCG64([seed, 7, 17]))
    skip = (rng.random((brows, bcols)) < skip_prob).astype(np.uint8)
    if bcols > 8:
        skip[0:8, 8:16] = 1
    if brows > 8:
        skip[8:16, 0:8] = 0
    return Frame(width, height, bitdepth, layout, src, recon, skip, damping, seed)


def cif_luma() -> Frame:
    """352x288 8-bit luma, filtered with (pri 4, sec 2) and damping 5."""
    return make_frame(352, 288, 8, LAYOUT_400, workload_seed(WL_CIF, 0), damping=5)


def hd1080_frame() -> Frame:
    """One 1920x1080 10-bit 4:2:0 frame for the full strength search (damping 3)."""
    return make_frame(1920, 1080, 10, LAYOUT_420, workload_seed(WL_1080P, 0), damping=3)


def uhd4k_frames(nframes: int = 8) -> List[Frame]:
    """Eight 3840x2160 10-bit 4:2:0 frames with 30% of 8x8 blocks skipped."""
    return [make_frame(3840, 2160, 10, LAYOUT_420, workload_seed(WL_4K, f), skip_prob=0.3, damping=3)
            for f in range(nframes)]


def mixed_frame_params(n: int, workload: int = WL_MIXED):
    """Resolution, bit depth and damping of each frame of an uneven batch."""
    rng = np.random.Generator(np.random.PCG64([workload_seed(workload, 0), 99]))
    out = []
    for _ in range(n):
        w, h = MIXED_RESOLUTIONS[int(rng.integers(0, len(MIXED_RESOLUTIONS)))]
        bd = int((8, 10)[int(rng.integers(0, 2))])
        d = int(rng.integers(3, 7))
        out.append((w, h, bd, d))
    return out


def mixed_frames(nframes: int = 64) -> List[Frame]:
    """An uneven batch of mixed resolution and bit depth frames."""
    return [make_frame(w, h, bd, LAYOUT_420, workload_seed(WL_MIXED, i), damping=d)
            for i, (w, h, bd, d) in enumerate(mixed_frame_params(nframes, WL_MIXED))]
