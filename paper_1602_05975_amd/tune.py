"""Autotuner for batched launches.

Every launch variant of cdef_batch_launch computes bit-identical results;
they differ in the occupancy bound (waves per SIMD, hence the register
budget), in the order in which filter blocks are dealt to the XCDs, and in
a flat grid (one workgroup per filter block) against persistent workgroups
that take filter blocks from per-XCD work queues.  The
tuner times each variant on the caller's prepared batch (HIP events on the
launch stream) and remembers the fastest per batch signature -- the GPU
architecture plus the multiset of (frame-size class, bit depth, layout,
mode) of the jobs -- in a small JSON cache.
"""
from __future__ import annotations

import json
import math
import os
import threading
from collections import Counter
from typing import Dict, Optional

from . import cdef

NUM_VARIANTS = cdef.BATCH_VARIANTS
VARIANT_NAMES = {
    0: "3 waves/SIMD, XCD-contiguous order",
    1: "2 waves/SIMD, XCD-contiguous order",
    2: "3 waves/SIMD, plain order",
    3: "2 waves/SIMD, plain order",
    4: "3 waves/SIMD, persistent workgroups on per-XCD queues",
    5: "2 waves/SIMD, persistent workgroups on per-XCD queues",
}
# the cdef_tuning of each variant (wg_per_cu, order, persistent)
VARIANT_TUNING = {0: (3, 0, 0), 1: (2, 0, 0), 2: (3, 1, 0), 3: (2, 1, 0), 4: (3, 0, 1),
                  5: (2, 0, 1)}
_lock = threading.Lock()


def cache_path() -> str:
    return os.environ.get("CDEF_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "cdef_mi355x",
                                       "tune.json"))


def _load_cache(path: str) -> Dict[str, dict]:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def signature(batch: "cdef.Batch") -> str:
    """Arch + job mix, with frame sizes bucketed by filter-block count."""
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    mix = Counter()
    for j in batch.jobs:
        nfb = ((j.recon.width + 63) // 64) * ((j.recon.height + 63) // 64)
        size_class = int(math.log2(max(1, nfb)))
        mix[(size_class, j.recon.bitdepth, j.recon.layout, j.mode)] += 1
    items = sorted(f"{k[0]}:{k[1]}:{k[2]}:{k[3]}x{v}" for k, v in mix.items())
    return arch + "|" + ",".join(items)


def time_variants(batch: "cdef.Batch", stream=None, reps: int = 3) -> Dict[int, float]:
    """Median launch time (ms) of every variant on this batch."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    out = {}
    keep = batch.plan.variant
    for v in range(NUM_VARIANTS):
        batch.plan.variant = v
        batch.launch(s)  # warm-up
        times = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(s)
            batch.launch(s)
            b.record(s)
            b.synchronize()
            times.append(a.elapsed_time(b))
        out[v] = sorted(times)[len(times) // 2]
    batch.plan.variant = keep
    return out


def tune(batch: "cdef.Batch", stream=None, reps: int = 3, use_cache: bool = True,
         path: Optional[str] = None) -> int:
    """Pick the fastest variant for `batch`, set it in the batch's plan and
    return it.  Cached results are reused without timing."""
    path = path or cache_path()
    sig = signature(batch)
    with _lock:
        cache = _load_cache(path) if use_cache else {}
    if sig in cache:
        v = int(cache[sig]["variant"])
    else:
        times = time_variants(batch, stream, reps)
        v = min(times, key=times.get)
        with _lock:
            cache = _load_cache(path)
            cache[sig] = {"variant": v, "ms": {str(k): t for k, t in times.items()}}
            try:
                os.makedirs(os.path.dirname(path), exist_ok=True)
                tmp = path + ".tmp"
                with open(tmp, "w") as f:
                    json.dump(cache, f, indent=1)
                os.replace(tmp, path)
            except OSError:
                pass  # a read-only home still tunes, it just does not remember
    batch.plan.variant = v
    return v
