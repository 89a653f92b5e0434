"""Benchmark of the CDEF hot path on one MI355X.

A step is one pass of the whole path -- tile staging, direction search,
per-block filter parameters, the constrained filter under all 64 strength
pairs and the fused SSE reduction -- over one batch of eight synthetic
3840x2160 10-bit 4:2:0 frames with 30 % of 8x8 blocks skipped: one
cdef_batch_launch over all their filter blocks (--per-frame: one
cdef_search_strengths launch per frame).  Inputs are resident in HBM before
the timed region.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--per-frame] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work of the fused search (frozen formula, independent of the
# kernel's instruction count): element operations per plane sample that is
# filtered (12 tap differences/magnitudes/clamp bounds 48, 15 primary
# strengths x 4 taps x 6 = 360, 3 secondary strengths x 8 taps x 6 = 144,
# 64 pairs x 8 = 512), per skipped sample (difference, square, accumulate),
# and per luma pixel for the direction search.
OPS_PER_FILTERED_SAMPLE = 1064
OPS_PER_SKIPPED_SAMPLE = 3
OPS_PER_LUMA_PX_DIRSEARCH = 10
# The 128-combination search adds, per filtered sample, the (19, 7) preset
# (4 primary taps x 6 + 8 secondary taps x 6 + 8 to combine), and per sample
# the unfiltered difference, square and accumulate over the whole block.
OPS_PER_SPECIAL_SAMPLE = 80
OPS_PER_SAMPLE_UNFILTERED = 3
# The weighted search (Eq. 14) keeps the 7 per-pair operations before the
# square and, per pair, forms d = e + s, d^2 and e^2 and sums d, d^2, e^2
# over the unit (13 instead of 8), and takes 6 source/reconstruction moments
# per sample; the per-unit double-precision weights are not counted.
OPS_PER_FILTERED_SAMPLE_W = OPS_PER_FILTERED_SAMPLE + 64 * (13 - 8)
OPS_PER_SAMPLE_MOMENTS = 6
# The decoder path (direction search + the filter at one signaled preset
# per filter block).  Per sample of a filtered block, each tap of a group
# whose strength is not 0 costs its difference and magnitude (2) and the
# constrained term at that strength (6: shift, saturating subtract, min,
# sign, weight, accumulate); a group at strength 0 adds nothing (f = 0).
# With both groups the sum of the two, and the clamp to the range of the 12
# taps (a max and a min per tap, then the clamp); with one group the clamp
# cannot bind (weights sum to 12/16).  Round (3) and add x (1) in every
# case.  Both groups: 127; primary only: 36; secondary only: 68; neither,
# or a skipped block: 0 (the sample is copied).
FILTER_OPS_PER_TAP = 2 + 6
FILTER_OPS_CLAMP = 2 * 12 + 2
FILTER_OPS_ROUND_ADD = 4


def filter_ops_per_sample(pri_on, sec_on):
    """Element operations per sample of a filtered block (arrays of bool)."""
    pri_on, sec_on = np.asarray(pri_on, bool), np.asarray(sec_on, bool)
    both = pri_on & sec_on
    return np.where(pri_on | sec_on, FILTER_OPS_ROUND_ADD, 0) + \
        FILTER_OPS_PER_TAP * (4 * pri_on + 8 * sec_on) + both * (FILTER_OPS_CLAMP + 1)


def adjusted_luma_strength(pri, var):
    """Eq. (13): the luma primary strength adjusted by the block variance v
    (0 below v = 2^10; the log term 0 while v < 2^16)."""
    pri, var = np.asarray(pri, np.int64), np.asarray(var, np.int64)
    q = var >> 16
    i = np.where(q > 0, np.minimum(np.floor(np.log2(np.maximum(q, 1))), 12), 0).astype(np.int64)
    return np.where(var < 1024, 0, (pri * (4 + i) + 8) // 16)


def filter_work(fr, strengths, var):
    """(algorithmic ops, filtered luma samples, filtered chroma samples) of
    the decoder path on one frame: strengths uint8 [fb_rows][fb_cols][4]
    without the skip condition bit or the special preset, var the 8x8
    blocks' variances from the direction search."""
    assert not (strengths[..., 1] & 0x80).any() and not (strengths[..., 3] & 0x80).any()
    assert (strengths[..., 0] < 16).all() and (strengths[..., 2] < 16).all()
    br, bc = fr.blk_rows, fr.blk_cols
    fb = strengths[np.arange(br)[:, None] // 8, np.arange(bc)[None, :] // 8].astype(np.int64)
    live = ~fr.skip.astype(bool)
    # samples of each 8x8 luma block and of its chroma blocks inside the frame
    ys = np.minimum(8, fr.height - 8 * np.arange(br))[:, None]
    xs = np.minimum(8, fr.width - 8 * np.arange(bc))[None, :]
    n_y = ys * xs
    ops = filter_ops_per_sample(adjusted_luma_strength(fb[..., 0], var) > 0,
                                fb[..., 1] > 0) * n_y * live
    n_c = 0
    if fr.nplanes == 3:
        sx, sy = synth_shift(fr.layout)
        cy = -(-ys // (1 << sy)) if sy else ys
        cx = -(-xs // (1 << sx)) if sx else xs
        n_c = 2 * cy * cx
        ops = ops + filter_ops_per_sample(fb[..., 2] > 0, fb[..., 3] > 0) * n_c * live
    ops = int(ops.sum()) + OPS_PER_LUMA_PX_DIRSEARCH * fr.width * fr.height
    return ops, int((n_y * live).sum()), int((n_c * live).sum())
# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T int32 lane-ops/s;
# packed 16-bit instructions do two element operations per lane.
PEAK_PACKED_I16_TOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
PEAK_HBM_GBS = 8000.0
# The subset workload's default: S^(p) in {0, 1, 2, 3, 4, 6, 8, 11}, every
# S^(s), skip condition bit 0 -- 32 of the 64 pairs.
DEFAULT_SUBSET = (0b0000100101011111 | (0b1111 << 16) | (0b01 << 20))
# bit depth and layout of the format workloads (luma 3840x2160, 8 frames)
FORMATS = {"search4k": (10, 1), "search128": (10, 1), "weighted": (10, 1), "subset": (10, 1),
           "search12": (12, 1), "search444": (10, 3), "search422": (10, 2)}
KERNEL_SOURCES = ["k_fused.hip", "cdef_device.hpp"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for s in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1602_05975_amd", "csrc", s), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def subset_counts(cand):
    """(non-zero S^(p) values, non-zero S^(s) values, (S^(p), S^(s)) pairs,
    skip condition bits) of a preset subset word (0: all presets)."""
    if not cand:
        return 15, 3, 64, 2
    pri = [p for p in range(16) if (cand >> p) & 1]
    sec = [i for i in range(4) if (cand >> (16 + i)) & 1]
    skb = [k for k in range(2) if (cand >> (20 + k)) & 1]
    return (len([p for p in pri if p]), len([i for i in sec if i]), len(pri) * len(sec), len(skb))


def ops_per_filtered_sample(cand=0):
    """OPS_PER_FILTERED_SAMPLE restricted to a subset's strengths and pairs."""
    npri, nsec, npairs, _ = subset_counts(cand)
    return 48 + 24 * npri + 48 * nsec + 8 * npairs


def frame_work(fr, full=False, weighted=False, cand=0):
    """(algorithmic ops, algorithmic HBM bytes) of one fused search launch
    (full: the 128-combination search, where the skipped blocks of filter
    blocks with residual are filtered under every preset too; cand: a preset
    subset, whose absent strengths and pairs cost nothing)."""
    filtered = skipped = 0
    sk = fr.skip.astype(bool)
    fb_all = np.zeros((fr.fb_rows, fr.fb_cols), bool)
    for by in range(fr.fb_rows):
        for bx in range(fr.fb_cols):
            fb_all[by, bx] = sk[8 * by:8 * by + 8, 8 * bx:8 * bx + 8].all()
    for p in range(fr.search_planes):
        w, h = fr.plane_dims(p)
        sx, sy = (0, 0) if p == 0 else synth_shift(fr.layout)
        bs, fs = 8 >> sx, 64 >> sx
        if full:  # every sample of a filter block with residual is filtered
            allsk = np.repeat(np.repeat(fb_all, fs, axis=0), fs, axis=1)[:h, :w]
            n_sk = int(allsk.sum())
        else:
            px_sk = np.repeat(np.repeat(sk, bs, axis=0), bs, axis=1)[:h, :w]
            n_sk = int(px_sk.sum())
        skipped += n_sk
        filtered += w * h - n_sk
    per_filtered = ops_per_filtered_sample(cand)
    if full and (not cand or (cand >> 21) & 1):
        per_filtered += OPS_PER_SPECIAL_SAMPLE
    if weighted:
        per_filtered = OPS_PER_FILTERED_SAMPLE_W
    ops = (per_filtered * filtered + OPS_PER_SKIPPED_SAMPLE * skipped
           + OPS_PER_LUMA_PX_DIRSEARCH * fr.width * fr.height)
    samples = filtered + skipped
    if full:
        ops += OPS_PER_SAMPLE_UNFILTERED * samples
    if weighted:
        ops += OPS_PER_SAMPLE_MOMENTS * samples
    nfb = fr.fb_rows * fr.fb_cols
    nblk = fr.blk_rows * fr.blk_cols
    ncand = 128 if full else 64
    bytes_ = 2 * 2 * samples + nblk + nfb * ncand * 8 * fr.search_planes + 5 * nblk
    return ops, bytes_


def synth_shift(layout):
    from paper_1602_05975_amd import synth
    return synth.chroma_shift(layout)


def _host_facts():
    """CPU model, logical CPUs, threads this process may use, the oracle's
    compiler and flags."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    from oracle import build as oracle_build
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_threads": usable,
            "oracle_build": "gcc " + " ".join(oracle_build.CFLAGS)}


def cpu_baseline(fr, fb_rows: int = 0, single_rows: int = 3, other_configs: bool = True):
    """The oracle, as it stands: on all host threads the box gives this
    process (max 16) over the first `fb_rows` filter-block rows of one frame
    (0: all; direction search of those rows + the search of their filter
    blocks), single-threaded over its first `single_rows` rows, and on all
    threads over the 1920x1080 10-bit search and the 352x288 8-bit filter.
    One whole 4K frame is about 35 s of CPU time."""
    from oracle import oracle
    from paper_1602_05975_amd import synth
    facts = _host_facts()
    cores = max(1, min(16, facts["usable_threads"]))

    def search_rows(f, rows_fb, threads):
        rows = min(f.height, 64 * rows_fb)
        t0 = time.perf_counter()
        d, v = oracle.find_dir(np.ascontiguousarray(f.recon[0][:rows]), f.bitdepth)
        dfull = np.zeros((f.blk_rows, f.blk_cols), np.uint8)
        vfull = np.zeros((f.blk_rows, f.blk_cols), np.int32)
        dfull[:d.shape[0]] = d
        vfull[:v.shape[0]] = v
        fbs = [(by, bx) for by in range(rows_fb) for bx in range(f.fb_cols)]
        oracle.search_fbs(f.recon, f.src, f.width, f.height, f.bitdepth, dfull, vfull,
                          f.skip, f.damping, fbs, threads=threads)
        return rows * f.width, time.perf_counter() - t0, len(fbs)

    fb_rows = fb_rows or fr.fb_rows
    px, t_all, nfb = search_rows(fr, fb_rows, cores)
    px1, t_one, nfb1 = search_rows(fr, single_rows, 1)
    out = {
        "value": px / t_all / 1e6,
        "unit": "Mpixel/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{nfb} filter blocks ({fb_rows} rows of 64) of one 3840x2160 10-bit "
                  f"4:2:0 frame, 30% skip: direction search + all-pair search, "
                  f"{t_all:.1f} s wall on {cores} threads",
        "single_thread": {"value": px1 / t_one / 1e6, "unit": "Mpixel/s", "cores": 1,
                          "sample": f"{nfb1} filter blocks ({single_rows} rows of 64) of the "
                                    f"same frame, {t_one:.1f} s"},
        **facts,
    }
    if other_configs:
        hd = synth.hd1080_frame()
        t0 = time.perf_counter()
        oracle.search(hd.recon, hd.src, hd.width, hd.height, hd.bitdepth, None, hd.damping,
                      threads=cores)
        t_hd = time.perf_counter() - t0
        out["search_1920x1080_10bit"] = {
            "value": hd.width * hd.height / t_hd / 1e6, "unit": "Mpixel/s", "cores": cores,
            "sample": f"the whole frame (510 filter blocks, no skip, damping 3), {t_hd:.2f} s"}
        cif = synth.cif_luma()
        st = np.zeros((cif.fb_rows, cif.fb_cols, 4), np.uint8)
        st[..., 0], st[..., 1] = 4, 2
        t0 = time.perf_counter()
        reps = 5
        for _ in range(reps):
            d, v = oracle.find_dir(cif.recon[0], 8)
            oracle.filter_frame(cif.recon, cif.width, cif.height, 8, d, v, None, cif.damping, st)
        t_cif = (time.perf_counter() - t0) / reps
        out["filter_352x288_8bit"] = {
            "value": cif.width * cif.height / t_cif / 1e6, "unit": "Mpixel/s", "cores": 1,
            "sample": f"direction search + filter at (4, 2), damping 5, {t_cif * 1e3:.1f} ms "
                      "per frame (single-threaded)"}
    return out


def record_traffic(name, kernel, fetch_dir, write_dir, copy_fetch_dir, copy_write_dir,
                   copy_mib=512):
    """profiles/<name>_4k_traffic.json from four rocprofv3 --pmc runs (csv
    output): FETCH_SIZE and WRITE_SIZE of one launch of `kernel` (KiB per
    dispatch, averaged over its dispatches), each scaled by what the same
    counter reads for a device copy of copy_mib MiB (bench.py
    --copy-calibration), together with the hash of the kernel sources."""
    import csv
    import glob

    def per_dispatch(d, counter, match, largest=False):
        vals = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                for row in csv.DictReader(fh):
                    if row["Counter_Name"] == counter and match in row["Kernel_Name"]:
                        vals.append(float(row["Counter_Value"]))
        assert vals, (d, counter, match)
        return max(vals) if largest else float(np.mean(vals))

    fetch = per_dispatch(fetch_dir, "FETCH_SIZE", kernel)
    write = per_dispatch(write_dir, "WRITE_SIZE", kernel)
    cfetch = per_dispatch(copy_fetch_dir, "FETCH_SIZE", "copyBuffer", largest=True)
    cwrite = per_dispatch(copy_write_dir, "WRITE_SIZE", "copyBuffer", largest=True)
    nbytes = copy_mib << 20
    fscale, wscale = nbytes / (cfetch * 1024), nbytes / (cwrite * 1024)
    rec = {"kernel_hash": kernel_hash(), "kernel": kernel, "fetch_kib_raw": fetch,
           "write_kib_raw": write, "copy_fetch_kib_raw": cfetch, "copy_write_kib_raw": cwrite,
           "fetch_scale": fscale, "write_scale": wscale,
           "hbm_bytes_per_launch": int(round(fetch * 1024 * fscale + write * 1024 * wscale)),
           "hbm_read_bytes_per_launch": int(round(fetch * 1024 * fscale)),
           "hbm_write_bytes_per_launch": int(round(write * 1024 * wscale))}
    path = os.path.join(ROOT, "profiles", f"{name}_4k_traffic.json")
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    return rec


def load_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 counter runs, valid
    only while the kernel sources are unchanged since they were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_4k_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def _device_search_jobs(frames, dev):
    import torch
    from paper_1602_05975_amd import cdef
    jobs = []
    for fr in frames:
        rec = cdef.Frame.from_numpy(fr.recon, fr.width, fr.height, fr.bitdepth, fr.layout, dev)
        src = cdef.Frame.from_numpy(fr.src, fr.width, fr.height, fr.bitdepth, fr.layout, dev)
        skip = torch.from_numpy(fr.skip).to(dev)
        sse = torch.empty((fr.nplanes, fr.fb_rows, fr.fb_cols, 16, 4), dtype=torch.int64,
                          device=dev)
        d = torch.empty((fr.blk_rows, fr.blk_cols), dtype=torch.uint8, device=dev)
        v = torch.empty((fr.blk_rows, fr.blk_cols), dtype=torch.int32, device=dev)
        jobs.append((rec, src, skip, fr.damping, sse, d, v))
    return jobs


def _time_steps(fn, steps, warmup, stream):
    """Wall time per step (ms) of `fn`, bracketed by device synchronization."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def measure_batching(nframes: int = 64, steps: int = 10):
    """The uneven batch (resolutions 426x240 .. 3840x2160, 8/10 bit,
    damping 3..6, 64-pair search): per-frame launches vs one batched launch,
    tuned, eager and replayed from a captured HIP graph.  Results of all
    paths are compared bit for bit before timing."""
    import torch
    from paper_1602_05975_amd import cdef, synth, tune
    log(f"generating the {nframes}-frame mixed batch")
    frames = synth.mixed_frames(nframes)
    dev = torch.device("cuda:0")
    jobs = _device_search_jobs(frames, dev)
    stream = torch.cuda.current_stream()
    px = sum(f.width * f.height for f in frames)

    def plain():
        for (rec, src, skip, D, sse, d, v) in jobs:
            cdef.cdef_search_strengths(rec, src, skip, D, sse, d, v, stream)

    plain()
    torch.cuda.synchronize()
    ref = [j[4].clone() for j in jobs]

    batch = cdef.Batch()
    for (rec, src, skip, D, sse, d, v) in jobs:
        batch.add_search(rec, src, skip, D, sse, d, v)
    batch.prepare(stream)
    torch.cuda.synchronize()
    per_variant = tune.time_variants(batch, stream, reps=5)
    best = min(per_variant, key=per_variant.get)
    batch.plan.variant = best
    for j in jobs:
        j[4].zero_()
    batch.launch(stream)
    torch.cuda.synchronize()
    exact = all(torch.equal(j[4], r) for j, r in zip(jobs, ref))

    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        batch.launch(side)
    side.synchronize()
    with torch.cuda.graph(graph, stream=side):
        batch.launch(side)
    for j in jobs:
        j[4].zero_()
    graph.replay()
    torch.cuda.synchronize()
    exact = exact and all(torch.equal(j[4], r) for j, r in zip(jobs, ref))

    log(f"timing {steps} steps of each batching path")
    t_plain = _time_steps(plain, steps, 2, stream)
    t_batch = _time_steps(lambda: batch.launch(stream), steps, 2, stream)
    t_graph = _time_steps(graph.replay, steps, 2, stream)
    return {
        "workload": f"{nframes} frames, resolutions uniform over 426x240..3840x2160, 8/10-bit, "
                    "damping 3..6, 4:2:0, full 64-pair search",
        "luma_px_per_step": px,
        "filter_blocks": batch.nitems,
        "bit_exact_vs_per_frame": bool(exact),
        "per_frame_launches": {"ms_per_step": round(t_plain, 4),
                               "mpixel_s": round(px / t_plain / 1e3, 1)},
        "batched_launch": {"ms_per_step": round(t_batch, 4),
                           "mpixel_s": round(px / t_batch / 1e3, 1)},
        "graph_replay": {"ms_per_step": round(t_graph, 4),
                         "mpixel_s": round(px / t_graph / 1e3, 1)},
        "speedup_graph_vs_per_frame": round(t_plain / t_graph, 3),
        "tuned_variant": best,
        "variant_ms": {tune.VARIANT_NAMES[k]: round(v, 4) for k, v in per_variant.items()},
    }


def run_batching(args):
    print(json.dumps(measure_batching(64, max(3, args.steps // 3))), flush=True)


def run_filter(args):
    """The decoder path on the eight 4K frames with random per-filter-block
    strengths: per frame cdef_find_dir + cdef_filter_frame (two launches),
    and the same work as one batched launch of filter jobs (direction search
    fused in).  Outputs of both are compared before timing."""
    import torch
    from paper_1602_05975_amd import cdef, synth
    log(f"generating {args.frames} synthetic 3840x2160 10-bit 4:2:0 frames")
    frames = synth.uhd4k_frames(args.frames)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    jobs = []
    for i, fr in enumerate(frames):
        rec = cdef.Frame.from_numpy(fr.recon, fr.width, fr.height, fr.bitdepth, fr.layout, dev)
        skip = torch.from_numpy(fr.skip).to(dev)
        st = torch.from_numpy(synth.random_strengths(fr, 600 + i)).to(dev)
        d = torch.empty((fr.blk_rows, fr.blk_cols), dtype=torch.uint8, device=dev)
        v = torch.empty((fr.blk_rows, fr.blk_cols), dtype=torch.int32, device=dev)
        plain = [torch.empty_like(p) for p in rec.planes[:fr.nplanes]]
        fused = [torch.empty_like(p) for p in rec.planes[:fr.nplanes]]
        jobs.append((fr, rec, skip, st, d, v, plain, fused))

    def step_plain():
        for fr, rec, skip, st, d, v, plain, _ in jobs:
            cdef.cdef_find_dir(rec, d, v, stream)
            cdef.cdef_filter_frame(rec, plain, d, v, skip, fr.damping, st, stream)

    batch = cdef.Batch()
    for fr, rec, skip, st, d, v, _, fused in jobs:
        batch.add_filter(rec, fused, skip, fr.damping, st)
    batch.prepare(stream)
    step_plain()
    batch.launch(stream)
    torch.cuda.synchronize()
    exact = all(torch.equal(a, b) for j in jobs for a, b in zip(j[6], j[7]))
    log(f"timing {args.steps} steps of each path")
    ms_plain = _time_steps(step_plain, args.steps, args.warmup, stream)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    for _ in range(args.warmup):
        batch.launch(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        batch.launch(stream)
        b.record(stream)
    torch.cuda.synchronize()
    ms_batch = (time.perf_counter() - t0) * 1e3 / args.steps
    launch_s = float(np.mean([a.elapsed_time(b) for a, b in ev])) / 1e3
    px = sum(f.width * f.height for f in frames)
    samples = sum(sum(int(np.prod(f.plane_dims(p))) for p in range(f.nplanes)) for f in frames)
    ops = sum(filter_work(fr, st.cpu().numpy(), v.cpu().numpy())[0]
              for fr, _, _, st, _, v, _, _ in jobs)
    bytes_ = 2 * 2 * samples + sum(f.blk_rows * f.blk_cols for f in frames)
    achieved = ops / launch_s / 1e12
    print(json.dumps({
        "metric": "Mpixel/s for dir+filter at one preset per filter block (decoder path), "
                  "4K 10-bit",
        "value": round(px / ms_batch / 1e3, 1), "unit": "Mpixel/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_batch, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int16",
        "data": "synthetic",
        "config": {"workload": f"{len(frames)}x3840x2160 10-bit 4:2:0 frames, 30% of 8x8 blocks "
                               "skipped, random per-filter-block strengths: direction search + "
                               "filter, one batched launch of filter jobs per step",
                   "frames_per_step": len(frames), "luma_px_per_step": px},
        "plain_path": {"launches_per_step": 2 * len(frames), "ms_per_step": round(ms_plain, 4),
                       "mpixel_s": round(px / ms_plain / 1e3, 1)},
        "bit_exact_plain_vs_batched": bool(exact),
        "roofline": {"bound": "alu", "achieved": round(achieved, 3),
                     "peak": round(PEAK_PACKED_I16_TOPS, 1), "unit": "TOP/s",
                     "frac": round(achieved / PEAK_PACKED_I16_TOPS, 4),
                     "traffic": load_traffic("k_filter_batch"),
                     "kernel": "k_filter_batch", "algorithmic_ops_per_launch": int(ops),
                     "hbm_gbs_algorithmic": round(bytes_ / launch_s / 1e9, 1),
                     "hbm_peak_gbs": PEAK_HBM_GBS},
    }), flush=True)


def run_presets(args):
    """Preset selection (Eq. 15) on the strength-search tables of the eight
    4K frames, 64 and 128 candidates, without and with two refinement
    passes: device time per frame from HIP events, and the oracle's time on
    one table."""
    import torch
    from paper_1602_05975_amd import cdef, synth
    from oracle import oracle
    log(f"generating {args.frames} synthetic 3840x2160 10-bit 4:2:0 frames")
    frames = synth.uhd4k_frames(args.frames)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    tables = {64: [], 128: []}
    for fr in frames:
        rec = cdef.Frame.from_numpy(fr.recon, fr.width, fr.height, fr.bitdepth, fr.layout, dev)
        src = cdef.Frame.from_numpy(fr.src, fr.width, fr.height, fr.bitdepth, fr.layout, dev)
        skip = torch.from_numpy(fr.skip).to(dev)
        for nc in (64, 128):
            tables[nc].append(cdef.search_strengths(rec, src, skip, fr.damping, full=nc == 128))
    torch.cuda.synchronize()
    lam = 2.0e4
    res = torch.zeros(360, dtype=torch.uint8, device=dev)
    ws = cdef.preset_workspace(dev)
    fbr, fbc = frames[0].fb_rows, frames[0].fb_cols
    fl = torch.empty((fbr, fbc), dtype=torch.uint8, device=dev)
    fc = torch.empty_like(fl)
    out = {"workload": f"{args.frames} tables of 3840x2160 10-bit 4:2:0 frames "
                       f"({fbr}x{fbc} filter blocks, 3 planes), lambda {lam}",
           "cases": []}
    for nc in (64, 128):
        for refine in (0, 2):
            def one(t):
                cdef.cdef_select_presets(t, lam, refine, res, fl, fc, ws, stream)
            for t in tables[nc][:2]:
                one(t)
            torch.cuda.synchronize()
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(args.steps)]
            for k in range(args.steps):
                t = tables[nc][k % len(tables[nc])]
                ev[k][0].record(stream)
                one(t)
                ev[k][1].record(stream)
            torch.cuda.synchronize()
            us = np.array([a.elapsed_time(b) * 1e3 for a, b in ev])
            table = tables[nc][0].cpu().numpy().view(np.uint64)
            t0 = time.perf_counter()
            ref = oracle.select_presets(table, lam, refine)
            t_cpu = time.perf_counter() - t0
            cdef.cdef_select_presets(tables[nc][0], lam, refine, res, fl, fc, ws, stream)
            torch.cuda.synchronize()
            r = cdef.CdefPresetResult.from_buffer_copy(res.cpu().numpy().tobytes())
            exact = (r.n == ref["n"] and np.array_equal(np.array(r.luma), ref["luma"])
                     and np.array_equal(np.array(r.chroma), ref["chroma"])
                     and np.array_equal(fl.cpu().numpy(), ref["fb_luma"])
                     and np.array_equal(fc.cpu().numpy(), ref["fb_chroma"]))
            table_bytes = table.nbytes
            out["cases"].append({
                "candidates": nc, "refine_passes": refine, "chosen_n": int(r.n),
                "us_per_frame_p50": round(float(np.percentile(us, 50)), 1),
                "us_per_frame_mean": round(float(us.mean()), 1),
                "table_bytes": int(table_bytes),
                "table_read_gbs": round(table_bytes / (us.mean() * 1e-6) / 1e9, 1),
                "oracle_ms_1_thread": round(t_cpu * 1e3, 1),
                "bit_exact_vs_oracle": bool(exact)})
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=int(os.environ.get("WORLD_SIZE", "1")))
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--frames", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-frames", type=int, default=64,
                    help="frames of the uneven batch measured in the headline line (0: skip)")
    ap.add_argument("--serve-host-frames", type=int, default=300,
                    help="frames of the host-memory serving trace in the headline line "
                         "(each a search and a filter request; 0: skip)")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="timed requests of the serving trace whose p50/p99 the headline "
                         "line reports (0: skip; report the batch launch time instead)")
    ap.add_argument("--variant", type=int, default=0,
                    help="launch variant of the batched launch (cdef_batch_plan.variant: "
                         "0 / 1: at most 3 / 2 waves per SIMD, XCD-contiguous filter-block "
                         "order; 2 / 3: the same in plain order)")
    ap.add_argument("--per-frame", action="store_true",
                    help="one cdef_search_strengths launch per frame instead of one batch")
    ap.add_argument("--workload", choices=["search4k", "search128", "weighted", "search12",
                                           "search444", "search422", "subset", "filter",
                                           "presets", "batch", "serve"],
                    default="search4k",
                    help="search4k: the headline line (default); search128: the same frames "
                         "under the 128-combination search; weighted: the same frames with the "
                         "Eq. (14) distortion; search12 / search444 / search422: 12-bit 4:2:0, "
                         "10-bit 4:4:4, 10-bit 4:2:2 frames of the same size; subset: the "
                         "headline frames under a preset subset (--subset); filter: the "
                         "decoder path (direction search + filter at one preset per filter "
                         "block); presets: Eq. (15) "
                         "preset "
                         "selection on their tables; batch: 64 mixed frames, "
                         "per-frame launches vs one tuned, graph-replayed batch; serve: "
                         "Poisson request stream, continuous batching vs one request per "
                         "launch")
    ap.add_argument("--subset", type=lambda x: int(x, 0), default=DEFAULT_SUBSET,
                    help="preset subset word of the subset workload: S^(p) mask | S^(s) index "
                         "mask << 16 | skip condition bit mask << 20")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB five times "
                         "(reference kernel for scaling HBM counters)")
    ap.add_argument("--record-traffic", nargs=6, metavar=("NAME", "KERNEL", "FETCH_DIR",
                                                        "WRITE_DIR", "COPY_FETCH_DIR",
                                                        "COPY_WRITE_DIR"),
                    help="only write profiles/NAME_4k_traffic.json from rocprofv3 --pmc "
                         "FETCH_SIZE / WRITE_SIZE runs of the workload and of "
                         "--copy-calibration 512 (no GPU needed)")
    args = ap.parse_args()
    if args.record_traffic:
        print(json.dumps(record_traffic(*args.record_traffic)))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(frames are independent: a batch shards across GPUs by frame with no exchange)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1602_05975_amd import cdef, synth
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        n = args.copy_calibration << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "reads": n, "writes": n}))
        return
    cdef.load()
    if args.workload == "batch":
        return run_batching(args)
    if args.workload == "serve":
        from paper_1602_05975_amd import serve
        return serve.bench_main(args)
    if args.workload == "presets":
        return run_presets(args)
    if args.workload == "filter":
        return run_filter(args)
    full = args.workload == "search128"
    weighted = args.workload == "weighted"
    cand = args.subset if args.workload == "subset" else 0
    if cand and (cand >> 21) & 1:
        full = True
    bd, layout = FORMATS[args.workload]
    lname = {0: "4:0:0", 1: "4:2:0", 2: "4:2:2", 3: "4:4:4"}[layout]

    log(f"generating {args.frames} synthetic 3840x2160 {bd}-bit {lname} frames")
    if (bd, layout) == (10, 1):
        frames = synth.uhd4k_frames(args.frames)
    else:
        frames = [synth.make_frame(3840, 2160, bd, layout, synth.workload_seed(synth.WL_4K, f),
                                   skip_prob=0.3, damping=3) for f in range(args.frames)]
    ops = sum(frame_work(f, full, weighted, cand)[0] for f in frames)
    algo_bytes = sum(frame_work(f, full, weighted, cand)[1] for f in frames)

    dev = torch.device("cuda:0")
    jobs = []
    for fr in frames:
        rec = cdef.Frame.from_numpy(fr.recon, fr.width, fr.height, fr.bitdepth, fr.layout, dev)
        src = cdef.Frame.from_numpy(fr.src, fr.width, fr.height, fr.bitdepth, fr.layout, dev)
        skip = torch.from_numpy(fr.skip).to(dev)
        shape = (fr.search_planes, fr.fb_rows, fr.fb_cols) + ((2, 16, 4) if full else (16, 4))
        sse = torch.empty(shape, dtype=torch.float64 if weighted else torch.int64, device=dev)
        d = torch.empty((fr.blk_rows, fr.blk_cols), dtype=torch.uint8, device=dev)
        v = torch.empty((fr.blk_rows, fr.blk_cols), dtype=torch.int32, device=dev)
        jobs.append((rec, src, skip, fr.damping, sse, d, v))
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    search_one = (cdef.cdef_search_weighted if weighted else
                  cdef.cdef_search_strengths128 if full else cdef.cdef_search_strengths)
    if cand:
        def search_one(rec, src, skip, D, sse, d, v, stream):
            cdef.cdef_search_subset(rec, src, skip, D, cand, sse, d, v, stream)
    batch = None
    if not args.per_frame:
        batch = cdef.Batch()
        for (rec, src, skip, D, sse, d, v) in jobs:
            batch.add_search(rec, src, skip, D, sse, d, v, full=full, weighted=weighted,
                             candidates=cand)
        batch.prepare(stream)
        batch.plan.variant = args.variant
        torch.cuda.synchronize()

    # launches of one step, each bracketed by HIP events on the launch stream
    def step(events=None):
        if batch is not None:
            if events is not None:
                events[0][0].record(stream)
            batch.launch(stream)
            if events is not None:
                events[0][1].record(stream)
            return
        for k, (rec, src, skip, D, sse, d, v) in enumerate(jobs):
            if events is not None:
                events[k][0].record(stream)
            search_one(rec, src, skip, D, sse, d, v, stream)
            if events is not None:
                events[k][1].record(stream)

    launches_per_step = 1 if batch is not None else len(jobs)
    log(f"warmup {args.warmup} steps")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    log(f"timing {args.steps} steps ({launches_per_step} launch(es) per step)")
    ev = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)]
           for _ in range(launches_per_step)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s_ in range(args.steps):
        step(ev[s_])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = np.array([[e[0].elapsed_time(e[1]) for e in st] for st in ev])

    px_per_step = sum(f.width * f.height for f in frames)
    ms_per_step = wall * 1e3 / args.steps
    value = px_per_step * args.steps / wall / 1e6
    avg_launch_s = float(launch_ms.mean()) / 1e3
    ops_per_launch = ops / launches_per_step
    bytes_per_launch = algo_bytes / launches_per_step
    achieved = ops_per_launch / avg_launch_s / 1e12
    frame_ms = launch_ms if batch is None else launch_ms  # a batch's frames finish together
    kname = "k_fused_batch" if batch is not None else "k_fused_one"
    suffix = {"search4k": "", "search128": "_full", "weighted": "_weighted"}.get(args.workload,
                                                                           "_" + args.workload)
    traffic = load_traffic(kname + suffix)
    npri, nsec, npairs, nskb = subset_counts(cand)
    what = ("all 128 (primary, secondary, skip condition) presets" if full and not cand else
            "all 64 (primary, secondary) strength pairs" if not cand else
            f"a subset of {npairs * nskb} presets (word {cand:#x})")
    if weighted:
        what += " with the Eq. (14) contrast-weighted distortion (float64 table)"
    fmt = f"{bd}-bit {lname}"
    result = {
        "metric": ("Mpixel/s for dir+filter+128-combination SSE search, 4K 10-bit" if full and not cand
                   else "Mpixel/s for dir+filter+all-strength Eq. (14) weighted search, 4K 10-bit"
                   if weighted else
                   f"Mpixel/s for dir+filter+subset SSE search, 4K 10-bit" if cand else
                   "Mpixel/s for dir+filter+all-strength SSE search, 4K 10-bit; p99 frame latency"
                   if (bd, layout) == (10, 1) else
                   f"Mpixel/s for dir+filter+all-strength SSE search, 4K {fmt}"),
        "value": round(value, 1),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int16",
        "data": "synthetic",
        "config": {
            "workload": f"{len(frames)}x3840x2160 {fmt} frames, 30% of 8x8 blocks "
                        f"skipped, damping 3: fused direction search + filter under {what} "
                        "+ per-64x64 SSE, "
                        + ("one launch per frame" if batch is None else
                           "one batched launch per step"),
            "frames_per_step": len(frames),
            "luma_px_per_step": px_per_step,
        },
        "roofline": {
            "bound": "alu",
            "achieved": round(achieved, 3),
            "peak": round(PEAK_PACKED_I16_TOPS, 1),
            "unit": "TOP/s",
            "frac": round(achieved / PEAK_PACKED_I16_TOPS, 4),
            "traffic": traffic,
            "kernel": kname,
            "algorithmic_ops_per_launch": int(ops_per_launch),
            "hbm_gbs_algorithmic": round(bytes_per_launch / avg_launch_s / 1e9, 1),
            "hbm_peak_gbs": PEAK_HBM_GBS,
        },
    }
    result["batch_launch_ms"] = {
        "p50": round(float(np.percentile(launch_ms, 50)), 4),
        "p99": round(float(np.percentile(launch_ms, 99)), 4),
        "note": "per-frame launch time" if batch is None else
                "launch time of the whole step (all frames of a step complete together)"}
    headline = args.workload == "search4k" and not args.per_frame
    if headline and args.serve_requests > 0:
        from paper_1602_05975_amd import serve
        tr = serve.latency_summary(n_req=args.serve_requests, warm=max(20, args.serve_requests // 10))
        result["frame_latency_ms"] = {
            "p50": tr["batched"]["p50_ms"], "p99": tr["batched"]["p99_ms"],
            "plain_p50": tr["plain"]["p50_ms"], "plain_p99": tr["plain"]["p99_ms"],
            "p99_gain_vs_plain": tr["p99_gain"], "p50_gain_vs_plain": tr["p50_gain"],
            "note": "serving trace: arrival to completion of each request, continuous batching "
                    "vs one request per launch on the same Poisson arrivals at "
                    f"{tr['rate_fraction_of_plain']} x the plain path's capacity"}
        result["serving"] = tr
    else:
        result["frame_latency_ms"] = dict(result["batch_launch_ms"])
    if headline and args.serve_host_frames > 0:
        from paper_1602_05975_amd import serve
        result["serving_host"] = serve.host_latency_summary(
            n_frames=args.serve_host_frames, warm=max(10, args.serve_host_frames // 10))
    if headline and args.batch_frames > 0:
        result["batching"] = measure_batching(args.batch_frames, 10)
    if not args.no_cpu_baseline and args.workload == "search4k":
        log("timing the CPU oracle on a bounded sample")
        result["cpu_baseline"] = cpu_baseline(frames[0])
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
