"""Compile the gfx950 HIP library (libcdef_hip.so) in-tree with hipcc."""
from __future__ import annotations

import json
import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libcdef_hip.so")
BUILD = os.path.join(HERE, "_build")
# per-kernel registers, spills, LDS and occupancy from the compiler's
# resource-usage remarks, written by build()
RESOURCES = os.path.join(BUILD, "kernel_resources.json")
# (source, object, extra flags): k_fused.hip is built once per kernel set so
# that its sets compile in parallel; a set leaves the shared helpers that
# only other sets use unreferenced, which is expected there
KSETS = 9
KSET_FLAGS = ["-Wno-unused-function", "-Wno-unneeded-internal-declaration"]
# Sets 7 and 8 hold the persistent batch kernels, whose item loop wraps the
# whole per-item body: machine-level loop-invariant code motion would hoist
# constants out of it and keep them in registers across every item (62
# spilled VGPRs at 3 waves/SIMD with it, 15 without).
LOOP_FLAGS = ["-mllvm", "-disable-machine-licm"]
SOURCES = [("k_fused.hip", f"k_fused_{k}.o",
            [f"-DCDEF_KSET={k}", *KSET_FLAGS, *(LOOP_FLAGS if k in (7, 8) else [])])
           for k in range(KSETS)] + [
    (src, src.replace(".hip", ".o"), []) for src in ("cdef_api.hip", "k_plain.hip", "k_presets.hip")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(HERE, "..", "include"),
]


def _compile(unit, extra):
    src, obj, defs = unit
    obj = os.path.join(BUILD, obj)
    cmd = [HIPCC, *FLAGS, "-Rpass-analysis=kernel-resource-usage", *defs, *extra, "-c",
           os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj, _resources(r.stderr)


def _resources(remarks: str) -> dict:
    """{kernel: {field: value}} from -Rpass-analysis=kernel-resource-usage."""
    out, cur = {}, None
    for line in remarks.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            cur = out.setdefault(m.group(1), {})
            continue
        m = re.search(r"remark:\s+([A-Za-z][^:\[]*?)(?: \[[^\]]*\])?: (\w+) \[", line)
        if cur is not None and m:
            v = m.group(2)
            cur[m.group(1).strip()] = int(v) if v.isdigit() else v
    return out


def build(extra=(), out=OUT, verbose=False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(min(len(SOURCES), os.cpu_count() or 1)) as ex:
        done = list(ex.map(lambda s: _compile(s, list(extra)), SOURCES))
    objs = [o for o, _ in done]
    res = {}
    for _, r in done:
        res.update(r)
    with open(RESOURCES, "w") as f:
        json.dump(res, f, indent=1, sort_keys=True)
    tmp = out + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    if verbose:
        print(out)
    return out


if __name__ == "__main__":
    build(extra=sys.argv[1:], verbose=True)
