"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds the oracle's C source with -fsanitize=address,undefined (halting on
the first undefined-behaviour report) into a temporary directory and runs the
oracle's CPU test files against that build in a child process (the ASan
runtime has to be preloaded into the Python interpreter there).  Any
sanitizer report, or any failing test, fails this test.
"""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_TESTS = ["test_oracle_pins.py", "test_presets_cpu.py", "test_full_search_cpu.py",
                "test_weighted_cpu.py", "test_layouts_cpu.py", "test_subset_cpu.py"]
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-fno-omit-frame-pointer", "-g"]


def _runtime(name):
    if shutil.which("gcc") is None:
        return None
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True,
                          text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_tests_pass_under_asan_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    from oracle import build
    lib = build.build(SAN_FLAGS, out=str(tmp_path / "libcdef_oracle_san.so"))
    logs = tmp_path / "san"
    env = dict(os.environ)
    env.update({
        "CDEF_ORACLE_LIB": lib,
        "LD_PRELOAD": asan,
        "ASAN_OPTIONS": f"detect_leaks=0:log_path={logs}",
        "UBSAN_OPTIONS": f"halt_on_error=1:print_stacktrace=1:log_path={logs}",
    })
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
           *[os.path.join(ROOT, "tests", t) for t in ORACLE_TESTS]]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    reports = sorted(glob.glob(str(logs) + "*"))
    text = "".join(open(p).read() for p in reports)
    assert not reports, "sanitizer reports:\n" + text[:4000]
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-2000:]
    assert " passed" in r.stdout
