"""bench.py's workloads run end to end on the GPU (one 4K frame, one step)
and print a well-formed JSON line; the driver and the measurements depend
on every one of them."""
import json
import sys

import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("workload", ["search4k", "search128", "weighted", "search12", "search444",
                                      "search422", "subset", "filter", "presets"])
def test_bench_workload_runs(workload, monkeypatch, capsys):
    import bench
    print(f"bench.py --workload {workload} --frames 1 --steps 1 --warmup 0", file=sys.stderr,
          flush=True)
    monkeypatch.setattr(sys, "argv", ["bench.py", "--workload", workload, "--frames", "1",
                                      "--steps", "1", "--warmup", "0", "--no-cpu-baseline",
                                      "--batch-frames", "0", "--serve-requests", "0",
                                      "--serve-host-frames", "0"])
    bench.main()
    lines = [ln for ln in capsys.readouterr().out.splitlines() if ln.startswith("{")]
    assert len(lines) == 1
    rec = json.loads(lines[0])
    if workload == "presets":
        assert len(rec["cases"]) == 4
        assert all(c["bit_exact_vs_oracle"] for c in rec["cases"])
        return
    assert rec["value"] > 0 and rec["n_gpus"] == 1 and rec["steps"] == 1
    assert rec["unit"] and rec["metric"] and isinstance(rec["config"], dict)
    r = rec["roofline"]
    assert r["peak"] > 0 and 0 < r["frac"] < 1.5 and r["achieved"] > 0


def test_bench_headline_line_carries_every_part(monkeypatch, capsys):
    # the default line: the batched search, the serving trace's latency
    # percentiles for both paths, the uneven batch, the CPU baseline (here on
    # one filter-block row); sizes cut down to keep the test short
    import bench
    full = bench.cpu_baseline
    monkeypatch.setattr(bench, "cpu_baseline",
                        lambda fr: full(fr, fb_rows=1, single_rows=1, other_configs=False))
    monkeypatch.setattr(sys, "argv", ["bench.py", "--frames", "1", "--steps", "2", "--warmup",
                                      "1", "--batch-frames", "6", "--serve-requests", "100",
                                      "--serve-host-frames", "40"])
    bench.main()
    lines = [ln for ln in capsys.readouterr().out.splitlines() if ln.startswith("{")]
    assert len(lines) == 1
    rec = json.loads(lines[0])
    lat = rec["frame_latency_ms"]
    assert 0 < lat["p50"] <= lat["p99"] and 0 < lat["plain_p50"] <= lat["plain_p99"]
    assert rec["serving"]["batched"]["requests"] == 100
    host = rec["serving_host"]
    assert host["batched"]["requests"] == 2 * 40 and host["plain"]["p99_ms"] > 0
    assert rec["batching"]["bit_exact_vs_per_frame"]
    cb = rec["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["single_thread"]["value"] > 0
    assert cb["cpu_model"] and cb["nproc"] >= 1 and "gcc" in cb["oracle_build"]
