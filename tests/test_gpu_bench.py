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
                                      "--steps", "1", "--warmup", "0", "--no-cpu-baseline"])
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
