"""bench.py's output contract: one JSON line with the headline metric, the
roofline object of the dominant kernel and the single-request latency on the
(H2O)30 headline workload; more
than one GPU is refused with a message before any device work."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


@pytest.mark.gpu
def test_bench_line_carries_the_contract_fields():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "2",
                        "--warmup", "1", "--no-cpu-baseline", "--no-evgw", "--no-core",
                        "--only", "bf16x3w"], capture_output=True, text=True, timeout=400)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "latency_ms", "paths"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1
    assert d["value"] > 0 and d["ms_per_step"] > 0 and d["higher_is_better"] is True
    assert d["vs_baseline"] is None and d["data"] == "synthetic"
    assert "workload" in d["config"]
    roof = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in roof, k
    assert roof["bound"] in ("hbm", "mfma", "alu")
    assert abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-3
    assert d["latency_ms"]["p50"] > 0 and d["latency_ms"]["p99"] >= d["latency_ms"]["p50"]
    assert d["paths"]["bf16x3w"]["states_checked"] >= 1
    assert d["paths"]["bf16x3w"]["max_err_mev_vs_oracle"] <= 1.0
    assert "(H2O)30" in d["config"]["workload"] and d["config"]["grid_points"] == 128
    assert roof["algorithmic_bytes"] > 0
