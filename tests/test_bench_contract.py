"""The benchmark's output contract: one JSON line with the metric, the step
timing, the roofline of the dominant kernel and the oracle's host baseline;
more than one GPU is refused."""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, timeout=300):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, cwd=ROOT,
                          capture_output=True, text=True, timeout=timeout)


@pytest.mark.gpu
def test_bench_line_fields():
    from gpu_helpers import device
    device()
    r = _run(["--steps", "2", "--warmup", "1"])
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip().startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
                "roofline", "cpu_baseline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1
    assert d["value"] > 0 and d["ms_per_step"] > 0
    assert "workload" in d["config"]
    roof = d["roofline"]
    assert roof["bound"] in ("hbm", "mfma", "alu")
    assert 0 < roof["frac"] <= 1 and abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-3
    assert "traffic" in roof
    cpu = d["cpu_baseline"]
    assert cpu["kind"] == "oracle" and cpu["value"] > 0 and cpu["cores"] >= 1 and cpu["sample"]
    # The GPU results the line reports were checked against the oracle.
    assert max(cpu["rel_err_gpu_vs_oracle"].values()) <= 1e-5


def test_more_than_one_gpu_is_refused():
    # Checked before anything touches a GPU (this runs in the CPU suite too).
    r = _run(["--gpus", "2"], timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr
