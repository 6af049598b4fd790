"""bench.py's output contract: one JSON line with the metric, the roofline object of
the dominant kernel and the CPU baseline; more than one GPU is refused with a message."""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=60, cwd=ROOT)
    assert res.returncode == 2
    assert "one GPU" in res.stderr


@pytest.mark.gpu
def test_bench_line_fields():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "5", "--warmup", "1",
                          "--no-autotune", "--race-objects", "0", "--cpu-seconds", "1", "--cpu-seconds-single", "1",
                          "--no-extra-workloads"],
                         capture_output=True, text=True, timeout=110, cwd=ROOT)
    print(res.stderr[-2000:], flush=True)
    assert res.returncode == 0
    lines = [ln for ln in res.stdout.splitlines() if ln.strip()]
    d = json.loads(lines[-1])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 5 and d["warmup"] == 1 and d["value"] > 0
    assert "workload" in d["config"]
    r = d["roofline"]
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert 0 < r["frac"] < 1 and abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-9
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and cb["value"] > 0 and cb["unit"] == "patterns/s"
    assert 0 < d["pcie_inclusive"]["value"] <= d["value"]
