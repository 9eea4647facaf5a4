"""The benchmark's output contract on the GPU: one JSON line with the fields the results are
read from, consistent with one another (a short run of the default workload)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_line_contract():
    r = subprocess.run([sys.executable, "bench.py", "--steps", "20", "--warmup", "2", "--no-extra",
                        "--no-round-trip", "--variants", "none", "--cpu-steps", "2"],
                       cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1, r.stdout[-2000:]
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "cpu_baseline", "kernel_source_sha256", "library_build_id"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 20 and d["warmup"] == 2
    assert d["unit"] == "MLUPS" and d["higher_is_better"] is True and d["data"] == "synthetic"
    assert d["config"]["nodes"] == 19195714 and d["config"]["instances"] == 256
    # MLUPS from the step time
    assert abs(d["value"] / (d["config"]["nodes"] / (d["ms_per_step"] * 1e3)) - 1) < 1e-3
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert rf["alg_bytes_per_lu"] == 168
    # achieved = algorithmic bytes of one launch / its time; frac = achieved / peak
    assert abs(rf["achieved"] / (rf["alg_bytes_per_launch"] / (d["ms_per_step"] * 1e-3) / 1e9) - 1) < 1e-3
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3
    assert 0 < rf["frac"] < 1 and 0 < rf["frac_of_copy"] < 1.5
    # the device's streaming rate, measured in the same run
    assert rf["copy_gbs"] > 0 and abs(rf["frac_of_copy"] - rf["achieved"] / rf["copy_gbs"]) < 1e-3
    # the launch configuration the autotuner chose, XCD dealing included
    deal = d["config"]["deal"]
    assert deal == "bands" or 1 <= deal <= 4096
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["value_1_thread"] > 0
    assert cb["cores"] >= 1 and cb["cores_1_thread"] == 1


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "8"], cwd=ROOT, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0 and r.stdout == "" and "one GPU" in r.stderr
