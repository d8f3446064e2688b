"""The benchmark's output on one GPU, on the small lattice: exactly one JSON
line on stdout with the throughput, the roofline of the timed kernel and the
CPU oracle baseline, and a roofline fraction that follows from its own
figures."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_prints_one_json_line_with_its_fields():
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--config", "small", "--steps", "6",
           "--warmup", "2", "--cpu-steps", "2", "--cpu-steps-1t", "1", "--companions", "0",
           "--adjoint-steps", "0"]
    print("running", " ".join(cmd[1:]), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-3000:]
    lines = [line for line in r.stdout.splitlines() if line.strip()]
    assert len(lines) == 1, r.stdout[-3000:]
    out = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
                "roofline", "cpu_baseline", "droplets", "row_averages"):
        assert key in out, key
    assert out["n_gpus"] == 1 and out["steps"] == 6 and out["warmup"] == 2
    assert out["unit"] == "MLUPS" and out["value"] > 0 and out["higher_is_better"] is True
    assert out["dtype"] == "f32" and out["data"] == "synthetic"
    assert out["config"]["workload"] == "small-128x64"
    roof = out["roofline"]
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    assert roof["achieved"] > 0
    # both are rounded in the line: frac to 1e-4, achieved to 0.1 GB/s
    assert roof["frac"] == pytest.approx(roof["achieved"] / roof["peak"], rel=2e-3, abs=1e-4)
    # achieved = algorithmic bytes per launch / launch time
    per_launch = roof["bytes_per_lattice_update"] * roof["nodes_per_launch"] * roof["updates_per_node"]
    assert roof["achieved"] == pytest.approx(per_launch / (roof["launch_us"] * 1e-6) / 1e9, rel=2e-3, abs=0.1)
    cpu = out["cpu_baseline"]
    assert cpu["kind"] == "oracle" and cpu["unit"] == "MLUPS" and cpu["value"] > 0 and cpu["cores"] >= 1
    assert cpu["single_thread"]["cores"] == 1
