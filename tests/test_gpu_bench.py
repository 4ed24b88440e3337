"""The bench's main leg exactly as the full test run calls it (side legs off)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.gpu
def test_bench_main_leg_prints_roofline_and_cpu_baseline():
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "20", "--warmup", "5",
           "--no-batched", "--no-learned", "--no-eos", "--no-table3", "--no-spheres",
           "--cpu-sweeps", "2", "--kernel-samples", "16"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["steps"] == 20 and line["n_gpus"] == 1 and line["value"] > 0
    assert "N=1048576" in line["config"]["workload"] and "phi=0.700" in line["config"]["workload"]
    assert line["config"]["timed_graph_launches"] == 2
    roof = line["roofline"]
    assert roof["bound"] == "hbm" and 0 < roof["frac"] < 1 and roof["peak"] == 8000.0
    # the counter figures of the committed profile (its source hash matches)
    assert roof["kernel"].startswith("k_sweep_fused<") and roof["traffic"] > 0
    assert roof["valu_busy"] > 0 and 0 < roof["alu"]["frac"] < 1
    cb = line["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1
    assert cb["one_thread"]["value"] > 0 and cb["host_cpu"]


@pytest.mark.gpu
def test_bench_separate_launches_report_the_subsweep():
    """--separate: the same chain as four sub-sweep launches and a rebuild
    per sweep; the line's roofline is then the sub-sweep kernel's, with its
    own profile's counters."""
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--separate", "--steps", "20",
           "--warmup", "5", "--block", "192", "--lanes", "1", "--no-batched", "--no-learned",
           "--no-eos", "--no-table3", "--no-spheres", "--no-cpu-baseline", "--kernel-samples", "16"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["value"] > 0 and line["config"]["sweep_kernel"].startswith("four sub-sweep")
    roof = line["roofline"]
    assert roof["kernel"].startswith("k_subsweep<") and roof["traffic"] > 0
    assert 0 < roof["frac"] < 1
