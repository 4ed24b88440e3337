"""Host-side checks of bench.py's warm-up plan (no GPU)."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("warmup", [-3, 0, 5, 200])
@pytest.mark.parametrize("steps", [1, 5, 16, 20, 1000])
def test_warmup_plan_never_negative(warmup, steps):
    b = _bench()
    p = b.warmup_plan(warmup, steps)
    assert p["tuner_sweeps"] == p["tuner_windows"] * p["tuner_window_sweeps"] > 0
    assert p["extra_sweeps"] == max(0, warmup)
    assert p["timed_graph_launches"] == steps // 16 + (1 if steps % 16 else 0)
    assert all(v >= 0 for v in p.values())


def test_warmup_plan_rejects_no_steps():
    with pytest.raises(ValueError):
        _bench().warmup_plan(5, 0)


def test_multi_gpu_request_is_refused():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU only" in r.stderr
