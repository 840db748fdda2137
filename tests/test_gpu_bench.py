"""The benchmark runs end to end on one GPU and prints one JSON line with the agreed
fields (a small grid and one timed step, so it stays a test, not a measurement)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.gpu
def test_bench_json_line_small():
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--n", "1024", "--steps", "1", "--warmup", "1",
           "--forms", "none", "--no-cpu-baseline"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=110)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
                "vs_baseline", "dtype", "data", "config", "roofline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 1 and d["dtype"] == "f64" and d["value"] > 0
    roof = d["roofline"]
    assert roof["bound"] == "hbm" and roof["peak"] == 8000.0 and 0 < roof["frac"] < 1
    assert roof["traffic"] is None  # the counter summary covers the 8192^2 launches only
    assert "workload" in d["config"] and "mixed" in d


def test_bench_refuses_several_gpus():
    """No GPU needed: the check comes before anything touches one."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode != 0 and "one GPU" in r.stderr
