"""The benchmark's command-line contract: one JSON line with the required keys, and a
clear refusal of more than one GPU."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")
KEYS = ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
        "vs_baseline", "dtype", "data", "config", "roofline")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


@pytest.mark.gpu
def test_short_run_prints_the_json_line():
    """A short FP64 run of the headline workload: every contract key, a roofline with the
    required fields, and a positive rate consistent with ms_per_step."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = subprocess.run([sys.executable, BENCH, "--steps", "3", "--warmup", "1", "--modes", "fp64",
                        "--latency-reps", "0", "--serve", "", "--no-cpu", "--no-configs", "--no-at-T"],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    line = json.loads(r.stdout.strip().splitlines()[-1])
    for k in KEYS:
        assert k in line, k
    assert line["n_gpus"] == 1 and line["steps"] == 3 and line["dtype"] == "f64"
    roof = line["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in roof, k
    assert 0.0 < roof["frac"] < 1.0
    dof = line["config"]["dof"]
    assert abs(line["value"] - dof / (line["ms_per_step"] * 1e-3) / 1e6) <= 1e-6 * line["value"]
