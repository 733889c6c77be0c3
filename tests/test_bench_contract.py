"""bench.py's output contract: one JSON line with the fields the driver and
the design notes read, and its refusals."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args, timeout=300):
    return subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=timeout)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2", timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "single GPU" in line["error"]


@pytest.mark.gpu
def test_bench_line_of_the_small_fp64_cloth():
    """One timed step of the 32x32 FP64 cloth: exit status 0 and one JSON
    line carrying the metric, the throughput, finite gradients, the roofline
    object and the CPU baseline of the oracle."""
    from tests._cases import needs_gpu
    needs_gpu()
    r = _run("--workload", "c1", "--steps", "1", "--warmup", "1", "--plain-steps", "0")
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 1 and d["dtype"] == "f64"
    assert d["value"] > 0 and d["grads_finite"] is True
    assert d["config"]["workload"] == "cloth32_distance_fp64"
    roof = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in roof, k
    assert roof["peak"] == 8000.0 and roof["unit"] == "GB/s"
    assert abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-3
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1
