"""bench.py's one-line JSON record on the GPU: the fields, types and internal
relations its contract fixes, from a shortened run (one timed solve of the
Nside-1024 workload, a small CPU sample, no batched, reduced-precision or
warm-start parts)."""
import json
import os
import subprocess
import sys

import pytest

from gpu_util import device

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_record_fields():
    device()  # skips without a GPU
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "1", "--warmup", "0",
           "--no-batch", "--no-configs", "--no-precision", "--no-learned",
           "--cpu-fraction", "0.02", "--pairs", "20"]
    print("running", " ".join(cmd), flush=True)
    run = subprocess.run(cmd, capture_output=True, text=True, timeout=400, cwd=ROOT)
    assert run.returncode == 0, run.stderr[-3000:]
    lines = [ln for ln in run.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1, run.stdout[-2000:]
    rec = json.loads(lines[0])

    assert isinstance(rec["metric"], str) and rec["metric"]
    assert rec["unit"] == "solves/s" and rec["higher_is_better"] is True
    assert rec["n_gpus"] == 1 and rec["steps"] == 1 and rec["warmup"] == 0
    assert rec["scaling"] == "weak" and rec["data"] == "synthetic" and rec["dtype"] == "f64"
    assert rec["vs_baseline"] is None
    assert rec["value"] > 0 and rec["ms_per_step"] > 0
    # whole-job throughput of one GPU: one solve per step
    assert rec["value"] == pytest.approx(1e3 / rec["ms_per_step"], rel=1e-9)
    cfg = rec["config"]
    assert cfg["nside"] == 1024 and cfg["lmax"] == 2048 and "1024" in cfg["workload"]

    roof = rec["roofline"]
    assert roof["bound"] in ("alu", "hbm", "mfma")
    assert roof["unit"] == "TFLOP/s" and roof["peak"] == 78.6
    assert roof["frac"] == pytest.approx(roof["achieved"] / roof["peak"], rel=1e-9)
    assert 0.0 < roof["frac"] < 1.0
    assert roof["traffic"] is None or roof["traffic"] > 0
    assert roof["avg_launch_ms"] > 0 and roof["launches"] > 0

    cpu = rec["cpu_baseline"]
    assert cpu["kind"] == "oracle" and cpu["unit"] == "solves/s"
    assert cpu["value"] > 0 and cpu["cores"] >= 1 and cpu["sample"]
