"""Host-side parts of bench.py that need no GPU: the one-GPU guard, the
algorithmic flop count the roofline is priced on, and the rule that a stored
HBM traffic figure is reported only while its kernel's source is unchanged."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    run = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert run.returncode == 2
    assert "one GPU" in run.stderr
    assert run.stdout == ""


def test_legendre_flops_match_the_triple_count():
    # T(l) = 2 Nside (l+1)(l+2)/2 triples, 8 flops each per direction: a pair
    # at Nside 1024, lmax 2048 is 6.88e10 flops, at Nside 16, lmax 32 2.9e5
    assert bench.legendre_flops(1024, 2048) == 8.0 * 2048 * 2049 * 2050 / 2
    assert 2 * bench.legendre_flops(1024, 2048) == pytest.approx(6.88e10, rel=2e-3)
    assert 2 * bench.legendre_flops(16, 32) == pytest.approx(2.87e5, rel=1e-2)
    assert bench.legendre_flops(16, -1) == 0.0
    # l_iter = m's lowest band: one l per m
    assert bench.legendre_flops(8, 0) == 8.0 * 16


def _summary(tmp_path, src_text, stored_text):
    (tmp_path / "k.hip").write_text(src_text)
    (tmp_path / "profiles").mkdir()
    rec = {"kernel": "k_leg_ana", "bytes_per_launch": 1234, "source": "k.hip",
           "source_sha256": hashlib.sha256(stored_text.encode()).hexdigest()}
    (tmp_path / "profiles" / "t.md").write_text("# x\n\ntraffic_json: " + json.dumps(rec) + "\n")


def test_traffic_figure_follows_its_kernel_source(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", "profiles/t.md")
    _summary(tmp_path, "kernel v1", "kernel v1")
    assert bench.measured_traffic("legendre_analysis") == 1234
    assert bench.measured_traffic("legendre_synthesis") is None  # no record for it
    assert bench.measured_traffic("no_such_class") is None
    (tmp_path / "k.hip").write_text("kernel v2")  # the kernel changed since
    assert bench.measured_traffic("legendre_analysis") is None


def test_committed_traffic_figures_describe_the_committed_kernels():
    for cls in bench.TRAFFIC_KERNELS:
        assert bench.measured_traffic(cls) is not None, cls
