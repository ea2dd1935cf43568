"""Host-side logic of bench.py (no GPU): the one-GPU contract, the gate that
reports measured HBM traffic only for the kernel source it was measured on,
and the algorithmic flop counts the roofline divides by."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_is_reported_only_for_the_measured_kernel_source(tmp_path, monkeypatch):
    f = tmp_path / "traffic.txt"
    f.write_text("# header: ignored\n"
                 f"kernel_source_sha256_16: {bench.kernel_source_hash()}\n"
                 "traffic_bytes_per_launch_f64: 12345\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("f64") == 12345.0
    assert bench.measured_traffic("f32") is None          # not measured for this storage
    f.write_text("kernel_source_sha256_16: 0000000000000000\ntraffic_bytes_per_launch_f64: 12345\n")
    assert bench.measured_traffic("f64") is None          # the kernel changed since
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic("f64") is None


@pytest.mark.parametrize("dim,nf,expected", [(2, 3.9, 407.1), (3, 4.0, 267.0), (3, 6.0, 368.0)])
def test_algorithmic_flops_per_update(dim, nf, expected):
    """One limited slope per (cell, velocity), every face flux once, source and
    updates: the per-update counts the roofline is priced with (cylinder's mean
    of 3.9 faces, tetrahedra, hexahedra)."""
    assert bench.alg_flops_per_update(dim, nf) == pytest.approx(expected, abs=0.06)
