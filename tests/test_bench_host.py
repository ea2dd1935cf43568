"""Host-side logic of bench.py (no GPU): the one-GPU contract, the gate that
reports measured HBM traffic only for the kernel source and sweep it was
measured on,
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


def test_traffic_is_reported_only_for_the_measured_kernel_source(tmp_path):
    f = tmp_path / "traffic.txt"
    f.write_text("# header: ignored\n"
                 f"kernel_source_sha256_16: {bench.kernel_source_hash()}\n"
                 "traffic_bytes_per_launch_f64: 12345\n")
    assert bench.measured_traffic("liftingbody", "f64", str(f)) == 12345.0
    assert bench.measured_traffic("liftingbody", "f32", str(f)) is None   # not measured for this storage
    assert bench.measured_traffic("liftingbody", "f64", str(f), sweep="push") is None   # sweep not stated
    f.write_text(f"kernel_source_sha256_16: {bench.kernel_source_hash()}\nsweep: push_unordered\n"
                 "traffic_bytes_per_launch_f64: 12345\n")
    assert bench.measured_traffic("liftingbody", "f64", str(f), sweep="push_unordered") == 12345.0
    assert bench.measured_traffic("liftingbody", "f64", str(f), sweep="push") is None   # another sweep
    f.write_text("kernel_source_sha256_16: 0000000000000000\ntraffic_bytes_per_launch_f64: 12345\n")
    assert bench.measured_traffic("liftingbody", "f64", str(f)) is None   # the kernel changed since
    assert bench.measured_traffic("liftingbody", "f64", str(tmp_path / "missing.txt")) is None
    assert bench.measured_traffic("sphere", "f64") is None                # no profile for this workload


def test_roofline_bound_is_the_roof_with_the_longer_least_time():
    """The bound is whichever roof gives the longer least time for the
    sweep: the vector ALUs when the method's flops per byte exceed the FP64
    ridge of 9.8 (2D FP64 f: about 407 flops per 32 B), HBM below it (the
    same flops over 4x the bytes); both figures are reported beside."""
    from paper_2412_06546_amd import cases
    c = cases.case_periodic_wave(nx=6, ny=4, nv=4)
    nc, nv = 20000, 3600
    fpu = bench.alg_flops_per_update(2, bench.mean_faces_per_cell(c))
    for bpu, bound in ((32, "alu"), (128, "hbm")):
        run = dict(nc=nc, nv=nv, sweep_ms_avg=3.0, achieved_gbs=nc * nv * bpu / 3e-3 / 1e9, bytes_per_update=bpu,
                   alg_bytes=nc * nv * bpu)
        assert (fpu / bpu > 78.6e12 / 8e12) == (bound == "alu")
        r = bench.roofline_of(c, run, "cylinder", "f64", "in-place")
        assert r["bound"] == bound and r["traffic"] is None
        assert r["hbm"]["unit"] == "GB/s" and r["hbm"]["peak"] == 8000.0
        assert r["hbm"]["frac"] == pytest.approx(nc * nv * bpu / 3e-3 / 1e9 / 8000.0, abs=1e-4)
        assert r["alu"]["unit"] == "TFLOP/s" and r["alu"]["peak"] == 78.6
        assert r["alu"]["achieved"] == pytest.approx(fpu * nc * nv / 3e-3 / 1e12, rel=1e-3)
        top = r[bound]
        assert (r["achieved"], r["peak"], r["unit"], r["frac"]) == (top["achieved"], top["peak"], top["unit"],
                                                                    top["frac"])
        assert r["least_ms"][bound] >= max(r["least_ms"].values())


@pytest.mark.parametrize("dim,nf,expected", [(2, 3.9, 407.1), (3, 4.0, 267.0), (3, 6.0, 368.0)])
def test_algorithmic_flops_per_update(dim, nf, expected):
    """One limited slope per (cell, velocity), every face flux once, source and
    updates: the per-update counts the roofline is priced with (cylinder's mean
    of 3.9 faces, tetrahedra, hexahedra)."""
    assert bench.alg_flops_per_update(dim, nf) == pytest.approx(expected, abs=0.06)


def test_json_line_has_no_nan():
    """Percentiles of an empty set of cases are NaN; the JSON line carries null."""
    import json
    line = bench.json_safe({"a": float("nan"), "b": [1.0, float("nan")], "c": {"d": float("nan"), "e": 2}})
    assert json.loads(json.dumps(line)) == {"a": None, "b": [1.0, None], "c": {"d": None, "e": 2}}
