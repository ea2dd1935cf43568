"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code
(no GPU needed).

* The library's host side (ugks_api.cpp: input validation, relabelling,
  geometry, the push sweep's colouring, the footprint plan) is compiled with
  both sanitizers for the host only and linked into a harness
  (tests/sanitize/host_harness.cpp) that drives it through the C ABI with
  valid and invalid inputs; the kernel launchers come from the built
  libugks.so.  Without a GPU, ugks_create runs every host step and stops at
  its first device allocation.
* The oracle (oracle/ugks_oracle.c) is compiled with both sanitizers and run
  for a few steps on cases that reach every face type (periodic, wall, far
  field), both dimensions, tabulated and scattered velocity sets, the
  residual, the macro gradients and the wall flux.

A sanitizer report ends the program with a non-zero status (undefined
behaviour is not recovered from), so each test checks the status and that no
report was printed.
"""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
LIB_DIR = os.path.join(ROOT, "paper_2412_06546_amd")

# sanitizer flags for host code only (each one after -Xarch_host)
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _no_report(text):
    return "ERROR: AddressSanitizer" not in text and "runtime error:" not in text and "LeakSanitizer" not in text


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_library_host_code_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    lib = os.path.join(LIB_DIR, "libugks.so")
    if not os.path.exists(lib):
        from paper_2412_06546_amd import build
        build.build(force=False)
    exe = str(tmp_path / "host_harness")
    cmd = [HIPCC, "--offload-arch=gfx950", "--cuda-host-only", "-O1", "-g", "-std=c++17", *HOST_SAN,
           "-I", os.path.join(ROOT, "include"), "-o", exe,
           os.path.join(ROOT, "tests", "sanitize", "host_harness.cpp"),
           os.path.join(LIB_DIR, "csrc", "ugks_api.cpp"),
           "-L", LIB_DIR, "-l:libugks.so", "-Wl,-rpath," + LIB_DIR]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and _no_report(out), out[-6000:]
    assert "0 failed" in r.stdout
    n = int(r.stdout.split()[0])
    assert n >= 200, r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    so = str(tmp_path / "libugks_oracle_san.so")
    cmd = ["gcc", "-O1", "-g", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_DEFAULT_SOURCE",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
           "-o", so, os.path.join(ROOT, "oracle", "ugks_oracle.c"), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    script = textwrap.dedent(f"""
        import sys
        sys.path.insert(0, {ROOT!r}); sys.path.insert(0, {os.path.join(ROOT, 'tests')!r})
        import numpy as np
        import oracle
        oracle._LIB = {so!r}
        oracle.build = lambda force=False: oracle._LIB
        from paper_2412_06546_amd import cases
        from special_cases import fallback_case
        cs = [cases.case_periodic_wave(nx=6, ny=4, nv=8),
              cases.case_cylinder_small(n_theta=12, n_r=5, nv=8),
              cases.case_channel_3d(n=3, kind="hex", nv=5),
              cases.case_box_wave_3d(n=3, kind="tet", nv=5),
              cases.case_box_wave_3d(n=3, kind="prism", nv=5),
              fallback_case()]
        c = cases.case_periodic_wave(nx=5, ny=3, nv=8)
        keep = (c["vgrid"]["u"] ** 2).sum(1) < 12.0          # a non-tabulated (disc) velocity set
        c["vgrid"] = dict(dim=2, u=np.ascontiguousarray(c["vgrid"]["u"][keep]),
                          w=np.ascontiguousarray(c["vgrid"]["w"][keep]))
        cs.append(c)
        for c in cs:
            o = oracle.Oracle(c, omp_threads=2)
            o.step(2)
            W, q = o.macros()
            r = o.residual()
            g, bad = o.macro_gradients()
            o.wall_flux()
            assert np.isfinite(W).all() and np.isfinite(r).all() and np.isfinite(o.f()).all()
        print("oracle ok", len(cs))
    """)
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True, timeout=600, env=env,
                       cwd=ROOT)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and _no_report(out), out[-6000:]
    assert "oracle ok" in r.stdout
