"""The C-ABI library loads and exports every entry point its header declares
(no compute call: runs without a GPU)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2412_06546_amd", "libugks.so")


def declared_functions():
    text = open(os.path.join(ROOT, "include", "ugks.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ugks_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_core_entry_points():
    names = declared_functions()
    for n in ("ugks_create", "ugks_step", "ugks_macros", "ugks_destroy"):
        assert n in names


def test_binding_constants_are_the_headers():
    """Every integer constant the header defines has the same value in the
    Python binding (status codes, storage and memory modes, boundary types,
    the default chunk)."""
    from paper_2412_06546_amd import ugks
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "ugks.h")).read(), flags=re.S)
    defs = dict(re.findall(r"^#define\s+(UGKS_[A-Z0-9_]+)\s+\(?(-?\d+)\)?\s*$", text, flags=re.M))
    assert len(defs) >= 16 and "UGKS_DEFAULT_CHUNK" in defs and "UGKS_ERR_STATE" in defs
    mismatched = {k: (v, getattr(ugks, k, None)) for k, v in defs.items() if getattr(ugks, k, None) != int(v)}
    assert not mismatched, mismatched


@pytest.mark.skipif(not os.path.exists(LIB), reason="libugks.so not built")
def test_library_exports_every_declared_symbol():
    import ctypes
    L = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libugks.so not built")
def test_binding_declares_the_same_names():
    from paper_2412_06546_amd import ugks
    L = ugks.load_library()
    for n in declared_functions():
        assert getattr(L, n).restype is not None or n in ("ugks_destroy", "ugks_batch_destroy")


def test_binding_fails_loudly_without_the_library(tmp_path):
    from paper_2412_06546_amd import ugks
    with pytest.raises(ImportError):
        ugks._lib = None
        try:
            ugks.load_library(str(tmp_path / "missing.so"))
        finally:
            ugks._lib = None


@pytest.mark.skipif(not os.path.exists(LIB), reason="libugks.so not built")
@pytest.mark.parametrize("what", ["no velocities", "no cells", "too many velocities", "dim 4",
                                  "bad storage", "Pr 0", "face out of range", "negative density",
                                  "normal not unit", "centroid not finite", "zero velocity weight"])
def test_create_rejects_degenerate_inputs_on_the_host(what):
    """ugks_create validates its arguments before any device call: each of
    these returns UGKS_ERR_ARG with a message, and no handle."""
    import ctypes
    import numpy as np
    from paper_2412_06546_amd import cases, ugks
    c = cases.case_periodic_wave(nx=4, ny=3, nv=6)
    m, vg, gas = c["mesh"], c["vgrid"], c["gas"]
    fstore = "f64"
    if what == "no velocities":
        c["vgrid"] = dict(dim=2, u=np.zeros((0, 2)), w=np.zeros(0))
    elif what == "no cells":
        c["mesh"] = dict(m, cell_volume=np.zeros(0), cell_centroid=np.zeros((0, 2)))
        c["prim0"] = np.zeros((0, 4))
    elif what == "too many velocities":
        c["vgrid"] = cases.tensor_vgrid(129, 6.0, 2)
    elif what == "dim 4":
        c["mesh"] = dict(m, dim=4)
    elif what == "bad storage":
        fstore = "f16"
    elif what == "Pr 0":
        c["gas"] = dict(gas, Pr=0.0)
    elif what == "face out of range":
        fc = m["face_cells"].copy()
        fc[3, 0] = len(m["cell_volume"])
        c["mesh"] = dict(m, face_cells=fc)
    elif what == "normal not unit":
        c["mesh"] = dict(m, face_normal=m["face_normal"] * 1.01)
    elif what == "centroid not finite":
        cc = m["cell_centroid"].copy()
        cc[2, 1] = np.nan
        c["mesh"] = dict(m, cell_centroid=cc)
    elif what == "zero velocity weight":
        w = vg["w"].copy()
        w[7] = 0.0
        c["vgrid"] = dict(vg, w=w)
    elif what == "negative density":
        c["prim0"] = c["prim0"].copy()
        c["prim0"][5, 0] = -1.0
    L = ugks.load_library()
    keep = []
    if fstore == "f16":
        ugks._FSTORE["f16"] = 7
    try:
        mesh, vgrid, g, prim0 = ugks._structs(c, fstore, keep)
    finally:
        ugks._FSTORE.pop("f16", None)
    h = ctypes.c_void_p(1)
    code = L.ugks_create(ctypes.byref(mesh), ctypes.byref(vgrid), ctypes.byref(g), prim0, None, ctypes.byref(h))
    assert code == ugks.UGKS_ERR_ARG, (what, code)
    assert not h.value
    assert L.ugks_last_error(None).decode()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libugks.so not built")
def test_binding_leaves_one_hip_runtime_in_the_process():
    """load_library() before any import of torch still leaves a single HIP
    runtime (and HSA runtime) mapped: the library binds to torch's."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2412_06546_amd import ugks\n"
            "ugks.load_library()\n"
            "import torch\n"
            "maps = [l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l or 'libhsa-runtime64' in l]\n"
            "print(len({m for m in maps if 'amdhip64' in m}), len({m for m in maps if 'hsa-runtime64' in m}))\n" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.split() == ["1", "1"], out.stdout


@pytest.mark.skipif(not os.path.exists(LIB), reason="libugks.so not built")
@pytest.mark.parametrize("dim", [2, 3])
def test_in_place_footprint_is_one_f_plus_the_ring(dim):
    """Host-side estimate (exactly what ugks_create allocates): the in-place
    form needs one f plus a ring of `chunk` velocities per cell, and nothing
    that grows with the number of chunks, so even one velocity per chunk
    stays below the two-buffer form; chunks beyond n_vel are capped."""
    from paper_2412_06546_amd import cases, ugks
    c = cases.case_periodic_wave() if dim == 2 else cases.case_channel_3d(n=3, kind="prism", nv=8)
    nc, nv = len(c["mesh"]["cell_volume"]), len(c["vgrid"]["w"])
    ncomp = 2 if dim == 2 else 1
    two = ugks.footprint_estimate(c, "f64", "two-buffers", sweep="gather")
    f_bytes = nc * ncomp * nv * 8
    # beyond one f and the ring: gather -- the moment sum and the wall
    # densities; push -- also the colour lists, the face -> wall ordinal and
    # the running moments about U^n: a few tens of doubles per cell at most
    for sweep, per_cell in (("gather", 16), ("push", 28), ("push_unordered", 28)):
        one = {ch: ugks.footprint_estimate(c, "f64", "in-place", ch, sweep=sweep) for ch in (1, 2, nv, 10 * nv)}
        assert one[1] < one[2] < one[nv] == one[10 * nv]
        assert one[1] < two
        extra = one[1] - (two - f_bytes) - nc * ncomp * 8
        assert 0 < extra <= nc * per_cell * 8 + 4096, (sweep, extra / nc)
        # the ring is the only part that grows with the chunk
        ring_growth = nc * ncomp * (nv - 1) * 8
        assert ring_growth <= one[nv] - one[1] <= ring_growth + 4096


@pytest.mark.parametrize("dim", [2, 3])
def test_unordered_push_allocates_what_the_push_sweep_does(dim):
    """The unordered push sweep keeps the push sweep's buffers (its one class
    lists every cell, as the colour lists do).  With BF16 f both keep FP32
    stage-1 sums: the second buffer in two buffers, the ring in place (2
    more bytes per value than BF16); the automatic choice gathers BF16 f."""
    from paper_2412_06546_amd import cases, ugks
    c = cases.case_periodic_wave() if dim == 2 else cases.case_channel_3d(n=3, kind="prism", nv=8)
    for fs in ("f64", "f32"):
        for mem in ("two-buffers", "in-place"):
            a = ugks.footprint_estimate(c, fs, mem, sweep="push")
            b = ugks.footprint_estimate(c, fs, mem, sweep="push_unordered")
            assert a == b > 0, (fs, mem)
    nc, nv = len(c["mesh"]["cell_volume"]), len(c["vgrid"]["w"])
    ncomp = 2 if dim == 2 else 1
    gather = ugks.footprint_estimate(c, "bf16", "two-buffers", sweep="gather")
    assert ugks.footprint_estimate(c, "bf16", "two-buffers") == gather
    for sw in ("push", "push_unordered"):
        bf = ugks.footprint_estimate(c, "bf16", "two-buffers", sweep=sw)
        f64push = ugks.footprint_estimate(c, "f64", "two-buffers", sweep=sw)
        assert bf == f64push - nc * ncomp * nv * (16 - 6), sw
        ch = min(ugks.UGKS_DEFAULT_CHUNK, nv)
        bf_ip = ugks.footprint_estimate(c, "bf16", "in-place", sweep=sw)
        f64_ip = ugks.footprint_estimate(c, "f64", "in-place", sweep=sw)
        assert bf_ip == f64_ip - nc * ncomp * (nv * (8 - 2) + ch * (8 - 4)), sw
