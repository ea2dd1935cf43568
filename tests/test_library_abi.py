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
