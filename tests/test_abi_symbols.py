"""The C-ABI library loads and exports every entry point include/mm.h
declares (no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mm.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mm_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared()
    for must in ("mm_naive", "mm_strassen", "mm_winograd", "mm_gemm_ex", "mm_workspace_size",
                 "mm_plan_create", "mm_plan_execute", "mm_plan_destroy", "mm_batched",
                 "mm_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2309_00628_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libmm.so not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_2309_00628_amd import _lib
    assert set(declared()) == set(_lib._SIGS)


def test_library_has_no_torch_dependency():
    from paper_2309_00628_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libmm.so not built")
    import subprocess
    out = subprocess.run(["readelf", "-d", _lib.LIB_PATH], stdout=subprocess.PIPE, text=True).stdout
    needed = re.findall(r"NEEDED.*\[(.*)\]", out)
    assert not [n for n in needed if "torch" in n or "c10" in n], needed
    assert any("amdhip64" in n for n in needed)


def test_error_message_without_device():
    from paper_2309_00628_amd import _lib
    lib = _lib.load()
    assert lib.mm_version() >= 1
    # invalid arguments are rejected before any device work
    st = lib.mm_naive(-1, 2, 2, None, None, None, 1, None)
    assert _lib.STATUS[st] == "MM_E_INVALID"
    assert "negative" in _lib.last_error()
