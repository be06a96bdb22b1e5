"""The C-ABI library loads on the CPU host and exports every entry point
declared in include/efe.h (no compute call is made without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    text = open(os.path.join(ROOT, "include", "efe.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(efe_[A-Za-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("efe_setup_mesh", "efe_apply_H", "efe_cheb_filter", "efe_rayleigh_ritz"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2607_06848_amd import efe
    if not os.path.exists(efe.LIB_PATH):
        pytest.skip("libefe.so not built (run __graft_entry__.build())")
    L = ctypes.CDLL(efe.LIB_PATH)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_declared_symbols():
    from paper_2607_06848_amd import efe
    assert set(declared()) <= set(efe.exported_symbols())


def test_setup_error_without_gpu_is_reported():
    """Bad arguments are rejected before any device work (no GPU needed)."""
    from paper_2607_06848_amd import efe
    if not os.path.exists(efe.LIB_PATH):
        pytest.skip("libefe.so not built")
    L = efe.lib()
    md = efe.MeshDesc()
    md.p = 0            # invalid order
    sd = efe.SystemDesc()
    h = ctypes.c_void_p()
    assert L.efe_setup_mesh(ctypes.byref(md), ctypes.byref(sd), None, ctypes.byref(h)) == -1
    assert not h.value
