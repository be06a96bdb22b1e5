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


# the binding's ctypes mirrors of the header's structs, field by field
STRUCTS = {"efe_mesh_desc": "MeshDesc", "efe_system_desc": "SystemDesc",
           "efe_cheb_params": "ChebParams", "efe_scf_params": "ScfParams",
           "efe_scf_report": "ScfReport", "efe_radial_params": "RadialParams",
           "efe_radial_report": "RadialReport"}


def test_struct_layouts_match_the_header(tmp_path):
    """Size and every field offset of each struct, as the C compiler lays it
    out from include/efe.h, equal the binding's ctypes mirror."""
    import shutil
    import subprocess
    from paper_2607_06848_amd import efe
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "efe.h"', "int main(void) {"]
    for cname, pyname in STRUCTS.items():
        py = getattr(efe, pyname)
        lines.append(f'printf("{pyname} size %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'printf("{pyname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            name, field, val = line.split()
            got[(name, field)] = int(val)
    for cname, pyname in STRUCTS.items():
        py = getattr(efe, pyname)
        assert got[(pyname, "size")] == ctypes.sizeof(py), pyname
        for f in py._fields_:
            assert got[(pyname, f[0])] == getattr(py, f[0]).offset, (pyname, f[0])
