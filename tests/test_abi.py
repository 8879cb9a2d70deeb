"""The C-ABI library loads and exports every entry point the header declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cutcell.h")
LIB = os.path.join(ROOT, "paper_1509_02572_amd", "libcutcell.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", text, re.M)
    return sorted(set(n for n in names if n.startswith(("cutcell_", "amr_"))))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1509_02572_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("cutcell_geometry", "cutcell_merge_map", "cutcell_tendency", "cutcell_rk_stage"):
        assert n in names
    assert len(names) >= 10


def test_library_exports_every_declared_symbol(lib):
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_version_and_argument_errors_without_device(lib):
    from paper_1509_02572_amd import cutcell as CC
    lib.cutcell_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.cutcell_version()
    L = CC.lib()
    # host-side argument checks return CC_EINVAL before touching the device
    g = CC.cc_grid(8, 8, 8, 8, 100.0, 100.0, 50.0, 3, 0)  # nsub not a power of two
    geom = CC.cc_geom()
    assert L.cutcell_geometry(ctypes.byref(g), ctypes.byref(geom), None, None) == CC.CC_EINVAL
    assert b"nsub" in L.cutcell_last_error()
    g = CC.cc_grid(8, 8, 8, 8, 100.0, 100.0, 50.0, 16, 0)
    assert L.cutcell_geometry(ctypes.byref(g), ctypes.byref(geom), None, None) == CC.CC_EINVAL
    assert b"null" in L.cutcell_last_error()
    g = CC.cc_grid(8, 8, 8, 4, 100.0, 100.0, 50.0, 16, 0)  # nzs < nz
    assert L.cutcell_merge_map(ctypes.byref(g), ctypes.byref(geom), None, None) == CC.CC_EINVAL
