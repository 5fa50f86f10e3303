"""The C-ABI library loads and exports every entry point of include/ibmx.h
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "ibmx.h")).read()
    return sorted(set(re.findall(r"IBMX_API\s+[\w\s\*]*?\b(ibmx_\w+)\s*\(", txt)))


def test_header_declares_the_api():
    from paper_2109_03972_amd import ibmx
    assert _declared() == sorted(ibmx.API)


def test_library_exports_every_declared_symbol():
    from paper_2109_03972_amd import ibmx
    if not os.path.exists(ibmx.LIB_PATH):
        pytest.fail("libibmx.so not built (run __graft_entry__.build())")
    L = ctypes.CDLL(ibmx.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name


def test_status_strings_and_version():
    from paper_2109_03972_amd import ibmx
    assert ibmx.status_string(ibmx.OK) == "ok"
    assert "wall" in ibmx.status_string(ibmx.EDOMAIN)
    assert ibmx.status_string(12345) == "unknown status"
    assert "gfx950" in ibmx.version()


def test_struct_layouts_match_header():
    """Field offsets of the ctypes mirrors follow the C declarations."""
    from paper_2109_03972_amd import ibmx
    assert ctypes.sizeof(ibmx.ibmx_grid) == 4 * 6 + 8 * 4
    assert ibmx.ibmx_params.two_alpha_dt.offset == 8
    assert ibmx.ibmx_params.disable_mode.offset == 8 + 8 * 13
    assert ibmx.ibmx_params.disable_seed.offset == 8 + 8 * 13 + 8
    assert ctypes.sizeof(ibmx.ibmx_params) == 8 + 8 * 13 + 8 + 8
