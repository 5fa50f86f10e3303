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


def test_struct_layouts_match_header(tmp_path):
    """Size and field offsets of the ctypes mirrors equal what the C
    compiler lays out for include/ibmx.h."""
    import subprocess
    from paper_2109_03972_amd import ibmx
    structs = (ibmx.ibmx_grid, ibmx.ibmx_params, ibmx.ibmx_stats)
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "ibmx.h"', "int main(void) {"]
    for S in structs:
        nme = S.__name__
        lines.append(f'printf("{nme} size %zu\\n", sizeof({nme}));')
        for f in S._fields_:
            lines.append(f'printf("{nme} {f[0]} %zu\\n", offsetof({nme}, {f[0]}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                           str(exe)])
    got = subprocess.check_output([str(exe)], text=True).split("\n")
    for row in got:
        if not row:
            continue
        nme, field, val = row.split()
        S = getattr(ibmx, nme)
        want = ctypes.sizeof(S) if field == "size" else getattr(S, field).offset
        assert int(val) == want, (nme, field, int(val), want)
    assert sum(1 for r in got if r) == sum(len(S._fields_) + 1 for S in structs)
