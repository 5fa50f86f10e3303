"""Host-side validation of the C ABI (the failure list of the boundary):
calls with invalid arguments return their status before any device work,
so these run without a GPU.  Each case changes one field of a valid plan
request."""
import ctypes

import numpy as np
import pytest

from paper_2109_03972_amd import ibmx, synth


def _create(n=(32, 32, 32), periodic=(1, 1, 0), moff=(0, 10, 25), **over):
    prm = synth.default_params()
    prm["n_iter"] = 3
    prm.update(over)
    grid = ibmx.make_grid(n, over.pop("h", 1.0), (0.0, 0.0, 0.0), periodic)
    p = ibmx.make_params(prm)
    m = np.ascontiguousarray(moff, dtype=np.int32)
    h = ctypes.c_void_p()
    st = ibmx.lib().ibmx_plan_create(ctypes.byref(h), ctypes.byref(grid), ctypes.byref(p),
                                     len(moff) - 1, m.ctypes.data_as(ctypes.c_void_p), ibmx.F32,
                                     None)
    return st, h


@pytest.mark.parametrize("over,code", [
    (dict(n_iter=0), ibmx.EINVAL),                     # fewer than one pass
    (dict(n_iter=65), ibmx.EINVAL),                    # above the library maximum
    (dict(c=0.0), ibmx.EINVAL),                        # c = 2 alpha dt must be nonzero
    (dict(c=float("nan")), ibmx.EINVAL),
    (dict(kernel=5), ibmx.EUNSUPPORTED),               # only the 3- and 4-point deltas
    (dict(normal_model=2), ibmx.EUNSUPPORTED),
    (dict(disable_mode=3), ibmx.EINVAL),
    (dict(disable_mode=1, eps_sep=1.5, gap_cut=2.9), ibmx.EINVAL),   # cut below 2 eps_sep
    (dict(e_dry=1.5), ibmx.EINVAL),
    (dict(T_c=0.0), ibmx.EINVAL),
    (dict(st_switch=2), ibmx.EINVAL),
])
def test_invalid_params(over, code):
    st, h = _create(**over)
    assert st == code
    assert not h.value


@pytest.mark.parametrize("moff", [(1, 10, 25), (0, 10, 5), (0, -1, 3)])
def test_invalid_marker_csr(moff):
    """Marker offsets must start at 0 and never decrease."""
    st, h = _create(moff=moff)
    assert st == ibmx.EINVAL
    assert not h.value


def test_invalid_grid():
    assert _create(n=(32, 0, 32))[0] == ibmx.EINVAL
    assert _create(n=(4, 32, 32), periodic=(1, 1, 1))[0] == ibmx.EINVAL   # < 2 supports
    assert _create(periodic=(2, 1, 1))[0] == ibmx.EINVAL


def test_null_handles():
    L = ibmx.lib()
    assert L.ibmx_plan_create(None, None, None, 0, None, 0, None) == ibmx.EINVAL
    assert L.ibmx_forcing(None, *([None] * 10)) == ibmx.EINVAL
    assert L.ibmx_plan_status(None) == ibmx.EINVAL
    assert L.ibmx_plan_destroy(None) == ibmx.EINVAL
