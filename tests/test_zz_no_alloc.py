"""ibmx_grid_mean_noalloc (the entry point that allocates nothing) against
ibmx_grid_mean through the C ABI: the same kernels in the same order, so the
means must agree bit for bit, on two calls in a row (the second on a smaller
grid) in both precisions, and after the static array has held another
call's partial sums."""
import ctypes

import numpy as np
import pytest

from paper_2109_03972_amd import ibmx, synth
from _util import require_gpu

pytestmark = pytest.mark.gpu


def _grid_case(n):
    return synth.Case(name="grid", n=tuple(n), h=1.0, origin=(0.0, 0.0, 0.0), periodic=(1, 1, 0),
                      xp=np.zeros((3, 0)), up=np.zeros((3, 0)), wp=np.zeros((3, 0)),
                      radius=np.zeros(0), mass=np.zeros(0), moff=np.zeros(1, dtype=np.int32),
                      body=np.zeros((3, 0)), dV=np.zeros(0), u0=None,
                      params=synth.default_params())


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_noalloc_mean_matches_plan_mean(precision):
    import torch
    dev = require_gpu()
    T = torch.float64 if precision == "f64" else torch.float32
    gen = torch.Generator(device="cpu").manual_seed(17)
    L = ibmx.lib()
    for n in ((96, 80, 72), (33, 17, 5)):       # second call: a smaller input
        print(f"noalloc mean {precision} n={n}", flush=True)
        f = torch.randn((3, n[2], n[1], n[0]), generator=gen, dtype=torch.float64).to(T).to(dev)
        plan = ibmx.Plan.from_case(_grid_case(n), precision)
        want = plan.grid_mean(f)
        got = torch.full((3,), float("nan"), dtype=torch.float64, device=dev)
        st = L.ibmx_grid_mean_noalloc(ctypes.c_void_p(f.data_ptr()), n[0] * n[1] * n[2],
                                      ibmx.F64 if precision == "f64" else ibmx.F32,
                                      ctypes.c_void_p(got.data_ptr()),
                                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == ibmx.OK
        torch.cuda.synchronize()
        assert torch.equal(got, want), (got, want)
        ref = f.double().mean(dim=(1, 2, 3))
        assert torch.allclose(got, ref, rtol=1e-12, atol=1e-14)
        plan.close()


def test_noalloc_mean_rejects_bad_sizes():
    import torch
    dev = require_gpu()
    f = torch.zeros(3, dtype=torch.float32, device=dev)
    m = torch.zeros(3, dtype=torch.float64, device=dev)
    L = ibmx.lib()
    for nn in (0, -5, 1 << 31):
        assert L.ibmx_grid_mean_noalloc(ctypes.c_void_p(f.data_ptr()), nn, ibmx.F32,
                                        ctypes.c_void_p(m.data_ptr()), None) == ibmx.EINVAL
    assert L.ibmx_grid_mean_noalloc(ctypes.c_void_p(f.data_ptr()), 1, 7,
                                    ctypes.c_void_p(m.data_ptr()), None) == ibmx.EINVAL
    assert L.ibmx_grid_mean_noalloc(None, 1, ibmx.F32, ctypes.c_void_p(m.data_ptr()),
                                    None) == ibmx.EINVAL
    # the binding's wrapper goes through the same entry point
    g = torch.arange(12, dtype=torch.float32, device=dev).reshape(3, 4)
    assert ibmx.grid_mean_noalloc(g).cpu().tolist() == [1.5, 5.5, 9.5]
