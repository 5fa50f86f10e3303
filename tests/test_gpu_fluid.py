"""Parity of the HIP pressure projection (ibmx_project, through the C ABI)
with the FP64 oracle: u, u_f, P and phi to 1e-12 in FP64 (FFT and
elimination orders differ from the oracle's), FP32 grids against the oracle
on the FP32-rounded inputs to 1e-5; at the bed's 512^3 size, properties
that hold at any size (the projected faces are divergence-free)."""
import numpy as np
import pytest

from oracle import projection as pj
from paper_2109_03972_amd import ibmx, synth
from tests._util import rel_err, require_gpu

pytestmark = pytest.mark.gpu


def _case(n, periodic, seed=0):
    """A grid without particles (the projection needs none)."""
    return synth.Case(name="grid", n=tuple(n), h=0.5 + 0.1 * (seed % 3), origin=(0.0, 0.0, 0.0),
                      periodic=tuple(periodic), xp=np.zeros((3, 0)), up=np.zeros((3, 0)),
                      wp=np.zeros((3, 0)), radius=np.zeros(0), mass=np.zeros(0),
                      moff=np.zeros(1, dtype=np.int32), body=np.zeros((3, 0)), dV=np.zeros(0),
                      u0=None, params=synth.default_params())


def _run(case, precision, u_np, P_np, theta):
    import torch
    dev = require_gpu()
    T = torch.float64 if precision == "f64" else torch.float32
    plan = ibmx.Plan.from_case(case, precision)
    u = torch.as_tensor(u_np).to(dev).to(T).contiguous()
    P = torch.as_tensor(P_np).to(dev).to(T).contiguous()
    uf, phi = plan.project(u, P, theta)
    plan.check("project")
    torch.cuda.synchronize()
    out = {k: v.double().cpu().numpy() for k, v in dict(u=u, uf=uf, P=P, phi=phi).items()}
    plan.close()
    return out


@pytest.mark.parametrize("n,periodic", [((16, 8, 8), (1, 1, 1)), ((32, 16, 13), (1, 1, 0)),
                                        ((8, 32, 1), (1, 1, 0)), ((8, 8, 64), (1, 1, 1)),
                                        ((64, 32, 20), (1, 1, 0))])
@pytest.mark.parametrize("theta", [0.0, 1.0])
def test_projection_parity_f64(n, periodic, theta):
    case = _case(n, periodic, seed=sum(n))
    rng = np.random.default_rng(7)
    shape = (n[2], n[1], n[0])
    u0 = rng.normal(0.0, 1.0, (3,) + shape)
    P0 = rng.normal(0.0, 1.0, shape)
    prm = case.params
    ref = pj.project(u0, P0, case.h, prm["c"], prm["nu_f"], theta, periodic)
    got = _run(case, "f64", u0, P0, theta)
    for k in ("u", "uf", "P", "phi"):
        e = rel_err(got[k], ref[k])
        assert e <= 1e-12, f"{k}: {e:.3e}"
    div = pj.face_div(got["uf"], case.h, periodic)
    assert np.abs(div).max() <= 1e-11 * np.abs(ref["div_star"]).max()


@pytest.mark.parametrize("n,periodic", [((32, 16, 13), (1, 1, 0)), ((16, 16, 16), (1, 1, 1))])
def test_projection_parity_f32(n, periodic):
    case = _case(n, periodic, seed=3)
    rng = np.random.default_rng(8)
    shape = (n[2], n[1], n[0])
    u0 = rng.normal(0.0, 1.0, (3,) + shape).astype(np.float32).astype(np.float64)
    P0 = rng.normal(0.0, 1.0, shape).astype(np.float32).astype(np.float64)
    prm = case.params
    ref = pj.project(u0, P0, case.h, prm["c"], prm["nu_f"], 0.0, periodic)
    got = _run(case, "f32", u0, P0, 0.0)
    for k in ("u", "uf", "P", "phi"):
        e = rel_err(got[k], ref[k])
        assert e <= 1e-5, f"{k}: {e:.3e}"


def test_unsupported_grids():
    import torch
    dev = require_gpu()
    for n, periodic in (((24, 16, 8), (1, 1, 0)), ((16, 16, 8), (1, 0, 1)),
                        ((16, 16, 12), (1, 1, 1))):
        case = _case(n, periodic, seed=1)
        plan = ibmx.Plan.from_case(case, "f64")
        u = torch.zeros((3, n[2], n[1], n[0]), dtype=torch.float64, device=dev)
        P = torch.zeros((n[2], n[1], n[0]), dtype=torch.float64, device=dev)
        with pytest.raises(ibmx.IbmxError):
            plan.project(u, P)
        plan.close()


def test_bed_512_divergence_free():
    """The bed workload's 512^3 grid with walls in z, FP32 grid, the
    synthetic velocity field: the projected face velocities are
    divergence-free to FP32 rounding and vanish on the upper wall."""
    import torch
    dev = require_gpu()
    case = synth.make_case("polydisperse_bed_512", lazy_field=True)
    plan = ibmx.Plan.from_case(case, "f32")
    u = case.field(device=dev).to(torch.float32).contiguous()
    shape = tuple(u.shape[1:])
    P = torch.zeros(shape, dtype=torch.float32, device=dev)
    uf, phi = plan.project(u, P, 0.0)
    plan.check("project bed")
    torch.cuda.synchronize()
    h = case.h
    ufd = uf.double()
    div = torch.zeros(shape, dtype=torch.float64, device=dev)
    for a, ax in enumerate((2, 1, 0)):
        inflow = torch.roll(ufd[a], 1, dims=ax)
        if a == 2:
            inflow[0] = 0.0
        div += (ufd[a] - inflow) / h
    scale = ufd.abs().max().item() / h
    print(f"bed: max |div u_f| {div.abs().max().item():.3e} (scale {scale:.3e})", flush=True)
    assert div.abs().max().item() <= 1e-5 * scale
    assert torch.all(uf[2][-1] == 0)
    plan.close()
