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
                                        ((64, 32, 20), (1, 1, 0)), ((16, 8, 70), (1, 1, 0)),
                                        # the bed's 512-point FFT lines, periodic and walled
                                        ((512, 512, 8), (1, 1, 1)), ((512, 512, 16), (1, 1, 0)),
                                        # the longest lines the solver takes (the shortest
                                        # periodic ones, 8 points, are above)
                                        ((1024, 8, 8), (1, 1, 1)), ((8, 1024, 5), (1, 1, 0))])
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


@pytest.mark.parametrize("n,periodic", [((32, 16, 13), (1, 1, 0)), ((16, 16, 16), (1, 1, 1)),
                                        ((512, 512, 8), (1, 1, 1)), ((512, 512, 16), (1, 1, 0))])
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


def _stage_inputs(shape, seed):
    rng = np.random.default_rng(seed)
    return (rng.normal(0.0, 1.0, (3,) + shape), rng.normal(0.0, 1.0, (3,) + shape),
            rng.normal(0.0, 1.0, shape), rng.normal(0.0, 0.1, (3,) + shape))


@pytest.mark.parametrize("n,periodic", [((16, 8, 8), (1, 1, 1)), ((32, 16, 13), (1, 1, 0)),
                                        ((8, 32, 1), (1, 1, 0)), ((64, 32, 20), (1, 1, 0)),
                                        ((16, 8, 70), (1, 1, 0)),
                                        ((512, 512, 8), (1, 1, 1)), ((512, 512, 16), (1, 1, 0)),
                                        ((1024, 8, 8), (1, 1, 1)), ((8, 1024, 5), (1, 1, 0))])
@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("theta", [0.0, 1.0])
def test_predictor_helmholtz_parity(n, periodic, precision, theta):
    """Steps a and e of one stage (alpha, gamma, zeta of the second RK stage)
    against the oracle; the forcing between them is stood in for by an
    arbitrary increment of u~."""
    import torch
    from oracle import fluid_stage as fs
    dev = require_gpu()
    T = torch.float64 if precision == "f64" else torch.float32
    shape = (n[2], n[1], n[0])
    u0, Np, P, df = _stage_inputs(shape, sum(n))
    if precision == "f32":
        u0, Np, P, df = (a.astype(np.float32).astype(np.float64) for a in (u0, Np, P, df))
    alpha, gamma, zeta, dt = 1.0 / 15.0, 5.0 / 12.0, -17.0 / 60.0, 0.4
    case = _case(n, periodic, seed=2)
    prm = dict(case.params)
    prm["c"] = 2.0 * alpha * dt
    prm["nu_f"] = 0.3
    case.params = prm
    fbar = np.array([0.05, -0.02, 0.01]) if all(periodic) else None
    ref_a = fs.predictor(u0, Np, P, case.h, prm["nu_f"], alpha, gamma, zeta, dt, periodic)
    plan = ibmx.Plan.from_case(case, precision)
    tu = lambda a: torch.as_tensor(a).to(dev).to(T).contiguous()
    u_d, N_d, P_d = tu(u0), tu(Np), tu(P)
    ut, lapnu = plan.fluid_predictor(u_d, N_d, P_d, dt, gamma, zeta)
    plan.check("predictor")
    tol = 1e-12 if precision == "f64" else 2e-6
    for k, got in (("u", ut), ("N", N_d), ("lapnu", lapnu)):
        e = rel_err(got.double().cpu().numpy(), ref_a[k])
        assert e <= tol, f"predictor {k}: {e:.3e}"
    # step e from the oracle's u~ plus a forcing increment
    uf_in = ref_a["u"] + df
    if precision == "f32":
        uf_in = uf_in.astype(np.float32).astype(np.float64)
    lap_in = ref_a["lapnu"].astype(np.float32).astype(np.float64) if precision == "f32" else ref_a["lapnu"]
    ref_e = fs.helmholtz(uf_in, lap_in, P, fbar, case.h, prm["nu_f"], alpha, theta, dt, periodic)
    us = tu(uf_in)
    fb_d = None if fbar is None else torch.as_tensor(fbar, dtype=torch.float64).to(dev)
    plan.fluid_helmholtz(us, tu(lap_in), P_d, dt, theta, fbar=fb_d)
    plan.check("helmholtz")
    torch.cuda.synchronize()
    e = rel_err(us.double().cpu().numpy(), ref_e)
    assert e <= (1e-12 if precision == "f64" else 1e-5), f"helmholtz: {e:.3e}"
    plan.close()


@pytest.mark.parametrize("n,periodic", [((20, 9, 67), (1, 1, 1)), ((70, 7, 70), (0, 1, 0)),
                                        ((8, 8, 64), (1, 0, 1)), ((3, 2, 33), (0, 0, 0))])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_predictor_parity_ragged(n, periodic, precision):
    """Step a alone on grids whose columns and z runs do not divide the
    kernel's blocking (ragged x and y edges, several runs of planes with a
    ragged last one), with walls on any axis."""
    import torch
    from oracle import fluid_stage as fs
    dev = require_gpu()
    T = torch.float64 if precision == "f64" else torch.float32
    shape = (n[2], n[1], n[0])
    u0, Np, P, _ = _stage_inputs(shape, 7 + sum(n))
    if precision == "f32":
        u0, Np, P = (a.astype(np.float32).astype(np.float64) for a in (u0, Np, P))
    alpha, gamma, zeta, dt = 4.0 / 15.0, 8.0 / 15.0, -17.0 / 60.0, 0.7
    case = _case(n, periodic, seed=1)
    prm = dict(case.params)
    prm["c"] = 2.0 * alpha * dt
    prm["nu_f"] = 0.2
    case.params = prm
    ref = fs.predictor(u0, Np, P, case.h, prm["nu_f"], alpha, gamma, zeta, dt, periodic)
    plan = ibmx.Plan.from_case(case, precision)
    tu = lambda a: torch.as_tensor(a).to(dev).to(T).contiguous()
    u_d, N_d, P_d = tu(u0), tu(Np), tu(P)
    ut, lapnu = plan.fluid_predictor(u_d, N_d, P_d, dt, gamma, zeta)
    plan.check("predictor")
    torch.cuda.synchronize()
    tol = 1e-12 if precision == "f64" else 2e-6
    for k, got in (("u", ut), ("N", N_d), ("lapnu", lapnu)):
        e = rel_err(got.double().cpu().numpy(), ref[k])
        assert e <= tol, f"predictor {k}: {e:.3e}"
    assert torch.equal(u_d, tu(u0))
    plan.close()


@pytest.mark.parametrize("theta", [0.0, 1.0])
def test_full_stage_chain(theta):
    """One Runge-Kutta stage of the collocated solver end to end (eq.
    fluid-solver a-i): predictor, the forcing loop on the particles, the
    implicit viscous step and the projection, each through the C ABI,
    against the same chain of oracle steps."""
    import torch
    import oracle
    from oracle import fluid_stage as fs
    dev = require_gpu()
    case = synth.small_case(41, n=(32, 32, 28), periodic=(1, 1, 0), n_iter=2, touch=0.3)
    alpha, gamma, zeta, dt = 4.0 / 15.0, 8.0 / 15.0, 0.0, 0.5
    prm = dict(case.params)
    prm["c"] = 2.0 * alpha * dt
    case.params = prm
    shape = (case.n[2], case.n[1], case.n[0])
    rng = np.random.default_rng(12)
    u0 = case.u0
    P0 = rng.normal(0.0, 0.01, shape)
    Np = np.zeros((3,) + shape)
    mask = oracle.marker_mask(case, oracle.pairs(case))
    # oracle chain
    a = fs.predictor(u0, Np, P0, case.h, prm["nu_f"], alpha, gamma, zeta, dt, (1, 1, 0))
    fo = oracle.forcing(case, u0=a["u"], mask=mask)
    us = fs.helmholtz(fo["u"], a["lapnu"], P0, None, case.h, prm["nu_f"], alpha, theta, dt,
                      (1, 1, 0))
    ref = pj.project(us, P0, case.h, prm["c"], prm["nu_f"], theta, (1, 1, 0))
    # HIP chain
    f64 = torch.float64
    tu = lambda x: torch.as_tensor(x, dtype=f64).to(dev).contiguous()
    plan = ibmx.Plan.from_case(case, "f64")
    D = {k: tu(getattr(case, k)) for k in ("xp", "up", "wp", "body", "dV")}
    plan.set_markers(D["body"], D["dV"])
    u_d, N_d, P_d = tu(u0), tu(Np), tu(P0)
    ut, lapnu = plan.fluid_predictor(u_d, N_d, P_d, dt, gamma, zeta)
    f = torch.zeros_like(ut)
    S, Tq = plan.forcing(ut, f, D["xp"], D["up"], D["wp"], mask=tu(mask).to(torch.uint8))
    plan.fluid_helmholtz(ut, lapnu, P_d, dt, theta)
    uf, phi = plan.project(ut, P_d, theta)
    plan.check("stage")
    torch.cuda.synchronize()
    for k, got, want in (("f_tot", f, fo["f_tot"]), ("S", S, fo["S"]), ("u", ut, ref["u"]),
                         ("uf", uf, ref["uf"]), ("P", P_d, ref["P"]), ("phi", phi, ref["phi"])):
        e = rel_err(got.cpu().numpy(), want)
        assert e <= 1e-11, f"{k}: {e:.3e}"
    plan.close()


def test_bed_512_predictor_planes_and_helmholtz_residual():
    """The bed's 512^3 grid, FP32 fields.  The predictor is local, so whole
    planes (the wall planes, their neighbours, one in the middle) are
    checked against the oracle run on the three-plane slab around each.  The
    implicit step is global: its equation's residual, evaluated in FP64 from
    the FP32 result, must be at FP32 rounding."""
    import torch
    from oracle import fluid_stage as fs
    dev = require_gpu()
    case = synth.make_case("polydisperse_bed_512", lazy_field=True)
    nx, ny, nz = case.n
    alpha, gamma, zeta, dt = 1.0 / 15.0, 5.0 / 12.0, -17.0 / 60.0, 1.0
    prm = dict(case.params)
    prm["c"] = 2.0 * alpha * dt
    prm["nu_f"] = 0.3
    case.params = prm
    plan = ibmx.Plan.from_case(case, "f32")
    u = case.field(device=dev).to(torch.float32).contiguous()
    g = torch.Generator(device=dev).manual_seed(3)
    Nb = (0.1 * torch.randn(u.shape, device=dev, generator=g)).contiguous()
    P = (0.01 * torch.randn(u.shape[1:], device=dev, generator=g)).contiguous()
    N0 = Nb.clone()
    ut, lapnu = plan.fluid_predictor(u, Nb, P, dt, gamma, zeta)
    plan.check("predictor bed")
    torch.cuda.synchronize()
    for k in (0, 1, nz // 2, nz - 2, nz - 1):
        lo, hi = max(k - 1, 0), min(k + 2, nz)
        sl = slice(lo, hi)
        slab = (1, 1, 0)
        uk = u[:, sl].double().cpu().numpy()
        ref = fs.predictor(uk, N0[:, sl].double().cpu().numpy(), P[sl].double().cpu().numpy(),
                           case.h, prm["nu_f"], alpha, gamma, zeta, dt, slab)
        m = k - lo
        # a slab edge that is not a real wall: only the middle plane counts
        for name, got in (("u", ut), ("N", Nb), ("lapnu", lapnu)):
            e = rel_err(got[:, k].double().cpu().numpy(), ref[name][:, m])
            assert e <= 2e-6, f"plane {k} {name}: {e:.3e}"
    # implicit step on the predictor's result; residual of
    # u* - beta L u* = rhs with rhs from the same inputs
    rhs_u = ut.clone()
    plan.fluid_helmholtz(ut, lapnu, P, dt, 1.0)
    plan.check("helmholtz bed")
    torch.cuda.synchronize()
    beta = alpha * dt * prm["nu_f"]
    us = ut.double()
    Pd = P.double()
    h = case.h
    worst = 0.0
    for b in range(3):
        ub = us[b]
        lap = torch.zeros_like(ub)
        for ax, periodic in ((2, True), (1, True), (0, False)):
            upn = torch.roll(ub, -1, dims=ax)
            dnn = torch.roll(ub, 1, dims=ax)
            if not periodic:
                upn[-1] = -ub[-1]
                dnn[0] = -ub[0]
            lap += (upn - 2.0 * ub + dnn) / (h * h)
        # grad P along b: mean of the face gradients, zero on wall faces
        axb = (2, 1, 0)[b]
        gp = (torch.roll(Pd, -1, dims=axb) - Pd) / h
        gm = (Pd - torch.roll(Pd, 1, dims=axb)) / h
        if b == 2:
            gp[-1] = 0.0
            gm[0] = 0.0
        gP = 0.5 * (gp + gm)
        rhs = rhs_u[b].double() + dt * (-alpha * lapnu[b].double() + 2.0 * alpha * gP)
        res = (ub - beta * lap - rhs).abs().max().item()
        worst = max(worst, res / rhs.abs().max().item())
    print(f"bed: Helmholtz relative residual {worst:.3e}", flush=True)
    assert worst <= 1e-5
    plan.close()
