"""Full-size checks of the forcing loop in the launch configuration the
benchmark times (its tuned tiles, 32x8x8 for FP32 and 16x16x8 for FP64, 256
threads per tile; eager launches and the call replayed as a HIP graph).

* bidisperse_bed_256x256x512: element-wise parity with the oracle on every
  output (the oracle finishes it in seconds).
* polydisperse_bed_512 (the benchmark's workload): element-wise parity with
  the oracle's five passes over the whole bed (about 40 s on one core), and
  the properties that hold at any size: u^n - u^0 = c f_tot node by node,
  total force on the grid equals the sum of the particle sums (Sec. 2.2.2
  spreading conserves the marker force), and the residual does not increase
  over the passes."""
import numpy as np
import pytest

import oracle
from paper_2109_03972_amd import synth
from _util import rel_err, require_gpu

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

BENCH_TILE = {"f32": (32, 8, 8), "f64": (32, 8, 8)}
TOL = {"f64": dict(U=1e-12, u=1e-12, f_tot=1e-12, S=1e-12, T=1e-12, resid=1e-12),
       "f32": dict(U=1e-5, u=1e-4, f_tot=1e-4, S=1e-4, T=1e-4, resid=1e-4)}


def _gpu_run(case, precision, u0_dev64, mask_dev, want_U, graph=True):
    import torch
    from paper_2109_03972_amd import ibmx
    dev = require_gpu()
    f64 = torch.float64
    T = f64 if precision == "f64" else torch.float32
    D = {k: torch.as_tensor(getattr(case, k), dtype=f64).to(dev).contiguous()
         for k in ("xp", "up", "wp", "body", "dV")}
    plan = ibmx.Plan.from_case(case, precision)
    plan.set_markers(D["body"], D["dV"])
    plan.set_tiles(*BENCH_TILE[precision])
    n_iter = int(case.params["n_iter"])
    u = u0_dev64.to(T).clone()   # the call updates u in place; keep u0
    f = torch.zeros_like(u)
    resid = torch.zeros(n_iter + 1, dtype=f64, device=dev)
    U = torch.zeros((n_iter, 3, case.nm), dtype=T, device=dev) if want_U else None
    S, Tq = plan.forcing(u, f, D["xp"], D["up"], D["wp"], mask=mask_dev, resid=resid,
                         U_debug=U, graph=graph)
    plan.check("full-size forcing")
    torch.cuda.synchronize()
    return plan, u, f, S, Tq, resid, U


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_bidisperse_bed_full_parity(precision):
    import torch
    dev = require_gpu()
    case = synth.make_case("bidisperse_bed_256x256x512")
    mask = oracle.marker_mask(case, oracle.pairs(case))
    print(f"bidisperse bed: nm={case.nm} active={int(mask.sum())}", flush=True)
    ref = oracle.forcing(case, mask=mask, want_U=True)
    u0 = torch.as_tensor(case.u0).to(dev)
    _, u, f, S, Tq, resid, U = _gpu_run(case, precision, u0, torch.as_tensor(mask).to(dev), True)
    act = mask.astype(bool)
    got = dict(u=u.double().cpu().numpy(), f_tot=f.double().cpu().numpy(), S=S.cpu().numpy(),
               T=Tq.cpu().numpy(), resid=resid.cpu().numpy(),
               U=U.double().cpu().numpy()[:, :, act])
    ref["U"] = ref["U"][:, :, act]
    for k, t in TOL[precision].items():
        e = rel_err(got[k], ref[k])
        print(f"{precision} {k}: {e:.3e}", flush=True)
        assert e <= t, f"{precision} {k}: {e:.3e} > {t}"


@pytest.fixture(scope="module")
def bidisperse_kernel4():
    """The bidisperse bed with the four-point delta (Sec. 2.2.3); its wider
    support needs markers 2h from the walls, so eps_sep = 2h (and the pair
    cut-off 2 eps_sep for the disable rule)."""
    case = synth.make_case("bidisperse_bed_256x256x512")
    case.params = dict(case.params, kernel=4, eps_sep=2.0, gap_cut=4.0)
    mask = oracle.marker_mask(case, oracle.pairs(case))
    ref = oracle.forcing(case, mask=mask, want_U=True)
    return case, mask, ref


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_bidisperse_bed_kernel4_full_parity(precision, bidisperse_kernel4):
    """Every output of the four-point path on a full bed (1.47M markers, five
    passes) in the bench's tiles, element by element against the oracle."""
    import torch
    dev = require_gpu()
    case, mask, ref = bidisperse_kernel4
    print(f"bidisperse bed, four-point delta: active={int(mask.sum())}", flush=True)
    u0 = torch.as_tensor(case.u0).to(dev)
    _, u, f, S, Tq, resid, U = _gpu_run(case, precision, u0, torch.as_tensor(mask).to(dev), True)
    act = mask.astype(bool)
    got = dict(u=u.double().cpu().numpy(), f_tot=f.double().cpu().numpy(), S=S.cpu().numpy(),
               T=Tq.cpu().numpy(), resid=resid.cpu().numpy(),
               U=U.double().cpu().numpy()[:, :, act])
    want = dict(ref, U=ref["U"][:, :, act])
    for k, t in TOL[precision].items():
        e = rel_err(got[k], want[k])
        print(f"{precision} kernel 4 {k}: {e:.3e}", flush=True)
        assert e <= t, f"{precision} kernel 4 {k}: {e:.3e} > {t}"


@pytest.fixture(scope="module")
def bed512():
    import torch
    dev = require_gpu()
    case = synth.make_case("polydisperse_bed_512", lazy_field=True)
    mask = oracle.marker_mask(case, oracle.pairs(case))
    u0 = case.field(device=dev)
    return case, mask, u0


@pytest.fixture(scope="module")
def bed512_ref(bed512):
    """The oracle's five passes over the whole bed (about 40 s on one core)."""
    case, mask, u0 = bed512
    print(f"bed512 oracle: nm={case.nm} active={int(mask.sum())}", flush=True)
    return oracle.forcing(case, u0=u0.cpu().numpy(), mask=mask, want_U=True)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_polydisperse_bed_full_parity(bed512, bed512_ref, precision):
    """Every output of the benchmark's workload against the oracle, element
    by element, in the benchmark's launch configuration: u and f_tot at every
    node, S and T of all 20,000 particles, the residual of every pass and the
    interpolated velocity of every active marker in every pass; plus the
    properties that hold at any size (u^n - u^0 = c f_tot node by node, the
    grid's total force equals the sum of the particle sums, residuals do not
    increase)."""
    import torch
    case, mask, u0 = bed512
    ref = bed512_ref
    c = float(case.params["c"])
    h3 = case.h ** 3
    mask_dev = torch.as_tensor(mask).to(u0.device)
    _, u, f, S, Tq, resid, U = _gpu_run(case, precision, u0, mask_dev, True)
    print(f"bed512 {precision}: nm={case.nm} active={int(mask.sum())}", flush=True)
    act = mask.astype(bool)
    got = dict(S=S.cpu().numpy(), T=Tq.cpu().numpy(), resid=resid.cpu().numpy())
    errs = {k: rel_err(got[k], ref[k]) for k in got}
    Ug = U.double().cpu().numpy()
    errs["U"] = max(rel_err(Ug[m][:, act], ref["U"][m][:, act]) for m in range(Ug.shape[0]))
    del Ug
    for k, g in (("u", u), ("f_tot", f)):
        a = g.double().cpu().numpy()
        errs[k] = rel_err(a, ref[k])
        del a
    for k, t in TOL[precision].items():
        print(f"bed512 {precision} {k}: {errs[k]:.3e}", flush=True)
        assert errs[k] <= t, f"{precision} {k}: {errs[k]:.3e} > {t}"

    # properties at any size
    du = (u.double() - u0.to(u.dtype).double())
    cf = c * f.double()
    e = float((du - cf).abs().max() / cf.abs().max())
    print(f"{precision} u^n - u^0 vs c f_tot: {e:.3e}", flush=True)
    assert e <= (1e-12 if precision == "f64" else 1e-4)
    tot_grid = (f.double().sum(dim=(1, 2, 3)) * h3).cpu().numpy()
    tot_part = S.sum(dim=1).cpu().numpy()
    scale = float(S.abs().sum())
    e = float(np.abs(tot_grid - tot_part).max() / scale)
    print(f"{precision} force conservation: {e:.3e}", flush=True)
    assert e <= (1e-12 if precision == "f64" else 1e-5)
    r = resid.cpu().numpy()
    assert np.all(np.diff(r) <= 1e-12 * r[0])

    # the eager launches the benchmark's headline times give the same bits
    _, u_e, f_e, S_e, T_e, resid_e, _ = _gpu_run(case, precision, u0, mask_dev, False,
                                                 graph=False)
    for k, a, b in (("u", u_e, u), ("f_tot", f_e, f), ("S", S_e, S), ("T", T_e, Tq),
                    ("resid", resid_e, resid)):
        assert torch.equal(a, b), f"{precision} eager vs graph: {k}"


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_polydisperse_bed_particle_integrals(bed512, precision):
    """Particle integrals of the 512^3 bed against the oracle, all 20000
    particles."""
    import torch
    from paper_2109_03972_amd import ibmx
    case, _, u0 = bed512
    f64 = torch.float64
    T = f64 if precision == "f64" else torch.float32
    plan = ibmx.Plan.from_case(case, precision)
    dev = u0.device
    xp = torch.as_tensor(case.xp, dtype=f64).to(dev).contiguous()
    rad = torch.as_tensor(case.radius, dtype=f64).to(dev).contiguous()
    u = u0.to(T).contiguous()
    Iu, Ir = plan.particle_integrals(u, xp, rad)
    plan.check("bed integrals")
    u_np = u.double().cpu().numpy()
    ref = oracle.particle_integrals(case, u=u_np)
    del u_np
    for k, got in (("Iu", Iu), ("Ir", Ir)):
        e = rel_err(got.cpu().numpy(), ref[k])
        print(f"bed512 {precision} {k}: {e:.2e}", flush=True)
        assert e <= 1e-11
