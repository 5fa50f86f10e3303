"""Parity of the particle integrals (level-set volume fraction, Sec. 2.2.9)
and of the grid mean (Sec. 2.2.4) with the oracle."""
import numpy as np
import pytest

import oracle
from paper_2109_03972_amd import synth
from _util import dev_case, rel_err, require_gpu

pytestmark = pytest.mark.gpu


def _gpu_integrals(case, precision, u=None, want_alpha=False):
    import torch
    from paper_2109_03972_amd import ibmx
    require_gpu()
    D = dev_case(case, precision, u0=u)
    plan = ibmx.Plan.from_case(case, precision)
    alpha = None
    if want_alpha:
        alpha = torch.full(D["u"].shape[1:], 3.0, dtype=D["u"].dtype, device=D["u"].device)
    Iu, Ir = plan.particle_integrals(D["u"], D["xp"], D["radius"], alpha=alpha)
    plan.check("particle integrals")
    out = dict(Iu=Iu.cpu().numpy(), Ir=Ir.cpu().numpy())
    if want_alpha:
        out["alpha"] = alpha.double().cpu().numpy()
    return out


@pytest.mark.parametrize("per", [(1, 1, 1), (1, 1, 0), (0, 1, 0)])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_integrals_small(per, precision):
    case = synth.small_case(301, n=(41, 36, 44), periodic=per, touch=0.4)
    u = case.u0
    if precision == "f32":
        u = u.astype(np.float32).astype(np.float64)   # the values the kernel reads
    ref = oracle.particle_integrals(case, u=u, want_alpha=True)
    got = _gpu_integrals(case, precision, u=u, want_alpha=True)
    tol = 1e-12 if precision == "f64" else 1e-11
    for k in ("Iu", "Ir"):
        e = rel_err(got[k], ref[k])
        print(precision, per, k, f"{e:.2e}", flush=True)
        assert e <= tol, (k, e)
    atol = 1e-13 if precision == "f64" else 2e-7   # alpha stored in the grid type
    np.testing.assert_allclose(got["alpha"], ref["alpha"], rtol=0, atol=atol)


@pytest.mark.parametrize("name", ["suspension_128", "bidisperse_bed_256x256x512"])
def test_integrals_workloads(name):
    case = synth.make_case(name)
    ref = oracle.particle_integrals(case)
    for precision, tol in (("f64", 1e-12), ("f32", 1e-6)):
        got = _gpu_integrals(case, precision)
        for k in ("Iu", "Ir"):
            e = rel_err(got[k], ref[k])
            print(name, precision, k, f"{e:.2e}", flush=True)
            assert e <= tol, (precision, k, e)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_grid_mean_of_the_ibm_force(precision):
    """The mean of f_tot after a forcing call: against the oracle's mean of
    the same field and against the particle sums (the spreading conserves
    the marker force: sum_x f h^3 = sum_p S_p)."""
    import torch
    from paper_2109_03972_amd import ibmx
    dev = require_gpu()
    case = synth.small_case(302, n=(40, 36, 44), periodic=(1, 1, 1), n_iter=2, touch=0.4)
    mask = oracle.marker_mask(case, oracle.pairs(case))
    D = dev_case(case, precision)
    plan = ibmx.Plan.from_case(case, precision)
    plan.set_markers(D["body"], D["dV"])
    S, _ = plan.forcing(D["u"], D["f"], D["xp"], D["up"], D["wp"],
                        mask=torch.as_tensor(mask).to(dev))
    mean = plan.grid_mean(D["f"])
    plan.check("grid mean")
    f = D["f"].double().cpu().numpy()
    ref = oracle.grid_mean(case, f)
    got = mean.cpu().numpy()
    assert rel_err(got, ref) <= 1e-12
    nodes = case.n[0] * case.n[1] * case.n[2]
    cons = S.sum(dim=1).cpu().numpy() / (nodes * case.h ** 3)
    tol = 1e-10 if precision == "f64" else 1e-5
    assert np.abs(got - cons).max() <= tol * np.abs(S.cpu().numpy()).sum() / nodes
