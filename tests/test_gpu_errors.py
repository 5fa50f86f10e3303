"""Failure handling of the C ABI on the device: a compute call before the
markers are attached (ESTATE), pair and wall lists over their capacity
(deferred ECAPACITY with the full counts still written), cell grids
beyond the cell capacity and radii above radius_max, and parameters or
tiles the plan cannot take (EINVAL).  Every case ends normally on the
device."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2109_03972_amd import ibmx, synth
from _util import dev_case, require_gpu

pytestmark = pytest.mark.gpu


def _small():
    return synth.small_case(401, n=(40, 36, 44), periodic=(1, 1, 0), n_iter=2, touch=0.5)


def test_forcing_before_set_markers_is_estate():
    import torch
    case = _small()
    D = dev_case(case, "f64")
    plan = ibmx.Plan.from_case(case, "f64")
    S = torch.empty((3, case.np_), dtype=torch.float64, device=D["u"].device)
    L = ibmx.lib()
    st = L.ibmx_forcing(plan.handle, D["u"].data_ptr(), D["f"].data_ptr(), D["xp"].data_ptr(),
                        D["up"].data_ptr(), D["wp"].data_ptr(), None, S.data_ptr(),
                        S.data_ptr(), None, None)
    assert st == ibmx.ESTATE
    with pytest.raises(ibmx.IbmxError) as ei:
        plan.forcing_backward(D["u"], D["xp"], D["up"], D["wp"], None, D["f"], None, None, None)
    assert ei.value.code == ibmx.ESTATE
    plan.close()


def test_list_capacity_exceeded_reports_and_counts():
    """Pair and wall capacities below the list lengths: ECAPACITY from the
    plan's status, the counts are the full lengths, the entries that fit
    are the first ones of the canonical order."""
    import torch
    case = synth.make_case("bidisperse_bed_256x256x512", lazy_field=True)
    ref = oracle.pairs(case)
    npairs, nwall = ref["pairs"].shape[1], ref["walls"].shape[1]
    assert npairs >= 3 and nwall >= 1, (npairs, nwall)
    D = dev_case(case, "f64")
    plan = ibmx.Plan.from_case(case, "f64")
    plan.set_markers(D["body"], D["dV"])
    for pc, wc in ((npairs - 2, nwall), (npairs, 0), (1, 1)):
        res = plan.pairs(D["xp"], D["radius"], D["mass"], D["up"], D["wp"], pair_cap=max(pc, 1)
                         if pc else 1, wall_cap=max(wc, 1) if wc else 1)
        st = plan.status()
        torch.cuda.synchronize()
        cnt = res["counts"].cpu().numpy().tolist()
        print(f"caps ({pc}, {wc}): status {st}, counts {cnt}", flush=True)
        assert cnt == [npairs, nwall]
        over = npairs > max(pc, 1) or nwall > max(wc, 1)
        assert st == (ibmx.ECAPACITY if over else ibmx.OK)
        k = min(npairs, max(pc, 1))
        assert np.array_equal(res["pairs"][:, :k].cpu().numpy(), ref["pairs"][:, :k])
    # the status is cleared once read; a call within capacity is clean again
    res = plan.pairs(D["xp"], D["radius"], D["mass"], D["up"], D["wp"])
    assert plan.status() == ibmx.OK
    plan.close()


def test_cell_capacity_and_bad_radius():
    import torch
    case = _small()
    D = dev_case(case, "f64")
    plan = ibmx.Plan.from_case(case, "f64")
    plan.set_markers(D["body"], D["dV"])
    with pytest.raises(ibmx.IbmxError) as ei:
        plan.pairs(D["xp"], D["radius"], D["mass"], D["up"], D["wp"], cell_cap=2)
    assert ei.value.code == ibmx.ECAPACITY
    with pytest.raises(ibmx.IbmxError) as ei:
        plan.pairs(D["xp"], D["radius"], D["mass"], D["up"], D["wp"], radius_max=0.0)
    assert ei.value.code == ibmx.EINVAL
    # a radius above radius_max is a deferred EINVAL
    plan.pairs(D["xp"], D["radius"], D["mass"], D["up"], D["wp"],
               radius_max=float(case.radius.max()) * 0.5)
    assert plan.status() == ibmx.EINVAL
    torch.cuda.synchronize()
    plan.close()


def test_params_and_tiles_the_plan_cannot_take():
    case = _small()
    plan = ibmx.Plan.from_case(case, "f32")
    prm = dict(case.params)
    with pytest.raises(ibmx.IbmxError) as ei:
        plan.set_params(dict(prm, n_iter=int(prm["n_iter"]) + 1))   # above the plan's n_iter
    assert ei.value.code == ibmx.EINVAL
    for bad in (dict(c=0.0), dict(n_iter=0), dict(disable_mode=1, gap_cut=1.0)):
        with pytest.raises(ibmx.IbmxError) as ei:
            plan.set_params(dict(prm, **bad))
        assert ei.value.code == ibmx.EINVAL
    for tiles in ((3, 16, 16), (16, 65, 16), (61, 8, 8)):
        with pytest.raises(ibmx.IbmxError) as ei:
            plan.set_tiles(*tiles)
        assert ei.value.code == ibmx.EINVAL
    # the plan still runs with its earlier settings
    assert plan.stats()["tile"] == (16, 16, 8)
    plan.close()
