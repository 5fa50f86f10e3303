"""Parity of the HIP forcing loop (ibmx_forcing, through the C ABI) with the
FP64 CPU oracle: FP64 to 1e-12, FP32 to 1e-5 on interpolated velocities and
1e-4 on the spread field and the updated velocity (normwise relative)."""
import numpy as np
import pytest

import oracle
from paper_2109_03972_amd import synth
from tests._util import gpu_forcing, rel_err

pytestmark = pytest.mark.gpu


def _mask_for(case):
    if case.params.get("disable_mode", 0) == 0:
        return None
    return oracle.marker_mask(case, oracle.pairs(case))


def _compare(case, precision, mask=None, want_U=True, tol=None, params=None):
    prm = dict(case.params if params is None else params)
    ref = oracle.forcing(case, mask=mask, n_iter=prm["n_iter"], c=prm["c"],
                         kernel=prm.get("kernel", 3), want_U=want_U)
    got = gpu_forcing(case, precision, mask=mask, want_U=want_U, params=prm)
    assert got["status"] == 0
    errs = {k: rel_err(got[k], ref[k]) for k in ("u", "f_tot", "S", "T", "resid")}
    if want_U:
        act = np.ones(case.nm, dtype=bool) if mask is None else mask.astype(bool)
        errs["U"] = rel_err(got["U"][:, :, act], ref["U"][:, :, act])
    print(case.name, precision, {k: f"{v:.2e}" for k, v in errs.items()})
    if precision == "f64":
        for k, v in errs.items():
            assert v <= 1e-12, (k, v)
    else:
        assert errs["U"] <= 1e-5
        for k in ("u", "f_tot"):
            assert errs[k] <= 1e-4, (k, errs[k])
        for k in ("S", "T", "resid"):
            assert errs[k] <= 1e-4, (k, errs[k])
    return got, ref


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_single_sphere(precision):
    c = synth.make_case("single_sphere_64")
    _compare(c, precision)
    prm = dict(c.params, n_iter=3)
    _compare(c, precision, params=prm)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_suspension_128(precision):
    c = synth.make_case("suspension_128")
    _compare(c, precision, mask=_mask_for(c))


@pytest.mark.parametrize("seed,periodic,kernel", [
    (101, (1, 1, 0), 3), (102, (1, 1, 1), 3), (103, (0, 1, 0), 3), (104, (1, 1, 0), 4),
    (105, (1, 1, 1), 4), (110, (0, 0, 0), 3), (111, (0, 0, 1), 4),
])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_small_ragged_cases(seed, periodic, kernel, precision):
    """Grids that are not multiples of any tile edge, walls on one or two
    axes, spheres crossing periodic seams, both delta kernels."""
    c = synth.small_case(seed, n=(41, 37, 45), periodic=periodic,
                         diameters=(12.0, 9.0, 7.0, 10.0, 11.0, 8.5), n_iter=3, touch=0.3)
    if kernel == 4:
        c.params.update(kernel=4, eps_sep=2.0, lub_C=4.0, gap_cut=4.0)
    mask = _mask_for(c)
    _compare(c, precision, mask=mask)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_maximum_passes(precision):
    """The largest pass count a plan takes (64): per-pass amplitude records,
    residual slots and sums at their full size, on a ragged grid with walls."""
    c = synth.small_case(106, n=(41, 37, 45), periodic=(1, 1, 0),
                         diameters=(12.0, 9.0, 7.0, 10.0), n_iter=64, touch=0.3)
    got, ref = _compare(c, precision, mask=_mask_for(c))
    assert got["resid"].shape == (65,)
    # the passes keep reducing the residual (Sec. 2.2.2)
    assert np.all(np.diff(ref["resid"]) <= 0.0)


def test_no_mask_and_all_masked():
    c = synth.small_case(106, n=(33, 35, 31), periodic=(1, 1, 1), disable_mode=0, n_iter=2)
    _compare(c, "f64")
    zero = np.zeros(c.nm, dtype=np.uint8)
    got = gpu_forcing(c, "f64", mask=zero)
    assert np.array_equal(got["u"], c.u0)
    assert np.abs(got["f_tot"]).max() == 0.0 and np.abs(got["S"]).max() == 0.0


def test_wall_crossing_support_is_reported():
    """A marker whose delta support leaves the grid through a wall is
    skipped and reported as EDOMAIN by ibmx_plan_status."""
    c = synth.small_case(107, n=(32, 32, 40), periodic=(1, 1, 0), disable_mode=0, n_iter=1)
    c.xp[2, 0] = c.radius[0] + 0.2      # its lowest markers sit 0.2h from the wall
    got = gpu_forcing(c, "f64")
    assert got["status"] == -2


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_no_particles(precision):
    """A plan with no particles: the forcing call leaves u and f_tot alone
    and the residuals are zero; the pair pass finds nothing."""
    import torch
    from paper_2109_03972_amd import ibmx
    from tests._util import require_gpu
    dev = require_gpu()
    c = synth.small_case(108, n=(32, 32, 36), periodic=(1, 1, 0), n_iter=2)
    empty = synth.Case(name="empty", n=c.n, h=c.h, origin=c.origin, periodic=c.periodic,
                       xp=np.zeros((3, 0)), up=np.zeros((3, 0)), wp=np.zeros((3, 0)),
                       radius=np.zeros(0), mass=np.zeros(0), moff=np.zeros(1, dtype=np.int32),
                       body=np.zeros((3, 0)), dV=np.zeros(0), u0=c.u0, params=c.params)
    T = torch.float64 if precision == "f64" else torch.float32
    f64 = torch.float64
    plan = ibmx.Plan.from_case(empty, precision)
    z = torch.zeros((3, 0), dtype=f64, device=dev)
    plan.set_markers(z, torch.zeros(0, dtype=f64, device=dev))
    u = torch.as_tensor(c.u0, device=dev).to(T).contiguous()
    u_before = u.clone()
    f = torch.zeros_like(u)
    resid = torch.full((3,), 7.0, dtype=f64, device=dev)
    S, Tq = plan.forcing(u, f, z, z, z, resid=resid)
    plan.check("no particles")
    assert torch.equal(u, u_before) and not f.any()
    assert S.shape == (3, 0) and Tq.shape == (3, 0)
    assert not resid.any()
    res = plan.pairs(z, torch.zeros(0, dtype=f64, device=dev), torch.zeros(0, dtype=f64, device=dev),
                     z, z, radius_max=1.0)
    plan.check("no particles pairs")
    assert res["counts"].cpu().tolist() == [0, 0]


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_particles_without_markers(precision):
    """Particles whose marker range is empty (marker_offset repeats) between
    particles that have markers: their sums are zero, the rest matches the
    oracle."""
    c = synth.small_case(109, n=(40, 36, 44), periodic=(1, 1, 1), n_iter=2)
    keep = [p for p in range(c.np_) if p % 2 == 0]
    assert 0 < len(keep) < c.np_
    segs = [np.arange(c.moff[p], c.moff[p + 1]) if p in keep else np.arange(0)
            for p in range(c.np_)]
    moff = np.zeros(c.np_ + 1, dtype=np.int32)
    moff[1:] = np.cumsum([len(g) for g in segs])
    idx = np.concatenate(segs)
    holed = synth.Case(name="holed", n=c.n, h=c.h, origin=c.origin, periodic=c.periodic,
                       xp=c.xp, up=c.up, wp=c.wp, radius=c.radius, mass=c.mass, moff=moff,
                       body=np.ascontiguousarray(c.body[:, idx]), dV=c.dV, u0=c.u0,
                       params=dict(c.params, disable_mode=0))
    got, ref = _compare(holed, precision)
    empty = [p for p in range(c.np_) if p not in keep]
    assert not np.any(got["S"][:, empty]) and not np.any(got["T"][:, empty])


@pytest.mark.parametrize("name", ["suspension_128", "small"])
def test_f32_arithmetic_and_end_to_end_errors(name):
    """FP32 forward errors of every output measured two ways:
    (i) against the oracle on the FP32-rounded velocity the kernels start
    from (the arithmetic error of the FP32 path) and (ii) against the oracle
    on the FP64 inputs (end to end, including the rounding of u0).  Both
    are held to the FP32 tolerances; (i) is the smaller."""
    if name == "small":
        c = synth.small_case(109, n=(41, 37, 45), periodic=(1, 1, 0), n_iter=3, touch=0.3)
    else:
        c = synth.make_case(name)
    mask = _mask_for(c)
    u32 = c.u0.astype(np.float32).astype(np.float64)
    ref_e2e = oracle.forcing(c, mask=mask, want_U=True)
    ref_ari = oracle.forcing(c, u0=u32, mask=mask, want_U=True)
    got = gpu_forcing(c, "f32", mask=mask, want_U=True)
    assert got["status"] == 0
    act = np.ones(c.nm, dtype=bool) if mask is None else mask.astype(bool)
    out = {}
    for k in ("U", "u", "f_tot", "S", "T", "resid"):
        g = got[k][:, :, act] if k == "U" else got[k]
        ra = ref_ari[k][:, :, act] if k == "U" else ref_ari[k]
        re = ref_e2e[k][:, :, act] if k == "U" else ref_e2e[k]
        out[k] = (rel_err(g, ra), rel_err(g, re))
        print(f"{name} f32 {k}: arithmetic {out[k][0]:.2e}  end-to-end {out[k][1]:.2e}",
              flush=True)
    assert out["U"][0] <= 1e-5 and out["U"][1] <= 1e-5
    for k in ("u", "f_tot", "S", "T", "resid"):
        assert out[k][0] <= 1e-4 and out[k][1] <= 1e-4, (k, out[k])
