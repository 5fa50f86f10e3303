"""Parity of the HIP pair pass (ibmx_pairs, through the C ABI) with the FP64
oracle: cell, pair and wall lists and the marker mask bit-exact; gaps,
forces, torques and spring history to 1e-12."""
import numpy as np
import pytest

import oracle
from paper_2109_03972_amd import ibmx, synth
from tests._util import dev_case, rel_err

pytestmark = pytest.mark.gpu


def _gpu_pairs(case, prev=None, plan=None):
    import torch
    D = dev_case(case, "f64")
    if plan is None:
        plan = ibmx.Plan.from_case(case, "f64")
        plan.set_markers(D["body"], D["dV"])
    res = plan.pairs(D["xp"], D["radius"], D["mass"], D["up"], D["wp"], prev=prev)
    st = plan.status()
    torch.cuda.synchronize()
    t = ibmx.trim_pairs(res)
    ncell = None
    out = dict(status=st, pairs=t["pairs"].cpu().numpy(), gap=t["gap"].cpu().numpy(),
               hist=t["hist"].cpu().numpy(), walls=t["walls"].cpu().numpy(),
               wgap=t["wgap"].cpu().numpy(), whist=t["whist"].cpu().numpy(),
               Fc=res["Fc"].cpu().numpy(), Tc=res["Tc"].cpu().numpy(),
               mask=res["mask"][:case.nm].cpu().numpy(),
               cell_start=res["cell_start"].cpu().numpy(),
               cell_particles=res["cell_particles"][:case.np_].cpu().numpy(),
               dev=dict(pairs=t["pairs"].contiguous(), hist=t["hist"].contiguous(),
                        walls=t["walls"].contiguous(), whist=t["whist"].contiguous()),
               plan=plan)
    return out


def _check(case, got, prev_host=None, ftol=1e-12):
    ref_l = oracle.pairs(case)
    assert got["status"] == 0
    assert np.array_equal(got["pairs"], ref_l["pairs"])
    assert np.array_equal(got["walls"], ref_l["walls"])
    assert rel_err(got["gap"], ref_l["gap"]) <= 1e-12
    assert rel_err(got["wgap"], ref_l["wgap"]) <= 1e-12
    cl = oracle.cell_list(case)
    ncell = len(cl["cell_start"]) - 1
    assert np.array_equal(got["cell_start"][:ncell + 1], cl["cell_start"])
    assert np.array_equal(got["cell_particles"], cl["cell_particles"])
    ref_f = oracle.pair_forces(case, ref_l, prev=prev_host)
    for k in ("Fc", "Tc"):
        assert rel_err(got[k], ref_f[k]) <= ftol, k
    for k in ("hist", "whist"):
        assert got[k].shape[0] == 4
        assert rel_err(got[k], ref_f[k]) <= ftol, k
    ref_m = oracle.marker_mask(case, ref_l)
    assert np.array_equal(got["mask"], ref_m)
    return ref_l, ref_f


def test_exact_regime_boundaries():
    """Gaps exactly on the regime boundaries (Sec. 2.2.5-2.2.7, reading
    c-13 and the disable threshold): touching spheres (gap 0: lubrication at
    zeta_min), a gap of exactly eps_sep (no force), exactly 2 eps_sep (the
    list's cut-off, strict: not listed), a slight overlap, and the same
    against a wall (gap 0 and eps_sep).  Binary-exact positions make every
    gap exact in FP64 on both sides."""
    R = 4.0
    rows = [(10.0, 18.0), (10.0, 19.5), (10.0, 21.0), (10.0, 17.75)]   # x pairs, gap 0 / 1.5 / 3 / -0.25
    xs, ys, zs = [], [], []
    for k, (a, b) in enumerate(rows):
        for x in (a, b):
            xs.append(x)
            ys.append(8.0 + 16.0 * k)
            zs.append(32.0)
    for k, z in enumerate((R, R + 1.5)):                                # wall gap 0 and eps_sep
        xs.append(40.0)
        ys.append(8.0 + 16.0 * k)
        zs.append(z)
    xp = np.array([xs, ys, zs])
    npart = xp.shape[1]
    diam = np.full(npart, 2.0 * R)
    rng = np.random.Generator(np.random.PCG64(211))
    moff, body, dV = synth.build_markers(diam, 1.0, rng)
    prm = synth.default_params()
    prm.update(disable_mode=1, eps_sep=1.5, gap_cut=3.0)
    case = synth.Case(name="boundaries", n=(64, 64, 64), h=1.0, origin=(0.0, 0.0, 0.0),
                      periodic=(1, 1, 0), xp=xp, up=rng.normal(0.0, 0.1, (3, npart)),
                      wp=rng.normal(0.0, 0.05, (3, npart)), radius=0.5 * diam,
                      mass=1.3 * np.pi / 6.0 * diam ** 3, moff=moff, body=body, dV=dV,
                      u0=None, params=prm)
    got = _gpu_pairs(case)
    ref_l, ref_f = _check(case, got)
    assert got["pairs"].T.tolist() == [[0, 1], [2, 3], [6, 7]]
    assert got["gap"].tolist() == [0.0, 1.5, -0.25]
    assert got["walls"].T.tolist() == [[8, 4], [9, 4]]
    assert got["wgap"].tolist() == [0.0, 1.5]
    # forces on the touching pair and the wall contact at gap 0 only
    # (the overlap also has its contact force); none at exactly eps_sep
    assert np.all(got["Fc"][:, [2, 3, 9]] == 0.0)
    assert np.any(got["Fc"][:, [0, 1, 6, 7, 8]] != 0.0, axis=0).all()


def test_half_box_separation():
    """Two spheres exactly half a periodic box apart along x, and a pair
    across the x seam: the minimum image (reading c-17) keeps +L/2 as it
    is, so both sides list the same pair with the same gap."""
    R = 14.0
    xp = np.array([[0.5, 32.5, 62.0, 2.5], [16.0, 16.0, 48.0, 48.0], [32.0, 32.0, 32.0, 32.0]])
    diam = np.array([2.0 * R, 2.0 * R, 4.0, 4.0])
    npart = xp.shape[1]
    rng = np.random.Generator(np.random.PCG64(212))
    moff, body, dV = synth.build_markers(diam, 1.0, rng)
    prm = synth.default_params()
    prm.update(disable_mode=1, eps_sep=1.5, gap_cut=5.0)
    case = synth.Case(name="half_box", n=(64, 64, 64), h=1.0, origin=(0.0, 0.0, 0.0),
                      periodic=(1, 1, 1), xp=xp, up=rng.normal(0.0, 0.1, (3, npart)),
                      wp=rng.normal(0.0, 0.05, (3, npart)), radius=0.5 * diam,
                      mass=1.3 * np.pi / 6.0 * diam ** 3, moff=moff, body=body, dV=dV,
                      u0=None, params=prm)
    got = _gpu_pairs(case)
    _check(case, got)
    assert got["pairs"].T.tolist() == [[0, 1], [2, 3]]
    assert got["gap"].tolist() == [32.0 - 2.0 * R, 4.5 - 4.0]


@pytest.mark.parametrize("name", ["suspension_128", "bidisperse_bed_256x256x512",
                                  "polydisperse_bed_512"])
def test_workload_pairs(name):
    c = synth.make_case(name, lazy_field=True)
    got = _gpu_pairs(c)
    ref_l, ref_f = _check(c, got)
    print(name, "pairs", ref_l["pairs"].shape[1], "walls", ref_l["walls"].shape[1],
          "contacts", int((ref_l["gap"] < 0).sum()), "masked", int((got["mask"] == 0).sum()))


def test_history_second_call():
    """A second call keyed by the first call's lists carries the tangential
    springs of persisting contacts."""
    c = synth.small_case(201, n=(48, 48, 48), periodic=(1, 1, 0),
                         diameters=(12.0, 9.0, 7.0, 10.0, 8.0, 11.0, 9.5, 6.0), touch=0.7,
                         min_gap=0.1)
    rng = np.random.default_rng(4)
    c.up = rng.normal(0, 0.3, c.up.shape)
    c.wp = rng.normal(0, 0.2, c.wp.shape)
    first = _gpu_pairs(c)
    ref_l, ref_f = _check(c, first)
    assert np.any(ref_l["gap"] < 0)
    c.xp = c.xp + rng.normal(0, 0.003, c.xp.shape)
    prev_host = dict(pairs=ref_l["pairs"], hist=ref_f["hist"], walls=ref_l["walls"],
                     whist=ref_f["whist"])
    second = _gpu_pairs(c, prev=first["dev"], plan=first["plan"])
    _check(c, second, prev_host=prev_host)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_disable_modes(mode):
    c = synth.small_case(202, n=(40, 44, 36), periodic=(1, 0, 1),
                         diameters=(12.0, 9.0, 7.0, 10.0, 8.0), touch=0.5, min_gap=0.2)
    c.params["disable_mode"] = mode
    got = _gpu_pairs(c)
    _check(c, got)


def test_small_periodic_box_dedup():
    """Fewer than three cells per axis: neighbour cells are visited once."""
    c = synth.small_case(203, n=(26, 26, 26), periodic=(1, 1, 1), diameters=(8.0, 7.0, 6.0),
                         min_gap=0.5)
    got = _gpu_pairs(c)
    _check(c, got)


@pytest.mark.parametrize("e_dry", [0.97, 0.8])
def test_hertz_model_and_impact_history(e_dry):
    """Hertz normal law with ACTM coefficients (the plan and the oracle
    solve the collision equation independently, to about 1e-13): forces on
    a first call, then a second call that carries the impact speeds."""
    c = synth.small_case(204, n=(48, 48, 48), periodic=(1, 1, 0),
                         diameters=(12.0, 9.0, 7.0, 10.0, 8.0, 11.0, 9.5, 6.0), touch=0.7,
                         min_gap=0.1)
    c.params.update(normal_model=1, e_dry=e_dry, gravity=(0.0, 0.0, -2e-3))
    rng = np.random.default_rng(6)
    c.up = rng.normal(0, 0.05, c.up.shape)
    c.wp = rng.normal(0, 0.02, c.wp.shape)
    first = _gpu_pairs(c)
    ref_l, ref_f = _check(c, first, ftol=1e-11)
    assert np.any(ref_l["gap"] < 0) and np.any(ref_f["hist"][3] > 0)
    c.xp = c.xp + rng.normal(0, 0.003, c.xp.shape)
    prev_host = dict(pairs=ref_l["pairs"], hist=ref_f["hist"], walls=ref_l["walls"],
                     whist=ref_f["whist"])
    second = _gpu_pairs(c, prev=first["dev"], plan=first["plan"])
    _check(c, second, prev_host=prev_host, ftol=1e-11)


@pytest.mark.parametrize("layout", ["one_near_wall", "one_overlapping_wall", "two_apart"])
def test_lists_without_pairs(layout):
    """Degenerate pair passes: a single particle (no pair possible) near or
    pressed into the lower wall, and two particles farther apart than the
    cut-off in a periodic box (empty pair and wall lists, zero forces, no
    marker disabled)."""
    if layout == "two_apart":
        c = synth.small_case(204, n=(48, 40, 44), periodic=(1, 1, 1), diameters=(10.0, 8.0),
                             min_gap=6.0)
    else:
        c = synth.small_case(205, n=(40, 36, 44), periodic=(1, 1, 0), diameters=(10.0,))
        c.xp[2, 0] = float(c.radius[0]) + (0.6 if layout == "one_near_wall" else -0.2)
    got = _gpu_pairs(c)
    ref_l, _ = _check(c, got)
    assert got["pairs"].shape[1] == 0
    if layout == "two_apart":
        assert got["walls"].shape[1] == 0
        assert np.all(got["Fc"] == 0.0) and np.all(got["Tc"] == 0.0)
        assert np.all(got["mask"] == 1)
    else:
        assert got["walls"].shape[1] == 1
        assert (got["wgap"][0] < 0) == (layout == "one_overlapping_wall")


def test_pair_pass_captured_on_its_first_call():
    """With its workspace reserved beforehand (ibmx_plan_reserve), the pair
    pass allocates nothing and synchronises nothing, so its very first call
    can be captured into a HIP graph.  Each replay, with eager work and
    synchronisations between them, gives the oracle's lists and mask and the
    bits of an eager call."""
    import torch
    case = synth.make_case("bidisperse_bed_256x256x512", lazy_field=True)
    D = dev_case(case, "f64")
    npart = case.np_
    caps = dict(pair_cap=16 * npart, wall_cap=2 * npart, cell_cap=1 << 16,
                radius_max=float(case.radius.max()))
    eager_plan = ibmx.Plan.from_case(case, "f64")
    eager_plan.set_markers(D["body"], D["dV"])
    eager = eager_plan.pairs(D["xp"], D["radius"], D["mass"], D["up"], D["wp"], **caps)
    eager_plan.check("eager pairs")
    plan = ibmx.Plan.from_case(case, "f64")
    plan.set_markers(D["body"], D["dV"])
    plan.reserve(caps["pair_cap"], caps["wall_cap"], caps["cell_cap"])
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        res = plan.pairs(D["xp"], D["radius"], D["mass"], D["up"], D["wp"], **caps)
    ref_l = oracle.pairs(case)
    ref_m = oracle.marker_mask(case, ref_l)
    k = ref_l["pairs"].shape[1]
    for rep in range(3):
        for key in ("pairs", "Fc", "mask"):
            res[key].fill_(-1 if key != "mask" else 7)
        g.replay()
        torch.cuda.synchronize()
        assert plan.status() == 0
        _ = (D["xp"] * 2.0).sum().item()     # eager work between replays
        kw = ref_l["walls"].shape[1]
        assert res["counts"].cpu().tolist() == [k, kw]
        assert np.array_equal(res["pairs"][:, :k].cpu().numpy(), ref_l["pairs"])
        assert np.array_equal(res["mask"][:case.nm].cpu().numpy(), ref_m)
        ncell = int(oracle.cell_list(case)["cell_start"].shape[0])
        got = dict(pairs=res["pairs"][:, :k], gap=res["gap"][:k], hist=res["hist"][:, :k],
                   walls=res["walls"][:, :kw], whist=res["whist"][:, :kw], Fc=res["Fc"],
                   Tc=res["Tc"], mask=res["mask"][:case.nm], cell=res["cell_start"][:ncell])
        want = dict(pairs=eager["pairs"][:, :k], gap=eager["gap"][:k], hist=eager["hist"][:, :k],
                    walls=eager["walls"][:, :kw], whist=eager["whist"][:, :kw], Fc=eager["Fc"],
                    Tc=eager["Tc"], mask=eager["mask"][:case.nm],
                    cell=eager["cell_start"][:ncell])
        for key in got:
            assert torch.equal(got[key], want[key]), f"replay {rep} {key}"


def test_unreserved_workspace_is_estate():
    """Without ibmx_plan_reserve the pair pass, the sub-stepping, the adjoint
    and the fluid solves refuse to run (ESTATE) instead of allocating."""
    import ctypes
    import torch
    case = synth.small_case(206, n=(32, 32, 32), periodic=(1, 1, 1), diameters=(8.0, 7.0))
    D = dev_case(case, "f64")
    plan = ibmx.Plan.from_case(case, "f64")
    plan.set_markers(D["body"], D["dV"])
    L = ibmx.lib()
    i32 = torch.int32
    cs = torch.zeros(4096, dtype=i32, device=D["xp"].device)
    cp = torch.zeros(case.np_, dtype=i32, device=D["xp"].device)
    lst = torch.zeros((2, 64), dtype=i32, device=D["xp"].device)
    gap = torch.zeros(64, dtype=torch.float64, device=D["xp"].device)
    hist = torch.zeros((4, 64), dtype=torch.float64, device=D["xp"].device)
    cnt = torch.zeros(2, dtype=i32, device=D["xp"].device)
    F = torch.zeros((3, case.np_), dtype=torch.float64, device=D["xp"].device)
    V = ctypes.c_void_p
    st = L.ibmx_pairs(plan.handle, V(D["xp"].data_ptr()), V(D["radius"].data_ptr()), 4.0,
                      V(D["mass"].data_ptr()), V(D["up"].data_ptr()), V(D["wp"].data_ptr()),
                      0, None, None, 0, None, None, V(cs.data_ptr()), 4096, V(cp.data_ptr()),
                      V(lst.data_ptr()), V(gap.data_ptr()), V(hist.data_ptr()), 64,
                      V(lst.data_ptr()), V(gap.data_ptr()), V(hist.data_ptr()), 64,
                      V(cnt.data_ptr()), V(F.data_ptr()), V(F.data_ptr()), None)
    assert st == ibmx.ESTATE
    st = L.ibmx_particle_substeps(plan.handle, 1.0, 2, V(D["xp"].data_ptr()),
                                  V(D["up"].data_ptr()), V(D["wp"].data_ptr()),
                                  V(D["radius"].data_ptr()), V(D["mass"].data_ptr()), None, None,
                                  V(cnt.data_ptr()), 64, V(lst.data_ptr()), 64,
                                  V(lst.data_ptr()), V(hist.data_ptr()), V(hist.data_ptr()),
                                  None, None)
    assert st == ibmx.ESTATE
    u = torch.zeros((3, 32, 32, 32), dtype=torch.float64, device=D["xp"].device)
    P = torch.zeros((32, 32, 32), dtype=torch.float64, device=D["xp"].device)
    assert L.ibmx_project(plan.handle, V(u.data_ptr()), V(u.data_ptr()), V(P.data_ptr()), None,
                          0.0) == ibmx.ESTATE
    st = L.ibmx_forcing_backward(plan.handle, V(u.data_ptr()), V(D["xp"].data_ptr()),
                                 V(D["up"].data_ptr()), V(D["wp"].data_ptr()), None, None, None,
                                 None, None, V(u.data_ptr()), V(F.data_ptr()), V(F.data_ptr()),
                                 V(F.data_ptr()))
    assert st == ibmx.ESTATE
    torch.cuda.synchronize()
    plan.close()
