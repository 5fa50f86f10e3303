"""Parity of the HIP particle sub-stepping (ibmx_particle_substeps, through
the C ABI) with the FP64 oracle on the same lists, histories and forces:
particle states, committed histories and the final collision force and
torque to 1e-11 (FP64 arithmetic in the same order on both sides; the
libraries' erf may differ in the last bit, and 91 contact evaluations
carry such differences forward)."""
import numpy as np
import pytest

import oracle
from paper_2109_03972_amd import ibmx, synth
from tests._util import dev_case, rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-11


def _oracle_lists(case):
    """Oracle lists and a history for them (one pair-pass evaluation)."""
    ref_l = oracle.pairs(case)
    ref_f = oracle.pair_forces(case, ref_l)
    return ref_l, ref_f


def _device_lists(plan, D, case, ref_l, ref_f, pair_cap=None, wall_cap=None):
    """The HIP pair pass's lists for the case (checked bit-exact against the
    oracle's) with the oracle's history copied into device arrays."""
    import torch
    plan.set_markers(D["body"], D["dV"])
    res = plan.pairs(D["xp"], D["radius"], D["mass"], D["up"], D["wp"], pair_cap=pair_cap,
                     wall_cap=wall_cap)
    torch.cuda.synchronize()
    t = ibmx.trim_pairs(res)
    assert np.array_equal(t["pairs"].cpu().numpy(), ref_l["pairs"])
    assert np.array_equal(t["walls"].cpu().numpy(), ref_l["walls"])
    dev = D["xp"].device
    hist = torch.zeros((4, res["pair_cap"]), dtype=torch.float64, device=dev)
    whist = torch.zeros((4, res["wall_cap"]), dtype=torch.float64, device=dev)
    k, kw = t["npairs"], t["nwall"]
    hist[:, :k] = torch.as_tensor(ref_f["hist"]).to(dev)
    whist[:, :kw] = torch.as_tensor(ref_f["whist"]).to(dev)
    return res, hist, whist, k, kw


def _run_both(case, dt_total, n_sub, seed=0, with_fh=True, pair_cap=None, wall_cap=None,
              precision="f64"):
    import torch
    rng = np.random.default_rng(seed)
    Fh = rng.normal(0, 1e-3, (3, case.np_)) if with_fh else None
    Th = rng.normal(0, 1e-3, (3, case.np_)) if with_fh else None
    ref_l, ref_f = _oracle_lists(case)
    ref = oracle.particle_substeps(case, ref_l, dt_total, n_sub, Fh=Fh, Th=Th,
                                   hist=ref_f["hist"], whist=ref_f["whist"])
    D = dev_case(case, "f64")
    plan = ibmx.Plan.from_case(case, precision)
    res, hist, whist, k, kw = _device_lists(plan, D, case, ref_l, ref_f, pair_cap, wall_cap)
    dev = D["xp"].device
    Fh_d = None if Fh is None else torch.as_tensor(Fh).to(dev).contiguous()
    Th_d = None if Th is None else torch.as_tensor(Th).to(dev).contiguous()
    Fc, Tc = plan.particle_substeps(dt_total, n_sub, D["xp"], D["up"], D["wp"], D["radius"],
                                    D["mass"], res, hist, whist, Fh=Fh_d, Th=Th_d)
    assert plan.status() == 0
    torch.cuda.synchronize()
    got = dict(xp=D["xp"].cpu().numpy(), up=D["up"].cpu().numpy(), wp=D["wp"].cpu().numpy(),
               hist=hist[:, :k].cpu().numpy(), whist=whist[:, :kw].cpu().numpy(),
               Fc=Fc.cpu().numpy(), Tc=Tc.cpu().numpy())
    return got, ref, ref_l


def _compare(got, ref, tol=TOL):
    # positions: the displacement over the call, relative to its size
    x0 = got["x0"]
    assert rel_err(got["xp"] - x0, ref["xp"] - x0) <= tol, "xp"
    for k in ("up", "wp", "hist", "whist", "Fc", "Tc"):
        assert rel_err(got[k], ref[k]) <= tol, f"{k}: {rel_err(got[k], ref[k]):.3e}"


def _cluster(seed, periodic=(1, 1, 1), n=48):
    c = synth.small_case(seed, n=(n, n, n), periodic=periodic,
                         diameters=(12.0, 9.0, 7.0, 10.0, 8.0, 11.0, 9.5, 6.0), touch=0.7,
                         min_gap=0.1)
    rng = np.random.default_rng(seed)
    c.up = rng.normal(0, 0.03, c.up.shape)
    c.wp = rng.normal(0, 0.01, c.wp.shape)
    c.params.update(gap_cut=3.0)
    return c


@pytest.mark.parametrize("model", [0, 1])
@pytest.mark.parametrize("periodic", [(1, 1, 1), (1, 1, 0)])
def test_cluster_parity(model, periodic):
    c = _cluster(301, periodic)
    c.params.update(normal_model=model, gravity=(0.0, 0.0, -2e-3))
    x0 = c.xp.copy()
    got, ref, ref_l = _run_both(c, 1.0, 15, seed=1)
    got["x0"] = x0
    assert np.any(ref_l["gap"] < 0)
    print(f"model {model} periodic {periodic}: pairs {ref_l['pairs'].shape[1]} walls "
          f"{ref_l['walls'].shape[1]}", flush=True)
    _compare(got, ref)


def _wall_layer(seed):
    """Spheres resting in and just above the lower wall, some overlapping it
    and each other."""
    rng = np.random.default_rng(seed)
    R = np.array([5.0, 4.0, 6.0, 4.5, 5.5, 3.5])
    x = np.array([[10.0, 19.2, 30.0, 40.4, 12.0, 24.0],
                  [10.0, 10.0, 11.0, 10.5, 21.0, 20.5],
                  [4.9, 3.95, 6.05, 4.6, 5.3, 3.4]])
    x[2] = np.minimum(x[2], R + rng.uniform(-0.2, 0.05, R.size))
    mass = 2.5 * 4.0 / 3.0 * np.pi * R ** 3
    prm = synth.default_params()
    prm.update(gap_cut=2.0, normal_model=1, gravity=(0.0, 0.0, -2e-3), disable_mode=0)
    npart = R.size
    return synth.Case(name="wall_layer", n=(48, 40, 32), h=1.0, origin=(0.0, 0.0, 0.0),
                      periodic=(1, 1, 0), xp=np.ascontiguousarray(x),
                      up=rng.normal(0, 0.03, (3, npart)), wp=rng.normal(0, 0.01, (3, npart)),
                      radius=R, mass=mass, moff=np.zeros(npart + 1, dtype=np.int32),
                      body=np.zeros((3, 0)), dV=np.ones(npart), u0=None, params=prm)


@pytest.mark.parametrize("model", [0, 1])
def test_wall_contacts(model):
    c = _wall_layer(306)
    c.params["normal_model"] = model
    x0 = c.xp.copy()
    got, ref, ref_l = _run_both(c, 1.0, 15, seed=6)
    got["x0"] = x0
    assert np.any(ref_l["wgap"] < 0) and np.any(ref_l["gap"] < 0)
    _compare(got, ref)


def test_fp32_plan():
    """The contact pass is FP64 whatever the plan's grid precision."""
    c = _wall_layer(308)
    x0 = c.xp.copy()
    got, ref, _ = _run_both(c, 1.0, 15, seed=7, precision="f32")
    got["x0"] = x0
    _compare(got, ref)


def test_st_switch_and_no_forcing():
    """The St switch with slow and fast contacts, with and without F_h; the
    switch drops F_h for some particles and not for others."""
    c = _wall_layer(307)
    c.params.update(st_switch=1, rho_f=1.0, nu_f=0.025)
    ref_l, ref_f = _oracle_lists(c)
    u_in = np.concatenate([ref_f["hist"][3], ref_f["whist"][3]])
    assert np.any(u_in > 0)
    rng = np.random.default_rng(2)
    Fh = rng.normal(0, 1e-3, (3, c.np_))
    on = oracle.particle_substeps(c, ref_l, 0.5, 4, Fh=Fh, hist=ref_f["hist"], whist=ref_f["whist"])
    # the particles the rule drops F_h for: some committed contact, none fast
    rhod = 3.0 * c.mass / (2.0 * np.pi * c.radius ** 2)
    u_crit = 9.0 * c.params["St_crit"] * c.params["rho_f"] * c.params["nu_f"]
    contacts = np.zeros(c.np_, int)
    fast = np.zeros(c.np_, int)
    for (i, j), u in zip(ref_l["pairs"].T, ref_f["hist"][3]):
        if u > 0:
            contacts[[i, j]] += 1
            fast[[i, j]] += u * 0.5 * (rhod[i] + rhod[j]) > u_crit
    for p, u in zip(ref_l["walls"][0], ref_f["whist"][3]):
        if u > 0:
            contacts[p] += 1
            fast[p] += u * rhod[p] > u_crit
    slow = (contacts > 0) & (fast == 0)
    assert np.any(slow) and not np.all(slow)
    Fh_off = Fh.copy()
    Fh_off[:, slow] = 0.0
    c.params["st_switch"] = 0
    off = oracle.particle_substeps(c, ref_l, 0.5, 4, Fh=Fh_off, hist=ref_f["hist"],
                                   whist=ref_f["whist"])
    c.params["st_switch"] = 1
    assert np.array_equal(on["up"], off["up"]) and np.array_equal(on["xp"], off["xp"])
    for with_fh in (True, False):
        x0 = c.xp.copy()
        got, ref, _ = _run_both(c, 0.5, 4, seed=2, with_fh=with_fh)
        got["x0"] = x0
        _compare(got, ref)


def test_single_substep_and_tight_caps():
    """n_sub = 1, lists filling their capacities exactly."""
    c = _cluster(303, (1, 1, 0))
    ref_l, _ = _oracle_lists(c)
    x0 = c.xp.copy()
    got, ref, _ = _run_both(c, 1.0, 1, seed=3, pair_cap=ref_l["pairs"].shape[1],
                            wall_cap=max(1, ref_l["walls"].shape[1]))
    got["x0"] = x0
    _compare(got, ref)


def test_no_contacts():
    """Particles far apart: only F_h, T_h and gravity act."""
    c = synth.small_case(304, n=(64, 64, 64), periodic=(1, 1, 1), diameters=(8.0, 6.0, 7.0),
                         min_gap=12.0)
    c.params.update(gap_cut=1.0, gravity=(1e-3, 0.0, -2e-3), disable_mode=0)
    ref_l, _ = _oracle_lists(c)
    assert ref_l["pairs"].shape[1] == 0
    x0 = c.xp.copy()
    got, ref, _ = _run_both(c, 2.0, 5, seed=4)
    got["x0"] = x0
    _compare(got, ref)


def test_split_call_matches_whole():
    """Two calls of dt/2 with n_sub/2 sub-steps follow one call of dt with
    n_sub: the second call starts at the first call's final state with its
    committed history."""
    import torch
    c = _cluster(305, (1, 1, 0))
    c.params.update(normal_model=1)
    ref_l, ref_f = _oracle_lists(c)
    out = []
    for parts in (1, 2):
        D = dev_case(c, "f64")
        plan = ibmx.Plan.from_case(c, "f64")
        res, hist, whist, k, kw = _device_lists(plan, D, c, ref_l, ref_f)
        for _ in range(parts):
            plan.particle_substeps(1.0 / parts, 8 // parts, D["xp"], D["up"], D["wp"],
                                   D["radius"], D["mass"], res, hist, whist, want_forces=False)
        torch.cuda.synchronize()
        out.append((D["xp"].cpu().numpy() - c.xp, D["up"].cpu().numpy(), hist[:, :k].cpu().numpy()))
    for a, b in zip(out[0], out[1]):
        assert rel_err(b, a) <= 1e-12


def test_polydisperse_bed_512_parity():
    """The bed workload's particles (20,000 polydisperse spheres on a wall),
    Hertz law, the paper's 15 sub-steps."""
    c = synth.make_case("polydisperse_bed_512", lazy_field=True)
    c.params.update(normal_model=1, gap_cut=max(c.params["gap_cut"], 2.0))
    x0 = c.xp.copy()
    got, ref, ref_l = _run_both(c, 1.0, 15, seed=5)
    got["x0"] = x0
    print(f"bed: np {c.np_} pairs {ref_l['pairs'].shape[1]} walls {ref_l['walls'].shape[1]} "
          f"contacts {int((ref_l['gap'] < 0).sum())}", flush=True)
    _compare(got, ref)


def test_bad_list_entries_are_skipped_and_reported():
    """Entries outside the particle range or on a periodic axis are skipped
    and latched as EINVAL; the valid ones still act."""
    import torch
    c = _wall_layer(309)
    ref_l, ref_f = _oracle_lists(c)
    D = dev_case(c, "f64")
    plan = ibmx.Plan.from_case(c, "f64")
    res, hist, whist, k, kw = _device_lists(plan, D, c, ref_l, ref_f)
    bad = dict(res)
    pairs = res["pairs"].clone()
    pairs[1, 0] = c.np_ + 5            # partner out of range
    walls = res["walls"].clone()
    walls[1, 0] = 0                    # x is periodic: no wall there
    bad["pairs"], bad["walls"] = pairs, walls
    plan.particle_substeps(1.0, 3, D["xp"], D["up"], D["wp"], D["radius"], D["mass"], bad, hist,
                           whist, want_forces=False)
    torch.cuda.synchronize()
    assert plan.status() == ibmx.EINVAL
    assert torch.isfinite(D["xp"]).all() and torch.isfinite(D["up"]).all()
