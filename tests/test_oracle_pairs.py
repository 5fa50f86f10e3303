"""Pins of the oracle's pair pass (Secs. 2.2.5-2.2.8): neighbour lists, collision
forces and marker disabling."""
import math

import numpy as np
import pytest

from paper_2109_03972_amd import synth


def _pcase(xp, radius, n=(40, 40, 40), periodic=(1, 1, 1), mass=None, up=None, wp=None,
           markers=None, **prm_over):
    npart = xp.shape[1]
    prm = synth.default_params()
    prm.update(prm_over)
    if markers is None:
        moff = np.zeros(npart + 1, dtype=np.int32)
        body = np.zeros((3, 0))
    else:
        moff, body = markers
    return synth.Case(name="p", n=tuple(n), h=1.0, origin=(0.0, 0.0, 0.0), periodic=tuple(periodic),
                      xp=np.ascontiguousarray(xp, dtype=np.float64),
                      up=np.zeros((3, npart)) if up is None else np.asarray(up, dtype=np.float64),
                      wp=np.zeros((3, npart)) if wp is None else np.asarray(wp, dtype=np.float64),
                      radius=np.asarray(radius, dtype=np.float64),
                      mass=np.ones(npart) if mass is None else np.asarray(mass, dtype=np.float64),
                      moff=moff, body=body, dV=np.ones(npart), u0=None, params=prm)


def test_pair_list_hand_cases(oracle_lib):
    """Known gaps, including a pair across the periodic seam and one just
    beyond the cut-off."""
    xp = np.array([[1.0, 38.0, 20.0, 20.0], [5.0, 5.0, 20.0, 20.0], [5.0, 5.0, 20.0, 30.1]])
    r = np.array([1.0, 1.0, 2.0, 3.0])
    c = _pcase(xp, r, gap_cut=3.0)
    pl = oracle_lib.pairs(c)
    # 0-1 across the seam: distance 3, gap 1; 2-3: distance 10.1, gap 5.1 > 3
    assert pl["pairs"].tolist() == [[0], [1]]
    assert pl["gap"][0] == pytest.approx(1.0, abs=1e-14)
    c2 = _pcase(xp, r, gap_cut=5.2)
    pl2 = oracle_lib.pairs(c2)
    assert pl2["pairs"].T.tolist() == [[0, 1], [2, 3]]
    assert pl2["gap"][1] == pytest.approx(5.1, abs=1e-12)


def test_pair_list_equals_numpy_bruteforce(oracle_lib):
    c = synth.make_case("suspension_128", lazy_field=True)
    pl = oracle_lib.pairs(c)
    x = c.xp.T
    d = x[None, :, :] - x[:, None, :]
    d -= 128.0 * np.round(d / 128.0)
    dist = np.sqrt((d ** 2).sum(-1))
    cut = c.radius[:, None] + c.radius[None, :] + c.params["gap_cut"]
    I, J = np.nonzero(np.triu(dist < cut, 1))
    assert np.array_equal(pl["pairs"], np.stack([I, J]).astype(np.int32))
    assert np.allclose(pl["gap"], dist[I, J] - c.radius[I] - c.radius[J], atol=1e-12)


def test_cell_list_invariants(oracle_lib):
    c = synth.make_case("bidisperse_bed_256x256x512", lazy_field=True)
    cl = oracle_lib.cell_list(c)
    nc = cl["nc"]
    rmax = c.radius.max()
    for a in range(3):
        assert nc[a] == max(1, int(math.floor(c.n[a] / (2 * rmax + c.params["gap_cut"]))))
    cs, cp = cl["cell_start"], cl["cell_particles"]
    assert cs[0] == 0 and cs[-1] == c.np_
    assert sorted(cp.tolist()) == list(range(c.np_))
    for cell in range(len(cs) - 1):
        seg = cp[cs[cell]:cs[cell + 1]]
        assert np.all(np.diff(seg) > 0)
        assert np.all(cl["cell_of"][seg] == cell)
    # every listed pair lies in neighbouring cells
    pl = oracle_lib.pairs(c)
    ncv = nc.astype(int)
    co = cl["cell_of"]
    cx, cy, cz = co % ncv[0], (co // ncv[0]) % ncv[1], co // (ncv[0] * ncv[1])
    for i, j in pl["pairs"].T:
        for a, cc in enumerate((cx, cy, cz)):
            dd = abs(int(cc[i]) - int(cc[j]))
            if c.periodic[a]:
                dd = min(dd, ncv[a] - dd)
            assert dd <= 1


def test_wall_list(oracle_lib):
    xp = np.array([[5.0, 15.0, 25.0, 35.0], [5.0, 5.0, 5.0, 5.0], [2.5, 20.0, 37.1, 37.0]])
    c = _pcase(xp, [2.0, 2.0, 2.0, 2.0], periodic=(1, 1, 0), gap_cut=1.0)
    pl = oracle_lib.pairs(c)
    # lower wall: gap 0.5; upper wall: gap 0.9 listed, exactly 1.0 not (strict)
    assert pl["walls"].T.tolist() == [[0, 4], [2, 5]]
    assert np.allclose(pl["wgap"], [0.5, 0.9], atol=1e-13)


def test_newton_third_law_and_angular_momentum(oracle_lib):
    """sum_p F_c = 0 and sum_p (x_p x F_c + T_c) = 0 for particle pairs
    (eq. f_int, with forces equal and opposite and the lever arms summing to
    the centre distance)."""
    rng = np.random.default_rng(2)
    c = synth.small_case(21, n=(48, 48, 48), periodic=(1, 1, 1),
                         diameters=(12.0, 9.0, 7.0, 10.0, 8.0, 11.0), touch=0.6, min_gap=0.2)
    c.up = rng.normal(0, 0.3, c.up.shape)
    c.wp = rng.normal(0, 0.1, c.wp.shape)
    pl = oracle_lib.pairs(c, gap_cut=3.0)
    assert pl["pairs"].shape[1] >= 2 and np.any(pl["gap"] < 0)
    prev = dict(pairs=pl["pairs"], hist=rng.normal(0, 0.01, (4, pl["pairs"].shape[1])),
                walls=pl["walls"], whist=np.zeros((4, pl["walls"].shape[1])))
    f = oracle_lib.pair_forces(c, pl, prev=prev)
    assert np.abs(f["Fc"].sum(axis=1)).max() < 1e-12 * max(1.0, np.abs(f["Fc"]).max())
    # angular momentum per pair, with the partner at its minimum image
    for k in range(pl["pairs"].shape[1]):
        i, j = (int(v) for v in pl["pairs"][:, k])
        one = dict(pairs=pl["pairs"][:, k:k + 1].copy(), gap=pl["gap"][k:k + 1].copy(),
                   walls=np.zeros((2, 0), np.int32), wgap=np.zeros(0))
        fk = oracle_lib.pair_forces(c, one, prev=prev)
        d = c.xp[:, j] - c.xp[:, i]
        d -= 48.0 * np.round(d / 48.0)
        xi, xj = c.xp[:, i], c.xp[:, i] + d
        tot = (np.cross(xi, fk["Fc"][:, i]) + np.cross(xj, fk["Fc"][:, j])
               + fk["Tc"][:, i] + fk["Tc"][:, j])
        scale = max(1.0, np.abs(fk["Fc"]).max() * 48)
        assert np.abs(tot).max() < 1e-12 * scale


def _collide(oracle_lib, R1, R2, m1, m2, v, dt_int, e_dry, T_c, lub=False, steps=None):
    """Integrate a head-on collision of two spheres with the oracle's pair
    force (velocity Verlet); returns contact duration and rebound ratio."""
    x = np.array([[10.0, 10.0 + R1 + R2 + 1e-9], [20.0, 20.0], [20.0, 20.0]])
    u = np.array([[v / 2, -v / 2], [0.0, 0.0], [0.0, 0.0]])
    prm = dict(e_dry=e_dry, T_c=T_c, nu_f=(0.025 if lub else 0.0), gap_cut=3.0)
    hist = dict(pairs=np.zeros((2, 0), np.int32), hist=np.zeros((4, 0)),
                walls=np.zeros((2, 0), np.int32), whist=np.zeros((4, 0)))
    m = np.array([m1, m2])
    t = 0.0
    t_in = t_out = None
    for _ in range(steps or 200000):
        c = _pcase(x, [R1, R2], n=(64, 64, 64), mass=m, up=u, dt=dt_int, **prm)
        pl = oracle_lib.pairs(c)
        f = oracle_lib.pair_forces(c, pl, prev=hist)
        hist = dict(pairs=pl["pairs"], hist=f["hist"], walls=pl["walls"], whist=f["whist"])
        a = f["Fc"] / m
        gap = (x[0, 1] - x[0, 0]) - R1 - R2
        if gap < 0 and t_in is None:
            t_in = t
        if t_in is not None and gap >= 0 and t_out is None:
            t_out = t
            break
        u = u + dt_int * a
        x = x + dt_int * u
        t += dt_int
    rel_out = u[0, 1] - u[0, 0]
    return t_out - t_in, rel_out / v


def test_linear_contact_restitution_and_duration(oracle_lib):
    """The linear spring-dashpot normal force gives a contact lasting T_c with
    rebound/impact speed e_dry (damped-oscillator solution, the linear form of
    eq. ode), for unequal masses."""
    Tc, e = 10.0, 0.97
    dur, ratio = _collide(oracle_lib, 6.0, 4.0, 2.0, 0.7, 0.05, Tc / 4000.0, e, Tc)
    assert dur == pytest.approx(Tc, rel=2e-3)
    assert ratio == pytest.approx(e, rel=2e-3)


def test_lubrication_textbook_limits(oracle_lib):
    """For small gaps (psi ~ 1) the lubrication force reduces to the
    Reynolds/Cox-Brenner results: 6 pi mu R^2 V / zeta for a sphere
    approaching a wall, and 6 pi mu (R/2)^2 V / zeta for two equal spheres."""
    mu = 1.0 * 0.025
    R, V, zeta = 5.0, 0.2, 0.1
    # sphere moving towards the lower z wall
    c = _pcase(np.array([[10.0], [10.0], [R + zeta]]), [R], periodic=(1, 1, 0),
               up=np.array([[0.0], [0.0], [-V]]))
    pl = oracle_lib.pairs(c)
    f = oracle_lib.pair_forces(c, pl)
    psi = 0.5 * math.erf(6 - 5.5 * zeta) + 0.5
    assert psi > 0.99999
    assert f["Fc"][2, 0] == pytest.approx(6 * math.pi * mu * R * R * V / zeta * psi, rel=1e-12)
    # two equal spheres approaching each other with relative speed V
    xp = np.array([[10.0, 10.0 + 2 * R + zeta], [20.0, 20.0], [20.0, 20.0]])
    c2 = _pcase(xp, [R, R], up=np.array([[V / 2, -V / 2], [0, 0], [0, 0]]))
    f2 = oracle_lib.pair_forces(c2, oracle_lib.pairs(c2))
    assert f2["Fc"][0, 0] == pytest.approx(-6 * math.pi * mu * (R / 2) ** 2 * V / zeta * psi, rel=1e-12)
    assert f2["Fc"][0, 1] == pytest.approx(-f2["Fc"][0, 0], rel=1e-15)
    # blended to ~7.31e-4 of the unblended value at eps_sep and zero beyond
    at = 1.5 - 1e-12
    xp3 = np.array([[10.0, 10.0 + 2 * R + at], [20.0, 20.0], [20.0, 20.0]])
    c3 = _pcase(xp3, [R, R], up=np.array([[V / 2, -V / 2], [0, 0], [0, 0]]))
    f3 = oracle_lib.pair_forces(c3, oracle_lib.pairs(c3))
    unblended = 6 * math.pi * mu * (R / 2) ** 2 * V / at
    assert -f3["Fc"][0, 0] / unblended == pytest.approx(7.31e-4, rel=2e-3)
    xp4 = np.array([[10.0, 10.0 + 2 * R + 1.5], [20.0, 20.0], [20.0, 20.0]])
    c4 = _pcase(xp4, [R, R], up=np.array([[V / 2, -V / 2], [0, 0], [0, 0]]))
    assert np.abs(oracle_lib.pair_forces(c4, oracle_lib.pairs(c4))["Fc"]).max() == 0.0


def test_tangential_coulomb_cap(oracle_lib):
    """A sphere pressed into a wall and sliding fast: the tangential force is
    capped at mu_k |F_n| and opposes the sliding (Sec. 2.2.8 tangential model);
    a slowly creeping contact sticks with |F_t| <= mu_s |F_n|."""
    R = 4.0
    x = np.array([[10.0], [10.0], [R - 0.02]])
    fast = _pcase(x, [R], periodic=(1, 1, 0), up=np.array([[0.5], [0.0], [0.0]]))
    f = oracle_lib.pair_forces(fast, oracle_lib.pairs(fast))
    Fz = f["Fc"][2, 0]
    assert Fz > 0
    assert f["Fc"][0, 0] == pytest.approx(-0.8 * Fz, rel=1e-12)
    slow = _pcase(x, [R], periodic=(1, 1, 0), up=np.array([[1e-6], [0.0], [0.0]]))
    f = oracle_lib.pair_forces(slow, oracle_lib.pairs(slow))
    assert abs(f["Fc"][0, 0]) <= 0.11 * f["Fc"][2, 0]
    assert f["Fc"][0, 0] < 0


def _splitmix64(x):
    M = 0xFFFFFFFFFFFFFFFF
    z = (x + 0x9E3779B97F4A7C15) & M
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
    return z ^ (z >> 31)


def test_marker_mask_rules(oracle_lib):
    """Marker disabling (Sec. 2.2.5): for each pair closer than 2 eps_sep
    exactly one particle loses markers (those within 2 eps_sep of the partner's
    surface); markers closer than eps_sep to a wall are off; nothing else."""
    c = synth.make_case("bidisperse_bed_256x256x512", lazy_field=True)
    pl = oracle_lib.pairs(c)
    mask = oracle_lib.marker_mask(c, pl)
    eps = c.params["eps_sep"]
    seed = c.params["disable_seed"]
    pid = np.repeat(np.arange(c.np_), np.diff(c.moff))
    X = c.xp[:, pid] + c.body
    expect = np.ones(c.nm, dtype=bool)
    L = np.array(c.n, dtype=np.float64)
    losers = set()
    for k, (p, q) in enumerate(pl["pairs"].T):
        if not pl["gap"][k] < 2 * eps:
            continue
        ch = p if (_splitmix64(seed ^ ((int(p) << 32) | int(q))) & 1) == 0 else q
        pa = q if ch == p else p
        losers.add(int(ch))
        sl = slice(c.moff[ch], c.moff[ch + 1])
        d = X[:, sl] - c.xp[:, pa:pa + 1]
        for a in range(2):
            d[a] -= L[a] * np.round(d[a] / L[a])
        expect[sl] &= ~((d ** 2).sum(0) < (c.radius[pa] + 2 * eps) ** 2)
    for k, (p, side) in enumerate(pl["walls"].T):
        if not pl["wgap"][k] < eps:
            continue
        sl = slice(c.moff[p], c.moff[p + 1])
        z = X[2, sl]
        dist = z if side == 4 else L[2] - z
        expect[sl] &= ~(dist < eps)
    assert np.array_equal(mask.astype(bool), expect)
    # at least one pair is close, and the particles that lost markers are
    # only those chosen (or near a wall)
    assert len(losers) > 10
    off_particles = set(np.unique(pid[mask == 0]).tolist())
    wall_p = set(pl["walls"][0][pl["wgap"] < eps].tolist())
    assert off_particles <= (losers | wall_p)
    # every remaining marker keeps its delta support inside the walls
    keep = mask.astype(bool)
    assert np.all(X[2, keep] >= 1.0) and np.all(X[2, keep] <= L[2] - 1.0)


def test_whole_mode_removes_all_markers_of_one(oracle_lib):
    xp = np.array([[10.0, 19.0], [10.0, 10.0], [10.0, 10.0]])
    body = np.concatenate([synth.spiral_points(50).T * 4.0] * 2, axis=1)
    moff = np.array([0, 50, 100], dtype=np.int32)
    c = _pcase(xp, [4.0, 4.0], markers=(moff, body), gap_cut=3.0, disable_seed=12345)
    pl = oracle_lib.pairs(c)
    m = oracle_lib.marker_mask(c, pl, mode=2)
    offs = [int((m[0:50] == 0).sum()), int((m[50:100] == 0).sum())]
    assert sorted(offs) == [0, 50]
    m1 = oracle_lib.marker_mask(c, pl, mode=1)
    loser = 0 if offs[0] == 50 else 1
    assert (m1[50 * loser:50 * loser + 50] == 0).sum() > 0
    assert (m1[50 * (1 - loser):50 * (1 - loser) + 50] == 0).sum() == 0
    assert np.all(oracle_lib.marker_mask(c, pl, mode=0) == 1)


def _wall_slide(oracle_lib, v0, steps, dt_int, nu_poi, overlap=0.05, mass=1.0, R=4.0,
                hold_velocity=False):
    """A sphere pressed into the lower z wall by a fixed overlap, rotation
    frozen, moving along x: only the tangential force changes its velocity
    (the normal one is balanced by holding the height).  Returns the time
    series of (x-velocity, tangential spring, F_x, F_z) over the evaluations,
    with the history passed from each evaluation to the next."""
    x = np.array([[10.0], [10.0], [R - overlap]])
    wl = dict(pairs=np.zeros((2, 0), np.int32), gap=np.zeros(0),
              walls=np.array([[0], [4]], np.int32), wgap=np.array([-overlap]))
    prev = dict(pairs=np.zeros((2, 0), np.int32), hist=np.zeros((4, 0)),
                walls=np.zeros((2, 0), np.int32), whist=np.zeros((4, 0)))
    u = v0
    out = []
    for _ in range(steps):
        c = _pcase(x, [R], periodic=(1, 1, 0), mass=[mass],
                   up=np.array([[u], [0.0], [0.0]]), dt=dt_int, nu_poi=nu_poi, nu_f=0.0)
        f = oracle_lib.pair_forces(c, wl, prev=prev)
        prev = dict(pairs=prev["pairs"], hist=prev["hist"], walls=wl["walls"], whist=f["whist"])
        out.append((u, f["whist"][0, 0], f["Fc"][0, 0], f["Fc"][2, 0]))
        if not hold_velocity:
            u = u + dt_int * f["Fc"][0, 0] / mass
    return np.array(out)


@pytest.mark.parametrize("nu_poi", [0.0, 0.3, 0.45])
def test_tangential_stick_is_damped_oscillator(oracle_lib, nu_poi):
    """Stick branch of the tangential model (Sec. 2.2.8, with k_t = kappa k_n and
    the damping of the normal law carried over, as the paper leaves them open):
    while |F_t| stays below mu_s |F_n| the tangential force is a linear
    spring-dashpot on the integrated slip, so the tangential motion obeys
    m zeta'' + d_t zeta' + k_t zeta = 0 with k_t = kappa k_n, kappa =
    2(1 - nu)/(2 - nu), and d_t = 2 sqrt(m k_t) (-ln e)/sqrt(pi^2 + ln^2 e).
    Its solution from zeta = 0 returns to zero after half a period
    pi / omega_d = T_c / sqrt(kappa), with velocity -e times the initial one:
    a dropped kappa, a k_t without the k_n factor, a d_t off by any factor or a
    sign error in the spring update each move one of the two numbers."""
    Tc, e = 10.0, 0.97
    kappa = 2.0 * (1.0 - nu_poi) / (2.0 - nu_poi)
    half = Tc / math.sqrt(kappa)
    dt_int = half / 4000.0
    v0 = 1e-3   # small enough that |F_t| << mu_s |F_n|: the contact sticks
    s = _wall_slide(oracle_lib, v0, 4400, dt_int, nu_poi)
    u, zt, Fx, Fz = s.T
    assert np.all(np.abs(Fx) <= 0.11 * Fz)          # never slips
    # first return of the spring to zero
    k = int(np.nonzero((zt[:-1] > 0) & (zt[1:] <= 0))[0][0])
    frac = zt[k] / (zt[k] - zt[k + 1])
    t_cross = (k + frac + 1) * dt_int   # zt[i] is the spring after i + 1 increments
    u_cross = u[k] + frac * (u[k + 1] - u[k])
    assert t_cross == pytest.approx(half, rel=2e-3)
    assert -u_cross / v0 == pytest.approx(e, rel=2e-3)


def test_tangential_slip_caps_and_resets_spring(oracle_lib):
    """Slip branch of the tangential model (Sec. 2.2.8, with the spring reset on
    slipping): under a
    constant normal force and a constant tangential slip speed the tangential
    force is mu_k |F_n| at every evaluation, opposed to the slip, and the
    spring is reset to -(F_t + d_t g_t)/k_t each time, so it does not grow
    after the first slip."""
    Tc, e, nu_poi, g = 10.0, 0.97, 0.3, 0.05
    s = _wall_slide(oracle_lib, g, 50, 0.1, nu_poi, hold_velocity=True)
    u, zt, Fx, Fz = s.T
    assert np.all(Fz > 0)
    assert np.allclose(Fx, -0.8 * Fz, rtol=1e-12, atol=0.0)
    le = math.log(e)
    kn = (math.pi ** 2 + le * le) / Tc ** 2         # m_eff = m_p = 1 for a wall
    kt = 2.0 * (1.0 - nu_poi) / (2.0 - nu_poi) * kn
    dt_ = 2.0 * math.sqrt(kt) * (-le) / math.sqrt(math.pi ** 2 + le * le)
    reset = -(Fx[0] + dt_ * g) / kt
    assert np.allclose(zt, reset, rtol=1e-12, atol=0.0)
    assert zt[-1] == zt[1]
