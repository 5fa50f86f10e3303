"""Pins of the oracle's particle sub-stepping (Sec. 2.2.10) and Hertz/ACTM
normal contact (Sec. 2.2.7): closed forms of the collision equation, exact
motion under constant forces, momentum conservation, the restitution and
contact time the coefficients are built for, and the resting overlap the
gravity stiffness sets."""
import math

import numpy as np
import pytest

from paper_2109_03972_amd import synth


def _pcase(xp, radius, n=(64, 64, 64), periodic=(1, 1, 1), mass=None, up=None, wp=None, **over):
    npart = xp.shape[1]
    prm = synth.default_params()
    prm.update(over)
    return synth.Case(name="p", n=tuple(n), h=1.0, origin=(0.0, 0.0, 0.0), periodic=tuple(periodic),
                      xp=np.ascontiguousarray(xp, dtype=np.float64),
                      up=np.zeros((3, npart)) if up is None else np.asarray(up, dtype=np.float64),
                      wp=np.zeros((3, npart)) if wp is None else np.asarray(wp, dtype=np.float64),
                      radius=np.asarray(radius, dtype=np.float64),
                      mass=np.ones(npart) if mass is None else np.asarray(mass, dtype=np.float64),
                      moff=np.zeros(npart + 1, dtype=np.int32), body=np.zeros((3, 0)),
                      dV=np.ones(npart), u0=None, params=prm)


def test_actm_closed_forms(oracle_lib):
    # undamped Hertz contact: duration 2 z_max int_0^1 (1 - x^(5/2))^(-1/2) dx
    # with z_max = (5 / 4K)^(2/5); the integral is (2/5) B(2/5, 1/2)
    J = 0.4 * math.gamma(0.4) * math.gamma(0.5) / math.gamma(0.9)
    K, D = oracle_lib.actm_coefficients(1.0, 1.5)
    assert D == 0.0
    assert K == pytest.approx(1.25 * (2.0 * J) ** 2.5, rel=1e-11)
    # linear law: z = exp(-D t/2) sin(pi t)/pi closes at t = 1 with rebound
    # exp(-D/2): K = pi^2 + ln^2 e, D = -2 ln e
    for e in (0.97, 0.8, 0.5):
        K, D = oracle_lib.actm_coefficients(e, 1.0)
        assert K == pytest.approx(math.pi ** 2 + math.log(e) ** 2, rel=1e-11)
        assert D == pytest.approx(-2.0 * math.log(e), rel=1e-11)
    # more damping for less restitution; the Hertz stiffness grows with it
    K97, D97 = oracle_lib.actm_coefficients(0.97)
    K80, D80 = oracle_lib.actm_coefficients(0.8)
    assert 0.0 < D97 < D80 and K97 < K80


def test_constant_force_motion_exact(oracle_lib):
    """No contacts: the update integrates constant F_h, T_h and gravity
    exactly (the 2 alpha_k sum to 1 and x takes the trapezoid of u)."""
    rng = np.random.default_rng(5)
    xp = rng.uniform(10, 50, (3, 4))
    xp[:, 1] = xp[:, 0] + 30.0
    c = _pcase(xp, [3.0, 4.0, 2.5, 3.5], mass=[2.0, 5.0, 1.0, 3.0], up=rng.normal(0, 0.1, (3, 4)),
               wp=rng.normal(0, 0.1, (3, 4)), gravity=(0.01, -0.02, -0.05), rho_f=1.0)
    Fh = rng.normal(0, 0.5, (3, 4))
    Th = rng.normal(0, 0.5, (3, 4))
    empty = dict(pairs=np.zeros((2, 0), np.int32), walls=np.zeros((2, 0), np.int32))
    T, nsub = 2.5, 7
    r = oracle_lib.particle_substeps(c, empty, T, nsub, Fh=Fh, Th=Th)
    rho_p = c.mass / (4.0 / 3.0 * math.pi * c.radius ** 3)
    g = np.array(c.params["gravity"])[:, None]
    acc = Fh / c.mass + (1.0 - c.params["rho_f"] / rho_p) * g
    I = 0.4 * c.mass * c.radius ** 2
    np.testing.assert_allclose(r["up"], c.up + acc * T, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(r["wp"], c.wp + Th / I * T, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(r["xp"], c.xp + c.up * T + 0.5 * acc * T * T, rtol=1e-13, atol=1e-12)
    assert np.all(r["Fc"] == 0.0)


def _touching_cluster(seed, n_side=40):
    c = synth.small_case(seed, n=(n_side,) * 3, periodic=(1, 1, 1),
                         diameters=(12.0, 9.0, 7.0, 10.0, 8.0, 11.0), touch=0.6, min_gap=0.2)
    rng = np.random.default_rng(seed)
    c.up = rng.normal(0, 0.02, c.up.shape)
    c.wp = rng.normal(0, 0.005, c.wp.shape)
    c.mass = 4.0 / 3.0 * math.pi * c.radius ** 3 * 2.5
    return c


@pytest.mark.parametrize("model", [0, 1])
def test_momentum_conserved(oracle_lib, model):
    """Periodic box, no walls, F_h = 0, no gravity: contact forces are equal
    and opposite at every evaluation, so sum m u is unchanged."""
    c = _touching_cluster(31)
    c.params.update(normal_model=model, gravity=(0.0, 0.0, 0.0), gap_cut=3.0)
    pl = oracle_lib.pairs(c)
    assert np.any(pl["gap"] < 0.0) and pl["walls"].shape[1] == 0
    r = oracle_lib.particle_substeps(c, pl, 1.0, 15)
    p0 = (c.mass * c.up).sum(axis=1)
    p1 = (c.mass * r["up"]).sum(axis=1)
    scale = (c.mass * np.abs(r["up"] - c.up)).sum()
    assert scale > 0.0
    assert np.abs(p1 - p0).max() < 1e-13 * max(scale, np.abs(c.mass * c.up).sum())
    assert np.all(r["Fc"].sum(axis=1) == pytest.approx(0.0, abs=1e-12 * np.abs(r["Fc"]).max()))
    # history is kept for contacts of the final state only
    pl1 = oracle_lib.pairs(c, xp=r["xp"])
    assert np.array_equal(pl1["pairs"], pl["pairs"])
    apart = pl1["gap"] >= 0.0
    assert np.all(r["hist"][:, apart] == 0.0)
    assert np.any(r["hist"][3, ~apart] > 0.0)


def _head_on(oracle_lib, model, e, T_c, v, n_sub=15, dt_call=0.05):
    """Two spheres approach head-on in vacuum (no fluid, no gravity); returns
    the contact duration and the rebound ratio of the normal speed."""
    R1, R2, m1, m2 = 5.0, 3.5, 3.0, 1.2
    xp = np.array([[20.0, 20.0 + R1 + R2 + 0.05], [30.0, 30.0], [30.0, 30.0]])
    up = np.array([[m2 * v / (m1 + m2), -m1 * v / (m1 + m2)], [0, 0], [0, 0]], dtype=np.float64)
    c = _pcase(xp, [R1, R2], mass=[m1, m2], up=up, normal_model=model, e_dry=e, T_c=T_c,
               rho_f=0.0, nu_f=0.0, gravity=(0.0, 0.0, 0.0), gap_cut=1.0)
    pl = oracle_lib.pairs(c)
    assert pl["pairs"].shape[1] == 1
    x, u, w = c.xp.copy(), c.up.copy(), c.wp.copy()
    hist = np.zeros((4, 1))
    gap_prev = (x[0, 1] - x[0, 0]) - R1 - R2
    t, t_in, t_out = 0.0, None, None
    while t_out is None and t < 20 * T_c:
        r = oracle_lib.particle_substeps(c, pl, dt_call, n_sub, hist=hist, whist=np.zeros((4, 0)),
                                         xp=x, up=u, wp=w)
        x, u, w, hist = r["xp"], r["up"], r["wp"], r["hist"]
        gap = (x[0, 1] - x[0, 0]) - R1 - R2
        if t_in is None and gap < 0.0:
            t_in = t + dt_call * gap_prev / (gap_prev - gap)
        elif t_in is not None and gap >= 0.0:
            t_out = t + dt_call * gap_prev / (gap_prev - gap)
        gap_prev = gap
        t += dt_call
    return t_out - t_in, (u[0, 1] - u[0, 0]) / v, hist


@pytest.mark.parametrize("model,e", [(0, 0.97), (1, 0.97), (1, 0.8)])
def test_collision_restitution_and_duration(oracle_lib, model, e):
    """The normal coefficients are built so that a collision lasts T_c and
    rebounds with e_dry times the impact speed (Sec. 2.2.7): for the Hertz
    law at any impact speed (ACTM), for the linear law by construction.
    The printed corrector (gamma_k at the predicted state, zeta_k at the
    stage's start) weighs the stage forces with first moment 0.883 instead
    of 1/2 over a step, so the sub-stepping converges at first order in
    dts: the errors at dts and dts/4 differ by a factor of 4 (once dts is
    small enough for the contact onset to be resolved), and their
    Richardson extrapolation reproduces e_dry and T_c."""
    T_c = 10.0
    for v in (0.05, 0.2):
        T1, r1, _ = _head_on(oracle_lib, model, e, T_c, v, n_sub=60)
        T4, r4, _ = _head_on(oracle_lib, model, e, T_c, v, n_sub=240)
        assert (e - r1) / (e - r4) == pytest.approx(4.0, rel=2e-3)
        assert (4.0 * r4 - r1) / 3.0 == pytest.approx(e, rel=1e-7)
        assert (4.0 * T4 - T1) / 3.0 == pytest.approx(T_c, abs=1e-6)
        assert abs(T1 - T_c) < 1e-3 and abs(r1 - e) < 1e-3


def test_resting_overlap_from_gravity_stiffness(oracle_lib):
    """A sphere settling on the lower wall with its impact speed below the
    critical one rests on k_n = max(k_n,crit, k_n,grav): with the gravity
    term dominant, the overlap at rest balances m g' by k_n,grav, i.e.
    eps d/2 (g'/g)^(2/3) (Sec. 2.2.7)."""
    R, m = 5.0, 3.0
    xp = np.array([[32.0], [32.0], [R + 0.02]])
    g = 1e-3
    c = _pcase(xp, [R], mass=[m], periodic=(1, 1, 0), normal_model=1, rho_f=1e-3, nu_f=0.5,
               gravity=(0.0, 0.0, -g), gap_cut=1.0, eps_sep=0.01, T_c=10.0, e_dry=0.5)
    pl = oracle_lib.pairs(c)
    assert pl["walls"].tolist() == [[0], [4]]
    rho_p = m / (4.0 / 3.0 * math.pi * R ** 3)
    u_crit = 9.0 * 5.0 * 1e-3 * 0.5 / (rho_p * 2 * R)
    r = oracle_lib.particle_substeps(c, pl, 3000.0, 30000, whist=np.zeros((4, 1)))
    assert 0.0 < r["whist"][3, 0] <= u_crit          # settled in the critical regime
    gp = (1.0 - 1e-3 / rho_p) * g
    delta = R - r["xp"][2, 0]
    assert delta == pytest.approx(1e-3 * R * (gp / g) ** (2.0 / 3.0), rel=1e-6)
    assert abs(r["up"][2, 0]) < 1e-9


def test_st_switch(oracle_lib):
    """With the switch on, F_h is dropped for a particle whose committed
    contacts are all slow (St <= St_crit) and kept for a particle without
    contacts or with a fast one."""
    xp = np.array([[20.0, 29.9, 45.0], [30.0, 30.0, 30.0], [30.0, 30.0, 30.0]])
    c = _pcase(xp, [5.0, 5.0, 5.0], st_switch=1, gap_cut=1.0, gravity=(0.0, 0.0, 0.0))
    pl = oracle_lib.pairs(c)
    assert pl["pairs"].T.tolist() == [[0, 1]]
    Fh = np.zeros((3, 3))
    Fh[2] = 1e-3
    rho_d = 3.0 / (2.0 * math.pi * 25.0)
    u_crit = 9.0 * 5.0 * c.params["rho_f"] * c.params["nu_f"] / rho_d
    for u_in, dropped in ((0.5 * u_crit, True), (2.0 * u_crit, False)):
        hist = np.array([[0.0], [0.0], [0.0], [u_in]])
        r = oracle_lib.particle_substeps(c, pl, 1.0, 3, Fh=Fh, hist=hist)
        r0 = oracle_lib.particle_substeps(c, pl, 1.0, 3, Fh=None, hist=hist)
        for p in (0, 1):
            same = np.array_equal(r["up"][2, p], r0["up"][2, p])
            assert same == dropped
        assert r["up"][2, 2] == pytest.approx(1e-3, rel=1e-12)   # no contact: F_h kept
