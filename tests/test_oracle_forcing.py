"""Pins of the oracle's outer forcing loop (Sec. 2.2.2) against facts fixed by
the paper and by the delta kernel's moment conditions, not by the oracle's
own formulas."""
import math

import numpy as np
import pytest

from paper_2109_03972_amd import synth


def _case(n, xp, body_list, dV, periodic=(1, 1, 1), h=1.0, u0=None, up=None, wp=None,
          n_iter=1, c=8.0 / 15.0, origin=(0.0, 0.0, 0.0)):
    npart = xp.shape[1]
    counts = [b.shape[1] for b in body_list]
    moff = np.zeros(npart + 1, dtype=np.int32)
    moff[1:] = np.cumsum(counts)
    body = np.concatenate(body_list, axis=1) if body_list else np.zeros((3, 0))
    prm = synth.default_params()
    prm.update(n_iter=n_iter, c=c)
    rng = np.random.default_rng(0)
    u0 = rng.standard_normal((3, n[2], n[1], n[0])) if u0 is None else u0
    return synth.Case(name="t", n=tuple(n), h=h, origin=origin, periodic=tuple(periodic),
                      xp=np.ascontiguousarray(xp, dtype=np.float64),
                      up=np.zeros((3, npart)) if up is None else up,
                      wp=np.zeros((3, npart)) if wp is None else wp,
                      radius=np.ones(npart), mass=np.ones(npart), moff=moff,
                      body=np.ascontiguousarray(body), dV=np.asarray(dV, dtype=np.float64),
                      u0=u0, params=prm)


def _node_coords(n, h, origin):
    return [origin[a] + (np.arange(n[a]) + 0.5) * h for a in range(3)]


def test_shell_volume_and_marker_counts():
    """N_l dV_l equals the shell volume 4/3 pi [(d/2+h/2)^3 - (d/2-h/2)^3]
    (Sec. 2.1) and the marker counts of the workloads are 805/453/1019."""
    assert [synth.n_markers(d) for d in (16.0, 12.0, 18.0)] == [805, 453, 1019]
    for d in (8.0, 12.0, 16.0, 18.0, 23.7):
        for h in (1.0, 0.5):
            nl = synth.n_markers(d, h)
            shell = 4.0 / 3.0 * math.pi * ((d / 2 + h / 2) ** 3 - (d / 2 - h / 2) ** 3)
            assert nl * synth.marker_volume(d, h, nl) == pytest.approx(shell, rel=1e-14)


def test_spiral_points_on_sphere_and_balanced():
    pts = synth.spiral_points(805)
    assert np.allclose(np.linalg.norm(pts, axis=1), 1.0, atol=1e-14)
    assert np.linalg.norm(pts.mean(axis=0)) < 5e-3


def test_interpolation_equals_full_grid_sum(oracle_lib):
    """U_l = sum over ALL nodes of u(x) delta_h(x - X_l) h^3 (Sec. 2.2.2, step 1)
    computed by brute force with minimum-image distances on a periodic grid;
    markers straddle the periodic seam."""
    n = (7, 6, 8)
    rng = np.random.default_rng(1)
    xp = np.array([[0.2], [5.7], [3.1]])
    body = rng.uniform(-1.0, 1.0, (3, 9))
    c = _case(n, xp, [body], [0.9], n_iter=1)
    res = oracle_lib.forcing(c, want_U=True)
    X = xp + body
    coords = _node_coords(n, 1.0, (0, 0, 0))
    for l in range(body.shape[1]):
        acc = np.zeros(3)
        for k in range(n[2]):
            for j in range(n[1]):
                for i in range(n[0]):
                    w = 1.0
                    for a, idx in enumerate((i, j, k)):
                        d = coords[a][idx] - X[a, l]
                        d -= n[a] * round(d / n[a])
                        w *= oracle_lib.phi3(d)
                    acc += w * c.u0[:, k, j, i]
        assert np.allclose(res["U"][0, :, l], acc, rtol=0, atol=1e-13)


def test_constant_and_linear_fields_interpolate_exactly(oracle_lib):
    """sum w = 1 and zero first moment make interpolation exact for constant
    and linear fields (walls in z, particle well inside)."""
    n = (24, 24, 24)
    h = 0.7
    coords = _node_coords(n, h, (0.0, 0.0, 0.0))
    Z, Y, Xg = np.meshgrid(coords[2], coords[1], coords[0], indexing="ij")
    a0 = np.array([0.3, -1.2, 2.0])
    B = np.array([[0.1, -0.4, 0.25], [0.7, 0.05, -0.3], [-0.2, 0.6, 0.15]])
    u_lin = np.stack([a0[cmp] + B[cmp, 0] * Xg + B[cmp, 1] * Y + B[cmp, 2] * Z for cmp in range(3)])
    xp = np.array([[8.3], [8.1], [8.6]])
    body = synth.spiral_points(200).T * 3.1
    c = _case(n, xp, [body], [0.5 * h ** 3], periodic=(1, 1, 0), h=h, u0=u_lin)
    U = oracle_lib.forcing(c, want_U=True)["U"][0]
    X = xp + body
    exact = a0[:, None] + B @ X
    assert np.abs(U - exact).max() < 1e-12
    c2 = _case(n, xp, [body], [0.5 * h ** 3], periodic=(1, 1, 0), h=h,
               u0=np.broadcast_to(a0[:, None, None, None], u_lin.shape).copy())
    U2 = oracle_lib.forcing(c2, want_U=True)["U"][0]
    assert np.abs(U2 - a0[:, None]).max() < 1e-13


def test_rigid_body_flow_gives_zero_forcing(oracle_lib):
    """A fluid already moving with the particle's rigid-body velocity
    u_p + omega_p x (x - x_p) needs no forcing: F = 0, f = 0, S = T = 0 and the
    velocity is unchanged (Sec. 2.1 desired velocity; interpolation exact for
    linear fields)."""
    n = (32, 32, 32)
    coords = _node_coords(n, 1.0, (0.0, 0.0, 0.0))
    Z, Y, Xg = np.meshgrid(coords[2], coords[1], coords[0], indexing="ij")
    xc = np.array([16.2, 15.7, 16.4])
    upv = np.array([0.3, -0.1, 0.2])
    w = np.array([0.05, -0.07, 0.02])
    R = np.stack([Xg - xc[0], Y - xc[1], Z - xc[2]])
    u = np.stack([upv[0] + w[1] * R[2] - w[2] * R[1],
                  upv[1] + w[2] * R[0] - w[0] * R[2],
                  upv[2] + w[0] * R[1] - w[1] * R[0]])
    body = synth.spiral_points(453).T * 6.0
    c = _case(n, xc[:, None], [body], [1.0], u0=u, up=upv[:, None], wp=w[:, None], n_iter=3)
    r = oracle_lib.forcing(c)
    assert np.abs(r["f_tot"]).max() < 1e-13
    assert np.abs(r["S"]).max() < 1e-11 and np.abs(r["T"]).max() < 1e-11
    assert np.abs(r["u"] - u).max() < 1e-13
    assert r["resid"].max() < 1e-11


def test_rigid_rotation_sign_matters(oracle_lib):
    """The reversed cross product (o x omega) does not reproduce the rigid
    rotation: guards the orientation of U^d."""
    n = (32, 32, 32)
    coords = _node_coords(n, 1.0, (0.0, 0.0, 0.0))
    Z, Y, Xg = np.meshgrid(coords[2], coords[1], coords[0], indexing="ij")
    xc = np.array([16.2, 15.7, 16.4])
    w = np.array([0.0, 0.0, 0.1])
    u = np.stack([-w[2] * (Y - xc[1]), w[2] * (Xg - xc[0]), 0 * Z])
    body = synth.spiral_points(100).T * 5.0
    good = _case(n, xc[:, None], [body], [1.0], u0=u, wp=w[:, None])
    bad = _case(n, xc[:, None], [body], [1.0], u0=u, wp=-w[:, None])
    assert oracle_lib.forcing(good)["resid"][0] < 1e-12
    assert oracle_lib.forcing(bad)["resid"][0] > 1.0


def test_force_and_torque_conservation(oracle_lib):
    """Spreading conserves the force and its first moment: sum_x f_tot h^3 =
    sum_p S_p and, for a particle away from the periodic seam,
    sum_x (x - x_p) x f_tot h^3 = T_p (Sec. 2.2.2 step 3 with the moment
    conditions)."""
    c = synth.make_case("single_sphere_64")
    c.params["n_iter"] = 3
    r = oracle_lib.forcing(c)
    h3 = c.h ** 3
    assert np.allclose(r["f_tot"].sum(axis=(1, 2, 3)) * h3, r["S"][:, 0], rtol=1e-12, atol=1e-10)
    coords = _node_coords(c.n, c.h, c.origin)
    Z, Y, Xg = np.meshgrid(coords[2], coords[1], coords[0], indexing="ij")
    xc = c.xp[:, 0]
    R = np.stack([Xg - xc[0], Y - xc[1], Z - xc[2]])
    f = r["f_tot"]
    mom = np.array([(R[1] * f[2] - R[2] * f[1]).sum(), (R[2] * f[0] - R[0] * f[2]).sum(),
                    (R[0] * f[1] - R[1] * f[0]).sum()]) * h3
    assert np.allclose(mom, r["T"][:, 0], rtol=1e-11, atol=1e-9)


def test_spread_is_adjoint_of_interpolation(oracle_lib):
    """<I v, F>_dV = <v, S F>_h^3 for arbitrary fields: the marker-volume
    weighted interpolation and the spreading are transposes (Sec. 2.2.2 steps
    1 and 3).  Uses a 4-particle polydisperse periodic case, one pass."""
    c = synth.small_case(7, periodic=(1, 1, 1), disable_mode=0, n_iter=1)
    rng = np.random.default_rng(9)
    v = rng.standard_normal(c.u0.shape)
    ru = oracle_lib.forcing(c, want_U=True)
    rv = oracle_lib.forcing(c, u0=v, want_U=True)
    F = np.zeros((3, c.nm))
    dVl = np.repeat(c.dV, np.diff(c.moff))
    pid = np.repeat(np.arange(c.np_), np.diff(c.moff))
    o = c.body
    Ud = c.up[:, pid] + np.cross(c.wp[:, pid].T, o.T).T
    F = (Ud - ru["U"][0]) / c.params["c"]
    lhs = np.sum(dVl * np.sum(rv["U"][0] * F, axis=0))
    rhs = np.sum(v * ru["f_tot"]) * c.h ** 3
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_update_independent_of_c(oracle_lib):
    """u^n and c f_tot do not depend on 2 alpha_k dt (steps 2 and 4)."""
    c = synth.small_case(8, periodic=(1, 1, 1), disable_mode=0, n_iter=3)
    a = oracle_lib.forcing(c, c=0.3)
    b = oracle_lib.forcing(c, c=1.7)
    assert np.abs(a["u"] - b["u"]).max() < 1e-12
    assert np.abs(0.3 * a["f_tot"] - 1.7 * b["f_tot"]).max() < 1e-12
    assert np.allclose(a["resid"], b["resid"], rtol=1e-12)


@pytest.mark.parametrize("kernel,sumsq", [(3, 0.5), (4, 0.375)])
def test_isolated_markers_closed_form_decay(oracle_lib, kernel, sumsq):
    """Markers whose supports do not overlap: each pass multiplies the no-slip
    error by exactly (1 - dV/h^3 (sum phi^2)^3), from steps 1-4 and the
    kernel's sum of squares (1/2 for phi3, 3/8 for phi4)."""
    n = (40, 40, 40)
    h = 1.0
    rng = np.random.default_rng(5)
    xp = np.array([[6.3, 17.1, 30.6], [8.7, 24.2, 12.5], [20.2, 9.9, 31.3]])
    bodies = [rng.uniform(-0.5, 0.5, (3, 1)) for _ in range(3)]
    dV = [0.8, 1.1, 1.4]
    upv = rng.standard_normal((3, 3))
    c = _case(n, xp, bodies, dV, n_iter=5, up=upv, c=0.41)
    c.params["kernel"] = kernel
    r = oracle_lib.forcing(c, want_U=True)
    for p in range(3):
        rs = [upv[:, p] - r["U"][m, :, p] for m in range(5)]
        fac = 1.0 - dV[p] * sumsq ** 3
        for m in range(4):
            assert np.allclose(rs[m + 1], fac * rs[m], rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("name", ["single_sphere_64", "suspension_128"])
def test_residual_decays_monotonically(oracle_lib, name):
    """More outer forcing passes reduce the no-slip error (Sec. 2.2.2)."""
    c = synth.make_case(name)
    mask = None
    if c.np_ > 1:
        pl = oracle_lib.pairs(c)
        mask = oracle_lib.marker_mask(c, pl)
    r = oracle_lib.forcing(c, mask=mask, n_iter=4)
    res = r["resid"]
    assert np.all(np.diff(res) < 0)
    assert res[-1] < 0.2 * res[0]


def test_smooth_field_interpolation_second_order(oracle_lib):
    """Interpolating the Taylor-Green field of Sec. 3.1 (sampled at the
    nodes) to a fixed circle of markers converges at second order in h."""
    errs = []
    L = 2.0
    for nn in (16, 32, 64):
        h = L / nn
        n = (nn, nn, 4)
        coords = _node_coords(n, h, (0.0, 0.0, 0.0))
        Z, Y, Xg = np.meshgrid(coords[2], coords[1], coords[0], indexing="ij")
        k = math.pi
        u = np.stack([np.sin(k * Xg) * np.cos(k * Y), -np.cos(k * Xg) * np.sin(k * Y), 0 * Z])
        th = np.linspace(0, 2 * math.pi, 60, endpoint=False)
        X = np.stack([1.0 + 0.45 * np.cos(th), 1.0 + 0.45 * np.sin(th), np.full_like(th, 2 * h)])
        xp = np.array([[1.0], [1.0], [2 * h]])
        c = _case(n, xp, [X - xp], [h ** 3], h=h, u0=u)
        U = oracle_lib.forcing(c, want_U=True)["U"][0]
        ex = np.stack([np.sin(k * X[0]) * np.cos(k * X[1]), -np.cos(k * X[0]) * np.sin(k * X[1])])
        errs.append(np.abs(U[:2] - ex).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.8 < r < 2.3 for r in rates), (errs, rates)


def test_wall_support_domain_error(oracle_lib):
    """A marker closer than 1h to a wall (cell-centred nodes) has a support
    node beyond the wall: the call is rejected; at >= 1h it is accepted."""
    n = (16, 16, 16)
    xp = np.array([[8.0], [8.0], [3.0]])
    ok = _case(n, xp, [np.array([[0.0], [0.0], [-2.0]])], [1.0], periodic=(1, 1, 0))
    oracle_lib.forcing(ok)
    bad = _case(n, xp, [np.array([[0.0], [0.0], [-2.05]])], [1.0], periodic=(1, 1, 0))
    with pytest.raises(oracle_lib.OracleError) as e:
        oracle_lib.forcing(bad)
    assert e.value.code == oracle_lib.EDOMAIN
    masked = oracle_lib.forcing(bad, mask=np.zeros(1, np.uint8))
    assert np.abs(masked["f_tot"]).max() == 0.0
