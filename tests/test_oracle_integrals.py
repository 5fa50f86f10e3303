"""Pins of the oracle's level-set volume fraction and particle integrals
(Sec. 2.2.9: alpha from the signed corner distances, the midpoint sums of u
and r x u over the particle) and of the grid mean (Sec. 2.2.4)."""
import math

import numpy as np
import pytest

from paper_2109_03972_amd import synth


def sphere_case(d, n, centres, periodic=(1, 1, 1), radii=None):
    centres = np.asarray(centres, dtype=np.float64).reshape(-1, 3).T
    k = centres.shape[1]
    radius = np.full(k, d / 2.0) if radii is None else np.asarray(radii, dtype=np.float64)
    return synth.Case(name="spheres", n=(n, n, n), h=1.0, origin=(0.0, 0.0, 0.0),
                      periodic=periodic, xp=np.ascontiguousarray(centres),
                      up=np.zeros((3, k)), wp=np.zeros((3, k)), radius=radius,
                      mass=np.ones(k), moff=np.zeros(k + 1, dtype=np.int32),
                      body=np.zeros((3, 0)), dV=np.ones(k), u0=None,
                      params=synth.default_params())


def node_coords(n):
    x = np.arange(n) + 0.5
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return X, Y, Z


def test_cell_alpha_closed_forms(oracle_lib):
    h = 1.0
    # all corners inside / outside
    assert oracle_lib.cell_alpha([-0.5, -0.5, -0.5], h, 5.0) == 1.0
    assert oracle_lib.cell_alpha([10.0, 0.0, 0.0], h, 5.0) == 0.0
    # a surface that is locally a plane x = f through the cell: the
    # level-set fraction is f exactly for a plane (linear phi)
    R = 1.0e6
    for f in (0.1, 0.37, 0.5, 0.83):
        # the cell spans [R - f, R - f + 1] along x from the centre: the
        # fraction f of it lies inside the surface x = R
        c0 = [R - f, -0.5, -0.5]
        a = oracle_lib.cell_alpha(c0, h, R)
        assert a == pytest.approx(f, abs=1e-6)
    # alpha lies in [0, 1] for random cells near the surface
    rng = np.random.default_rng(3)
    for _ in range(200):
        c0 = rng.uniform(-7, 6, 3)
        a = oracle_lib.cell_alpha(c0, h, 6.0)
        assert 0.0 <= a <= 1.0


def test_volume_second_order(oracle_lib):
    errs = []
    for d in (8, 16, 32):
        n = int(1.5 * d) + 4
        ctr = [n / 2 + 0.37, n / 2 + 0.11, n / 2 + 0.23]
        c = sphere_case(d, n, [ctr])
        u = np.zeros((3, n, n, n))
        u[0] = 1.0
        V = oracle_lib.particle_integrals(c, u=u)["Iu"][0, 0]
        errs.append((V - math.pi * d ** 3 / 6) / (math.pi * d ** 3 / 6))
    for a, b in zip(errs, errs[1:]):
        assert 3.5 < a / b < 4.5
    assert abs(errs[-1]) < 2e-3


def test_rigid_rotation_moment_of_inertia(oracle_lib):
    w = np.array([0.3, -0.2, 1.0])
    errs = []
    for d in (8, 16, 32):
        n = int(1.5 * d) + 4
        ctr = np.array([n / 2 + 0.37, n / 2 + 0.11, n / 2 + 0.23])
        c = sphere_case(d, n, [ctr])
        X, Y, Z = node_coords(n)
        rx, ry, rz = X - ctr[0], Y - ctr[1], Z - ctr[2]
        u = np.stack([w[1] * rz - w[2] * ry, w[2] * rx - w[0] * rz, w[0] * ry - w[1] * rx])
        Ir = oracle_lib.particle_integrals(c, u=u)["Ir"][:, 0]
        I = 8 * math.pi * (d / 2) ** 5 / 15           # unit-density sphere
        errs.append(np.abs(Ir - I * w).max() / (I * np.abs(w).max()))
    assert errs[2] < errs[1] < errs[0] < 3e-3


def test_uniform_field_and_symmetric_first_moment(oracle_lib):
    n, d = 40, 14
    ctr = [20.5, 19.5, 20.5]            # a cell centre: its box is mirror-symmetric
    c = sphere_case(d, n, [ctr])
    U = np.array([0.7, -1.3, 2.1])
    u = np.broadcast_to(U[:, None, None, None], (3, n, n, n)).copy()
    r = oracle_lib.particle_integrals(c, u=u)
    V = r["Iu"][0, 0] / U[0]
    np.testing.assert_allclose(r["Iu"][:, 0], V * U, rtol=1e-12)
    # sum alpha r = 0 by the mirror symmetries of the placement, so
    # Ir = (sum alpha h^3 r) x U vanishes
    assert np.abs(r["Ir"][:, 0]).max() < 1e-11 * V * d * np.abs(U).max()


def test_periodic_images_and_alpha_field(oracle_lib):
    """A particle across the periodic seams gives the same integrals as the
    same particle shifted by whole cells into the interior; alpha summed over
    the grid equals the volume."""
    n, d = 32, 12
    rng = np.random.default_rng(7)
    X, Y, Z = node_coords(n)
    u = np.stack([np.sin(2 * np.pi * X / n) + 0.3 * Y / n, np.cos(2 * np.pi * Z / n),
                  0.2 * X / n + np.sin(2 * np.pi * Y / n)])
    inner = np.array([15.27, 16.61, 14.93])
    shift = np.array([-13, 17, -12])          # whole cells: seams on every axis
    seam = (inner + shift) % n
    a = oracle_lib.particle_integrals(sphere_case(d, n, [inner]),
                                      u=np.roll(u, shift=(12, -17, 13), axis=(1, 2, 3)),
                                      want_alpha=True)
    b = oracle_lib.particle_integrals(sphere_case(d, n, [seam]), u=u, want_alpha=True)
    np.testing.assert_allclose(b["Iu"], a["Iu"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(b["Ir"], a["Ir"], rtol=1e-12, atol=1e-12)
    ones = np.zeros((3, n, n, n))
    ones[0] = 1.0
    V = oracle_lib.particle_integrals(sphere_case(d, n, [seam]), u=ones)["Iu"][0, 0]
    assert b["alpha"].sum() == pytest.approx(V, rel=1e-12)
    assert b["alpha"].min() >= 0.0 and b["alpha"].max() <= 1.0


def test_wall_cells_skipped(oracle_lib):
    """On a wall axis the cells beyond the wall are not summed: a sphere
    overlapping the lower z wall loses exactly the part of its volume
    fraction that lies below it."""
    n, d = 32, 12
    ones = np.zeros((3, n, n, n))
    ones[0] = 1.0
    free = sphere_case(d, n, [[16.3, 15.8, 16.4]], periodic=(1, 1, 0))
    cut = sphere_case(d, n, [[16.3, 15.8, 4.4]], periodic=(1, 1, 0))
    Vf = oracle_lib.particle_integrals(free, u=ones)["Iu"][0, 0]
    r = oracle_lib.particle_integrals(cut, u=ones, want_alpha=True)
    assert r["Iu"][0, 0] < Vf
    assert r["alpha"].sum() == pytest.approx(r["Iu"][0, 0], rel=1e-12)


def test_grid_mean(oracle_lib):
    n = 12
    c = sphere_case(4, n, [[6.0, 6.0, 6.0]])
    X, Y, Z = node_coords(n)
    f = np.stack([np.sin(2 * np.pi * X / n) + 1.5, np.cos(2 * np.pi * Y / n) - 2.0,
                  0.25 * np.ones_like(Z)])
    np.testing.assert_allclose(oracle_lib.grid_mean(c, f), [1.5, -2.0, 0.25], atol=1e-14)
