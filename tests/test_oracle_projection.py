"""Pins of the oracle's pressure projection (Sec. 2.2.1, eq. fluid-solver
steps f-i): the projected face velocities are discretely divergence-free,
the Poisson solution matches a dense solve of the same operator assembled
cell by cell, single Fourier modes and a through-wall flow have closed forms."""
import numpy as np
import pytest

from oracle import projection as pj


def _field(seed, shape):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, 1.0, (3,) + shape)


@pytest.mark.parametrize("periodic,shape", [((1, 1, 1), (8, 16, 8)), ((1, 1, 0), (7, 8, 16)),
                                            ((1, 1, 0), (1, 4, 4))])
def test_projected_faces_are_divergence_free(periodic, shape):
    u = _field(1, shape)
    P0 = np.random.default_rng(2).normal(size=shape)
    r = pj.project(u, P0, 0.5, 0.3, 0.02, 0.0, periodic)
    div = pj.face_div(r["uf"], 0.5, periodic)
    assert np.abs(div).max() <= 1e-12 * np.abs(r["div_star"]).max()
    assert abs(r["phi"].mean()) < 1e-14 * np.abs(r["phi"]).max()
    # the Poisson equation itself
    res = pj.compact_laplacian(r["phi"], 0.5, periodic) - r["div_star"] / 0.3
    assert np.abs(res).max() <= 1e-11 * np.abs(r["div_star"] / 0.3).max()
    if not periodic[2]:
        assert np.all(r["uf"][2][-1] == 0.0)


def _dense_laplacian(shape, h, periodic):
    """The compact Laplacian written cell by cell: each face between two
    cells couples them with weight 1/h^2; wall faces couple nothing."""
    nz, ny, nx = shape
    n = nx * ny * nz
    A = np.zeros((n, n))
    idx = lambda i, j, k: (k * ny + j) * nx + i
    dims = (nx, ny, nz)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                c = idx(i, j, k)
                for a in range(3):
                    for d in (-1, 1):
                        q = [i, j, k]
                        q[a] += d
                        if not 0 <= q[a] < dims[a]:
                            if not periodic[a]:
                                continue
                            q[a] %= dims[a]
                        A[c, idx(*q)] += 1.0 / (h * h)
                        A[c, c] -= 1.0 / (h * h)
    return A


@pytest.mark.parametrize("periodic,shape", [((1, 1, 1), (4, 4, 8)), ((1, 1, 0), (5, 4, 4)),
                                            ((1, 1, 0), (3, 8, 2)), ((1, 1, 0), (13, 16, 8)),
                                            ((1, 1, 1), (8, 16, 16))])
def test_poisson_matches_dense_solve(periodic, shape):
    rng = np.random.default_rng(3)
    rhs = rng.normal(size=shape)
    rhs -= rhs.mean()
    phi = pj.poisson(rhs, 0.7, periodic)
    A = _dense_laplacian(shape, 0.7, periodic)
    ref = np.linalg.lstsq(A, rhs.ravel(), rcond=None)[0]    # minimum norm: zero mean
    np.testing.assert_allclose(phi.ravel(), ref, atol=1e-12 * np.abs(ref).max())


def test_single_fourier_mode():
    nz, ny, nx, h = 8, 16, 32, 0.25
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    kx, ky, kz = 3, 2, 1
    rhs = np.cos(2 * np.pi * (kx * x / nx + ky * y / ny + kz * z / nz))
    lam = sum((2 * np.cos(2 * np.pi * k / n) - 2) / h ** 2 for k, n in ((kx, nx), (ky, ny), (kz, nz)))
    phi = pj.poisson(rhs, h, (1, 1, 1))
    np.testing.assert_allclose(phi, rhs / lam, atol=1e-13)


def test_through_wall_flow_is_removed():
    """A uniform vertical velocity w between walls: the projected z faces
    carry no flow, the cells next to the walls keep w/2 (their face
    gradients are w/c and 0) and the interior cells 0; horizontal
    components are untouched."""
    nz, ny, nx, w, c = 9, 4, 8, 0.6, 0.25
    u = np.zeros((3, nz, ny, nx))
    u[2] = w
    u[0] = 0.3
    r = pj.project(u, np.zeros((nz, ny, nx)), 1.0, c, 0.01, 1.0, (1, 1, 0))
    assert np.abs(r["uf"][2]).max() < 1e-13
    expect = np.zeros(nz)
    expect[0] = expect[-1] = w / 2
    np.testing.assert_allclose(r["u"][2][:, 0, 0], expect, atol=1e-13)
    np.testing.assert_allclose(r["u"][0], 0.3, atol=1e-15)


def test_pressure_update_forms():
    """theta = 0 adds phi - (c/2) nu L phi to the previous pressure, theta = 1
    replaces it."""
    shape = (6, 8, 8)
    u = _field(4, shape)
    P0 = np.random.default_rng(5).normal(size=shape)
    a = pj.project(u, P0, 1.0, 0.5, 0.1, 0.0, (1, 1, 0))
    b = pj.project(u, P0, 1.0, 0.5, 0.1, 1.0, (1, 1, 0))
    np.testing.assert_allclose(a["P"] - P0, b["P"], atol=1e-13)
    np.testing.assert_allclose(b["P"], a["phi"] - 0.25 * 0.1 * a["div_star"] / 0.5, atol=1e-12)
