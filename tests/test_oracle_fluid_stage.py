"""Pins of the oracle's predictor steps of the collocated fluid solver (eq.
fluid-solver, steps a and e): the difference operators on Fourier modes and
on a wall profile, the advection of a two-mode field, and the implicit
viscous solve against a dense operator assembled cell by cell."""
import numpy as np
import pytest

from oracle import fluid_stage as fs


def _grid(nz, ny, nx, h):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return z, y, x


def test_laplacian_of_fourier_mode():
    nz, ny, nx, h = 8, 16, 32, 0.5
    z, y, x = _grid(nz, ny, nx, h)
    th = 2 * np.pi * (3 * x / nx + 2 * y / ny + 1 * z / nz)
    u = np.stack([np.cos(th), np.sin(th), 2.0 * np.cos(th)])
    lam = sum((2 * np.cos(2 * np.pi * k / n) - 2) / h ** 2 for k, n in ((3, nx), (2, ny), (1, nz)))
    np.testing.assert_allclose(fs.laplacian(u, h, (1, 1, 1)), lam * u, atol=1e-12)


def test_laplacian_of_wall_profile():
    """u = z (distance from the lower wall face) between walls: zero
    Laplacian except in the top cell, where the ghost -u gives -2 nz / h."""
    nz, ny, nx, h = 7, 4, 4, 0.5
    zc = (np.arange(nz) + 0.5) * h
    u = np.zeros((3, nz, ny, nx))
    u[0] = zc[:, None, None]
    L = fs.laplacian(u, h, (1, 1, 0))
    expect = np.zeros(nz)
    expect[-1] = -2.0 * nz / h
    np.testing.assert_allclose(L[0][:, 1, 2], expect, atol=1e-12)
    assert np.all(L[1:] == 0.0)


def test_advection_of_two_modes():
    """u = (cos(2 pi m y / ny), sin(2 pi l x / nx), 0): central differences of
    a mode are the mode's derivative times sin(k h)/(k h)."""
    nz, ny, nx, h, m, l = 4, 16, 8, 0.25, 3, 2
    z, y, x = _grid(nz, ny, nx, h)
    ty, tx = 2 * np.pi * m * y / ny, 2 * np.pi * l * x / nx
    u = np.stack([np.cos(ty), np.sin(tx), np.zeros_like(tx)])
    N = fs.advection(u, h, (1, 1, 1))
    np.testing.assert_allclose(N[0], np.sin(tx) * (-np.sin(ty) * np.sin(2 * np.pi * m / ny) / h),
                               atol=1e-12)
    np.testing.assert_allclose(N[1], np.cos(ty) * (np.cos(tx) * np.sin(2 * np.pi * l / nx) / h),
                               atol=1e-12)
    assert np.all(N[2] == 0.0)


def _dense_helmholtz(shape, h, beta, periodic):
    """I - beta L written cell by cell: each neighbour couples with 1/h^2; a
    missing neighbour behind a wall contributes the ghost -u (-1/h^2 on the
    diagonal)."""
    nz, ny, nx = shape
    n = nx * ny * nz
    A = np.eye(n)
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
                        A[c, c] += beta * 2.0 / (2 * h * h)      # the -2/h^2 of L, half per side
                        if not 0 <= q[a] < dims[a]:
                            if not periodic[a]:
                                A[c, c] += beta / (h * h)        # ghost -u
                                continue
                            q[a] %= dims[a]
                        A[c, idx(*q)] -= beta / (h * h)
    return A


@pytest.mark.parametrize("periodic,shape", [((1, 1, 1), (4, 4, 8)), ((1, 1, 0), (5, 4, 4)),
                                            ((1, 1, 0), (1, 4, 8)), ((1, 1, 0), (13, 16, 8)),
                                            ((1, 1, 1), (8, 16, 16))])
def test_helmholtz_matches_dense_solve(periodic, shape):
    rng = np.random.default_rng(9)
    rhs = rng.normal(size=shape)
    beta, h = 0.37, 0.8
    x = fs.helmholtz_solve(rhs, beta, h, periodic)
    A = _dense_helmholtz(shape, h, beta, periodic)
    ref = np.linalg.solve(A, rhs.ravel())
    np.testing.assert_allclose(x.ravel(), ref, atol=1e-12 * np.abs(ref).max())
    # and the operator form with the vector Laplacian
    u = np.stack([x, np.zeros_like(x), np.zeros_like(x)])
    res = x - beta * fs.laplacian(u, h, periodic)[0] - rhs
    assert np.abs(res).max() < 1e-12 * np.abs(rhs).max()


def test_predictor_and_helmholtz_without_viscosity():
    """nu = 0: the predictor is the explicit pressure and advection update
    and the implicit step adds nothing but the forcing correction terms."""
    rng = np.random.default_rng(10)
    shape = (6, 8, 8)
    u = rng.normal(size=(3,) + shape)
    Np = rng.normal(size=(3,) + shape)
    P = rng.normal(size=shape)
    h, a, g, z, dt = 0.5, 1 / 15, 5 / 12, -17 / 60, 0.3
    r = fs.predictor(u, Np, P, h, 0.0, a, g, z, dt, (1, 1, 0))
    assert np.all(r["lapnu"] == 0.0)
    us = fs.helmholtz(r["u"], r["lapnu"], P, [0.1, 0.0, -0.2], h, 0.0, a, 1.0, dt, (1, 1, 0))
    gP = fs.cell_grad(P, h, (1, 1, 0))
    expect = r["u"] - 2 * a * dt * np.array([0.1, 0.0, -0.2])[:, None, None, None] + dt * 2 * a * gP
    np.testing.assert_allclose(us, expect, atol=1e-13)
