"""Plain FP64 numpy oracle of the pressure projection of the collocated
fluid solver (Sec. 2.2.1 and eq. fluid-solver, steps f-i).

TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.  It shares no
code with the HIP library.

Grid conventions: fields are [nz][ny][nx] (vectors [3][nz][ny][nx]) at cell
centres, spacing h.  Axis a is periodic or bounded by walls at its two ends
(cell faces).  Face arrays hold, per cell, the normal velocity on the face
between the cell and its +a neighbour; on a wall axis the last cell's +a face
is the wall (always 0) and the first cell's -a face is the other wall.

Steps for one Runge-Kutta stage with c = 2 alpha_k dt:
  u_f* = I(u*): the mean of the two cells next to the face (linear, second
         order, as the paper states for the interpolation operator);
  div  = sum_a (u_f*[cell] - u_f*[cell - e_a]) / h, wall faces 0;
  L phi = div / c, L the compact Laplacian of the face gradients
         (phi_+ - 2 phi + phi_-)/h^2 per axis, zero normal gradient at walls;
         phi is fixed by zero mean;
  u   = u* - c grad(phi), the cell gradient being the mean of the two face
         gradients of the cell (central difference, wall face gradient 0);
  u_f = u_f* - c (phi_+ - phi)/h on interior faces;
  P   = (1 - theta) P_prev + phi - (c/2) nu L phi.
The printed pressure update multiplies the whole bracket by theta, which
would freeze P under projection (theta = 0) against the original solver's
step; it is read as incremental for theta = 0 and as a fresh pressure for
theta = 1.
"""
from __future__ import annotations

import numpy as np

AXES = (2, 1, 0)   # array axis of x, y, z in a [nz][ny][nx] field


def _shift(f, a, d):
    """f at the cell d steps along axis a (periodic wrap; callers mask walls)."""
    return np.roll(f, -d, axis=AXES[a])


def _last_mask(shape, a):
    m = np.zeros(shape, dtype=bool)
    idx = [slice(None)] * 3
    idx[AXES[a]] = -1
    m[tuple(idx)] = True
    return m


def face_interp(u, periodic):
    """u_f*[a] on the +a face of every cell (wall faces 0)."""
    uf = np.empty_like(u)
    for a in range(3):
        uf[a] = 0.5 * (u[a] + _shift(u[a], a, 1))
        if not periodic[a]:
            uf[a][_last_mask(u[a].shape, a)] = 0.0
    return uf


def face_div(uf, h, periodic):
    """Divergence of a face field: outflow minus inflow over h per axis."""
    div = np.zeros(uf.shape[1:])
    for a in range(3):
        inflow = _shift(uf[a], a, -1)
        if not periodic[a]:
            idx = [slice(None)] * 3
            idx[AXES[a]] = 0
            inflow[tuple(idx)] = 0.0           # the lower wall
        div += (uf[a] - inflow) / h
    return div


def face_grad(phi, h, periodic):
    """(phi_+ - phi)/h on the +a faces; 0 on wall faces."""
    g = np.empty((3,) + phi.shape)
    for a in range(3):
        g[a] = (_shift(phi, a, 1) - phi) / h
        if not periodic[a]:
            g[a][_last_mask(phi.shape, a)] = 0.0
    return g


def compact_laplacian(phi, h, periodic):
    return face_div(face_grad(phi, h, periodic), h, periodic)


def cell_grad(phi, h, periodic):
    """Mean of the two face gradients of each cell."""
    fg = face_grad(phi, h, periodic)
    g = np.empty_like(fg)
    for a in range(3):
        lower = _shift(fg[a], a, -1)
        if not periodic[a]:
            idx = [slice(None)] * 3
            idx[AXES[a]] = 0
            lower[tuple(idx)] = 0.0
        g[a] = 0.5 * (fg[a] + lower)
    return g


def poisson(rhs, h, periodic):
    """Zero-mean phi with compact_laplacian(phi) = rhs (rhs must sum to 0).

    Periodic x and y: discrete Fourier modes, eigenvalue (2 cos(2 pi k/n) - 2)/h^2
    per axis.  z periodic: the same; z walls: per (kx, ky) mode the tridiagonal
    second difference with zero-gradient ends, solved by elimination (the
    singular (0, 0) mode with its last value pinned, then shifted to zero mean).
    """
    if not (periodic[0] and periodic[1]):
        raise ValueError("the projection needs periodic x and y")
    nz, ny, nx = rhs.shape
    lam = lambda n: (2.0 * np.cos(2.0 * np.pi * np.arange(n) / n) - 2.0) / (h * h)
    lxy = lam(ny)[:, None] + lam(nx)[None, :]
    if periodic[2]:
        R = np.fft.fftn(rhs)
        L = lam(nz)[:, None, None] + lxy[None, :, :]
        L[0, 0, 0] = 1.0
        Phi = R / L
        Phi[0, 0, 0] = 0.0
        return np.real(np.fft.ifftn(Phi))
    R = np.fft.fft2(rhs, axes=(1, 2))
    Phi = np.empty_like(R)
    for j in range(ny):
        for i in range(nx):
            A = np.zeros((nz, nz))
            for k in range(nz):
                if k > 0:
                    A[k, k - 1] = 1.0
                    A[k, k] -= 1.0
                if k < nz - 1:
                    A[k, k + 1] = 1.0
                    A[k, k] -= 1.0
            A = A / (h * h) + lxy[j, i] * np.eye(nz)
            b = R[:, j, i].copy()
            if i == 0 and j == 0:
                A[-1, :] = 0.0
                A[-1, -1] = 1.0
                b[-1] = 0.0
            Phi[:, j, i] = np.linalg.solve(A, b)
    phi = np.real(np.fft.ifft2(Phi, axes=(1, 2)))
    return phi - phi.mean()


def project(u_star, P_prev, h, c, nu, theta, periodic):
    """One projection: returns u, u_f, P, phi and the divergence of u_f*."""
    periodic = tuple(bool(p) for p in periodic)
    uf_star = face_interp(u_star, periodic)
    div = face_div(uf_star, h, periodic)
    phi = poisson(div / c, h, periodic)
    u = u_star - c * cell_grad(phi, h, periodic)
    uf = uf_star - c * face_grad(phi, h, periodic)
    P = (1.0 - theta) * P_prev + phi - 0.5 * c * nu * compact_laplacian(phi, h, periodic)
    return dict(u=u, uf=uf, P=P, phi=phi, div_star=div)
