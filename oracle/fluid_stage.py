"""Plain FP64 numpy oracle of the predictor steps of the collocated fluid
solver (eq. fluid-solver, steps a and e).

TEST INFRASTRUCTURE ONLY: used by the test suite and the smoke check,
never by the product path.  It shares no code with the HIP library.

Conventions as in oracle.projection.  Velocity vanishes on a wall face: a
cell next to a wall sees the ghost value -u of its own cell (the linear
profile through zero on the face); pressure has zero normal gradient there
(ghost value = its own).  With c = 2 alpha_k dt:

  step a:  u~ = u + dt (2 alpha nu L u - 2 alpha grad P - gamma N - zeta N_prev)
           N = (u . grad) u, both with second-order central differences;
  step e:  (I - alpha dt nu L) u* = u_f - c fbar + dt (-alpha nu L u + 2 alpha theta grad P)
           where u_f = u~ + c f_IBM is the velocity after the forcing loop,
           fbar the mean IBM force (triply periodic cases, else 0) and L u
           the Laplacian of the stage's input velocity (kept from step a).
L is the 7-point Laplacian, grad P the mean of the cell's two face
gradients (oracle.projection.cell_grad).
"""
from __future__ import annotations

import numpy as np

from .projection import AXES, cell_grad


def _nb(f, a, d, periodic, ghost_sign):
    """f at the neighbour d (+1/-1) along axis a; past a wall the ghost
    ghost_sign * f of the cell itself."""
    g = np.roll(f, -d, axis=AXES[a])
    if not periodic[a]:
        idx = [slice(None)] * 3
        idx[AXES[a]] = -1 if d > 0 else 0
        g[tuple(idx)] = ghost_sign * f[tuple(idx)]
    return g


def laplacian(u, h, periodic):
    """Vector 7-point Laplacian with zero velocity on wall faces."""
    out = np.zeros_like(u)
    for b in range(3):
        acc = np.zeros(u.shape[1:])
        for a in range(3):
            acc += (_nb(u[b], a, 1, periodic, -1.0) - 2.0 * u[b] + _nb(u[b], a, -1, periodic, -1.0)) / (h * h)
        out[b] = acc
    return out


def advection(u, h, periodic):
    """N_b = sum_a u_a (u_b(+a) - u_b(-a)) / 2h."""
    out = np.zeros_like(u)
    for b in range(3):
        acc = np.zeros(u.shape[1:])
        for a in range(3):
            d = (_nb(u[b], a, 1, periodic, -1.0) - _nb(u[b], a, -1, periodic, -1.0)) / (2.0 * h)
            acc += u[a] * d
        out[b] = acc
    return out


def predictor(u, N_prev, P, h, nu, alpha, gamma, zeta, dt, periodic):
    """Step a: returns u~, N = (u.grad)u and nu L u of the input velocity."""
    periodic = tuple(bool(p) for p in periodic)
    lapnu = nu * laplacian(u, h, periodic)
    N = advection(u, h, periodic)
    gP = cell_grad(P, h, periodic)
    ut = u + dt * (2.0 * alpha * lapnu - 2.0 * alpha * gP - gamma * N - zeta * N_prev)
    return dict(u=ut, N=N, lapnu=lapnu)


def helmholtz_solve(rhs, beta, h, periodic):
    """x with x - beta L x = rhs (one component, wall faces x = 0).

    Fourier modes along periodic x and y; along z either modes (periodic)
    or, per (kx, ky), the dense matrix of the wall-bounded second difference.
    """
    if not (periodic[0] and periodic[1]):
        raise ValueError("the Helmholtz solve needs periodic x and y")
    nz, ny, nx = rhs.shape
    lam = lambda n: (2.0 * np.cos(2.0 * np.pi * np.arange(n) / n) - 2.0) / (h * h)
    lxy = lam(ny)[:, None] + lam(nx)[None, :]
    if periodic[2]:
        R = np.fft.fftn(rhs)
        L = lam(nz)[:, None, None] + lxy[None, :, :]
        return np.real(np.fft.ifftn(R / (1.0 - beta * L)))
    R = np.fft.fft2(rhs, axes=(1, 2))
    X = np.empty_like(R)
    D = np.zeros((nz, nz))
    for k in range(nz):
        D[k, k] = -2.0
        if k > 0:
            D[k, k - 1] = 1.0
        if k < nz - 1:
            D[k, k + 1] = 1.0
    D[0, 0] = D[-1, -1] = -3.0 if nz > 1 else -4.0
    D /= h * h
    for j in range(ny):
        for i in range(nx):
            A = np.eye(nz) - beta * (D + lxy[j, i] * np.eye(nz))
            X[:, j, i] = np.linalg.solve(A, R[:, j, i])
    return np.real(np.fft.ifft2(X, axes=(1, 2)))


def helmholtz(u_forced, lapnu, P, fbar, h, nu, alpha, theta, dt, periodic):
    """Step e: u* from the forced velocity (see the module text)."""
    periodic = tuple(bool(p) for p in periodic)
    c = 2.0 * alpha * dt
    gP = cell_grad(P, h, periodic)
    fb = np.zeros(3) if fbar is None else np.asarray(fbar, dtype=np.float64)
    out = np.empty_like(u_forced)
    for b in range(3):
        rhs = u_forced[b] - c * fb[b] + dt * (-alpha * lapnu[b] + 2.0 * alpha * theta * gP[b])
        out[b] = helmholtz_solve(rhs, alpha * dt * nu, h, periodic)
    return out
