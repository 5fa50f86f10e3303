"""Grids whose components span 4 GB or more (FP64 1024 x 1024 x 512, FP32
1024^3), where the forcing kernels address the grid by 64-bit offsets instead
of 32-bit ones.  One sphere sits in a velocity field of period 64 along every
axis, so its local problem is the same as that of the sphere at the same
position modulo 64 in a periodic 64^3 grid, which runs with 32-bit offsets
and with the tiles aligned alike (64 is a multiple of every tile edge used).
The marker positions x_p + o and the field's cosines round differently at the
two magnitudes, so the two runs agree to rounding, not bit for bit: u and f_tot over the 64^3 window
around the sphere and the particle sums must match to the precision's
tolerance, the rest of the large grid stay untouched, and the 64^3 result
must agree with the oracle."""
import numpy as np
import pytest

import oracle
from paper_2109_03972_amd import ibmx, synth
from _util import rel_err, require_gpu

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-4}


def _case(n, xp, seed=11):
    rng = np.random.default_rng(seed)
    diam = np.array([16.0])
    moff, body, dV = synth.build_markers(diam, 1.0, rng)
    params = synth.default_params()
    params["n_iter"] = 3
    params["disable_mode"] = 0
    return synth.Case(name="one_sphere", n=tuple(n), h=1.0, origin=(0.0, 0.0, 0.0),
                      periodic=(1, 1, 1), xp=np.asarray(xp, dtype=np.float64).reshape(3, 1),
                      up=np.array([[0.03], [-0.05], [0.02]]), wp=np.array([[0.01], [0.02], [-0.015]]),
                      radius=0.5 * diam, mass=1.3 * np.pi / 6.0 * diam ** 3, moff=moff, body=body,
                      dV=dV, u0=None, params=params)


def _field(n, dtype, dev):
    """u_c(i, j, k) = a_c cos(2 pi (m_c i / 64 + p_c)) cos(2 pi q_c j / 64) cos(2 pi r_c k / 64
    + s_c): period 64 along every axis, built by broadcasting on the device."""
    import torch
    nx, ny, nz = n
    modes = [(1.0, 1, 0.1, 2, 3, 0.3), (-0.7, 2, 0.0, 1, 1, 0.7), (0.5, 3, 0.4, 4, 2, 0.2)]
    u = torch.empty((3, nz, ny, nx), dtype=dtype, device=dev)
    two_pi = 2.0 * np.pi
    for c, (a, m, p, q, r, s) in enumerate(modes):
        cx = torch.cos(two_pi * (m * torch.arange(nx, dtype=torch.float64, device=dev) / 64.0 + p))
        cy = torch.cos(two_pi * q * torch.arange(ny, dtype=torch.float64, device=dev) / 64.0)
        cz = torch.cos(two_pi * (r * torch.arange(nz, dtype=torch.float64, device=dev) / 64.0 + s))
        u[c] = (a * cz[:, None, None] * cy[None, :, None] * cx[None, None, :]).to(dtype)
    return u


def _run(case, u, dev, tile):
    import torch
    f64 = torch.float64
    prec = "f64" if u.dtype == torch.float64 else "f32"
    D = {k: torch.as_tensor(getattr(case, k), dtype=f64).to(dev).contiguous()
         for k in ("xp", "up", "wp", "body", "dV")}
    plan = ibmx.Plan.from_case(case, prec)
    plan.set_markers(D["body"], D["dV"])
    plan.set_tiles(*tile)
    f = torch.zeros_like(u)
    resid = torch.zeros(int(case.params["n_iter"]) + 1, dtype=f64, device=dev)
    S, Tq = plan.forcing(u, f, D["xp"], D["up"], D["wp"], resid=resid)
    plan.check("forcing")
    torch.cuda.synchronize()
    plan.close()
    return f, S, Tq, resid


@pytest.mark.parametrize("precision,n", [("f64", (1024, 1024, 512)), ("f32", (1024, 1024, 1024))])
def test_component_over_4gb_matches_periodic_window(precision, n):
    import torch
    dev = require_gpu()
    T = torch.float64 if precision == "f64" else torch.float32
    elem = 8 if precision == "f64" else 4
    assert n[0] * n[1] * n[2] * elem >= 1 << 32     # the 64-bit offset kernels
    tile = (16, 16, 8)
    x_small = np.array([30.3, 33.7, 28.9])
    block = np.array([9, 3, 5])                      # the window of the large grid
    x_big = x_small + 64.0 * block
    print(f"large grid {precision} {n}: sphere at {x_big}", flush=True)

    small = _case((64, 64, 64), x_small)
    u_s = _field((64, 64, 64), T, dev)
    u_s0 = u_s.clone()
    f_s, S_s, T_s, r_s = _run(small, u_s, dev, tile)

    big = _case(n, x_big)
    u_b = _field(n, T, dev)
    x0, y0, z0 = (64 * block).tolist()
    win = (slice(None), slice(z0, z0 + 64), slice(y0, y0 + 64), slice(x0, x0 + 64))
    u_b0_win = u_b[win].clone()
    f_b, S_b, T_b, r_b = _run(big, u_b, dev, tile)

    tol = TOL[precision]
    for name, a, b in (("S", S_b, S_s), ("T", T_b, T_s), ("u window", u_b[win], u_s),
                       ("f_tot window", f_b[win], f_s), ("resid", r_b, r_s)):
        e = rel_err(a.double().cpu().numpy(), b.double().cpu().numpy())
        assert e <= tol, f"{name}: large grid against the 64^3 window {e:.3e}"
    # outside the window nothing moved: f_tot zero, u still the field
    assert torch.count_nonzero(f_s).item() > 0
    f_b[win] = 0
    assert torch.count_nonzero(f_b).item() == 0
    del f_b
    u_b[win] = u_b0_win
    assert torch.equal(u_b, _field(n, T, dev))
    del u_b
    torch.cuda.empty_cache()

    # the 64^3 problem against the oracle
    ref = oracle.forcing(small, u0=u_s0.double().cpu().numpy())
    for name, got in (("u", u_s), ("f_tot", f_s), ("S", S_s), ("T", T_s)):
        e = rel_err(got.double().cpu().numpy(), ref[name])
        assert e <= tol, f"{name}: {e:.3e}"


def test_fluid_steps_over_4gb():
    """The fluid stencils on a 1024 x 1024 x 512 grid with walls in z (FP32
    fields; the FP64 real grid spans 4 GB, so they address by 64-bit
    offsets): predictor planes at the walls and in the middle against the
    oracle run on the three-plane slab around each, the projected faces
    divergence-free to FP32 rounding, and the implicit step (pressure term
    included) leaving the real-space residual of its equation at FP32
    rounding on sampled planes."""
    import torch
    from oracle import fluid_stage as fs
    dev = require_gpu()
    n = (1024, 1024, 512)
    nx, ny, nz = n
    assert nx * ny * nz * 8 >= 1 << 32
    case = _case(n, [100.5, 200.5, 300.5])
    case.periodic = (1, 1, 0)
    alpha, gamma, zeta, dt = 1.0 / 15.0, 5.0 / 12.0, -17.0 / 60.0, 1.0
    prm = dict(case.params)
    prm["c"] = 2.0 * alpha * dt
    prm["nu_f"] = 0.3
    case.params = prm
    plan = ibmx.Plan.from_case(case, "f32")
    g = torch.Generator(device=dev).manual_seed(5)
    u = torch.randn((3, nz, ny, nx), device=dev, generator=g)
    Nb = (0.1 * torch.randn((3, nz, ny, nx), device=dev, generator=g)).contiguous()
    P = (0.01 * torch.randn((nz, ny, nx), device=dev, generator=g)).contiguous()
    N0 = Nb.clone()
    ut, lapnu = plan.fluid_predictor(u, Nb, P, dt, gamma, zeta)
    plan.check("predictor")
    torch.cuda.synchronize()
    for k in (0, 1, nz // 2, nz - 2, nz - 1):
        lo, hi = max(k - 1, 0), min(k + 2, nz)
        ref = fs.predictor(u[:, lo:hi].double().cpu().numpy(), N0[:, lo:hi].double().cpu().numpy(),
                           P[lo:hi].double().cpu().numpy(), case.h, prm["nu_f"], alpha, gamma,
                           zeta, dt, (1, 1, 0))
        for name, got in (("u", ut), ("N", Nb), ("lapnu", lapnu)):
            e = rel_err(got[:, k].double().cpu().numpy(), ref[name][:, k - lo])
            assert e <= 2e-6, f"plane {k} {name}: {e:.3e}"
    del N0, Nb
    # implicit step with the pressure term; residual on sampled planes
    rhs_u = ut.clone()
    plan.fluid_helmholtz(ut, lapnu, P, dt, 1.0)
    plan.check("helmholtz")
    torch.cuda.synchronize()
    beta = alpha * dt * prm["nu_f"]
    for k in (0, nz // 3, nz - 1):
        lo, hi = max(k - 1, 0), min(k + 2, nz)
        for b in range(3):
            us = ut[b, lo:hi].double()
            m = k - lo
            lap = torch.zeros_like(us[m])
            for ax in (0, 1):
                lap += (torch.roll(us[m], -1, dims=ax) - 2.0 * us[m] + torch.roll(us[m], 1, dims=ax))
            up = us[m + 1] if k + 1 < nz else -us[m]
            dn = us[m - 1] if k > 0 else -us[m]
            lap += up - 2.0 * us[m] + dn
            Pd = P[lo:hi].double()
            if b == 2:
                gp = (Pd[m + 1] - Pd[m]) if k + 1 < nz else torch.zeros_like(Pd[m])
                gm = (Pd[m] - Pd[m - 1]) if k > 0 else torch.zeros_like(Pd[m])
            else:
                ax = 1 - b   # x is the last axis of a plane, y the first
                gp = torch.roll(Pd[m], -1, dims=ax) - Pd[m]
                gm = Pd[m] - torch.roll(Pd[m], 1, dims=ax)
            rhs = rhs_u[b, k].double() + dt * (-alpha * lapnu[b, k].double() + alpha * (gp + gm))
            res = (us[m] - beta * lap - rhs).abs().max().item() / rhs.abs().max().item()
            assert res <= 1e-5, f"helmholtz plane {k} component {b}: {res:.3e}"
    del rhs_u, lapnu, ut
    # projection of the first velocity: faces divergence-free
    Pz = torch.zeros((nz, ny, nx), device=dev)
    uf, _ = plan.project(u, Pz, 0.0, want_phi=False)
    plan.check("project")
    torch.cuda.synchronize()
    worst = 0.0
    for k in (0, nz // 2, nz - 1):
        div = torch.zeros((ny, nx), dtype=torch.float64, device=dev)
        div += uf[0, k].double() - torch.roll(uf[0, k].double(), 1, dims=1)
        div += uf[1, k].double() - torch.roll(uf[1, k].double(), 1, dims=0)
        div += uf[2, k].double() - (uf[2, k - 1].double() if k > 0 else 0.0)
        worst = max(worst, div.abs().max().item())
    scale = uf.abs().max().item()
    assert worst <= 1e-5 * scale, f"max |div u_f| {worst:.3e} (scale {scale:.3e})"
    assert torch.all(uf[2][-1] == 0)
    plan.close()
