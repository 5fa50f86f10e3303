"""Edge cases of the forcing loop on the GPU against the FP64 oracle:
markers placed exactly on the ties of the delta's support (the marker
coordinate an integer number of h away from a node's cell face, where the
last support node has weight exactly zero and counts as outside the support)
at tile faces, at periodic seams and exactly 1.0h (three-point delta) or
1.5h (four-point delta) from a wall, where the last support node has zero
weight and may lie beyond the wall (such a marker is accepted).  The grids have walls in x
with n_x not a multiple of four, so the velocity is staged element by element
next to the x walls, in the forward and the adjoint kernels."""
import numpy as np
import pytest

import oracle
from paper_2109_03972_amd import synth
from _util import dev_case, rel_err, require_gpu

pytestmark = pytest.mark.gpu

TOL = {"f64": dict(U=1e-12, u=1e-12, f_tot=1e-12, S=1e-12, T=1e-12, resid=1e-12),
       "f32": dict(U=1e-5, u=1e-4, f_tot=1e-4, S=1e-4, T=1e-4, resid=1e-4)}


def _tie_points(n, periodic, kernel, tile, rng):
    """Marker positions with exact ties on one or all axes."""
    off = 0.0 if kernel == 3 else 0.5           # s - base shift integral
    wall = 1.0 if kernel == 3 else 1.5          # closest accepted wall distance
    L = [float(v) for v in n]
    ties = []
    for a in range(3):
        vals = [k * tile[a] + d + off for k in (1, 2) for d in (-1, 0) if k * tile[a] + 2 < n[a]]
        if periodic[a]:
            vals += [off, L[a] - 1.0 + off, L[a] - 2.0 + off]
        else:
            vals += [wall, L[a] - wall]
        ties.append(vals)
    pts = []
    for a in range(3):
        for v in ties[a]:
            # other coordinates on a 1/64 lattice: x_p + o stays exact
            X = [round(float(rng.uniform(3.0, L[b] - 3.0)) * 64.0) / 64.0 for b in range(3)]
            X[a] = v
            pts.append(X)
    # ties on all three axes at once (tile corners, seams, walls)
    for k in range(8):
        pts.append([ties[a][(k + a) % len(ties[a])] for a in range(3)])
    return np.array(pts).T


def _tie_case(seed, n, periodic, kernel, n_iter=3, tile=(16, 16, 8)):
    base = synth.small_case(seed, n=n, periodic=periodic, diameters=(9.0, 8.0, 7.0),
                            n_iter=n_iter, touch=0.0)
    if kernel == 4:
        base.params.update(kernel=4, eps_sep=2.0, lub_C=4.0, gap_cut=4.0)
    mask = oracle.marker_mask(base, oracle.pairs(base))
    rng = np.random.default_rng(seed)
    X = _tie_points(n, periodic, kernel, tile, rng)
    # a particle whose centre and offsets are exact binary fractions, so that
    # x_p + o reproduces the tie positions exactly
    xc = np.array([[n[0] / 2 + 0.25], [n[1] / 2 - 0.25], [n[2] / 2 + 0.125]])
    body = X - xc
    assert np.array_equal(xc + body, X)
    nt = X.shape[1]
    c = synth.Case(name=f"ties_{seed}", n=base.n, h=base.h, origin=base.origin,
                   periodic=base.periodic,
                   xp=np.ascontiguousarray(np.concatenate([base.xp, xc], axis=1)),
                   up=np.concatenate([base.up, rng.normal(0, 0.1, (3, 1))], axis=1),
                   wp=np.concatenate([base.wp, rng.normal(0, 0.05, (3, 1))], axis=1),
                   radius=np.concatenate([base.radius, [2.0]]),
                   mass=np.concatenate([base.mass, [1.0]]),
                   moff=np.concatenate([base.moff, [base.moff[-1] + nt]]).astype(np.int32),
                   body=np.ascontiguousarray(np.concatenate([base.body, body], axis=1)),
                   dV=np.concatenate([base.dV, [0.9]]), u0=base.u0, params=dict(base.params))
    mask = np.concatenate([mask, np.ones(nt, dtype=np.uint8)])
    return c, mask


def _run(case, precision, mask, tile):
    import torch
    from paper_2109_03972_amd import ibmx
    dev = require_gpu()
    D = dev_case(case, precision)
    plan = ibmx.Plan.from_case(case, precision)
    plan.set_markers(D["body"], D["dV"])
    plan.set_tiles(*tile)
    n_iter = int(case.params["n_iter"])
    resid = torch.zeros(n_iter + 1, dtype=torch.float64, device=dev)
    U = torch.zeros((n_iter, 3, case.nm), dtype=D["u"].dtype, device=dev)
    mk = torch.as_tensor(mask).to(dev)
    S, T = plan.forcing(D["u"], D["f"], D["xp"], D["up"], D["wp"], mask=mk, resid=resid,
                        U_debug=U)
    st = plan.status()
    torch.cuda.synchronize()
    return dict(u=D["u"].double().cpu().numpy(), f_tot=D["f"].double().cpu().numpy(),
                S=S.cpu().numpy(), T=T.cpu().numpy(), resid=resid.cpu().numpy(),
                U=U.double().cpu().numpy(), status=st), plan, D


CASES = [
    # seed, grid, periodic, kernel
    (301, (37, 40, 36), (0, 1, 1), 3),
    (302, (45, 38, 34), (0, 1, 1), 4),
    (303, (41, 36, 37), (1, 1, 0), 3),
    (304, (39, 42, 40), (1, 1, 0), 4),
]


@pytest.mark.parametrize("tile", [(16, 16, 8), (8, 8, 8)])
@pytest.mark.parametrize("seed,n,per,kernel", CASES)
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_support_ties_forward(seed, n, per, kernel, precision, tile):
    case, mask = _tie_case(seed, n, per, kernel, tile=tile)
    print(f"ties seed={seed} n={n} periodic={per} kernel={kernel} tile={tile} {precision} "
          f"nm={case.nm}", flush=True)
    ref = oracle.forcing(case, mask=mask, want_U=True)
    got, _, _ = _run(case, precision, mask, tile)
    assert got["status"] == 0
    act = mask.astype(bool)
    got["U"] = got["U"][:, :, act]
    ref["U"] = ref["U"][:, :, act]
    for k, t in TOL[precision].items():
        e = rel_err(got[k], ref[k])
        assert np.all(np.isfinite(got[k])), k
        print(f"  {k}: {e:.2e}", flush=True)
        assert e <= t, (k, e)


@pytest.mark.parametrize("seed,n,per,kernel", CASES[:2])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_support_ties_backward(seed, n, per, kernel, precision):
    """The adjoint kernels stage the cotangent grids over the same regions
    next to the x walls."""
    import torch
    case, mask = _tie_case(seed, n, per, kernel, n_iter=2)
    print(f"ties backward seed={seed} kernel={kernel} {precision}", flush=True)
    rng = np.random.default_rng(seed + 7)
    shape = (3, case.n[2], case.n[1], case.n[0])
    cot = dict(g_f=rng.standard_normal(shape), g_u=rng.standard_normal(shape),
               g_S=rng.standard_normal((3, case.np_)), g_T=rng.standard_normal((3, case.np_)))
    u0 = case.u0
    if precision == "f32":
        u0 = u0.astype(np.float32).astype(np.float64)
        for k in ("g_f", "g_u"):
            cot[k] = cot[k].astype(np.float32).astype(np.float64)
    ref = oracle.forcing_adjoint(case, u0=u0, mask=mask, **cot)
    from paper_2109_03972_amd import ibmx
    dev = require_gpu()
    D = dev_case(case, precision)
    Tt = D["u"].dtype
    plan = ibmx.Plan.from_case(case, precision)
    plan.set_markers(D["body"], D["dV"])

    def to(a, dt):
        return torch.as_tensor(a, dtype=torch.float64).to(dev).to(dt).contiguous()

    gu0, gxp, gup, gwp = plan.forcing_backward(
        D["u"], D["xp"], D["up"], D["wp"], torch.as_tensor(mask).to(dev), to(cot["g_f"], Tt),
        to(cot["g_u"], Tt), to(cot["g_S"], torch.float64), to(cot["g_T"], torch.float64))
    assert plan.status() == 0
    tol = 1e-10 if precision == "f64" else 1e-5
    for k, g in (("gu0", gu0), ("gxp", gxp), ("gup", gup), ("gwp", gwp)):
        a = g.double().cpu().numpy()
        assert np.all(np.isfinite(a)), k
        e = rel_err(a, ref[k])
        print(f"  {k}: {e:.2e}", flush=True)
        assert e <= tol, (k, e)


@pytest.mark.parametrize("kernel", [3, 4])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_dense_markers_spread_exactly(precision, kernel):
    """A caller's marker set far denser than the paper's (about 150 markers
    per h^2 of surface, so that some node lies in the supports of over a
    thousand markers): the spreading's fixed-point sums would need more
    than 32 bits at the scale of an ordinary bed, and the per-tile scale
    bound keeps them exact; every output still matches the oracle."""
    base = synth.small_case(311, n=(36, 36, 40), periodic=(1, 1, 0), diameters=(8.0,),
                            n_iter=2, touch=0.0, disable_mode=0)
    if kernel == 4:
        base.params.update(kernel=4, eps_sep=2.0, lub_C=4.0, gap_cut=4.0)
    d = 8.0
    nl = 30000
    body = np.ascontiguousarray(synth.spiral_points(nl).T * (0.5 * d))
    case = synth.Case(name="dense", n=base.n, h=base.h, origin=base.origin,
                      periodic=base.periodic, xp=base.xp, up=base.up, wp=base.wp,
                      radius=base.radius, mass=base.mass,
                      moff=np.array([0, nl], dtype=np.int32), body=body,
                      dV=np.array([synth.marker_volume(d, base.h, nl)]), u0=base.u0,
                      params=dict(base.params))
    ref = oracle.forcing(case, want_U=True)
    got, plan, _ = _run(case, precision, np.ones(nl, dtype=np.uint8), (16, 16, 8))
    assert got["status"] == 0
    print(f"dense markers {precision} kernel {kernel}: nm={nl} shell={plan.stats()['shell_nodes']}",
          flush=True)
    for k, t in TOL[precision].items():
        e = rel_err(got[k], ref[k])
        print(f"  {k}: {e:.2e}", flush=True)
        assert e <= t, (k, e)
