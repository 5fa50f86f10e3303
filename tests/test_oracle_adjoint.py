"""Pin of the oracle's reverse-mode derivative of the forcing loop against
central finite differences of the oracle's own forward loop (FP64)."""
import numpy as np
import pytest

from paper_2109_03972_amd import synth


def _tiny(seed=31, n=(14, 13, 16), periodic=(1, 1, 0)):
    rng = np.random.default_rng(seed)
    xp = np.array([[4.3, 9.6], [5.2, 7.9], [7.7, 8.4]])
    nm_each = (23, 17)
    bodies = [synth.spiral_points(k).T * r for k, r in zip(nm_each, (2.6, 2.1))]
    moff = np.array([0, nm_each[0], sum(nm_each)], dtype=np.int32)
    prm = synth.default_params()
    prm.update(n_iter=3, c=0.47)
    c = synth.Case(name="adj", n=n, h=1.0, origin=(0.0, 0.0, 0.0), periodic=periodic,
                   xp=xp, up=rng.normal(0, 0.2, (3, 2)), wp=rng.normal(0, 0.1, (3, 2)),
                   radius=np.array([2.6, 2.1]), mass=np.ones(2), moff=moff,
                   body=np.concatenate(bodies, axis=1), dV=np.array([0.9, 1.1]),
                   u0=rng.standard_normal((3, n[2], n[1], n[0])), params=prm)
    mask = np.ones(c.nm, dtype=np.uint8)
    mask[5] = 0
    return c, mask


def _loss(oracle_lib, c, mask, cot, **kw):
    r = oracle_lib.forcing(c, mask=mask, final_resid=False, **kw)
    return (np.sum(cot["g_f"] * r["f_tot"]) + np.sum(cot["g_u"] * r["u"])
            + np.sum(cot["g_S"] * r["S"]) + np.sum(cot["g_T"] * r["T"]))


def test_adjoint_matches_central_differences(oracle_lib):
    c, mask = _tiny()
    rng = np.random.default_rng(77)
    cot = dict(g_f=rng.standard_normal(c.u0.shape), g_u=rng.standard_normal(c.u0.shape),
               g_S=rng.standard_normal((3, 2)), g_T=rng.standard_normal((3, 2)))
    adj = oracle_lib.forcing_adjoint(c, mask=mask, **cot)
    # no marker coordinate sits near a kink of phi3'' (integer s)
    pid = np.repeat(np.arange(2), np.diff(c.moff))
    s = c.xp[:, pid] + c.body
    assert np.min(np.abs(s - np.round(s))) > 1e-4
    eps = 1e-6
    for trial in range(20):
        v = dict(u0=rng.standard_normal(c.u0.shape), xp=rng.standard_normal((3, 2)),
                 up=rng.standard_normal((3, 2)), wp=rng.standard_normal((3, 2)))
        plus = _loss(oracle_lib, c, mask, cot, u0=c.u0 + eps * v["u0"], xp=c.xp + eps * v["xp"],
                     up=c.up + eps * v["up"], wp=c.wp + eps * v["wp"])
        minus = _loss(oracle_lib, c, mask, cot, u0=c.u0 - eps * v["u0"], xp=c.xp - eps * v["xp"],
                      up=c.up - eps * v["up"], wp=c.wp - eps * v["wp"])
        fd = (plus - minus) / (2 * eps)
        an = (np.sum(adj["gu0"] * v["u0"]) + np.sum(adj["gxp"] * v["xp"])
              + np.sum(adj["gup"] * v["up"]) + np.sum(adj["gwp"] * v["wp"]))
        assert fd == pytest.approx(an, rel=1e-7, abs=1e-7)


def test_adjoint_position_gradient_alone(oracle_lib):
    """The position gradient (delta-derivative terms) on its own, per
    component, against central differences."""
    c, mask = _tiny(seed=5)
    rng = np.random.default_rng(8)
    cot = dict(g_f=rng.standard_normal(c.u0.shape), g_u=np.zeros(c.u0.shape),
               g_S=rng.standard_normal((3, 2)), g_T=rng.standard_normal((3, 2)))
    adj = oracle_lib.forcing_adjoint(c, mask=mask, **cot)
    eps = 1e-6
    for p in range(2):
        for a in range(3):
            dx = np.zeros((3, 2))
            dx[a, p] = eps
            fd = (_loss(oracle_lib, c, mask, cot, xp=c.xp + dx)
                  - _loss(oracle_lib, c, mask, cot, xp=c.xp - dx)) / (2 * eps)
            assert fd == pytest.approx(adj["gxp"][a, p], rel=1e-6, abs=1e-7)
