"""The seeded generators: determinism and the structure of each workload."""
import math

import numpy as np
import pytest

from paper_2109_03972_amd import synth


def test_deterministic():
    a = synth.make_case("suspension_128")
    b = synth.make_case("suspension_128")
    for k in ("xp", "up", "wp", "body", "dV", "u0"):
        assert np.array_equal(getattr(a, k), getattr(b, k))
    assert a.params["disable_seed"] == b.params["disable_seed"]


@pytest.mark.parametrize("name,np_,nm,periodic", [
    ("single_sphere_64", 1, 805, (1, 1, 1)),
    ("suspension_128", 200, 90600, (1, 1, 1)),
    ("bidisperse_bed_256x256x512", 2000, 1472000, (1, 1, 0)),
])
def test_workload_shapes(name, np_, nm, periodic):
    c = synth.make_case(name, lazy_field=True)
    assert c.np_ == np_ and c.nm == nm and c.periodic == periodic
    assert c.moff[-1] == nm
    # markers sit on the sphere surfaces
    pid = np.repeat(np.arange(c.np_), np.diff(c.moff))
    rr = np.linalg.norm(c.body, axis=0)
    assert np.allclose(rr, c.radius[pid], rtol=1e-13)


def test_suspension_min_gap_and_fraction():
    c = synth.make_case("suspension_128", lazy_field=True)
    x = c.xp.T
    d = x[None] - x[:, None]
    d -= 128.0 * np.round(d / 128.0)
    dist = np.sqrt((d ** 2).sum(-1)) + np.eye(c.np_) * 1e9
    assert (dist - 12.0).min() >= 0.5
    phi = c.np_ * math.pi / 6 * 12.0 ** 3 / 128.0 ** 3
    assert phi == pytest.approx(0.086, abs=1e-3)


def test_bed_slab_and_contacts():
    c = synth.make_case("bidisperse_bed_256x256x512", lazy_field=True)
    z = c.xp[2]
    assert np.all(z - c.radius >= 0.0)
    vol = np.sum(math.pi / 6 * (2 * c.radius) ** 3)
    H = vol / (0.3 * 256 * 256)
    assert np.all(z + c.radius <= H + 1e-9)
    x = c.xp.T
    d = x[None] - x[:, None]
    for a in range(2):
        d[..., a] -= 256.0 * np.round(d[..., a] / 256.0)
    gap = np.sqrt((d ** 2).sum(-1)) - c.radius[None] - c.radius[:, None] + np.eye(c.np_) * 1e9
    assert gap.min() >= -0.05 - 1e-9
    assert (gap < 0).sum() // 2 >= 10       # the contact branch is exercised
