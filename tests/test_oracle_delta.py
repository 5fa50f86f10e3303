"""Pins of the oracle's regularized delta functions (Sec. 2.1 and 2.2.3).

The three-point function of Roma et al. and the four-point function of
Peskin are fixed by closed-form values and by their discrete moment
conditions; a wrong branch, sign or constant breaks at least one of these.
"""
import math

import numpy as np
import pytest


def test_phi3_closed_form_values(oracle_lib):
    o = oracle_lib
    assert o.phi3(0.0) == pytest.approx(2.0 / 3.0, abs=1e-15)
    for r in (0.5, -0.5):
        assert o.phi3(r) == pytest.approx(0.5, abs=1e-15)
    for r in (1.0, -1.0):
        assert o.phi3(r) == pytest.approx(1.0 / 6.0, abs=1e-15)
    for r in (1.5, -1.5, 1.7, -2.0, 3.0):
        assert o.phi3(r) == pytest.approx(0.0, abs=1e-15)


def test_phi3_continuity_and_c1(oracle_lib):
    o = oracle_lib
    e = 1e-9
    for b in (0.5, 1.5):
        for s in (1.0, -1.0):
            r = s * b
            assert abs(o.phi3(r - e) - o.phi3(r + e)) < 1e-8
            assert abs(o.dphi3(r - e) - o.dphi3(r + e)) < 1e-4
    assert o.dphi3(0.5) == pytest.approx(-1.0, abs=1e-12)
    assert o.dphi3(-0.5) == pytest.approx(1.0, abs=1e-12)
    assert o.dphi3(1.5) == pytest.approx(0.0, abs=1e-12)


@pytest.mark.parametrize("fn,dfn,half", [("phi3", "dphi3", 1.5), ("phi4", "dphi4", 2.0)])
def test_derivative_matches_finite_difference(oracle_lib, fn, dfn, half):
    o = oracle_lib
    f, df = getattr(o, fn), getattr(o, dfn)
    rng = np.random.default_rng(11)
    for r in rng.uniform(-half, half, 400):
        # stay away from the branch points where the second derivative jumps
        if min(abs(abs(r) - b) for b in (0.0, 0.5, 1.0, 1.5, 2.0)) < 1e-3:
            continue
        e = 1e-6
        fd = (f(r + e) - f(r - e)) / (2 * e)
        assert abs(fd - df(r)) < 1e-6 * max(1.0, abs(fd))


def _stencil_sums(f, s, half, power=1, moment=0, parity=None):
    tot = 0.0
    for j in range(int(math.floor(s - half)) - 1, int(math.ceil(s + half)) + 2):
        if parity is not None and (j % 2) != parity:
            continue
        r = s - j
        tot += (r ** moment) * f(r) ** power
    return tot


def test_phi3_moment_conditions(oracle_lib):
    """sum phi3 = 1 (the condition stated for the three-point function),
    zero first moment and sum phi3^2 = 1/2 for every shift."""
    o = oracle_lib
    rng = np.random.default_rng(3)
    for s in np.concatenate([rng.uniform(-3, 3, 2000), [0.0, 0.5, 1.0, -0.5]]):
        assert abs(_stencil_sums(o.phi3, s, 1.5) - 1.0) < 1e-14
        assert abs(_stencil_sums(o.phi3, s, 1.5, moment=1)) < 1e-14
        assert abs(_stencil_sums(o.phi3, s, 1.5, power=2) - 0.5) < 1e-14


def test_phi4_even_odd_condition(oracle_lib):
    """sum over even nodes = sum over odd nodes = 1/2 (Sec. 2.2.3), zero first
    moment and sum phi4^2 = 3/8 (Peskin 2002)."""
    o = oracle_lib
    rng = np.random.default_rng(4)
    for s in np.concatenate([rng.uniform(-3, 3, 2000), [0.0, 0.5, 1.0]]):
        assert abs(_stencil_sums(o.phi4, s, 2.0, parity=0) - 0.5) < 1e-14
        assert abs(_stencil_sums(o.phi4, s, 2.0, parity=1) - 0.5) < 1e-14
        assert abs(_stencil_sums(o.phi4, s, 2.0, moment=1)) < 1e-14
        assert abs(_stencil_sums(o.phi4, s, 2.0, power=2) - 0.375) < 1e-14


def test_phi4_values(oracle_lib):
    o = oracle_lib
    assert o.phi4(0.0) == pytest.approx(0.5, abs=1e-15)
    assert o.phi4(1.0) == pytest.approx(0.25, abs=1e-15)
    assert o.phi4(-1.0) == pytest.approx(0.25, abs=1e-15)
    assert o.phi4(2.0) == pytest.approx(0.0, abs=1e-15)
    assert o.phi4(-2.0) == pytest.approx(0.0, abs=1e-15)
    # mirror symmetry of the four branches
    for r in np.linspace(0.01, 1.99, 50):
        assert o.phi4(r) == pytest.approx(o.phi4(-r), abs=1e-15)


def test_splitmix64_published_vector(oracle_lib):
    """SplitMix64 seeded with 0 gives 0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4,
    0x06c45d188009454f as its first outputs (Steele, Lea & Flood 2014)."""
    o = oracle_lib
    g = 0x9E3779B97F4A7C15
    outs = [o.splitmix64((k * g) & 0xFFFFFFFFFFFFFFFF) for k in range(3)]
    assert outs == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
