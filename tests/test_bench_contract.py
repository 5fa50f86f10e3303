"""Host logic of bench.py: the one-GPU refusal and the algorithmic byte
counts its roofline divides by (records per marker, values per shell node)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


@pytest.mark.parametrize("s", [4, 8])
def test_forcing_bytes_per_launch(s):
    n, S = 1000, 7000
    # interpolation: packed node + fractions (4 + 3s), U^d and dV (4s), G written (3s),
    # pass sum read and written (6s); the shell read once (3s per node)
    assert bench.algorithmic_bytes("interp", s, n, S) == n * (4 + 3 * s + 4 * s + 3 * s + 6 * s) + S * 3 * s
    # spreading: node + fractions and G per record; u read and written per shell node,
    # f_tot as well when the call has a single pass
    assert bench.algorithmic_bytes("spread", s, n, S, n_iter=5) == n * (4 + 6 * s) + S * 6 * s
    assert bench.algorithmic_bytes("spread", s, n, S, n_iter=1) == n * (4 + 6 * s) + S * 12 * s
    assert bench.algorithmic_bytes("ftot", s, n, S) == n * (4 + 6 * s) + S * 6 * s
    with pytest.raises(KeyError):
        bench.algorithmic_bytes("other", s, n, S)


def test_fluid_bytes_per_call():
    N = 512 ** 3
    # predictor: u, N, P read (7 fields of 4 B), u~, N, nu L u written (9)
    assert bench.fluid_bytes("predictor", 4, N) == 16 * 4 * N
    # one solve between walls: y passes (32 B per node) and the elimination (32 B)
    spec_walls, spec_per = 64, 80
    assert bench.fluid_bytes("helmholtz", 4, N) == 3 * ((2 * 4 + 8) + spec_walls + (8 + 4)) * N
    assert bench.fluid_bytes("helmholtz", 4, N, walls_z=False) == 3 * ((2 * 4 + 8) + spec_per + (8 + 4)) * N
    assert bench.fluid_bytes("project", 8, N) == ((6 * 8 + 8) + 16 + spec_walls + 16 + (8 + 14 * 8)) * N
