"""Host logic of bench.py: the one-GPU refusal and the algorithmic byte
counts its roofline divides by (records per marker-update, values per shell
node)."""
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
def test_pass_bytes(s):
    n, S, H = 1000, 4100, 600
    # the roofline's bytes per pass: a 20 B (FP32) or 32 B (FP64) record per
    # marker-update, four accesses of the three components per shell node
    rec = 20 if s == 4 else 32
    assert bench.pass_bytes(s, n, S) == n * rec + S * 4 * 3 * s
    # FP32 at S/N = 4.08: about 216 B per marker-update
    assert 215 < bench.pass_bytes(4, 1000, 4080) / 1000 < 217
    # the tile kernels' own lower bounds: T4 records (4s) per marker entry,
    # the halo list, three components per shell node read (and written)
    assert bench.design_bytes("interp", s, n, S, H) == n * 3 * 4 * s + S * 3 * s
    assert bench.design_bytes("spread", s, n, S, H) == (n + H) * 2 * 4 * s + H * 4 + S * 6 * s
    with pytest.raises(KeyError):
        bench.design_bytes("other", s, n, S, H)


def test_fluid_bytes_per_call():
    N = 512 ** 3
    # predictor: u, N, P read (7 fields of 4 B), u~, N, nu L u written (9)
    assert bench.fluid_bytes("predictor", 4, N) == 16 * 4 * N
    # one solve between walls: y passes (32 B per node) and the elimination (32 B)
    spec_walls, spec_per = 64, 80
    assert bench.fluid_bytes("helmholtz", 4, N) == 3 * ((2 * 4 + 8) + spec_walls + (8 + 4)) * N
    assert bench.fluid_bytes("helmholtz", 4, N, walls_z=False) == 3 * ((2 * 4 + 8) + spec_per + (8 + 4)) * N
    assert bench.fluid_bytes("project", 8, N) == ((6 * 8 + 8) + 16 + spec_walls + 16 + (8 + 14 * 8)) * N


def test_kernel_hash_ignores_comments(tmp_path, monkeypatch):
    # the counter summary stays valid across comment edits, not code edits
    src = "int f(int a) { // sum\n  /* twice */ return a + a;\n}\n"
    assert bench._strip_comments(src) == bench._strip_comments(
        "// header\nint f(int a) {\n  return a + a;  // same code\n}\n")
    assert bench._strip_comments(src) != bench._strip_comments(src.replace("a + a", "a * 2"))
    files = []
    for i, f in enumerate(bench.KERNEL_SOURCES):
        p = tmp_path / f"k{i}.hip"
        with open(bench.os.path.join(bench.ROOT, f)) as fh:
            p.write_text(fh.read())
        files.append(str(p))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", tuple(files))
    h0 = bench.kernel_sources_hash()
    with open(files[0], "a") as fh:
        fh.write("\n// a new comment\n")
    assert bench.kernel_sources_hash() == h0
    with open(files[0], "a") as fh:
        fh.write("\nstatic int unused_code = 0;\n")
    assert bench.kernel_sources_hash() != h0
