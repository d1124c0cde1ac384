"""Host-side logic of the library that needs no GPU, compiled and run here."""
import os
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run_cpp(src):
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "check")
        subprocess.run(["/opt/rocm/bin/hipcc", "-O2", "-std=c++17",
                        "-I", os.path.join(ROOT, "include"),
                        "-I", os.path.join(ROOT, "paper_1701_04733_amd", "csrc"),
                        os.path.join(ROOT, "tests", "cpp", src), "-o", exe],
                       check=True, capture_output=True, timeout=300)
        return subprocess.run([exe], capture_output=True, text=True, timeout=120)


def test_tile_plans_cover_every_output_once():
    r = _run_cpp("tile_plan_check.cpp")
    assert r.returncode == 0, r.stdout + r.stderr
    assert "tile plan failures: 0" in r.stdout


def test_pool_allocator_never_overlaps_and_coalesces():
    r = _run_cpp("range_alloc_check.cpp")
    assert r.returncode == 0, r.stdout + r.stderr
    assert "range allocator failures: 0" in r.stdout
