"""The benchmark's command-line contract that can be checked without a GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_peak_derivation():
    sys.path.insert(0, ROOT)
    import bench
    # 256 CUs x 128 fp32 lanes x 2.4 GHz lane-slots, 1.5 slots per term, 2 ops per term
    assert abs(bench.PEAK_TOPS - 256 * 128 * 2.4e9 / 1.5 * 2 / 1e12) < 1e-9
    assert 104.8 < bench.PEAK_TOPS < 104.9
