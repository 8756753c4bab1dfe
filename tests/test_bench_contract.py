"""Host-side checks of bench.py: the one-GPU guard, and that the committed
HBM byte records of the three hot kernels belong to the current sources
(a kernel changed since its counters were taken reports null traffic)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_records_match_the_sources():
    for prof, src in ((bench.PASS1_PROFILE, bench.PASS1_SOURCES),
                      (bench.SELECT_PROFILE, bench.SELECT_SOURCES),
                      (bench.PASS2_PROFILE, bench.PASS2_SOURCES)):
        t = bench.kernel_traffic(prof, src)
        assert t is not None and t > 0, prof


def test_algorithmic_bytes_per_particle():
    # 24 + 4 + 4 L + 24 + L + 12 + 32 with L = 77.5 list entries
    assert abs(bench.SELECT_BYTES_PER_PARTICLE - 483.5) < 1e-9
    assert bench.PASS2_BYTES_PER_PARTICLE == 749
