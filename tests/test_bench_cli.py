"""Host-side pieces of bench.py (no GPU): the one-GPU guard, the algorithmic
work per sweep used by the roofline, and the profile fields it reads."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_ops_per_sweep():
    import bench
    # c3: m = 500 - 3 points per sweep, p = 5: 2pm + m ceil(log2 m) + 2m
    assert bench.algorithmic_ops(497, 5) == 2 * 5 * 497 + 497 * 9 + 2 * 497 == 10437


def test_profile_has_the_fields_bench_reads():
    import bench
    txt = open(bench.PROFILE).read()
    assert re.search(r"kernel_sources_sha256: [0-9a-f]{16}", txt)
    assert re.search(r"traffic_bytes_per_launch: [0-9.e+]+", txt)
    assert len(bench.kernel_fingerprint()) == 16
