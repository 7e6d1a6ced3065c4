"""CPU checks of bench.py's host logic (no GPU): the one-GPU refusal of
--gpus N > 1, and the counter-traffic field, which is reported only for a
probed kernel with counters and only while the kernel source has the hash
the counters were taken with."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "--gpus 1" in r.stderr


def test_traffic_only_for_measured_kernels_of_the_current_source(monkeypatch):
    t = bench.traffic_fields("post_u", 100e6)
    assert t["traffic"] == bench.TRAFFIC["post_u"]["bytes_per_launch"]
    ratio = t["traffic_over_algorithmic"]
    assert abs(ratio - 122.7 / 104.8) < 1e-12
    assert abs(t["traffic_per_average_launch"] - ratio * 100e6) < 1e-3
    assert bench.traffic_fields("cheb_u", 100e6) == {"traffic": None}
    stale = {k: dict(v, kernels_sha256_prefix="0000000000000000") for k, v in bench.TRAFFIC.items()}
    monkeypatch.setattr(bench, "TRAFFIC", stale)
    assert bench.traffic_fields("post_u", 100e6) == {"traffic": None}

