"""Host-side checks of bench.py: the one-GPU contract and the committed
counter record the roofline entry reads."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_record_matches_the_kernel_source():
    """The FETCH/WRITE record is keyed by the source hash of the fused 2D
    kernels; the committed record belongs to the committed source, covers
    every tile height the autotuner can pick, and is close to the
    algorithmic bytes (34 B per point, 2047^2 points)."""
    with open(bench.TRAFFIC_FILE) as f:
        t = json.load(f)
    assert t["src_sha"] == bench.src_hash()
    alg = 34 * 2047 * 2047
    assert t["algorithmic_bytes_per_launch"] == alg
    for th in (4, 8, 16):
        v = bench.measured_traffic("post", th)
        assert v is not None, th
        assert 0.9 * alg < v < 1.1 * alg, (th, v)
    # calibration by a 1 GiB copy: FETCH_SIZE counts half the bytes read
    c = t["calibration"]
    assert abs(c["fetch_factor"] - 2.0) < 0.01 and abs(c["write_factor"] - 1.0) < 0.01
