"""bench.py contract checks that need no GPU."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "single" in r.stderr


def test_traffic_record_names_existing_sources():
    sys.path.insert(0, ROOT)
    import bench
    for rel in bench.TRAFFIC["sources"]:
        assert os.path.isfile(os.path.join(ROOT, rel))
    assert len(bench.TRAFFIC["sha256"]) == 64
    # a changed kernel source reports no traffic instead of a stale figure
    assert bench.measured_traffic("C5") is None
    json.dumps(bench.TRAFFIC)
