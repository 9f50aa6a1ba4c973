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
    path = os.path.join(ROOT, bench.TRAFFIC["source"])
    assert os.path.isfile(path)
    with open(path) as f:
        assert bench.TRAFFIC["through"] in f.read()
    assert len(bench.TRAFFIC["sha256"]) == 64
    # the counters were taken on the sweep kernel as it stands
    assert bench.measured_traffic("C3") is not None
    # another workload reports no traffic instead of a figure measured on C3
    assert bench.measured_traffic("C5") is None
    json.dumps(bench.TRAFFIC)


def test_traffic_record_is_dropped_when_the_kernel_changes(monkeypatch, tmp_path):
    """An edit of the sweep kernel (or of anything before it in its file)
    makes bench.py report no traffic rather than a stale figure."""
    sys.path.insert(0, ROOT)
    import bench
    with open(os.path.join(ROOT, bench.TRAFFIC["source"])) as f:
        text = f.read()
    at = text.index(bench.TRAFFIC["through"])
    edited = text[:at] + "// edit\n" + text[at:]
    src = tmp_path / "paper_1706_05586_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "solve.hip").write_text(edited)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("C3") is None
