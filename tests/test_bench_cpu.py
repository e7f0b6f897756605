"""CPU: bench.py's contract pieces that need no GPU -- more than one GPU is refused with
a message, and the measured HBM traffic is reported only while the kernel sources match
the hash it was measured on."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_only_for_the_measured_sources(tmp_path, monkeypatch):
    path = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.measured_traffic("k_forward") is None            # no file
    entry = {"kernels": {"k_forward": {"bytes_per_launch": 123}}}
    path.write_text(json.dumps(dict(entry, source_hash="0" * 16)))
    assert bench.measured_traffic("k_forward") is None            # other sources
    path.write_text(json.dumps(dict(entry, source_hash=bench.kernel_source_hash())))
    assert bench.measured_traffic("k_forward") == 123
    assert bench.measured_traffic("k_cone_gather") is None        # kernel not measured
    path.write_text("{ not json")
    assert bench.measured_traffic("k_forward") is None
