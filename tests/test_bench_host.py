"""Host logic of bench.py that runs without a GPU."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_traffic_is_reported_only_for_the_current_kernel_sources(tmp_path, monkeypatch):
    path = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.traffic_entry("fp32", 17.5) is None                     # no summary
    path.write_text(json.dumps({"kernel_hash": bench.kernel_hash(), "fp32": {"bytes_per_launch": 123}}))
    assert bench.traffic_entry("fp32", 17.5) == 123
    assert bench.traffic_entry("fp16", 8.9) is None                      # storage not profiled
    path.write_text(json.dumps({"kernel_hash": "0" * 16, "fp32": {"bytes_per_launch": 123}}))
    assert bench.traffic_entry("fp32", 17.5) is None                     # kernel changed since
