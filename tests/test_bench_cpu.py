"""Host-side pieces of bench.py: the keying of the stored HBM-traffic record
to the step kernel's source, and the one-GPU contract."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_code_only_drops_comments_and_blank_lines():
    text = "int a = 1;  // one\n\n// whole-line comment\n  b();\n"
    assert bench.code_only(text) == "int a = 1;\n  b();"


def test_traffic_record_is_keyed_to_the_source(tmp_path, monkeypatch):
    rec = {"source_sha256": bench.step_source_hash(), "bytes_per_launch": 123.0}
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.measured_traffic() == 123.0
    rec["source_sha256"] = "0" * 64
    path.write_text(json.dumps(rec))
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic() is None


def test_committed_traffic_record_matches_the_committed_source():
    with open(bench.TRAFFIC_FILE) as f:
        rec = json.load(f)
    assert rec["source_sha256"] == bench.step_source_hash()
    assert rec["bytes_per_launch"] > 0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
