"""Host-side pieces of bench.py: the keying of the stored kernel-trace and
HBM-traffic records to each kernel's sources, and the one-GPU contract."""
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
    step, digit = bench.STEP_KERNEL_PREFIX, bench.DIGIT_KERNEL_PREFIX
    rec = {"records": {step: {"source_sha256": bench.step_source_hash(), "bytes_per_launch": 123.0},
                       digit: {"source_sha256": bench.source_hash(bench.DIGIT_SOURCES), "bytes_per_launch": 7.0}}}
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.measured_traffic(step) == 123.0
    assert bench.measured_traffic(digit) == 7.0
    rec["records"][step]["source_sha256"] = "0" * 64
    path.write_text(json.dumps(rec))
    assert bench.measured_traffic(step) is None
    assert bench.measured_traffic(digit) == 7.0
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic(step) is None


def test_committed_kernel_records_match_the_committed_sources():
    for path, key in ((bench.TRAFFIC_FILE, "bytes_per_launch"), (bench.TRACE_FILE, "avg_ns")):
        with open(path) as f:
            rec = json.load(f)
        for frag, sources in bench.RECORDED_KERNELS.items():
            r = rec["records"][frag]
            assert r["source_sha256"] == bench.source_hash(sources), (path, frag)
            assert r[key] > 0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
