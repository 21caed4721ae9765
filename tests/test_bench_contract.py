"""Host-side parts of bench.py's contract that need no GPU: the one-GPU
refusal and the counter-traffic record, which is used only while the
half-iteration kernel's sources are the ones it was measured on."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_traffic_record_follows_the_kernel_sources(monkeypatch, tmp_path):
    srcs = ["fs1_large.hip", "fs1_frame.h"]
    rec = {"entries": {"c4:f64": {"kernel_sources": srcs,
                                  "kernel_source_sha": bench.source_hash(srcs),
                                  "bytes_per_launch": 123}}}
    p = tmp_path / "t.json"
    p.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(p))
    assert bench.measured_traffic("f64", "c4") == 123
    assert bench.measured_traffic("f32", "c4") is None  # no such record
    rec["entries"]["c4:f64"]["kernel_source_sha"] = "0" * 16  # sources changed since
    p.write_text(json.dumps(rec))
    assert bench.measured_traffic("f64", "c4") is None


def test_committed_traffic_records_name_existing_sources():
    if not os.path.exists(bench.TRAFFIC_FILE):
        return
    with open(bench.TRAFFIC_FILE) as f:
        rec = json.load(f)
    for key, e in rec["entries"].items():
        assert all(os.path.exists(os.path.join(bench.CSRC, s)) for s in e["kernel_sources"]), key
        assert 1.0 <= e["bytes_per_launch"] / e["alg_bytes_per_launch"] < 1.5, key


def test_algorithmic_bytes_per_point():
    # binary64: psi-half 32 B (phi, nu, old psi, new psi), phi-half 24 B
    assert bench.ALG_BYTES_PER_POINT["f64"] == 28
    # binary32: psi-half 4 + 4 + 4 + 4 + 8 (binary64 nu for the error), phi-half 12
    assert bench.ALG_BYTES_PER_POINT["f32"] == 18


def test_source_hash_ignores_comments_only():
    # a counter record stays valid across comment edits, not across code edits
    a = "int f(int x) { // twice\n  return 2 * x; /* doubled */ }\n"
    b = "// a new header comment\nint f(int x) {\n  return 2 * x;  // still doubled\n}\n"
    c = "int f(int x) { return 3 * x; }\n"
    d = 'const char* s = "// not a comment"; int g;'
    assert bench.code_text(a) == bench.code_text(b)
    assert bench.code_text(a) != bench.code_text(c)
    assert "// not a comment" in bench.code_text(d)
