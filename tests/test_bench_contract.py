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


def test_traffic_record_follows_the_kernel_sources(monkeypatch):
    with open(bench.TRAFFIC_FILE) as f:
        rec = json.load(f)
    want = rec["entries"]["c2:f64"]["bytes_per_launch"]
    # the record describes a per-launch volume near the algorithmic bytes
    assert 1.0 <= want / rec["entries"]["c2:f64"]["alg_bytes_per_launch"] < 1.5
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: rec["kernel_source_sha"])
    assert bench.measured_traffic("f64", "c2") == want
    assert bench.measured_traffic("f32", "c2") is None  # no such record
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic("f64", "c2") is None  # sources changed since


def test_kernel_source_hash_covers_the_fused_kernel_sources():
    names = {os.path.basename(p) for p in bench.KERNEL_SOURCES}
    assert {"fs1_fused.hip", "fs1_frame.h", "fs1_device.h", "fs1_tile.h"} <= names
    assert all(os.path.exists(p) for p in bench.KERNEL_SOURCES)
    assert len(bench.kernel_source_hash()) == 16
