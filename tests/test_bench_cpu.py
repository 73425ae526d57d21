"""The benchmark's host side: it refuses more than one GPU before touching
any device, and the committed HBM traffic record is well formed — every
recorded operation's measured bytes lie within 1% of its algorithmic bytes,
and a record is only reported for the kernel sources it was taken on."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_record_is_consistent():
    with open(bench.TRAFFIC) as f:
        rec = json.load(f)
    assert 1.9 < rec["fetch_scale"] < 2.1 and 0.9 < rec["write_scale"] < 1.1
    assert set(rec["ops"]) == set(bench.KERNEL_SOURCES)
    for op, e in rec["ops"].items():
        assert e["kernels"], op
        assert abs(e["traffic_bytes"] / e["algorithmic_bytes"] - 1) < 0.01, op
        t = bench.measured_traffic(op)
        # reported exactly when the sources still hash to the recorded value
        assert (t == e["traffic_bytes"]) == (e["source_sha256"] == bench.source_hash(op)), op
        assert t is None or t == e["traffic_bytes"]


def test_traffic_withheld_after_a_source_change(tmp_path, monkeypatch):
    with open(bench.TRAFFIC) as f:
        rec = json.load(f)
    rec["ops"]["ger_f64"]["source_sha256"] = "0" * 64   # as if ger.hip had changed since
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC", str(p))
    assert bench.measured_traffic("ger_f64") is None
    assert bench.measured_traffic("no_such_op") is None
