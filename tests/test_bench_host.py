"""Host logic of bench.py that needs no GPU: the stored HBM-traffic lookup
behind roofline.traffic and the one-GPU guard."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_committed_traffic_summary_has_the_lookup_fields():
    tf = json.load(open(bench.TRAFFIC_FILE))
    assert tf["size"] == 1 << 30 and len(tf["kernel_hash"]) == 16
    for d in ("encode", "decode"):
        e = tf[d]
        assert e["bytes_per_launch"] > 0 and e["algorithmic_bytes"] > 0
        # measured traffic within 1% of the algorithmic bytes (no re-reads)
        assert abs(e["bytes_per_launch"] / e["algorithmic_bytes"] - 1) < 0.01


def test_stored_traffic_matches_only_same_size_and_sources(tmp_path, monkeypatch):
    f = tmp_path / "t.json"
    h = bench.kernel_hash()
    doc = {"size": 1 << 30, "kernel_hash": h, "decode": {"bytes_per_launch": 123}, "encode": {"bytes_per_launch": 7}}
    f.write_text(json.dumps(doc))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.stored_traffic("decode", 1 << 30) == 123
    assert bench.stored_traffic("encode", 1 << 30) == 7
    assert bench.stored_traffic("decode", 1 << 20) is None  # other size
    doc["kernel_hash"] = "0" * 16
    f.write_text(json.dumps(doc))
    assert bench.stored_traffic("decode", 1 << 30) is None  # other kernel sources
    f.write_text("not json")
    assert bench.stored_traffic("decode", 1 << 30) is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.stored_traffic("decode", 1 << 30) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0 and "one GPU" in (r.stdout + r.stderr)
