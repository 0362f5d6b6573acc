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


def test_serving_mismatch_count_closed_forms():
    """The serving check's closed forms: encode lengths, clean decode
    lengths, and the first injected byte inside a corrupted slice."""
    import types

    import numpy as np

    banks = types.SimpleNamespace(text_len=1000, inject_pos=np.array([10, 50, 300], np.int64))
    req = {"op": np.array([0, 0, 1, 1, 1, 1], np.uint8),
           "in_len": np.array([5, 3, 40, 40, 100, 8], np.int64),
           "in_begin": np.array([0, 7, 0, 1000 + 8, 1000 + 40, 1000 + 100], np.int64)}
    # encode 5 -> 8, 3 -> 4; clean decode 40 -> 30; corrupted at 10 (offset 2),
    # at 50 (offset 10), and a slice [100, 108) holding no injected byte
    res = {"t_done": np.ones(6), "out_len": np.array([8, 4, 30, -1, -1, 6], np.int64),
           "err_off": np.array([-1, -1, -1, 2, 10, -1], np.int64)}
    assert bench.serving_mismatches(req, res, banks) == (0, 3)
    res["err_off"][4] = 11
    res["out_len"][0] = 9
    assert bench.serving_mismatches(req, res, banks) == (2, 3)
    res["t_done"][0] = -1.0  # not completed: not counted
    assert bench.serving_mismatches(req, res, banks) == (1, 3)


def test_stored_batch_traffic_lookup(tmp_path, monkeypatch):
    """Per-configuration traffic of the batched and whitespace kernels comes
    from the committed summary only for the same kernel sources, kernel and
    (for the tile and per-wave layouts) launch shape."""
    tf = json.load(open(bench.BATCH_TRAFFIC_FILE))
    for key, e in tf["entries"].items():
        assert e["bytes_per_launch"] > 0 and 0.99 < e["ratio_to_algorithmic"] < 1.2, key
    f = tmp_path / "b.json"
    doc = {"batch_kernel_hash": bench.sources_hash(["b64_modes.hpp", "b64_device.hpp", "b64_batch.hip"]),
           "ws_kernel_hash": "0" * 16,
           "entries": {"uneven.encode": {"kernel": "k_batch_s<0, 4>", "grid_threads": 1, "block": 256,
                                         "bytes_per_launch": 10, "algorithmic_bytes": 9, "ratio_to_algorithmic": 1.1},
                       "heavy.decode": {"kernel": "k_dec_batch_t<4>", "grid_threads": 4096 * 1024, "block": 1024,
                                        "bytes_per_launch": 5, "algorithmic_bytes": 5, "ratio_to_algorithmic": 1.0},
                       "mime.decode": {"kernel": "k_dec_ws", "bytes_per_launch": 3, "algorithmic_bytes": 3,
                                       "ratio_to_algorithmic": 1.0}}}
    f.write_text(json.dumps(doc))
    monkeypatch.setattr(bench, "BATCH_TRAFFIC_FILE", str(f))
    k2 = bench.batch_kernel_name(0, {"layout": 2, "units_per_lane": 4})
    assert k2 == "k_batch_s<0, 4>" and bench.stored_batch_traffic("uneven.encode", k2, 256, 99)["bytes_per_launch"] == 10
    assert bench.stored_batch_traffic("uneven.encode", "k_batch_s<0, 2>", 256, 99) is None  # other kernel
    k0 = bench.batch_kernel_name(1, {"layout": 0, "units_per_lane": 4})
    assert bench.stored_batch_traffic("heavy.decode", k0, 1024, 4096)["ratio"] == 1.0
    assert bench.stored_batch_traffic("heavy.decode", k0, 512, 4096) is None  # other shape
    assert bench.stored_batch_traffic("mime.decode") is None  # other whitespace sources
    assert bench.stored_batch_traffic("uneven.decode") is None  # not measured
