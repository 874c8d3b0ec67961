"""Host-side logic of bench.py (no GPU): the one-GPU rule and the traffic bookkeeping."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_only_for_the_profiled_source_and_tile(tmp_path, monkeypatch):
    import hashlib
    src = os.path.join(ROOT, "paper_2010_04768_amd", "csrc", "gemm.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    cache = tmp_path / "tune.json"
    t = bench.TRAFFIC["fp64"]
    # counters taken on another GEMM source are not reported
    cache.write_text(json.dumps({"entries": [{"key": t["key"], "cfg": 5, "name": t["tile"], "ms": 1.0}]}))
    monkeypatch.setitem(bench.TRAFFIC, "gemm_src_sha256_16", "0" * 16)
    assert bench.traffic_for("fp64", str(cache)) == (None, None)
    # the profiled source: reported when the tuned tile is the profiled one
    monkeypatch.setitem(bench.TRAFFIC, "gemm_src_sha256_16", sha)
    cache.write_text(json.dumps({"entries": [{"key": t["key"], "cfg": 5, "name": t["tile"], "ms": 1.0}]}))
    traffic, detail = bench.traffic_for("fp64", str(cache))
    assert traffic == (t["fetch_GB"] + t["write_GB"]) * 1e9 and detail["tile"] == t["tile"]
    cache.write_text(json.dumps({"entries": [{"key": t["key"], "cfg": 4, "name": "db128x128", "ms": 1.0}]}))
    traffic, detail = bench.traffic_for("fp64", str(cache))
    assert traffic is None and detail == {"tuned_tile": "db128x128", "profiled_tile": t["tile"]}
    assert bench.traffic_for("fp64", None) == (None, None)
