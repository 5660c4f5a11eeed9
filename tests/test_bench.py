"""Host-side checks of the benchmark driver: it refuses a multi-GPU request
without touching a GPU, and the committed HBM-traffic record it reads is
self-consistent."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_multi_gpu_request_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr and "nothing was run" in r.stderr
    assert r.stdout == ""


def test_traffic_record_is_self_consistent():
    """bytes_per_launch = FETCH_SIZE x fetch scale + WRITE_SIZE x write scale
    (KiB per dispatch), the scales are those of the 1 GiB copy, and the
    algorithmic bytes are 2 K Q 4 per cell of the 256^3 workload."""
    t = json.load(open(bench.TRAFFIC_FILE))
    ref = t["copy_reference"]
    fs = ref["bytes"] / 1024 / ref["fetch_kib"]
    ws = ref["bytes"] / 1024 / ref["write_kib"]
    assert abs(fs - ref["fetch_scale"]) < 1e-5 and abs(ws - ref["write_scale"]) < 1e-5
    tb = (t["fetch_kib_per_dispatch_median"] * fs + t["write_kib_per_dispatch_median"] * ws) * 1024
    assert abs(tb - t["bytes_per_launch"]) <= 1.0
    assert t["algorithmic_bytes_per_launch"] == 2 * 17 * 7 * 4 * 256 ** 3
    assert abs(t["bytes_per_launch"] / t["algorithmic_bytes_per_launch"] - t["ratio_to_algorithmic"]) < 1e-5
    assert len(t["kernel_source_hash"]) == 16


def test_stale_traffic_record_is_not_reported(tmp_path, monkeypatch):
    """A record taken on other kernel sources gives no traffic figure."""
    t = json.load(open(bench.TRAFFIC_FILE))
    t["kernel_source_hash"] = "0" * 16
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps(t))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(p))
    assert bench.measured_traffic() is None
