"""Host-side logic of bench.py: the refusal of more than one GPU, the
raggedness summary, the traffic record's source check and the algorithmic
byte formulas.  No GPU is touched."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_ragged_summary_bins_and_percentiles():
    counts = np.array([0, 0, 1, 3, 4, 700, 1024, 5000], np.int32)
    s = bench.ragged_summary(counts)
    bins = dict(zip(s["bins"], s["rays"]))
    assert bins["[0,1)"] == 2 and bins["[1,2)"] == 1 and bins["[2,4)"] == 1
    assert bins["[4,8)"] == 1 and bins["[512,1024)"] == 1 and bins["[1024,2048)"] == 1
    assert bins["[4096,inf)"] == 1
    assert sum(s["rays"]) == counts.size
    assert s["percentiles"]["0"] == 0.0 and s["percentiles"]["100"] == 5000.0
    assert s["mean"] == counts.mean()
    json.dumps(s)  # part of the JSON line


def test_traffic_record_lapses_when_sources_change(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel v1\n")
    import hashlib
    rec = {"kernel": "render_bwd", "bytes_per_launch": 123.0, "sources": ["k.hip"],
           "sources_sha256": hashlib.sha256(b"kernel v1\n").hexdigest()}
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", str(path))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("render_bwd") == 123.0
    assert bench.measured_traffic("render_fwd") is None  # another kernel
    src.write_text("kernel v2\n")
    assert bench.measured_traffic("render_bwd") is None  # the kernel changed


def test_algorithmic_bytes_per_launch():
    N, Sm, S = 1 << 20, 300_000_000, 263_000_000
    assert bench.BYTES["render_bwd"](N, Sm, S) == 28 * N + 40 * S
    assert bench.BYTES["render_fwd"](N, Sm, S) == 36 * N + 24 * S
    assert bench.BYTES["march_fill"](N, Sm, S) == 32 * N + 12 * Sm
