"""Host-side logic of bench.py (no GPU): the one-GPU contract and the
traffic summary lookup."""
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


def test_traffic_summary_matches_or_is_dropped(tmp_path, monkeypatch):
    f = tmp_path / "t.txt"
    f.write_text(f"kernel: k\nsource_hash: {bench.source_hash()}\nfetch_bytes_per_launch: 100\n"
                 f"write_bytes_per_launch: 23\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic() == 123.0
    f.write_text("source_hash: 0000\nfetch_bytes_per_launch: 100\nwrite_bytes_per_launch: 23\n")
    assert bench.measured_traffic() is None  # kernel changed since the counters were taken


def test_committed_traffic_summary_is_parseable():
    kv = {}
    with open(bench.TRAFFIC_FILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith((" ", "#")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    assert float(kv["fetch_bytes_per_launch"]) > 0 and float(kv["write_bytes_per_launch"]) > 0
    assert len(kv["source_hash"]) == 16
