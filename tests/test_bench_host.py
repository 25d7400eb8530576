"""Host-side logic of bench.py (no GPU): the one-GPU contract and the
lookup of the committed PMC counter summary."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


COUNTER_LINES = ("fetch_bytes_per_launch: 100\nwrite_bytes_per_launch: 23\nvalu_busy_pct: 55.5\n"
                 "valu_utilization_pct: 40.25\nvalu_insts_per_launch: 7\ncounted_flops_fp32_per_launch: 1000\n"
                 "counted_flops_fp64_per_launch: 24\n")


def test_counter_summary_matches_or_is_dropped(tmp_path, monkeypatch):
    f = tmp_path / "t.txt"
    f.write_text(f"kernel: k\nsource_hash: {bench.source_hash()}\n" + COUNTER_LINES)
    monkeypatch.setattr(bench, "COUNTERS_FILE", str(f))
    c = bench.measured_counters()
    assert c == dict(traffic=123.0, valu_busy_pct=55.5, valu_utilization_pct=40.25, valu_insts=7.0,
                     per_kernel_bytes={}, per_kernel_valu={}, kernel="k")
    # per-kernel rows of the table (MB fetched, MB written) are summed per kernel; full rows also give
    # the counted TFLOP/s, its fraction of the unpacked FMA rate and the VALU issue fraction
    f.write_text(f"kernel: k\nsource_hash: {bench.source_hash()}\n" + COUNTER_LINES +
                 "k_trace_tiles<float>  1.5  2.5  80.0\nrtw::k_raster<float>  10.0  0.5  50.0\n"
                 "k_retrace64  2.2  175.2  49.4  92.8  28.89  0.107  1.651  17.66  0.225  0.100  0.473\n")
    c = bench.measured_counters()
    assert c["per_kernel_bytes"] == pytest.approx({"k_trace_tiles<float>": 4.0e6, "rtw::k_raster<float>": 10.5e6,
                                                   "k_retrace64": 177.4e6})
    assert c["per_kernel_valu"] == {"k_retrace64": dict(tflops=17.66, frac_unpacked=0.225, issue_frac=0.473)}
    f.write_text("source_hash: 0000\n" + COUNTER_LINES)
    assert bench.measured_counters() is None  # kernel changed since the counters were taken


def test_committed_counter_summary_is_parseable():
    kv = {}
    with open(bench.COUNTERS_FILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith((" ", "#")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    assert float(kv["fetch_bytes_per_launch"]) > 0 and float(kv["write_bytes_per_launch"]) > 0
    assert 0 < float(kv["valu_busy_pct"]) <= 100 and 0 < float(kv["valu_utilization_pct"]) <= 100
    assert float(kv["valu_insts_per_launch"]) > 0
    assert len(kv["source_hash"]) == 16


def test_committed_batch_trace_summary_is_parseable():
    kv = {}
    with open(os.path.join(ROOT, "profiles", "k_trace_batch4096_valu.txt")) as fh:
        for line in fh:
            if ":" in line and not line.startswith((" ", "#")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    assert 0 < float(kv["trace_valu_issue_frac"]) <= 1.0 and len(kv["source_hash"]) == 16


class _FakeProfiler:
    """Records the bench's profiling calls and the launches between them."""

    def __init__(self):
        self.log, self.on, self.only, self.launches = [], False, None, []

    def profile_enable(self, on):
        self.on = on
        self.log.append(("enable", on))

    def profile_only(self, name):
        self.only = name
        self.log.append(("only", name))

    def profile_read(self):
        self.log.append(("read",))
        rec = [x for x in self.launches if x[0]]
        self.launches = []
        out = {}
        for _, only in rec:
            for k, ms in (("k_a", 1.0), ("k_b", 3.0)):
                if only in (None, k):
                    t, n = out.get(k, (0.0, 0))
                    out[k] = (t + ms, n + 1)
        return out

    def launch(self):
        self.launches.append((self.on, self.only))


def test_timed_steps_brackets_only_the_dominant_kernel(monkeypatch):
    """Warm-up unprofiled, a profiled pass that names the dominant kernel,
    then exactly `steps` timed launches with events around that kernel only
    and the filter cleared afterwards."""
    import torch
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    f = _FakeProfiler()
    ms, prof, (dom, t, n) = bench.timed_steps(f, f.launch, steps=7, warmup=3, prof_steps=2)
    assert prof == {"k_a": (2.0, 2), "k_b": (6.0, 2)}
    assert (dom, t, n) == ("k_b", 21.0, 7)
    assert ms >= 0.0
    assert f.only is None and f.on is False
    assert ("only", "k_b") in f.log and f.log[-2:] == [("only", None), ("read",)]
