"""CPU checks of bench.py's contract that need no GPU: more than one GPU is
refused with a message, and the committed counter summary is used only
while the evaluation kernel's sources still match its digest."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_only_while_the_sources_match(monkeypatch):
    with open(bench.COUNTERS) as fh:
        c = json.load(fh)
    monkeypatch.setattr(bench, "eval_sources_digest", lambda: c["eval_sources_digest"])
    assert bench.measured_traffic() == c["hbm_bytes_per_dispatch"] > 0
    monkeypatch.setattr(bench, "eval_sources_digest", lambda: "0" * 16)
    assert bench.measured_traffic() is None


def test_counter_summary_scaling_is_consistent():
    """Scaled bytes = KiB per dispatch x 1024 x (copy size / copy reading)."""
    with open(bench.COUNTERS) as fh:
        c = json.load(fh)
    tot = 0.0
    for name in ("FETCH_SIZE", "WRITE_SIZE"):
        k = c["counters"][name]
        assert abs(k["factor"] - 262144.0 / k["copy_kib"]) < 1e-9
        tot += k["kib_per_dispatch"] * 1024 * k["factor"]
    assert abs(tot - c["hbm_bytes_per_dispatch"]) < 1e-3 * tot
