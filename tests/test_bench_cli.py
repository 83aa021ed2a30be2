"""CPU checks of bench.py's contract that need no GPU: more than one GPU is
refused with a message, the committed counter summary is used only while
the evaluation kernel's sources still match its digest, its HBM bytes are
the counters scaled by a plain copy's readings, and the VALU roofline
follows from its instruction counts."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _summary():
    if not os.path.exists(bench.COUNTERS):
        pytest.skip("no counter summary committed")
    with open(bench.COUNTERS) as fh:
        return json.load(fh)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_counters_only_while_the_sources_match(monkeypatch):
    c = _summary()
    case = sorted(c["cases"])[0]
    monkeypatch.setattr(bench, "eval_sources_digest", lambda: c["eval_sources_digest"])
    assert bench.eval_counters(case) == c["cases"][case]
    monkeypatch.setattr(bench, "eval_sources_digest", lambda: "0" * 16)
    assert bench.eval_counters(case) is None
    r = bench.valu_roofline(None, 1000, 1e-3, 1)
    assert r["achieved"] is None and r["frac"] is None and r["bound"] == "alu"


def test_counter_summary_scaling_is_consistent():
    """Scaled bytes = KiB per dispatch x 1024 x (copy size / copy reading)."""
    c = _summary()
    cal = c["copy_calibration"]
    for name in ("FETCH_SIZE", "WRITE_SIZE"):
        k = cal[name]
        assert abs(k["factor"] - k["copy_bytes"] / 1024.0 / k["copy_kib"]) < 1e-9
    for case, v in c["cases"].items():
        tot = (v["FETCH_SIZE_kib"] * cal["FETCH_SIZE"]["factor"] +
               v["WRITE_SIZE_kib"] * cal["WRITE_SIZE"]["factor"]) * 1024
        assert abs(tot - v["hbm_bytes"]) <= 1e-6 * tot, case


def test_valu_roofline_from_the_counts():
    ctr = {"SQ_INSTS_VALU": 614.4e3, "pairs": 1000.0, "hbm_bytes": 8e6,
           "SQ_INSTS_LDS": 100.0, "SQ_LDS_BANK_CONFLICT": 50.0}
    # 1000 pairs in 1 us: 614.4e3 instructions per us = the peak issue rate
    r = bench.valu_roofline(ctr, 1000, 1e-6, 1)
    assert abs(r["frac"] - 1.0) < 1e-12
    assert abs(r["hbm_measured"]["GBps"] - 8000.0) < 1e-9
    assert r["lds"]["bank_conflict_cycles_per_lds_instruction"] == 0.5
    assert abs(bench.VALU_PEAK_GIPS - 614.4) < 1e-9
