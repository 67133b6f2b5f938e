"""Host logic of bench.py (no GPU): the algorithmic work and byte counts
the roofline figures divide by, the traffic record that is reported only
for the kernel sources it was measured on, and the one-GPU contract."""
from __future__ import annotations

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_algorithmic_counts():
    f2 = bench.flops_per_stage_cell()
    assert f2["per_stage_cell"] == 2522 and f2["midpoint"] == 1202
    assert bench.flops_per_stage_cell_1d()["per_stage_cell"] == 872
    # read U^(k) and write U^(k+1) every stage, read U^n in two of three
    assert bench.bytes_per_stage_cell() == pytest.approx((3 * 32 + 2 * 32 + 3 * 32) / 3.0)


def test_traffic_record_follows_the_kernel_sources(monkeypatch):
    with open(bench.TRAFFIC_FILE) as f:
        rec = json.load(f)["quadrant2d_2048"]
    b = (rec["fetch_KiB_per_launch"] * rec["copy_fetch_factor"]
         + rec["write_KiB_per_launch"] * rec["copy_write_factor"]) * 1024
    assert rec["hbm_bytes_per_launch"] == pytest.approx(b)
    if rec["source_hash"] == bench.kernel_source_hash():
        assert bench.measured_traffic("quadrant2d_2048") == rec["hbm_bytes_per_launch"]
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic("quadrant2d_2048") is None
    assert bench.measured_traffic("no_such_workload") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""
