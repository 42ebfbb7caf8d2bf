"""bench.py on the CPU: the roofline arithmetic on synthetic launch records,
the refusal of more than one GPU, and the lookup of the committed HBM
traffic record by kernel-source hash."""

import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _recs():
    # two applies: per apply 2 stage launches (kind 1), one projection (0), one reconstruction (2)
    one = [dict(kind=0, ms=0.5, flops=1e9, bytes=1e9), dict(kind=1, ms=2.0, flops=8e12, bytes=4e9),
           dict(kind=1, ms=2.0, flops=8e12, bytes=4e9), dict(kind=2, ms=0.5, flops=1e9, bytes=1e9)]
    return one + one


def test_mfma_roofline_is_stage_flops_over_stage_time():
    r = bench.roofline(_recs(), 2, "c64")
    # 4 launches of 8e12 flops in 8 ms: 4e3 TFLOP/s over 157.3
    assert r["launches"] == 4 and r["avg_launch_ms"] == 2.0
    assert abs(r["achieved"] - 4000.0) < 1e-6 and abs(r["frac"] - round(4000.0 / 157.3, 4)) < 1e-9
    assert r["alg_flops_per_step"] == 16e12 and r["alg_bytes_per_step"] == 8e9
    assert abs(r["kernel_share_of_step"] - 0.8) < 1e-9
    s = bench.roofline(_recs(), 2, "bf16x3")
    assert s["executed_flops_factor"] == 3.0 and abs(s["achieved"] - 12000.0) < 1e-6


def test_hbm_roofline_per_launch_and_whole_apply():
    r = bench.hbm_roofline(_recs())
    assert abs(r["achieved"] - 2000.0) < 1e-6 and r["peak"] == 8000.0 and "whole_apply_gbps" not in r
    w = bench.hbm_roofline(_recs(), steps=2, ms_per_step=4.0, side_by_side=True)
    # per-launch view unchanged; whole apply: 10e9 bytes per step over 4 ms
    assert abs(w["achieved"] - 2000.0) < 1e-6 and abs(w["whole_apply_gbps"] - 2500.0) < 1e-6


def test_breakdown_is_milliseconds_per_step_by_kind():
    b = bench.breakdown(_recs(), 2)
    assert b == {"leaf_project": 0.5, "stages": 4.0, "leaf_reconstruct": 0.5}


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert p.returncode == 2 and "one GPU" in p.stderr


def test_traffic_record_is_used_only_for_the_hashed_kernel_source():
    path = os.path.join(ROOT, "profiles", "hbm_traffic_dft2d_n512_rhs256.json")
    rec = json.load(open(path))
    src = os.path.join(ROOT, rec["kernel_source"])
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    traffic, info = bench.measured_traffic(rec["workload"], rec["prec"])
    if sha == rec["kernel_source_sha256_16"]:
        assert traffic == rec["traffic_bytes_per_launch"] and info["command"]
    else:
        assert traffic is None
    assert bench.measured_traffic("no_such_workload", "c64") == (None, None)
