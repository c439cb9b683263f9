"""bench.py's host logic (no GPU): the algorithmic bytes of the near-field
product for either storage of its values, the storage option, the committed
HBM-traffic table (its source hash must match the gridding kernels as they
stand, or the bench reports no traffic), and the one-GPU refusal."""
import argparse
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
import paper_1305_3162_amd as slp  # noqa: E402


def _info(stored, packed):
    return {"extent": [80, 80, 80], "_n": [64, 64, 64], "n_targets": 1000, "n_src": 3000,
            "_stored": stored, "_packed": packed}


@pytest.mark.parametrize("packed", [True, False])
def test_near_bytes_follow_the_value_storage(packed):
    st = 256 * 1000
    b64, unit, bound = bench.algorithmic_units("near", _info(st, packed), 8, 8)
    assert unit == "byte" and bound == "hbm"
    b32, *_ = bench.algorithmic_units("near", dict(_info(st, packed), _near_esz=4), 8, 8)
    assert b64 - b32 == 4 * st
    colb = 2 * st + 4 * (st // 256) if packed else 4 * st
    assert b64 == 8 * st + colb + 1001 * 8 + 3000 * 8 + 16 * 1000


def test_near_storage_option():
    a = argparse.Namespace(near_storage="context")
    assert bench.near_storage(a, slp, slp.FP32) == slp.FP32
    a.near_storage = "fp32"
    assert bench.near_storage(a, slp, slp.FP64) == slp.FP32
    a.near_storage = "fp64"
    assert bench.near_storage(a, slp, slp.FP32) == slp.FP64


def test_traffic_table_matches_the_kernels_as_they_stand():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic_cube64.json")))
    args = argparse.Namespace(workload="cube64", precision="fp64", window="gauss",
                              near_tol=None, near_storage="context", integrated=0)
    t = bench.measured_traffic(args, 8, "spread_bins", 1)
    assert t is not None and t == rec["entries"]["cube64/fp64/gauss/m8"]["bytes_per_launch"]
    # configurations no counter run covers report none
    assert bench.measured_traffic(args, 8, "interp", 1) is None
    assert bench.measured_traffic(args, 8, "spread_bins", 2) is None
    args.near_tol, args.near_storage = 1e-4, "fp32"
    assert bench.measured_traffic(args, 8, "near", 1) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
