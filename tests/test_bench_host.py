"""bench.py's host logic (no GPU): the algorithmic bytes of the near-field
product for either storage of its values, the storage option, the committed
HBM-traffic table (its source hashes must match the kernels as they stand, or
the bench reports no traffic), the window choice at the precision gates, and
the one-GPU refusal."""
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
    """Every committed counter entry is reported only while the kernel sources
    it was taken on are unchanged (comments aside); a changed kernel source
    makes the bench report no traffic until the counters are retaken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        assert bench.measured_traffic("film512/fp64/kb/m4", "spread_bins", 1) is None
        return
    rec = json.load(open(path))
    for key, e in rec["entries"].items():
        t = bench.measured_traffic(key, e["stage"], 1)
        assert t == e["bytes_per_launch"], key
        # another stage, a batch, or an unknown workload report none
        assert bench.measured_traffic(key, "no_such_stage", 1) is None
        assert bench.measured_traffic(key, e["stage"], 2) is None
    assert bench.measured_traffic("no/such/key", "spread_bins", 1) is None


def test_traffic_keys():
    assert bench.traffic_key("film512", "fp64", "kb", 4) == "film512/fp64/kb/m4"
    assert bench.traffic_key("cube64", "fp64", "gauss", 8, 1e-4, "fp32") == \
        "cube64/fp64/gauss/m8/near0.0001/storedfp32"
    assert bench.traffic_key("cube64", "fp64", "gauss", 8, 1e-4, "context") == \
        "cube64/fp64/gauss/m8/near0.0001"


def test_window_choice_follows_the_precision_gate():
    a = argparse.Namespace(m=None, window=None, tol=None, precision="fp64")
    assert bench.resolve_window(a, slp, slp.FP64) == slp.choose_cutoff(1e-6, slp.FP64)
    a.precision = "fp32"
    assert bench.resolve_window(a, slp, slp.FP32) == slp.choose_cutoff(1e-4, slp.FP32)
    a.window = "gauss"
    w, m = bench.resolve_window(a, slp, slp.FP32)
    assert w == slp.WINDOW_GAUSS and (w, m) == slp.choose_cutoff(1e-4, slp.FP32, slp.WINDOW_GAUSS)
    a.m = 6
    assert bench.resolve_window(a, slp, slp.FP32) == (slp.WINDOW_GAUSS, 6)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
