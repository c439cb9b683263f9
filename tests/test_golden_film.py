"""The stored film-size values (written by tests/golden/make_film512_golden.py
through the oracle's NDFT route) agree with the oracle's independent pair-sum
route at one sampled node, and cover the intended sample (CPU only, ~1 min)."""
import os

import numpy as np
import pytest

from oracle import direct
from synth.workloads import make_workload

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "film512_phi_sample.npz")


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="golden values not generated")
def test_film_golden_matches_pair_sum():
    g = np.load(GOLDEN)
    assert g["idx"].size == 10000 and np.all(np.diff(g["idx"]) > 0)
    rng = np.random.default_rng(3003)
    assert np.array_equal(np.sort(rng.choice(544770, size=10000, replace=False)), g["idx"])
    wl = make_workload("film512")
    p = direct.prepare_workload(wl)
    assert p.omega.size == int(g["terms"])
    k = 5000
    r1 = direct.phi_pairs(p, g["idx"][[k]], chunk=65536)[0]
    assert abs(r1 - g["phi"][k]) <= 1e-12 * abs(g["phi"][k])
