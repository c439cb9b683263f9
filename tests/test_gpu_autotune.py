"""The gridding split (slp_params.seg_share) and the timing autotuner on the
device: every split gives the automatic split's potential up to rounding, the
segment count follows the share, the tuner keeps the fastest timed candidate
and reads it back from its cache, and the tuned window and cut-off meet the
requested tolerance against the oracle's non-uniform DFT."""
import numpy as np
import pytest

import paper_1305_3162_amd as slp
from paper_1305_3162_amd import autotune as at
from oracle import direct
from synth.workloads import cube_random, sphere_random
from slp_testlib import es_for, log, oracle_problem, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    slp.load_library()


@pytest.mark.parametrize("prec,m,window", [(slp.FP64, 8, slp.WINDOW_GAUSS),
                                           (slp.FP32, 3, slp.WINDOW_KB)])
def test_split_does_not_change_the_potential(prec, m, window):
    wl = cube_random(16, 2, 64, m)
    w, g = es_for(wl)
    d = torch.as_tensor(wl.dens).cuda()
    G0 = slp.Geometry(wl.nodes, wl.tris, wl.grid, m, w, g, wl.alpha, prec, wl.eta2, window=window)
    ref = G0.solve(d).cpu().numpy()
    auto, nseg0 = G0.info["seg_share"], G0.info["n_segments"]
    log(f"case split prec={prec} m={m}: auto share {auto}, {nseg0} segments")
    assert auto >= 64 and nseg0 >= 1
    last = None
    for share in (64, 100, 256, 1 << 24):
        G = slp.Geometry(wl.nodes, wl.tris, wl.grid, m, w, g, wl.alpha, prec, wl.eta2,
                         window=window, seg_share=share)
        got = G.solve(d).cpu().numpy()
        torch.cuda.synchronize()
        nseg = G.info["n_segments"]
        assert G.info["seg_share"] == share
        if last is not None:
            assert nseg <= last                   # fewer pieces as the share grows
        last = nseg
        e = rel_l2(got, ref)
        log(f"  share {share}: {nseg} segments, rel-L2 vs automatic split {e:.2e}")
        assert e <= (1e-13 if prec == slp.FP64 else 1e-6)
        G.close()
    assert last <= nseg0
    G0.close()


def test_tune_share_keeps_the_fastest_and_caches(tmp_path):
    wl = sphere_random(4, 5, 64, 6)
    w, g = es_for(wl)
    cache = str(tmp_path / "tune.json")
    r = at.tune_share(wl.nodes, wl.tris, wl.grid, 6, w, g, wl.alpha, slp.FP64, wl.eta2,
                      cache=cache, reps=5)
    log(f"case tune sphere_l4 m=6: {r}")
    assert not r["cached"] and r["candidates"]
    assert r["us"] == min(c["us"] for c in r["candidates"])
    assert r["seg_share"] in [c["seg_share"] for c in r["candidates"]]
    assert any(c["seg_share"] == r["auto_share"] for c in r["candidates"])
    r2 = at.tune_share(wl.nodes, wl.tris, wl.grid, 6, w, g, wl.alpha, slp.FP64, wl.eta2,
                       cache=cache, reps=5)
    assert r2["cached"] and r2["seg_share"] == r["seg_share"]
    G, r3 = at.tuned_geometry(wl.nodes, wl.tris, wl.grid, 6, w, g, wl.alpha, slp.FP64, wl.eta2,
                              cache=cache)
    assert r3["cached"] and G.info["seg_share"] == r["seg_share"]
    d = torch.as_tensor(wl.dens).cuda()
    got = G.solve(d).cpu().numpy()
    G0 = slp.Geometry(wl.nodes, wl.tris, wl.grid, 6, w, g, wl.alpha, slp.FP64, wl.eta2)
    ref = G0.solve(d).cpu().numpy()
    torch.cuda.synchronize()
    assert rel_l2(got, ref) <= 1e-13
    G.close()
    G0.close()


@pytest.mark.parametrize("prec,tol", [(slp.FP64, 1e-6), (slp.FP32, 1e-4)])
def test_tune_cutoff_meets_the_tolerance(prec, tol, tmp_path):
    wl = sphere_random(3, 4, 64, 8)
    w, g = es_for(wl)
    r = at.tune_cutoff(tol, wl.nodes, wl.tris, wl.grid, w, g, wl.alpha, prec, wl.eta2,
                       cache=str(tmp_path / "tune.json"), reps=5)
    log(f"case tune cutoff prec={prec} tol={tol}: {r}")
    assert (r["window"], r["m"]) in [(c["window"], c["m"]) for c in r["candidates"]]
    assert r["us"] == min(c["us"] for c in r["candidates"])
    G = slp.Geometry(wl.nodes, wl.tris, wl.grid, r["m"], w, g, wl.alpha, prec, wl.eta2,
                     window=r["window"], seg_share=r["seg_share"])
    got = G.solve(torch.as_tensor(wl.dens).cuda()).cpu().numpy()
    torch.cuda.synchronize()
    ref = direct.phi_ndft(oracle_problem(wl))
    e = rel_l2(got, ref)
    log(f"  rel-L2 vs oracle NDFT {e:.2e}")
    assert e <= tol
    G.close()
