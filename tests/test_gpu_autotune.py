"""The gridding split (slp_params.seg_share), the block-sum form
(slp_params.reduce_cells) and the timing autotuner on the device: every split
and both block-sum forms give the automatic potential up to rounding, the
segment count follows the share, the tuner keeps the
fastest timed candidate and reads it back from its cache, and the tuned window
and cut-off meet the requested tolerance against the oracle's non-uniform
DFT."""
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
    assert (r["seg_share"], r["reduce_cells"]) in [(c["seg_share"], c["reduce_cells"])
                                                   for c in r["candidates"]]
    assert any(c["seg_share"] == r["auto_share"] for c in r["candidates"])
    # both block-sum forms timed at the fastest split
    assert {c["reduce_cells"] for c in r["candidates"]} == {1, 2}
    r2 = at.tune_share(wl.nodes, wl.tris, wl.grid, 6, w, g, wl.alpha, slp.FP64, wl.eta2,
                       cache=cache, reps=5)
    assert r2["cached"] and r2["seg_share"] == r["seg_share"]
    assert r2["reduce_cells"] == r["reduce_cells"]
    G, r3 = at.tuned_geometry(wl.nodes, wl.tris, wl.grid, 6, w, g, wl.alpha, slp.FP64, wl.eta2,
                              cache=cache)
    assert r3["cached"] and G.info["seg_share"] == r["seg_share"]
    assert G.info["reduce_cells"] == r["reduce_cells"]
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


@pytest.mark.parametrize("prec,m,window", [(slp.FP64, 4, slp.WINDOW_KB), (slp.FP32, 3, slp.WINDOW_KB),
                                           (slp.FP64, 8, slp.WINDOW_GAUSS)])
def test_block_sum_forms_agree(prec, m, window):
    """slp_params.reduce_cells: one or two cells per thread of the block sum add
    each cell's terms in one order, so the potentials differ only by the
    gridding's own rounding order (its LDS accumulation order varies with
    scheduling), single and batched. The region of this cube (512 or 729
    tiles) takes one cell per thread automatically, and two in a batch of four
    densities (at least 2048 tiles)."""
    wl = cube_random(32, 3, 128, m)
    w, g = es_for(wl)
    geos = {c: slp.Geometry(wl.nodes, wl.tris, wl.grid, m, w, g, wl.alpha, prec, wl.eta2,
                            window=window, reduce_cells=c) for c in (0, 1, 2)}
    tiles = int(np.prod(geos[0].info["tiles"]))
    log(f"case block-sum forms prec={prec} m={m}: {tiles} tiles")
    assert tiles < 2048 <= 4 * tiles
    assert [geos[c].info["reduce_cells"] for c in (0, 1, 2)] == [1, 1, 2]
    tol = 1e-14 if prec == slp.FP64 else 1e-6
    rng = np.random.default_rng(11)
    dens = [torch.as_tensor(rng.normal(size=wl.n_src)).cuda() for _ in range(4)]
    single = {c: geos[c].solve(dens[0]) for c in (0, 1, 2)}
    batched = {}
    for c in (0, 1, 2):
        phis = [torch.full((wl.n_nodes,), float("nan"), dtype=torch.float64, device="cuda")
                for _ in range(4)]
        slp.eval_batched([geos[c].handle] * 4, dens, phis)
        batched[c] = [p.cpu().numpy() for p in phis]
    torch.cuda.synchronize()
    single = {c: v.cpu().numpy() for c, v in single.items()}
    assert np.isfinite(single[1]).all()
    for c in (0, 2):
        assert rel_l2(single[c], single[1]) <= tol, c
    for k in range(4):
        assert np.isfinite(batched[1][k]).all()
        for c in (0, 2):
            assert rel_l2(batched[c][k], batched[1][k]) <= tol, (c, k)
    assert rel_l2(batched[2][0], single[1]) <= tol
    for G in geos.values():
        G.close()


def test_block_sum_forms_on_the_smallest_regions():
    """Both block-sum forms on regions of one to a few tiles (an icosphere on
    16^3 and 32^3 grids), where the two-cell form has more threads' cells on
    the region's edge than inside it."""
    for level, grid, m in ((1, 16, 3), (2, 32, 4), (2, 32, 2)):
        wl = sphere_random(level, 90 + level, grid, m)
        w, g = es_for(wl)
        d = torch.as_tensor(wl.dens).cuda()
        out = {}
        for c in (1, 2):
            G = slp.Geometry(wl.nodes, wl.tris, wl.grid, m, w, g, wl.alpha, slp.FP64, wl.eta2,
                             window=slp.WINDOW_KB, reduce_cells=c)
            out[c] = G.solve(d).cpu().numpy()
            tiles = G.info["tiles"]
            G.close()
        log(f"case block-sum forms small region: level {level}, grid {grid}, m {m}, tiles {tiles}")
        assert np.isfinite(out[1]).all()
        assert rel_l2(out[2], out[1]) <= 1e-14
        e = rel_l2(out[2], direct.phi_ndft(oracle_problem(wl)))
        log(f"  rel-L2 vs oracle NDFT {e:.2e}")
        assert e <= 4 * np.exp(-2 * np.pi * m / 3)
