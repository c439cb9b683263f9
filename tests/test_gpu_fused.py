"""Fused multi-geometry batches (slp_eval_batched_mode with SLP_BATCH_FUSED):
one launch per stage for items on different meshes, the workgroups taken from
device work lists. Every item must equal its own single solve, which the
other GPU tests pin to the oracle; the accumulation order of the gridding's
LDS blocks differs between the two, so the bar is rounding: rel-L2 <= 1e-14
in FP64, <= 1e-6 in FP32 (the grid is stored in FP32 after FP64 block sums).
One item is also checked against the oracle's NUFFT (R3) directly."""
import numpy as np
import pytest

import paper_1305_3162_amd as slp
from oracle import nufft
from synth.workloads import sphere_random, cube_random, Workload, expsum_interval
from synth import box_surface, RandomSmoothMagnetisation, density_from_magnetisation
from slp_testlib import make_geometry, oracle_problem, rel_l2, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    slp.load_library()


def _film(seed, grid, m):
    """A small thin box (anisotropic grid: the passes have different lengths)."""
    nodes, tris = box_surface((1.0, 1.0, 0.1), (12, 12, 2))
    mf = RandomSmoothMagnetisation(seed, nodes.min(0), nodes.max(0))
    dens = density_from_magnetisation(nodes, tris, mf)
    lo, hi = expsum_interval(nodes)
    return Workload(f"box_s{seed}", nodes, tris, dens, grid, m, es_r_lo=lo, es_r_hi=hi)


def _mix(m):
    # different mesh sizes, grid edges and anisotropic grids (the smallest
    # grids that the stencils of this m fit)
    g = 16 if m <= 4 else 32
    return [sphere_random(2, 41, 32, m), sphere_random(3, 42, 64, m), sphere_random(4, 43, 128, m),
            cube_random(8, 44, 64, m), _film(45, (64, 64, g), m), sphere_random(1, 46, g, m)]


def _check(geos, order, dens, phis, tol):
    for k, i in enumerate(order):
        G, wl = geos[i]
        ref = G.solve(dens[k])
        torch.cuda.synchronize()
        e = rel_l2(phis[k].cpu().numpy(), ref.cpu().numpy())
        assert e <= tol, (k, i, e)


@pytest.mark.parametrize("prec,m", [(slp.FP64, 4), (slp.FP32, 3), (slp.FP64, 8)])
def test_fused_equals_single(prec, m):
    log(f"case fused mix prec={prec} m={m}")
    wls = _mix(m)
    geos = [(make_geometry(wl, m, prec), wl) for wl in wls]
    order = [0, 1, 2, 3, 4, 5, 2, 0, 4, 0]        # repeats use further buffer slots
    rng = np.random.default_rng(7)
    dens = [torch.as_tensor(rng.normal(size=geos[i][1].n_src)).cuda() for i in order]
    tol = 1e-14 if prec == slp.FP64 else 1e-6
    for rep in range(2):                          # the second call reuses the cached tables
        phis = [torch.full((geos[i][1].n_nodes,), float("nan"), dtype=torch.float64,
                           device="cuda") for i in order]
        slp.eval_batched([geos[i][0].handle for i in order], dens, phis, mode=slp.BATCH_FUSED)
        sums = torch.stack([p.sum() for p in phis])    # on the caller's stream, after the batch
        torch.cuda.synchronize()
        assert torch.isfinite(sums).all().item(), rep
        _check(geos, order, dens, phis, tol)
    for G, _ in geos:
        G.close()


def test_fused_item_against_oracle():
    """A fused item against the oracle's NUFFT at the same m (R3: the same
    gridding, FFT and interpolation steps on the CPU)."""
    log("case fused item vs R3")
    m = 5
    wla, wlb = sphere_random(2, 51, 32, m), sphere_random(3, 52, 64, m)
    Ga, Gb = make_geometry(wla, m), make_geometry(wlb, m)
    dens = [torch.as_tensor(wla.dens).cuda(), torch.as_tensor(wlb.dens).cuda()]
    phis = [torch.empty(wla.n_nodes, dtype=torch.float64, device="cuda"),
            torch.empty(wlb.n_nodes, dtype=torch.float64, device="cuda")]
    slp.eval_batched([Ga.handle, Gb.handle], dens, phis, mode=slp.BATCH_FUSED)
    torch.cuda.synchronize()
    for wl, phi in ((wla, phis[0]), (wlb, phis[1])):
        e = rel_l2(phi.cpu().numpy(), nufft.phi_nufft(oracle_problem(wl), m))
        log(f"  {wl.name}: rel-L2 vs R3 {e:.3e}")
        assert e <= 1e-10
    Ga.close()
    Gb.close()


def test_fused_with_near_field_and_lanes_agree():
    """A near field on one of the geometries (applied per geometry after the
    fused interpolation); the lanes mode gives the same results."""
    log("case fused with near field")
    m = 4
    wls = [sphere_random(3, 61, 64, m), sphere_random(2, 62, 32, m), cube_random(6, 63, 64, m)]
    geos = [(make_geometry(wl, m), wl) for wl in wls]
    G0 = geos[0][0]
    G0.setup_near_field(G0.near_radius(1e-3))
    order = [0, 1, 2, 0, 1]
    rng = np.random.default_rng(8)
    dens = [torch.as_tensor(rng.normal(size=geos[i][1].n_src)).cuda() for i in order]
    out = {}
    for mode in (slp.BATCH_FUSED, slp.BATCH_LANES, slp.BATCH_AUTO):
        phis = [torch.empty(geos[i][1].n_nodes, dtype=torch.float64, device="cuda") for i in order]
        slp.eval_batched([geos[i][0].handle for i in order], dens, phis, mode=mode)
        torch.cuda.synchronize()
        _check(geos, order, dens, phis, 1e-14)
        out[mode] = [p.cpu().numpy() for p in phis]
    for a, b in zip(out[slp.BATCH_FUSED], out[slp.BATCH_LANES]):
        assert rel_l2(a, b) <= 1e-14
    for G, _ in geos:
        G.close()


def test_fused_more_items_than_one_launch():
    """70 items on three geometries: launches of at most 64 items, per-item
    buffers grown as a geometry repeats (cached tables rebuilt for them)."""
    log("case fused 70 items")
    m = 3
    wls = [sphere_random(2, 71, 32, m), sphere_random(1, 72, 16, m), cube_random(4, 73, 32, m)]
    geos = [(make_geometry(wl, m, slp.FP32), wl) for wl in wls]
    order = [k % 3 for k in range(70)]
    rng = np.random.default_rng(10)
    dens = [torch.as_tensor(rng.normal(size=geos[i][1].n_src)).cuda() for i in order]
    phis = [torch.full((geos[i][1].n_nodes,), float("nan"), dtype=torch.float64, device="cuda")
            for i in order]
    slp.eval_batched([geos[i][0].handle for i in order], dens, phis)   # AUTO: fused
    torch.cuda.synchronize()
    assert all(torch.isfinite(p).all().item() for p in phis)
    sel = [0, 1, 2, 31, 63, 64, 65, 69]
    _check(geos, [order[k] for k in sel], [dens[k] for k in sel], [phis[k] for k in sel], 1e-6)
    for G, _ in geos:
        G.close()


def test_fused_rejects_mixed_cutoff():
    log("case fused rejects mixed m")
    wla, wlb = sphere_random(1, 81, 16, 3), sphere_random(1, 82, 16, 4)
    Ga, Gb = make_geometry(wla, 3), make_geometry(wlb, 4)
    dens = [torch.as_tensor(wla.dens).cuda(), torch.as_tensor(wlb.dens).cuda()]
    phis = [torch.empty(wla.n_nodes, dtype=torch.float64, device="cuda"),
            torch.empty(wlb.n_nodes, dtype=torch.float64, device="cuda")]
    with pytest.raises(slp.SlpError):
        slp.eval_batched([Ga.handle, Gb.handle], dens, phis, mode=slp.BATCH_FUSED)
    # AUTO falls back to the lanes
    slp.eval_batched([Ga.handle, Gb.handle], dens, phis)
    torch.cuda.synchronize()
    _check([(Ga, wla), (Gb, wlb)], [0, 1], dens, phis, 1e-14)
    Ga.close()
    Gb.close()
