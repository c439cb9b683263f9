"""Integrated-window gridding (Sec. 3.1, eq. gridding2, the matrix A) on the
device: the complete smooth part against the oracle's integrated route on
spheres and a cube in both windows and precisions, batched launches against
single ones, switching back to the point gridding, the combination with the
near-field correction (the paper's complete method) against the oracle and
the exact surface integrals, and the combination the library refuses."""
import numpy as np
import pytest

import paper_1305_3162_amd as slp
from oracle import direct, geometry, integrated as iwo
from synth.workloads import cube_random, sphere_random
from slp_testlib import es_for, log, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _geometry(wl, m, prec, window):
    w, g = es_for(wl)
    return slp.Geometry(wl.nodes, wl.tris, wl.grid, m, w, g, wl.alpha, prec, wl.eta2, window=window)


CASES = {
    "sphere_l2_gauss8_fp64": (lambda: sphere_random(2, 4, 32, 8), 8, slp.FP64, slp.WINDOW_GAUSS, 1e-6),
    "sphere_l3_kb4_fp64": (lambda: sphere_random(3, 4, 64, 4), 4, slp.FP64, slp.WINDOW_KB, 1e-6),
    "sphere_l3_gauss5_fp32": (lambda: sphere_random(3, 4, 64, 5), 5, slp.FP32, slp.WINDOW_GAUSS, 1e-4),
    "cube16_kb4_fp64": (lambda: cube_random(16, 2, 64, 4), 4, slp.FP64, slp.WINDOW_KB, 1e-6),
}


@pytest.mark.parametrize("name", list(CASES))
def test_integrated_gridding_against_oracle(name):
    make, m, prec, window, tol = CASES[name]
    wl = make()
    log(f"case integrated {name}: {wl.tris.shape[0]} triangles, grid {wl.grid}")
    prob = direct.prepare_workload(wl)
    G = _geometry(wl, m, prec, window)
    d = torch.as_tensor(wl.dens).cuda()
    point = G.solve(d).cpu().numpy()
    G.setup_integrated_gridding(8)
    info = G.integrated_gridding_info()
    got = G.solve(d).cpu().numpy()
    torch.cuda.synchronize()
    ref = iwo.phi_integrated(prob, wl.nodes, wl.tris, m, "kb" if window == slp.WINDOW_KB else "gauss",
                             n=12)
    e = rel_l2(got, ref)
    log(f"  {info}; rel-L2 vs oracle {e:.3e}; integrated vs point gridding {rel_l2(got, point):.3e}")
    assert info["order"] == 8
    # one stored integral per (triangle, cell of its index box), eq. indexset2:
    # floor(t_min) - m + 1 .. floor(t_max) + m per axis, t the vertices in grid units
    t = (geometry.to_torus(wl.nodes, prob.c, prob.s) + 0.5) * np.asarray(wl.grid, dtype=np.float64)
    tv = t[wl.tris]                                   # [M, 3 vertices, 3 axes]
    # (vertices on a cell face may round either way: bounds with t -/+ 1e-9)
    lo = np.floor(tv.max(axis=1) - 1e-9) - np.floor(tv.min(axis=1) + 1e-9) + 2 * m
    hi = np.floor(tv.max(axis=1) + 1e-9) - np.floor(tv.min(axis=1) - 1e-9) + 2 * m
    assert int(np.prod(lo, axis=1).sum()) <= info["nnz"] <= int(np.prod(hi, axis=1).sum())
    assert np.all(np.isfinite(got)) and e <= tol
    # the route changed (three-point quadrature vs the window integral)
    assert rel_l2(got, point) > 1e-9
    # back to the point gridding
    G.setup_integrated_gridding(0)
    again = G.solve(d).cpu().numpy()
    assert rel_l2(again, point) <= (1e-13 if prec == slp.FP64 else 1e-6)
    G.close()


@pytest.mark.parametrize("prec,tol", [(slp.FP64, 1e-6), (slp.FP32, 1e-4)])
def test_integrated_gridding_volume_targets(prec, tol):
    """Every node of the 16-cell tetrahedral lattice of the cube as an
    evaluation point (the paper's targets), with integrated-window gridding,
    against the oracle's integrated route at the same points."""
    from synth import cube_volume_nodes
    wl = cube_random(16, 2, 64, 4)
    tg = cube_volume_nodes(16)
    log(f"case integrated volume targets prec={prec}: {tg.shape[0]} points")
    prob = direct.prepare(wl.nodes, wl.tris, wl.dens, wl.grid, wl.alpha, wl.es_h, wl.es_r_lo,
                          wl.es_r_hi, wl.es_tol, wl.eta2, targets=tg)
    w, g = es_for(wl)
    G = slp.Geometry(wl.nodes, wl.tris, wl.grid, 4, w, g, wl.alpha, prec, wl.eta2,
                     window=slp.WINDOW_KB, targets=tg)
    G.setup_integrated_gridding(8)
    got = G.solve(torch.as_tensor(wl.dens).cuda()).cpu().numpy()
    torch.cuda.synchronize()
    ref = iwo.phi_integrated(prob, wl.nodes, wl.tris, 4, "kb", n=12)
    e = rel_l2(got, ref)
    log(f"  rel-L2 vs oracle {e:.3e}")
    assert got.shape == (tg.shape[0],) and e <= tol
    G.close()


def test_integrated_batched_equals_single():
    wl = sphere_random(2, 7, 32, 6)
    G = _geometry(wl, 6, slp.FP64, slp.WINDOW_GAUSS)
    G.setup_integrated_gridding(6)
    rng = np.random.default_rng(8)
    dens = [torch.as_tensor(rng.normal(size=wl.n_src)).cuda() for _ in range(11)]
    phis = [torch.full((wl.n_nodes,), float("nan"), dtype=torch.float64, device="cuda") for _ in dens]
    slp.eval_batched([G.handle] * len(dens), dens, phis)
    torch.cuda.synchronize()
    for k in (0, 3, 8, 10):
        ref = G.solve(dens[k])
        torch.cuda.synchronize()
        assert rel_l2(phis[k].cpu().numpy(), ref.cpu().numpy()) <= 1e-14, k
    G.close()


def test_integrated_gridding_with_near_field():
    """The paper's complete method: integrated-window gridding plus the
    near-field correction whose smooth share is integrated with the same rule.
    Against the oracle's integrated route (10^-6), the exact surface integrals
    (the Fourier error), in either setup order; switching the gridding off
    rebuilds the near field for the point sources."""
    from oracle import nearfield as nfo
    wl = sphere_random(2, 4, 64, 8)
    prob = direct.prepare_workload(wl)
    eps = nfo.near_radius(prob, 1e-3, wl.es_r_hi)
    log(f"case integrated + near field sphere_l2, eps {eps:.4f}")
    d = torch.as_tensor(wl.dens).cuda()
    G = _geometry(wl, 8, slp.FP64, slp.WINDOW_GAUSS)
    G.setup_integrated_gridding(8)
    G.setup_near_field(eps)
    got = G.solve(d).cpu().numpy()
    G2 = _geometry(wl, 8, slp.FP64, slp.WINDOW_GAUSS)
    G2.setup_near_field(eps)
    point = G2.solve(d).cpu().numpy()
    G2.setup_integrated_gridding(8)
    got2 = G2.solve(d).cpu().numpy()
    torch.cuda.synchronize()
    near_i, *_ = iwo.phi_near_integrated(prob, wl.nodes, wl.tris, eps, n=12)
    ref = iwo.phi_integrated(prob, wl.nodes, wl.tris, 8, "gauss", 12) + near_i
    gbar = nfo.element_mean_density(prob, wl.tris.shape[0])
    exact = nfo.phi_exact_integrals(wl.nodes, wl.tris, gbar, wl.nodes)
    e = rel_l2(got, ref)
    ex_i = np.abs(got - exact).max() / np.abs(exact).max()
    ex_3 = np.abs(point - exact).max() / np.abs(exact).max()
    log(f"  rel-L2 vs oracle {e:.3e}; vs exact integrals: integrated {ex_i:.3e}, three-point {ex_3:.3e}")
    assert e <= 1e-6 and rel_l2(got2, got) <= 1e-13
    assert ex_i <= 2e-4 and ex_3 >= 10 * ex_i
    # back to the point sources: the near field follows
    G.setup_integrated_gridding(0)
    back = G.solve(d).cpu().numpy()
    assert rel_l2(back, point) <= 1e-13
    G.close()
    G2.close()


def test_integrated_gridding_refusals():
    wl = sphere_random(2, 4, 32, 4)
    G = _geometry(wl, 4, slp.FP64, slp.WINDOW_KB)
    with pytest.raises(slp.SlpError, match="order"):
        G.setup_integrated_gridding(17)
    G.setup_integrated_gridding(4)
    with pytest.raises(slp.SlpError, match="captured"):
        slp.set_graph(G.handle, True)
    G.close()
