"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances:
  * against R3 (the same gridding/FFT/NFFT steps on the CPU, same m): the
    difference is rounding only: rel-L2 <= 1e-10 in FP64, <= 2e-5 in FP32;
  * against the definition R1/R2 (no window): the window error plus rounding,
    gated at rel-L2 <= 1e-6 in FP64 (m >= 7) and <= 1e-4 in FP32 (m >= 5);
  * at other m the error against the definition is printed and bounded by
    the Gaussian-window estimate 4 exp(-2 pi m / 3) (alpha = 2).
"""
import numpy as np
import pytest

import paper_1305_3162_amd as slp
from oracle import direct, nufft
from synth.workloads import make_workload, sphere_random
from synth import icosphere
from slp_testlib import gpu_phi, oracle_problem, rel_l2, log, make_geometry

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    slp.load_library()


def _region_map(info, grid):
    """R3 array indices of the GPU region cells along each axis."""
    lo, ext = info["lo"], info["extent"]
    return [np.mod(np.arange(lo[q], lo[q] + ext[q]) - grid[q] // 2, grid[q]) for q in range(3)]


@pytest.mark.parametrize("grid,m,alpha", [((16, 16, 16), 2, 2), ((32, 16, 64), 3, 2),
                                          ((64, 64, 64), 4, 4), ((8, 8, 8), 1, 2)])
def test_stagewise_against_cpu_nufft(grid, m, alpha):
    wl = sphere_random(1, 7, grid[0], m)
    wl.grid, wl.alpha = grid, alpha
    log(f"case grid={grid} m={m} alpha={alpha}")
    p = oracle_problem(wl)
    phi3, st = nufft.phi_nufft(p, m, stages=True)
    G = make_geometry(wl, m)
    info = G.info
    d = torch.as_tensor(wl.dens).cuda()
    phi = G.solve(d)
    P = [8 * t for t in info["tiles"]]
    ext = info["extent"]
    a_gpu = torch.empty(P[2] * P[1] * P[0], dtype=torch.float64, device="cuda")
    g_gpu = torch.empty(ext[2] * ext[1] * ext[0], dtype=torch.float64, device="cuda")
    slp.debug_copy(G.handle, 0, a_gpu)
    slp.debug_copy(G.handle, 1, g_gpu)
    torch.cuda.synchronize()
    b = info["window_b"]
    a_gpu = a_gpu.cpu().numpy().reshape(P[2], P[1], P[0])
    g_gpu = g_gpu.cpu().numpy().reshape(ext[2], ext[1], ext[0])
    ix, iy, iz = _region_map(info, grid)
    a_ref = st["a"][np.ix_(ix, iy, iz)].transpose(2, 1, 0) * (np.pi * b) ** 1.5
    assert np.abs(a_gpu[:ext[2], :ext[1], :ext[0]] - a_ref).max() <= 1e-13 * np.abs(a_ref).max()
    assert np.all(a_gpu[ext[2]:] == 0) and np.all(a_gpu[:, ext[1]:] == 0) and np.all(a_gpu[:, :, ext[0]:] == 0)
    # the whole grid outside the region is zero in the oracle too
    assert np.isclose(np.abs(st["a"]).sum() * (np.pi * b) ** 1.5, np.abs(a_gpu).sum(), rtol=1e-12)
    g_ref = np.real(st["g"])[np.ix_(ix, iy, iz)].transpose(2, 1, 0) * (np.pi * b) ** -1.5 / (4 * np.pi)
    assert np.abs(g_gpu - g_ref).max() <= 1e-11 * np.abs(g_ref).max()
    phi = phi.cpu().numpy()
    e3 = rel_l2(phi, phi3)
    e1 = rel_l2(phi, direct.phi_pairs(p))
    log(f"  vs R3 {e3:.3e}  vs R1 {e1:.3e}")
    assert e3 <= 1e-10
    assert e1 <= 4 * np.exp(-2 * np.pi * m / 3) * (2.0 / alpha) ** 0 + 1e-12
    G.close()


@pytest.fixture(scope="module")
def sphere_l3():
    wl = make_workload("sphere_l3")
    p = oracle_problem(wl)
    return wl, p, direct.phi_ndft(p)


@pytest.mark.parametrize("m", [4, 6, 8])
def test_sphere_l3_fp64(sphere_l3, m):
    wl, p, ref = sphere_l3
    log(f"case sphere_l3 fp64 m={m}")
    phi = gpu_phi(wl, m, slp.FP64)
    e_def = rel_l2(phi, ref)
    e_r3 = rel_l2(phi, nufft.phi_nufft(p, m))
    log(f"  rel-L2 vs definition {e_def:.3e}, vs R3 {e_r3:.3e}")
    assert e_r3 <= 1e-10
    assert e_def <= 4 * np.exp(-2 * np.pi * m / 3)
    if m >= 7:
        assert e_def <= 1e-6


@pytest.mark.parametrize("m", [4, 5, 6])
def test_sphere_l3_fp32(sphere_l3, m):
    wl, p, ref = sphere_l3
    log(f"case sphere_l3 fp32 m={m}")
    phi = gpu_phi(wl, m, slp.FP32)
    e_def = rel_l2(phi, ref)
    e_r3 = rel_l2(phi, nufft.phi_nufft(p, m))
    log(f"  rel-L2 vs definition {e_def:.3e}, vs R3 {e_r3:.3e}")
    assert e_r3 <= 2e-5
    if m >= 5:
        assert e_def <= 1e-4


@pytest.fixture(scope="module")
def cube64():
    wl = make_workload("cube64")
    p = oracle_problem(wl)
    return wl, p, direct.phi_ndft(p)


@pytest.mark.parametrize("m,prec,tol", [(8, slp.FP64, 1e-6), (5, slp.FP32, 1e-4),
                                        (4, slp.FP64, None), (4, slp.FP32, None)])
def test_cube64_against_definition(cube64, m, prec, tol):
    wl, p, ref = cube64
    log(f"case cube64 m={m} prec={'fp64' if prec == slp.FP64 else 'fp32'}")
    phi = gpu_phi(wl, m, prec)
    e = rel_l2(phi, ref)
    log(f"  rel-L2 vs definition {e:.3e} over {phi.size} nodes")
    if tol is not None:
        assert e <= tol
    assert e <= 4 * np.exp(-2 * np.pi * m / 3)


def test_determinism_and_linearity():
    wl = sphere_random(2, 3, 64, 6)
    log("case determinism/linearity sphere_l2 grid 64 m=6")
    G = make_geometry(wl, 6, slp.FP64)
    rng = np.random.default_rng(1)
    g1 = torch.as_tensor(rng.normal(size=wl.n_src)).cuda()
    g2 = torch.as_tensor(rng.normal(size=wl.n_src)).cuda()
    a = G.solve(g1)
    a2 = G.solve(g1)
    b = G.solve(g2)
    c = G.solve(2 * g1 - 3 * g2)
    torch.cuda.synchronize()
    # LDS accumulation order of the gridding may differ between runs: rounding only
    assert rel_l2(a.cpu().numpy(), a2.cpu().numpy()) <= 1e-14
    assert rel_l2((c).cpu().numpy(), (2 * a - 3 * b).cpu().numpy()) <= 1e-12
    z = G.solve(torch.zeros_like(g1))
    assert torch.count_nonzero(z).item() == 0
    G.close()


def test_batched_equals_single():
    log("case batched vs single")
    wla = sphere_random(2, 5, 64, 5)
    wlb = make_workload("sphere_l3", 5)
    Ga, Gb = make_geometry(wla, 5), make_geometry(wlb, 5)
    rng = np.random.default_rng(2)
    dens = [torch.as_tensor(rng.normal(size=wla.n_src)).cuda(),
            torch.as_tensor(wlb.dens).cuda(),
            torch.as_tensor(rng.normal(size=wla.n_src)).cuda()]
    geoms = [Ga.handle, Gb.handle, Ga.handle]
    phis = [torch.empty(wla.n_nodes, dtype=torch.float64, device="cuda"),
            torch.empty(wlb.n_nodes, dtype=torch.float64, device="cuda"),
            torch.empty(wla.n_nodes, dtype=torch.float64, device="cuda")]
    slp.eval_batched(geoms, dens, phis)
    solo = [Ga.solve(dens[0]), Gb.solve(dens[1]), Ga.solve(dens[2])]
    torch.cuda.synchronize()
    for x, y in zip(phis, solo):
        assert rel_l2(x.cpu().numpy(), y.cpu().numpy()) <= 1e-14
    Ga.close()
    Gb.close()


def test_single_open_triangle_and_min_grid():
    """One triangle (an open surface, 3 sources, 3 targets) on the smallest grid."""
    log("case single triangle grid 8 m=1")
    nodes = np.array([[0.0, 0.0, 0.0], [1.0, 0.2, 0.1], [0.3, 0.9, -0.2]])
    tris = np.array([[0, 1, 2]], dtype=np.int32)
    from synth.workloads import Workload, expsum_interval
    lo, hi = expsum_interval(nodes)
    wl = Workload("tri", nodes, tris, np.array([1.0, -0.5, 2.0]), (8, 8, 8), 1,
                  es_r_lo=lo, es_r_hi=hi)
    p = oracle_problem(wl)
    phi = gpu_phi(wl)
    assert rel_l2(phi, nufft.phi_nufft(p, 1)) <= 1e-10


def test_timing_reports_every_stage():
    wl = make_workload("sphere_l3", 4)
    G = make_geometry(wl, 4)
    slp.set_timing(G.handle, True)
    d = torch.as_tensor(wl.dens).cuda()
    for _ in range(40):                      # more than the event ring holds
        G.solve(d)
    ms, cnt = slp.stage_times(G.handle, reset=True)
    assert cnt == 40
    # without a near field its stage takes no time
    assert all(v > 0 for k, v in ms.items() if k != "near") and ms["near"] == 0.0, ms
    G.setup_near_field(G.near_radius(1e-2))
    for _ in range(5):
        G.solve(d)
    ms, cnt = slp.stage_times(G.handle, reset=True)
    assert cnt == 5 and all(v > 0 for v in ms.values()), ms
    G.close()


@pytest.mark.parametrize("prec", [slp.FP64, slp.FP32])
def test_multi_density_batch_equals_single(prec):
    """Consecutive items on one geometry share every launch (grid y = item):
    70 items on one sphere run as 64 + 6, interleaved with another geometry."""
    log(f"case multi-density batch prec={prec}")
    wla = sphere_random(2, 21, 64, 5)
    wlb = sphere_random(1, 22, 32, 3)
    Ga, Gb = make_geometry(wla, 5, prec), make_geometry(wlb, 3, prec)
    rng = np.random.default_rng(4)
    geoms, dens, phis = [], [], []
    for k in range(71):
        G, wl = (Gb, wlb) if k == 35 else (Ga, wla)
        geoms.append(G.handle)
        dens.append(torch.as_tensor(rng.normal(size=wl.n_src)).cuda())
        phis.append(torch.full((wl.n_nodes,), float("nan"), dtype=torch.float64, device="cuda"))
    slp.eval_batched(geoms, dens, phis)
    torch.cuda.synchronize()
    tol = 1e-14 if prec == slp.FP64 else 1e-6
    for k in (0, 1, 34, 35, 36, 63, 64, 70):
        G = Gb if k == 35 else Ga
        ref = G.solve(dens[k])
        torch.cuda.synchronize()
        assert rel_l2(phis[k].cpu().numpy(), ref.cpu().numpy()) <= tol, k
    assert all(torch.isfinite(p).all().item() for p in phis)
    Ga.close()
    Gb.close()


@pytest.mark.parametrize("with_dphi", [False, True])
def test_density_from_nodal_m(with_dphi):
    """Element-constant density from a nodal magnetisation (P1 ansatz) formed on
    the device, then the whole solve, against the oracle's density and definition."""
    from synth import RandomSmoothMagnetisation
    from oracle import geometry
    wl = make_workload("sphere_l3", 6)
    log(f"case density_from_m sphere_l3 m=6 dphi={with_dphi}")
    mf = RandomSmoothMagnetisation(21, wl.nodes.min(0), wl.nodes.max(0))
    m_nodes = mf(wl.nodes)
    rng = np.random.default_rng(22)
    dphi = rng.normal(size=wl.tris.shape[0]) if with_dphi else None
    g_ref = geometry.density_p1(wl.nodes, wl.tris, m_nodes, dphi)
    G = make_geometry(wl, 6, slp.FP64)
    G.set_density_from_m(torch.as_tensor(m_nodes).cuda().contiguous(),
                         None if dphi is None else torch.as_tensor(dphi).cuda())
    phi = torch.empty(wl.n_nodes, dtype=torch.float64, device="cuda")
    G.eval(phi)
    dev_g = torch.empty(wl.n_src, dtype=torch.float64, device="cuda")
    slp.debug_copy(G.handle, 2, dev_g)
    torch.cuda.synchronize()
    assert np.allclose(dev_g.cpu().numpy(), g_ref, rtol=1e-14, atol=1e-15)
    # the same solve from the oracle's density through set_density
    phi2 = G.solve(torch.as_tensor(g_ref).cuda())
    torch.cuda.synchronize()
    assert rel_l2(phi.cpu().numpy(), phi2.cpu().numpy()) <= 1e-13
    # against the definition (NDFT route) with the oracle's density
    p = oracle_problem(wl)
    p.g = g_ref
    e = rel_l2(phi.cpu().numpy(), direct.phi_ndft(p))
    log(f"  rel-L2 vs definition {e:.3e}")
    assert e <= 4 * np.exp(-2 * np.pi * 6 / 3)
    G.close()


def test_multi_mesh_batch_overlaps_and_joins():
    """Items on six geometries (two precisions, more geometries than overlap
    lanes, repeats interleaved) in one batched call, twice in a row: every result
    equals its single solve, and work queued on the caller's stream afterwards
    sees the finished results."""
    log("case multi-mesh batch (6 geometries, lanes)")
    specs = [(sphere_random(1, 31, 32, 3), 3, slp.FP64), (sphere_random(2, 32, 64, 5), 5, slp.FP32),
             (sphere_random(3, 33, 64, 4), 4, slp.FP64), (sphere_random(2, 34, 64, 6), 6, slp.FP64),
             (sphere_random(1, 35, 32, 2), 2, slp.FP32), (sphere_random(3, 36, 128, 5), 5, slp.FP32)]
    geos = [(make_geometry(wl, m, p), wl, p) for wl, m, p in specs]
    rng = np.random.default_rng(9)
    order = [0, 1, 2, 3, 4, 5, 5, 2, 0, 0, 3, 1, 4]
    dens = [torch.as_tensor(rng.normal(size=geos[i][1].n_src)).cuda() for i in order]
    torch.cuda.synchronize()
    for rep in range(2):
        phis = [torch.full((geos[i][1].n_nodes,), float("nan"), dtype=torch.float64, device="cuda")
                for i in order]
        slp.eval_batched([geos[i][0].handle for i in order], dens, phis)
        sums = torch.stack([p.sum() for p in phis])        # on the caller's stream
        torch.cuda.synchronize()
        assert torch.isfinite(sums).all().item(), rep
        for k, i in enumerate(order):
            G, wl, p = geos[i]
            ref = G.solve(dens[k])
            torch.cuda.synchronize()
            tol = 1e-14 if p == slp.FP64 else 1e-6
            assert rel_l2(phis[k].cpu().numpy(), ref.cpu().numpy()) <= tol, (rep, k)
    for G, _, _ in geos:
        G.close()
