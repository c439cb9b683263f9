"""The Kaiser-Bessel window (Sec. 3.2, eq. KBfct / eq. cFB) on the GPU against
the oracle: stage by stage against the step-by-step NUFFT with the same window
(rounding only), and against the definition (the window error, within the
bound of eq. error_bound_nufft; the FP64 gate 1e-6 at m = 4, FP32 1e-4 at m = 3)."""
import numpy as np
import pytest

import paper_1305_3162_amd as slp
from oracle import direct, nufft
from synth.workloads import make_workload, sphere_random
from slp_testlib import es_for, log, oracle_problem, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    slp.load_library()


def _kb_bound(m, alpha=2):
    return 4 * np.pi * (np.sqrt(m) + m) * (1 - 1 / alpha) ** 0.25 * np.exp(
        -2 * np.pi * m * np.sqrt(1 - 1 / alpha))


def _geom(wl, m, prec, grid=None):
    w, g = es_for(wl)
    return slp.Geometry(wl.nodes, wl.tris, grid or wl.grid, m, w, g, wl.alpha, prec, wl.eta2,
                        window=slp.WINDOW_KB)


def _solve(G, dens):
    phi = G.solve(torch.as_tensor(dens).cuda())
    torch.cuda.synchronize()
    return phi.cpu().numpy()


@pytest.mark.parametrize("grid,m,alpha", [((16, 16, 16), 2, 2), ((32, 16, 64), 3, 2),
                                          ((64, 64, 64), 4, 4), ((8, 8, 8), 1, 2)])
def test_kb_stagewise_against_cpu_nufft(grid, m, alpha):
    wl = sphere_random(1, 7, grid[0], m)
    wl.grid, wl.alpha = grid, alpha
    log(f"case kb grid={grid} m={m} alpha={alpha}")
    p = oracle_problem(wl)
    phi3, st = nufft.phi_nufft(p, m, stages=True, window="kb")
    G = _geom(wl, m, slp.FP64)
    info = G.info
    b = info["window_b"]
    assert np.isclose(b, np.pi * (2 - 1 / alpha))
    phi = G.solve(torch.as_tensor(wl.dens).cuda())
    P = [8 * t for t in info["tiles"]]
    ext = info["extent"]
    a_gpu = torch.empty(P[2] * P[1] * P[0], dtype=torch.float64, device="cuda")
    g_gpu = torch.empty(ext[2] * ext[1] * ext[0], dtype=torch.float64, device="cuda")
    slp.debug_copy(G.handle, 0, a_gpu)
    slp.debug_copy(G.handle, 1, g_gpu)
    torch.cuda.synchronize()
    # the kernels evaluate the window scaled to 1 at tau = 0: pi m / sinh(b m) times eq. KBfct
    c1 = np.pi * m / np.sinh(b * m)
    lo = info["lo"]
    ix, iy, iz = [np.mod(np.arange(lo[q], lo[q] + ext[q]) - grid[q] // 2, grid[q]) for q in range(3)]
    a_gpu = a_gpu.cpu().numpy().reshape(P[2], P[1], P[0])
    g_gpu = g_gpu.cpu().numpy().reshape(ext[2], ext[1], ext[0])
    a_ref = st["a"][np.ix_(ix, iy, iz)].transpose(2, 1, 0) * c1 ** 3
    assert np.abs(a_gpu[:ext[2], :ext[1], :ext[0]] - a_ref).max() <= 1e-13 * np.abs(a_ref).max()
    g_ref = np.real(st["g"])[np.ix_(ix, iy, iz)].transpose(2, 1, 0) / (4 * np.pi * c1 ** 3)
    assert np.abs(g_gpu - g_ref).max() <= 1e-11 * np.abs(g_ref).max()
    phi = phi.cpu().numpy()
    e3 = rel_l2(phi, phi3)
    e1 = rel_l2(phi, direct.phi_pairs(p))
    log(f"  vs R3 {e3:.3e}  vs R1 {e1:.3e}")
    assert e3 <= 1e-10
    assert e1 <= _kb_bound(m, alpha)
    G.close()


@pytest.fixture(scope="module")
def sphere_l3():
    wl = make_workload("sphere_l3")
    p = oracle_problem(wl)
    return wl, p, direct.phi_ndft(p)


@pytest.mark.parametrize("m,prec", [(3, slp.FP64), (4, slp.FP64), (6, slp.FP64),
                                    (3, slp.FP32), (4, slp.FP32)])
def test_kb_sphere_l3(sphere_l3, m, prec):
    wl, p, ref = sphere_l3
    log(f"case kb sphere_l3 m={m} prec={prec}")
    G = _geom(wl, m, prec)
    phi = _solve(G, wl.dens)
    G.close()
    e_def = rel_l2(phi, ref)
    e_r3 = rel_l2(phi, nufft.phi_nufft(p, m, window="kb"))
    log(f"  rel-L2 vs definition {e_def:.3e}, vs R3 {e_r3:.3e}")
    assert e_r3 <= (1e-10 if prec == slp.FP64 else 2e-5)
    assert e_def <= _kb_bound(m) + (0 if prec == slp.FP64 else 2e-5)
    if prec == slp.FP64 and m >= 4:
        assert e_def <= 1e-6
    if prec == slp.FP32 and m >= 3:
        assert e_def <= 1e-4


@pytest.mark.parametrize("m,prec,tol", [(4, slp.FP64, 1e-6), (5, slp.FP64, 1e-6),
                                        (3, slp.FP32, 1e-4), (4, slp.FP32, 1e-4)])
def test_kb_cube64_against_definition(m, prec, tol):
    wl = make_workload("cube64", m)
    log(f"case kb cube64 m={m} prec={prec}")
    ref = direct.phi_ndft(oracle_problem(wl))
    G = _geom(wl, m, prec)
    phi = _solve(G, wl.dens)
    G.close()
    e = rel_l2(phi, ref)
    log(f"  rel-L2 vs definition {e:.3e}")
    assert e <= tol


@pytest.mark.parametrize("tol,prec,window", [(1e-6, slp.FP64, None), (1e-6, slp.FP64, slp.WINDOW_GAUSS),
                                             (1e-4, slp.FP32, None), (1e-4, slp.FP32, slp.WINDOW_GAUSS)])
def test_chosen_cutoff_meets_tolerance(tol, prec, window):
    """The window and m picked by slp_choose_cutoff reach the tolerance on cube64."""
    w_, m = slp.choose_cutoff(tol, prec, window)
    wl = make_workload("cube64", m)
    log(f"case chosen cutoff tol={tol} prec={prec} -> window={w_} m={m}")
    ref = direct.phi_ndft(oracle_problem(wl))
    w, g = es_for(wl)
    G = slp.Geometry(wl.nodes, wl.tris, wl.grid, m, w, g, wl.alpha, prec, wl.eta2, window=w_)
    phi = _solve(G, wl.dens)
    G.close()
    e = rel_l2(phi, ref)
    log(f"  rel-L2 vs definition {e:.3e}")
    assert e <= tol
