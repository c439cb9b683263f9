"""The potential at every node of a volume mesh (the paper evaluates phi at all
tetrahedral nodes, Sec. 2 and Tables 3-4): the structured tetrahedral mesh of
the unit cube, whose boundary is the cube's surface triangulation. Parity with
the definition (NDFT route at the same points) within the stated tolerances,
and on the boundary points the same values as the boundary-node evaluation."""
import numpy as np
import pytest

import paper_1305_3162_amd as slp
from oracle import direct
from synth import cube, cube_volume_nodes, RandomSmoothMagnetisation, density_from_magnetisation
from synth.workloads import expsum_interval
from slp_testlib import log, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cube16():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    nodes, tris = cube(16)
    mf = RandomSmoothMagnetisation(23, nodes.min(0), nodes.max(0))
    dens = density_from_magnetisation(nodes, tris, mf)
    tg = cube_volume_nodes(16)
    r_lo, r_hi = expsum_interval(nodes)
    grid = (64, 64, 64)
    p = direct.prepare(nodes, tris, dens, grid, es_r_lo=r_lo, es_r_hi=r_hi, targets=tg)
    return nodes, tris, dens, tg, grid, (r_lo, r_hi), direct.phi_ndft(p)


@pytest.mark.parametrize("m,prec,window,tol", [(8, slp.FP64, slp.WINDOW_GAUSS, 1e-6),
                                               (4, slp.FP64, slp.WINDOW_KB, 1e-6),
                                               (5, slp.FP32, slp.WINDOW_GAUSS, 1e-4),
                                               (3, slp.FP32, slp.WINDOW_KB, 1e-4)])
def test_volume_nodes_against_definition(cube16, m, prec, window, tol):
    nodes, tris, dens, tg, grid, (r_lo, r_hi), ref = cube16
    log(f"case volume targets cube16 ({tg.shape[0]} points) m={m} prec={prec} window={window}")
    w, g = slp.expsum_sinc(0.2, r_lo, r_hi, 1e-12)
    G = slp.Geometry(nodes, tris, grid, m, w, g, 2, prec, window=window, targets=tg)
    assert G.info["n_targets"] == tg.shape[0] and G.info["n_nodes"] == nodes.shape[0]
    d = torch.as_tensor(dens).cuda()
    phi = G.solve(d)
    # the boundary-node context on the same mesh
    B = slp.Geometry(nodes, tris, grid, m, w, g, 2, prec, window=window)
    phib = B.solve(d)
    torch.cuda.synchronize()
    phi, phib = phi.cpu().numpy(), phib.cpu().numpy()
    G.close()
    B.close()
    e = rel_l2(phi, ref)
    log(f"  rel-L2 vs definition {e:.3e}")
    assert e <= tol
    # lattice points on the boundary are the surface nodes
    key = {tuple(np.round(x * 32).astype(int)): i for i, x in enumerate(nodes)}
    idx = [(i, key[tuple(np.round(x * 32).astype(int))]) for i, x in enumerate(tg)
           if tuple(np.round(x * 32).astype(int)) in key]
    assert len(idx) == nodes.shape[0]
    a = np.array([phi[i] for i, _ in idx])
    b = np.array([phib[j] for _, j in idx])
    assert rel_l2(a, b) <= (1e-13 if prec == slp.FP64 else 1e-6)
