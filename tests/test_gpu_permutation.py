"""Invariance of the result under a reordering of the input at full size: the
thin film (1,089,536 triangles, 544,770 nodes, grid 1024 x 1024 x 64) with its
triangles shuffled (the density follows its triangles: value s of triangle j
sits at j + s M) and its nodes renumbered (the triangles' vertex indices
follow, the potential comes back in the new node order). The binning sorts
sources and targets afresh, so every gridding segment, run and tile sees the
same points in another order: the potential must agree to rounding (FP64
rel-L2 <= 1e-13, FP32 <= 1e-6), in both windows."""
import numpy as np
import pytest

import paper_1305_3162_amd as slp
from synth.workloads import make_workload
from slp_testlib import es_for, log, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def film():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return make_workload("film512")


def _phi(wl, nodes, tris, dens, prec, window, m):
    w, g = es_for(wl)
    G = slp.Geometry(nodes, tris, wl.grid, m, w, g, wl.alpha, prec, wl.eta2, window=window)
    out = G.solve(torch.as_tensor(dens, device="cuda")).cpu().numpy()
    G.close()
    return out


@pytest.mark.parametrize("prec,window,m,tol", [(slp.FP64, slp.WINDOW_KB, 4, 1e-13),
                                               (slp.FP32, slp.WINDOW_KB, 3, 1e-6),
                                               (slp.FP32, slp.WINDOW_GAUSS, 5, 1e-6)])
def test_film_invariant_under_reordering(film, prec, window, m, tol):
    wl = film
    M, N = wl.tris.shape[0], wl.n_nodes
    rng = np.random.default_rng(77)
    tperm = rng.permutation(M)              # new triangle j came from tperm[j]
    nperm = rng.permutation(N)              # new node i is old node nperm[i]
    inv = np.empty(N, dtype=np.int64)
    inv[nperm] = np.arange(N)
    tris2 = inv[wl.tris[tperm]].astype(np.int32)
    nodes2 = wl.nodes[nperm]
    d = wl.dens.reshape(3, M)[:, tperm].reshape(-1)
    log(f"case film512 reordered, prec={'fp64' if prec == slp.FP64 else 'fp32'} "
        f"window={'kb' if window == slp.WINDOW_KB else 'gauss'} m={m}")
    ref = _phi(wl, wl.nodes, wl.tris, wl.dens, prec, window, m)
    got = _phi(wl, nodes2, tris2, d, prec, window, m)
    e = rel_l2(got, ref[nperm])
    log(f"  rel-L2 between the orderings {e:.3e}")
    assert e <= tol
