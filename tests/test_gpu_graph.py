"""Evaluations replayed through captured HIP graphs give the results of direct
launches: several replays in a row with different densities and outputs, eager
work queued between replays, batched replays, a capture dropped and redone when
the batch capacity grows, and direct launches again after switching off."""
import numpy as np
import pytest

import paper_1305_3162_amd as slp
from synth.workloads import sphere_random, cube_random
from slp_testlib import es_for, log, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("kind,m,prec,window", [("sphere", 6, slp.FP64, slp.WINDOW_GAUSS),
                                                ("cube", 3, slp.FP32, slp.WINDOW_KB)])
def test_graph_replays_equal_direct_launches(kind, m, prec, window):
    wl = sphere_random(3, 41, 64, m) if kind == "sphere" else cube_random(16, 42, 64, m)
    log(f"case graph {kind} m={m} prec={prec} window={window}")
    w, g = es_for(wl)
    G = slp.Geometry(wl.nodes, wl.tris, wl.grid, m, w, g, 2, prec, wl.eta2, window=window)
    rng = np.random.default_rng(43)
    dens = [torch.as_tensor(rng.normal(size=wl.n_src)).cuda() for _ in range(5)]
    ref = [G.solve(d) for d in dens]
    torch.cuda.synchronize()
    tol = 1e-14 if prec == slp.FP64 else 1e-6
    stream = torch.cuda.current_stream()
    slp.set_graph(G.handle, True)
    outs = []
    for k, d in enumerate(dens):
        d2 = d * 2.0                                   # eager work between replays
        phi = torch.full((wl.n_nodes,), float("nan"), dtype=torch.float64, device="cuda")
        G.set_density(d2 if k % 2 else d, stream)
        G.eval(phi, stream)
        outs.append(phi)
    torch.cuda.synchronize()
    for k, phi in enumerate(outs):
        want = ref[k] * (2.0 if k % 2 else 1.0)
        assert rel_l2(phi.cpu().numpy(), want.cpu().numpy()) <= tol, k
    # batched replays on the same geometry, then a larger batch (capacity grows,
    # the capture is redone)
    for nb in (3, 5, 3):
        phis = [torch.full((wl.n_nodes,), float("nan"), dtype=torch.float64, device="cuda")
                for _ in range(nb)]
        slp.eval_batched([G.handle] * nb, dens[:nb], phis, stream)
        torch.cuda.synchronize()
        for k in range(nb):
            assert rel_l2(phis[k].cpu().numpy(), ref[k].cpu().numpy()) <= tol, (nb, k)
    slp.set_graph(G.handle, False)
    phi = G.solve(dens[4])
    torch.cuda.synchronize()
    assert rel_l2(phi.cpu().numpy(), ref[4].cpu().numpy()) <= tol
    G.close()
