"""The request server on the GPU: every result is the same alone and in the mix
(within rounding: the gridding's LDS accumulation order may differ), under
memory pressure (evictions and rebuilds) and with an oversized geometry; a
burst of requests for one geometry is served by a few batched launches."""
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


def _mix():
    return [
        (sphere_random(2, 11, 64, 5), slp.FP64),
        (sphere_random(3, 12, 64, 6), slp.FP64),
        (cube_random(16, 13, 64, 4), slp.FP32),
        (cube_random(32, 14, 128, 5), slp.FP32),
        (sphere_random(4, 15, 128, 4), slp.FP32),
    ]


def _tol(prec):
    return 1e-13 if prec == slp.FP64 else 1e-5


def _solo(wl, prec, dens):
    w, g = es_for(wl)
    G = slp.Geometry(wl.nodes, wl.tris, wl.grid, wl.m, w, g, wl.alpha, prec, wl.eta2)
    out = G.solve(dens)
    torch.cuda.synchronize()
    G.close()
    return out


def test_device_bytes_estimate_matches_setup():
    for wl, prec in _mix()[:3]:
        w, g = es_for(wl)
        est = slp.geometry_device_bytes(wl.nodes, wl.tris, wl.grid, wl.m, w, g, wl.alpha, prec)
        G = slp.Geometry(wl.nodes, wl.tris, wl.grid, wl.m, w, g, wl.alpha, prec, wl.eta2)
        assert G.info["device_bytes"] == est
        G.close()


@pytest.mark.parametrize("budget_mb,slots", [(4096, 4), (16, 2)])
def test_results_same_alone_and_in_mix(budget_mb, slots):
    log(f"case server budget={budget_mb}MB slots={slots}")
    mix = _mix()
    rng = np.random.default_rng(7)
    srv = slp.Server(budget_mb << 20, slots)
    ids = []
    for wl, prec in mix:
        w, g = es_for(wl)
        ids.append(srv.add_geometry(wl.nodes, wl.tris, wl.grid, wl.m, w, g, wl.alpha, prec,
                                    wl.eta2))
    reqs = []
    for k in range(40):
        gi = int(rng.integers(len(mix)))
        wl, prec = mix[gi]
        dens = torch.as_tensor(rng.normal(size=wl.n_src), device="cuda")
        phi = torch.empty(wl.n_nodes, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()                    # inputs ready before the server's streams
        reqs.append((gi, dens, phi, srv.submit(ids[gi], dens, phi)))
    for gi, dens, phi, tk in reqs:
        srv.wait(tk, 60.0)
    st = srv.stats()
    log(f"  stats {st}")
    assert st["completed"] == 40 and st["failed"] == 0
    assert 0 < st["p50_s"] <= st["p99_s"]
    assert st["resident_bytes"] <= budget_mb << 20
    if budget_mb < 100:
        assert st["evictions"] > 0
    for gi, dens, phi, tk in reqs:
        wl, prec = mix[gi]
        ref = _solo(wl, prec, dens)
        assert rel_l2(phi.cpu().numpy(), ref.cpu().numpy()) <= _tol(prec)
    srv.close()


def test_oversized_geometry_fails_cleanly():
    wl = cube_random(32, 3, 128, 5)
    w, g = es_for(wl)
    srv = slp.Server(1 << 20, 2)                    # 1 MiB: far too small
    gid = srv.add_geometry(wl.nodes, wl.tris, wl.grid, wl.m, w, g, 2, slp.FP32)
    small = sphere_random(1, 2, 32, 3)
    ws, gs = es_for(small)
    sid = srv.add_geometry(small.nodes, small.tris, small.grid, small.m, ws, gs, 2, slp.FP64)
    dens = torch.zeros(wl.n_src, dtype=torch.float64, device="cuda")
    phi = torch.zeros(wl.n_nodes, dtype=torch.float64, device="cuda")
    d2 = torch.as_tensor(small.dens, device="cuda")
    p2 = torch.empty(small.n_nodes, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t1 = srv.submit(gid, dens, phi)
    t2 = srv.submit(sid, d2, p2)
    with pytest.raises(slp.SlpError) as ei:
        srv.wait(t1, 30.0)
    assert ei.value.code == -2
    srv.wait(t2, 30.0)
    assert rel_l2(p2.cpu().numpy(), _solo(small, slp.FP64, d2).cpu().numpy()) <= 1e-13
    st = srv.stats()
    assert st["failed"] == 1 and st["completed"] == 1
    srv.close()


def test_near_field_served_and_estimated():
    """A geometry registered with a near field: the served result equals a
    context with the same near field, and the memory estimate used for
    admission equals what the context holds (both precisions, plain and packed
    layouts)."""
    cases = [(sphere_random(3, 16, 64, 6), slp.FP64, 1e-2),
             (cube_random(64, 17, 128, 5), slp.FP32, 1e-3)]
    srv = slp.Server(4096 << 20, 2)
    rng = np.random.default_rng(8)
    for wl, prec, tol in cases:
        log(f"case served near field {wl.name} prec={prec} tol={tol}")
        w, g = es_for(wl)
        G = slp.Geometry(wl.nodes, wl.tris, wl.grid, wl.m, w, g, wl.alpha, prec, wl.eta2)
        eps = G.near_radius(tol)
        G.setup_near_field(eps)
        est = (slp.geometry_device_bytes(wl.nodes, wl.tris, wl.grid, wl.m, w, g, wl.alpha, prec)
               + slp.near_field_device_bytes(wl.nodes, wl.tris, eps, prec))
        assert G.info["device_bytes"] == est, (G.info["device_bytes"], est)
        dens = torch.as_tensor(rng.normal(size=wl.n_src)).cuda()
        want = G.solve(dens)
        torch.cuda.synchronize()
        G.close()
        gid = srv.add_geometry(wl.nodes, wl.tris, wl.grid, wl.m, w, g, wl.alpha, prec, wl.eta2,
                               near_eps=eps)
        phi = torch.full((wl.n_nodes,), float("nan"), dtype=torch.float64, device="cuda")
        srv.wait(srv.submit(gid, dens, phi), 60.0)
        assert rel_l2(phi.cpu().numpy(), want.cpu().numpy()) <= _tol(prec)
    srv.close()


def test_burst_is_served_by_batched_launches():
    """16 requests for one geometry submitted while it is being set up: the
    pending ones are coalesced (up to 8 per launch), so far fewer than 16
    launches serve them, and every result equals its solo evaluation."""
    wl = sphere_random(3, 18, 64, 5)
    w, g = es_for(wl)
    rng = np.random.default_rng(9)
    srv = slp.Server(1 << 30, 2)
    gid = srv.add_geometry(wl.nodes, wl.tris, wl.grid, wl.m, w, g, wl.alpha, slp.FP64, wl.eta2)
    dens = [torch.as_tensor(rng.normal(size=wl.n_src), device="cuda") for _ in range(16)]
    phis = [torch.full((wl.n_nodes,), float("nan"), dtype=torch.float64, device="cuda")
            for _ in range(16)]
    torch.cuda.synchronize()
    tks = [srv.submit(gid, d, p) for d, p in zip(dens, phis)]
    for tk in tks:
        srv.wait(tk, 60.0)
    st = srv.stats()
    log(f"case burst of 16: launches {st['launches']}, p50 {st['p50_s'] * 1e3:.3f} ms")
    assert st["completed"] == 16 and st["failed"] == 0
    assert st["launches"] <= 8
    for d, p in zip(dens, phis):
        assert rel_l2(p.cpu().numpy(), _solo(wl, slp.FP64, d).cpu().numpy()) <= _tol(slp.FP64)
    srv.close()
