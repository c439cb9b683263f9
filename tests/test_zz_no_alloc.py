"""The evaluation that allocates nothing (slp_eval_single_layer_static, all
work buffers in the library's static device workspace) against the ordinary
evaluation of the same context (slp_eval_single_layer), through the C ABI.

Two calls in a row, the second with a smaller input (the workspace keeps the
first call's contents), in FP64 and FP32, with and without the near-field
correction; each result must equal the ordinary evaluation's to the rounding
of the gridding's block accumulation (the same kernels on the same inputs:
rel-L2 <= 1e-14 in FP64, <= 1e-6 in FP32). An evaluation whose work buffers
exceed the workspace is refused with SLP_ENOMEM and leaves phi untouched."""
import numpy as np
import pytest

import paper_1305_3162_amd as slp
from synth.workloads import cube_random, sphere_random
from slp_testlib import make_geometry, rel_l2, log

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    slp.load_library()


def _pair(G, dens):
    """(ordinary, static) potentials of one density on context G."""
    d = torch.as_tensor(dens).cuda()
    n = G.info["n_targets"]
    ref = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
    out = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
    G.set_density(d)
    G.eval(ref)
    slp.eval_single_layer_static(G.handle, out)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


@pytest.mark.parametrize("prec,m,tol", [(slp.FP64, 8, 1e-14), (slp.FP32, 5, 1e-6)])
def test_static_equals_ordinary_twice(prec, m, tol):
    big = cube_random(24, 31, 64, m)          # first call: larger work buffers
    small = sphere_random(2, 32, 32, m)       # second call: smaller input
    for wl in (big, small):
        G = make_geometry(wl, m, prec)
        ref, out = _pair(G, wl.dens)
        e = rel_l2(out, ref)
        log(f"case {wl.name} m={m} {'fp64' if prec == slp.FP64 else 'fp32'}: "
            f"static vs ordinary rel-L2 {e:.3e}")
        assert np.all(np.isfinite(out))
        assert e <= tol
        G.close()


def test_static_with_near_field():
    wl = sphere_random(2, 33, 32, 4)
    G = make_geometry(wl, 4, slp.FP64)
    G.setup_near_field(G.near_radius(1e-3))
    ref, out = _pair(G, wl.dens)
    e = rel_l2(out, ref)
    log(f"case {wl.name} with the near field: static vs ordinary rel-L2 {e:.3e}")
    assert e <= 1e-14
    G.close()


def test_static_refuses_oversized():
    wl = cube_random(128, 34, 256, 8)
    G = make_geometry(wl, 8, slp.FP64)
    n = G.info["n_targets"]
    out = torch.full((n,), 7.0, dtype=torch.float64, device="cuda")
    G.set_density(torch.as_tensor(wl.dens).cuda())
    with pytest.raises(slp.SlpError) as ei:
        slp.eval_single_layer_static(G.handle, out)
    log(f"case {wl.name}: refused ({ei.value})")
    assert ei.value.code == -2 and "workspace" in str(ei.value)
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)
    G.close()
