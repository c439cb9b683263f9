"""The FFT passes on long lines, against the oracle's CPU NUFFT (R3, same m).

The grids of the other parity tests have at most 128 points per axis; the
thin film has 1024 along x and y. Here a slender box (extent ratio equal to
the grid ratio, so that the body spans 0.4 of every axis) puts 1024 or 2048
points on one axis and 64 on the others, for each axis in turn, so that every
pass (x contiguous, y and z strided, the fused z pass) runs at those lengths;
and a plate shaped like the film (1 x 1 x 0.02, coarse cells) runs on the
film's own 1024 x 1024 x 64 grid. Checked: the grid after the inverse FFT
(region cells) and the potential, FP64 to rounding (1e-11 / 1e-10), FP32 to
its rounding (2e-5)."""
import numpy as np
import pytest

import paper_1305_3162_amd as slp
from oracle import direct, nufft
from synth import RandomSmoothMagnetisation, density_from_magnetisation
from synth.meshes import box_surface
from synth.workloads import _finish
from slp_testlib import make_geometry, rel_l2, log

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    slp.load_library()


def _workload(extent, cells, grid, m, seed):
    nodes, tris = box_surface(extent, cells)
    mf = RandomSmoothMagnetisation(seed, nodes.min(0), nodes.max(0))
    return _finish("box", nodes, tris, density_from_magnetisation(nodes, tris, mf), grid, m)


def _region_map(info, grid):
    lo, ext = info["lo"], info["extent"]
    return [np.mod(np.arange(lo[q], lo[q] + ext[q]) - grid[q] // 2, grid[q]) for q in range(3)]


def _check(wl, m, prec):
    p = direct.prepare_workload(wl)
    phi3, st = nufft.phi_nufft(p, m, stages=True)
    G = make_geometry(wl, m, prec)
    info = G.info
    phi = G.solve(torch.as_tensor(wl.dens).cuda())
    ext = info["extent"]
    dt = torch.float64 if prec == slp.FP64 else torch.float32
    g_gpu = torch.empty(ext[2] * ext[1] * ext[0], dtype=dt, device="cuda")
    slp.debug_copy(G.handle, 1, g_gpu)
    torch.cuda.synchronize()
    g_gpu = g_gpu.double().cpu().numpy().reshape(ext[2], ext[1], ext[0])
    b = info["window_b"]
    ix, iy, iz = _region_map(info, wl.grid)
    g_ref = np.real(st["g"])[np.ix_(ix, iy, iz)].transpose(2, 1, 0) * (np.pi * b) ** -1.5 / (4 * np.pi)
    eg = np.abs(g_gpu - g_ref).max() / np.abs(g_ref).max()
    e3 = rel_l2(phi.cpu().numpy(), phi3)
    G.close()
    log(f"  grid after the inverse FFT: max-norm rel {eg:.3e}; phi vs R3 {e3:.3e}")
    if prec == slp.FP64:
        assert eg <= 1e-11
        assert e3 <= 1e-10
    else:
        assert eg <= 2e-5
        assert e3 <= 2e-5


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("N", [1024, 2048])
@pytest.mark.parametrize("prec", [slp.FP64, slp.FP32])
def test_long_axis(axis, N, prec):
    grid = [64, 64, 64]
    grid[axis] = N
    extent = [1.0, 1.0, 1.0]
    extent[axis] = N / 64
    cells = [4, 4, 4]
    cells[axis] = N // 16
    log(f"case slender box along axis {axis}, grid {tuple(grid)}, "
        f"{'fp64' if prec == slp.FP64 else 'fp32'}, m=3")
    _check(_workload(extent, cells, tuple(grid), 3, 20 + axis), 3, prec)


@pytest.mark.parametrize("prec", [slp.FP64, slp.FP32])
def test_film_shaped_plate(prec):
    log(f"case plate 1 x 1 x 0.02 (64 x 64 x 2 cells), grid 1024 x 1024 x 64, "
        f"{'fp64' if prec == slp.FP64 else 'fp32'}, m=3")
    _check(_workload((1.0, 1.0, 0.02), (64, 64, 2), (1024, 1024, 64), 3, 11), 3, prec)
