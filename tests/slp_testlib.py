"""Helpers shared by the GPU tests: run the HIP path through the binding and
prepare the matching oracle problem from the same seeded workload."""
import sys
import time

import numpy as np

import paper_1305_3162_amd as slp
from oracle import direct


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def es_for(wl):
    return slp.expsum_sinc(wl.es_h, wl.es_r_lo, wl.es_r_hi, wl.es_tol)


def make_geometry(wl, m=None, precision=slp.FP64, grid=None):
    import torch  # noqa: F401
    w, g = es_for(wl)
    return slp.Geometry(wl.nodes, wl.tris, grid or wl.grid, m if m is not None else wl.m, w, g,
                        wl.alpha, precision, wl.eta2)


def gpu_phi(wl, m=None, precision=slp.FP64, dens=None, geom=None):
    """phi_s at the nodes computed by libslp (float64 numpy array)."""
    import torch
    own = geom is None
    if own:
        geom = make_geometry(wl, m, precision)
    d = torch.as_tensor(wl.dens if dens is None else dens, dtype=torch.float64).cuda()
    phi = geom.solve(d)
    torch.cuda.synchronize()
    out = phi.cpu().numpy()
    if own:
        geom.close()
    return out


def oracle_problem(wl):
    return direct.prepare_workload(wl)


class Timer:
    def __enter__(self):
        self.t = time.perf_counter()
        return self

    def __exit__(self, *a):
        self.dt = time.perf_counter() - self.t
