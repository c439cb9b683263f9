"""Write tests/golden/film512_phi_sample.npz: the smooth-part potential of the
thin-film workload (1 x 1 x 0.02, 1,089,536 triangles, 544,770 nodes, seed 3,
grid 1024 x 1024 x 64) at 10,000 nodes drawn without replacement (seed 3003),
computed by the oracle's NDFT route of the definition (eq. smooth_phi; no
window, no FFT). Calls only `oracle` and `synth`. About 1e14 flops of host
BLAS: tens of minutes on a few cores.

Usage: python tests/golden/make_film512_golden.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import direct            # noqa: E402
from synth.workloads import make_workload   # noqa: E402

OUT = os.path.join(HERE, "film512_phi_sample.npz")


def main():
    t0 = time.time()
    wl = make_workload("film512")
    p = direct.prepare_workload(wl)
    rng = np.random.default_rng(3003)
    idx = np.sort(rng.choice(wl.n_nodes, size=10000, replace=False))
    print(f"prepared: S'={p.omega.size} n={p.n} s={p.s} ({time.time() - t0:.1f} s)", flush=True)
    b = direct.ndft_b(p)
    print(f"b done ({time.time() - t0:.1f} s)", flush=True)
    phi = direct.phi_ndft(p, idx, b=b)
    np.savez_compressed(OUT, idx=idx, phi=phi, terms=p.omega.size, n=p.n, s=p.s, c=p.c)
    print(f"wrote {OUT} ({time.time() - t0:.1f} s)", flush=True)


if __name__ == "__main__":
    main()
