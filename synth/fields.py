"""Seeded magnetisation fields m(x) (unit vectors)."""
from __future__ import annotations

import numpy as np


def uniform_magnetisation(direction=(0.0, 0.0, 1.0)):
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)

    def m(x):
        x = np.asarray(x, dtype=np.float64)
        return np.broadcast_to(d, x.shape).copy()

    return m


class RandomSmoothMagnetisation:
    """Unit-normalised sum of four random Fourier modes.

    v(x) = sum_j a_j cos(2 pi k_j . xh + theta_j), m = v/|v|, where xh maps the
    body's bounding box onto [0, 1]^3, k_j has integer components in -3..3 with
    1 <= max|k_j| <= 3, a_j ~ N(0, I_3) and theta_j ~ U[0, 2 pi). Drawn from
    numpy's PCG64 generator seeded with `seed`. Where |v| < 1e-12 the field
    falls back to (0, 0, 1).
    """

    def __init__(self, seed: int, bbox_min, bbox_max, modes: int = 4, kmax: int = 3):
        rng = np.random.default_rng(int(seed))
        ks = []
        while len(ks) < modes:
            k = rng.integers(-kmax, kmax + 1, size=3)
            if 1 <= np.max(np.abs(k)) <= kmax:
                ks.append(k)
        self.k = np.array(ks, dtype=np.float64)
        self.a = rng.standard_normal((modes, 3))
        self.theta = rng.uniform(0.0, 2.0 * np.pi, size=modes)
        self.lo = np.asarray(bbox_min, dtype=np.float64)
        ext = np.asarray(bbox_max, dtype=np.float64) - self.lo
        self.ext = np.where(ext > 0, ext, 1.0)

    def __call__(self, x):
        x = np.asarray(x, dtype=np.float64)
        xh = (x - self.lo) / self.ext
        ph = 2.0 * np.pi * (xh @ self.k.T) + self.theta      # [P, modes]
        v = np.cos(ph) @ self.a                              # [P, 3]
        nv = np.linalg.norm(v, axis=-1, keepdims=True)
        out = np.where(nv < 1e-12, np.array([0.0, 0.0, 1.0]), v / np.where(nv < 1e-12, 1.0, nv))
        return out
