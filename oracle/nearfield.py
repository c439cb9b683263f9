"""Near-field correction of the single-layer potential (Sec. 3.4) and the exact
surface integrals it is built from.

Test infrastructure only (see oracle/__init__.py).

The kernel is split as 1/r = N_NF(r) + N_s(r) with N_NF = 1/r - N_s (eq.
splitting1), N_s the truncated exponential sum of Sec. 3.3. The smooth part is
the NUFFT sum (R1 in `direct`); the near field adds, for every target x_i and
every triangle S_j no further than eps from it (index set of eq. nf_index),

  C_ij  = int_{S_j} dsigma(y) / |x_i - y|  -  (|S_j| / 3) sum_s N_s(|x_i - y_{j,s}|)
  phi_NF(x_i) = 1/(4 pi) sum_{j in I_eps(x_i)} gbar_j C_ij               (eq. nfcorr)

with y_{j,s} the three quadrature points of S_j and gbar_j the mean of the
three density values of S_j (the element-constant g_j of Sec. 2 when the
density comes from the P1 ansatz). The second term of C_ij takes the smooth
kernel with the same three-point rule the gridding uses, so that on near
pairs the Fourier-series contribution of the smooth part is replaced by the
exact integral of 1/r (up to the Fourier error N_s - K_F of eq. splitting2).

  phi_complete = phi_s (R1, pair sum with K_F) + phi_NF          (Alg. 1, last steps)

The integrals of 1/r over a flat triangle are evaluated by decomposing the
triangle into three signed sub-triangles with apex at the foot point p of x
in the triangle's plane; in each sub-triangle the radial integral in polar
coordinates about p is done in closed form and the remaining integral along
the opposite edge numerically (composite Gauss-Legendre after the substitution
s = t sinh(u)). The paper's own treatment of the singular case (x a vertex of
S_j: Duffy substitution, tensor Gauss rule) is `vertex_potential_duffy`, used
as an independent pin.
"""
from __future__ import annotations

import numpy as np

from . import direct, geometry

FOUR_PI = 4.0 * np.pi

_GL_X, _GL_W = np.polynomial.legendre.leggauss(16)


def _unit_normals(a, b, c):
    n = np.cross(b - a, c - a)
    return n / np.linalg.norm(n, axis=-1, keepdims=True)


def _edge_integral(t, su, sv, d):
    """J = int_{su}^{sv} t ds / (sqrt(s^2 + t^2 + d^2) + |d|) for t > 0.

    This is the area integral of 1/sqrt(|y-p|^2 + d^2) over the triangle with
    apex p, whose opposite edge lies on a line at distance t from p, with
    along-edge coordinates su < sv measured from the foot of p on that line:
    in polar coordinates about p the radial integral of rho/sqrt(rho^2+d^2) up
    to the edge is sqrt(R^2 + d^2) - |d|, and with s = t tan(angle) the angular
    integral becomes the one above. s = t sinh(u) moves every singularity of
    the integrand to distance pi/2 from the real u axis; panels of width <= 1
    with 16 Gauss points then converge to rounding. Vectorised over arrays."""
    t = np.asarray(t, dtype=np.float64)
    ad = np.abs(np.asarray(d, dtype=np.float64))
    ua = np.arcsinh(su / t)
    ub = np.arcsinh(sv / t)
    span = ub - ua
    panels = np.maximum(1, np.ceil(span / 1.0)).astype(np.int64)
    out = np.zeros_like(t)
    for p in np.unique(panels):
        sel = panels == p
        a, b = ua[sel], ub[sel]
        tt, dd = t[sel], ad[sel]
        h = (b - a) / p
        acc = np.zeros_like(a)
        for k in range(int(p)):
            lo = a + k * h
            u = lo[:, None] + 0.5 * h[:, None] * (_GL_X[None, :] + 1.0)
            ch = np.cosh(u)
            s = tt[:, None] * np.sinh(u)
            f = tt[:, None] ** 2 * ch / (np.sqrt(s * s + tt[:, None] ** 2 + dd[:, None] ** 2)
                                        + dd[:, None])
            acc += 0.5 * h * (f @ _GL_W)
        out[sel] = acc
    return out


def triangle_potential(x, a, b, c):
    """int_T dsigma(y) / |x - y| over the flat triangle T = (a, b, c).

    Arrays broadcast: x [..., 3], a/b/c [..., 3]. The integral is split into the
    three signed sub-triangles (p, u, v) over the edges (u, v) of T, p the foot
    point of x in the plane of T; each contributes sign * J (see
    `_edge_integral`), the sign being + when p lies on the interior side of the
    edge. Sub-triangles of zero area (p on an edge line) contribute nothing."""
    x, a, b, c = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64) for v in (x, a, b, c)))
    shape = x.shape[:-1]
    x, a, b, c = (v.reshape(-1, 3) for v in (x, a, b, c))
    nrm = _unit_normals(a, b, c)
    d = np.einsum("ij,ij->i", x - a, nrm)
    p = x - d[:, None] * nrm
    scale = np.maximum.reduce([np.linalg.norm(b - a, axis=1), np.linalg.norm(c - b, axis=1),
                               np.linalg.norm(a - c, axis=1)])
    total = np.zeros(x.shape[0])
    for u, v in ((a, b), (b, c), (c, a)):
        el = np.linalg.norm(v - u, axis=1)
        e = (v - u) / el[:, None]
        out = np.cross(e, nrm)                       # in-plane, away from the interior
        t = np.einsum("ij,ij->i", u - p, out)        # > 0: p on the interior side
        su = np.einsum("ij,ij->i", u - p, e)
        sv = np.einsum("ij,ij->i", v - p, e)
        ok = np.abs(t) > 1e-14 * scale
        if np.any(ok):
            J = _edge_integral(np.abs(t[ok]), su[ok], sv[ok], d[ok])
            total[ok] += np.sign(t[ok]) * J
    return total.reshape(shape)


def vertex_potential_duffy(apex, p1, p2, order=24):
    """int_T dsigma(y) / |apex - y| for T = (apex, p1, p2), by the paper's
    treatment of the weakly singular case (Sec. 3.4): parametrise T from the
    singular vertex, y = apex + s (p1 - apex) + t (p2 - p1) on the unit triangle
    0 <= t <= s <= 1, substitute t = s t' (Jacobian s), and integrate the
    now regular integrand over the unit square with a tensor Gauss rule.
    Here the s-integrand is constant, so the rule reduces to t'."""
    apex, p1, p2 = (np.asarray(v, dtype=np.float64) for v in (apex, p1, p2))
    xg, wg = np.polynomial.legendre.leggauss(order)
    tp = 0.5 * (xg + 1.0)
    two_area = np.linalg.norm(np.cross(p1 - apex, p2 - apex))
    acc = 0.0
    sg = 0.5 * (xg + 1.0)
    for si, ws in zip(sg, 0.5 * wg):
        # y - apex = s * (e1 + t' e2); |.| = s |e1 + t' e2|; Jacobian 2|T| s
        e = (p1 - apex)[None, :] + tp[:, None] * (p2 - p1)[None, :]
        f = two_area * si / (si * np.linalg.norm(e, axis=1))
        acc += ws * (0.5 * wg) @ f
    return acc


def point_triangle_distance(x, a, b, c):
    """d(x, T) = min over y in T of |x - y| (eq. nf_index): the distance to the
    foot point when it lies inside T, else the distance to the nearest edge
    segment. Broadcasting as in `triangle_potential`."""
    x, a, b, c = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64) for v in (x, a, b, c)))
    nrm = _unit_normals(a, b, c)
    d = np.einsum("...j,...j->...", x - a, nrm)
    p = x - d[..., None] * nrm
    inside = np.ones(d.shape, dtype=bool)
    seg = np.full(d.shape, np.inf)
    for u, v in ((a, b), (b, c), (c, a)):
        e = v - u
        inside &= np.einsum("...j,...j->...", np.cross(e, p - u), nrm) >= 0.0
        tt = np.clip(np.einsum("...j,...j->...", x - u, e) / np.einsum("...j,...j->...", e, e),
                     0.0, 1.0)
        q = u + tt[..., None] * e
        seg = np.minimum(seg, np.linalg.norm(x - q, axis=-1))
    return np.where(inside, np.abs(d), seg)


def near_pairs(nodes, tris, targets, eps):
    """Index sets of eq. (nf_index) for every target, by brute force over all
    triangles: returns (rowptr [P+1], cols, dist) with the triangles of each
    row in increasing order and their distances."""
    nodes = np.asarray(nodes, dtype=np.float64)
    targets = np.asarray(targets, dtype=np.float64)
    A, B, Cc = nodes[tris[:, 0]], nodes[tris[:, 1]], nodes[tris[:, 2]]
    rowptr = [0]
    cols, dist = [], []
    for x in targets:
        dd = point_triangle_distance(x[None, :], A, B, Cc)
        j = np.nonzero(dd <= eps)[0]
        cols.append(j)
        dist.append(dd[j])
        rowptr.append(rowptr[-1] + j.size)
    return (np.asarray(rowptr, dtype=np.int64),
            np.concatenate(cols).astype(np.int64) if cols else np.zeros(0, np.int64),
            np.concatenate(dist) if dist else np.zeros(0))


def smooth_kernel(prob, r):
    """N_s(r) = sum_t omega_t exp(-gamma_t r^2) over the kept terms (eq. expsum,
    physical units)."""
    r = np.asarray(r, dtype=np.float64)
    return np.exp(-np.multiply.outer(r * r, prob.gamma)) @ prob.omega


def near_values(prob, nodes, tris, targets, rowptr, cols):
    """C_ij for the pairs of a CSR pattern (rows = targets, cols = triangles)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    targets = np.asarray(targets, dtype=np.float64)
    M = tris.shape[0]
    area, _ = geometry.triangle_areas_normals(nodes, tris)
    rows = np.repeat(np.arange(len(rowptr) - 1), np.diff(rowptr))
    x = targets[rows]
    j = np.asarray(cols, dtype=np.int64)
    exact = triangle_potential(x, nodes[tris[j, 0]], nodes[tris[j, 1]], nodes[tris[j, 2]])
    smooth = np.zeros(j.size)
    for s in range(3):
        r = np.linalg.norm(x - prob.y[j + s * M], axis=1)
        smooth += smooth_kernel(prob, r)
    return exact - area[j] / 3.0 * smooth


def element_mean_density(prob, n_tris):
    """gbar_j = (g_{j,0} + g_{j,1} + g_{j,2}) / 3 for the long index k = j + s M."""
    return prob.g.reshape(3, n_tris).mean(axis=0)


def phi_near(prob, nodes, tris, eps, targets=None, pattern=None):
    """phi_NF at the targets (the nodes unless given): eq. (nfcorr) over the
    index sets of eq. (nf_index), divided by 4 pi. Returns (phi, rowptr, cols,
    vals)."""
    tg = nodes if targets is None else targets
    if pattern is None:
        rowptr, cols, _ = near_pairs(nodes, tris, tg, eps)
    else:
        rowptr, cols = pattern
    vals = near_values(prob, nodes, tris, tg, rowptr, cols)
    gbar = element_mean_density(prob, tris.shape[0])
    rows = np.repeat(np.arange(len(rowptr) - 1), np.diff(rowptr))
    phi = np.bincount(rows, weights=vals * gbar[cols], minlength=len(rowptr) - 1) / FOUR_PI
    return phi, rowptr, cols, vals


def phi_complete(prob, nodes, tris, eps, targets=None):
    """phi_s + phi_NF (Alg. 1): the NUFFT sum R1 plus the near-field correction."""
    far = direct.phi_pairs(prob)
    near, *_ = phi_near(prob, nodes, tris, eps, targets)
    return far + near


def phi_exact_integrals(nodes, tris, gbar, targets, block=64):
    """1/(4 pi) sum_j gbar_j int_{S_j} dsigma / |x - y|: the single layer
    potential of an element-constant density with the exact kernel and exact
    integrals (eq. slayer3), dense over all pairs."""
    nodes = np.asarray(nodes, dtype=np.float64)
    targets = np.asarray(targets, dtype=np.float64)
    A, B, Cc = nodes[tris[:, 0]], nodes[tris[:, 1]], nodes[tris[:, 2]]
    out = np.empty(targets.shape[0])
    for i0 in range(0, targets.shape[0], block):
        xs = targets[i0:i0 + block]
        I = triangle_potential(xs[:, None, :], A[None], B[None], Cc[None])
        out[i0:i0 + block] = I @ gbar / FOUR_PI
    return out


def near_radius(prob, tol, r_max, ratio=0.999):
    """Smallest eps on the geometric scan r_k = r_max ratio^k such that the
    kept exponential sum matches the Newton kernel to |N_s(r) - 1/r| <= tol / r
    at every scan point from eps up to r_max (Sec. 3.3: the truncated sum is
    accurate on [eps, 1/2] only)."""
    r = r_max
    last_ok = None
    while r > 1e-6 * r_max:
        if abs(smooth_kernel(prob, np.array([r]))[0] * r - 1.0) <= tol:
            last_ok = r
        else:
            break
        r *= ratio
    return last_ok
