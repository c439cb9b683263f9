"""P1 finite elements for the Dirichlet problem of phi_1 (Sec. 2, eq. GR1, and
Sec. 2.1 'FEM for the Dirichlet problem'), the normal derivative that enters
the surface density, and the complete scalar potential phi = phi_1 + phi_2 of
Alg. 1.

Test infrastructure only (see oracle/__init__.py).

  -Laplace phi_1 = -div m in Omega, phi_1 = 0 on the boundary        (eq. GR1)
  weak form: int grad phi_1 . grad v = int m . grad v for v in H^1_0    (eq. varu1)
  S(fn, fn) x(fn) = b(fn),  S_km = sum_T int_T grad eta_m . grad eta_k,
                            b_k  = sum_T int_T m . grad eta_k            (eq. poisson)
  g_j = mean of m.n over S_j - d phi_1 / dn on S_j                       (Sec. 2.2)
  phi = phi_1 + phi_2,  phi_2 = single-layer potential of g at every node  (Alg. 1)

m is the nodal P1 interpolant, so int_T m = |T| times the mean of its four
vertex values, and grad eta_k is constant on each tetrahedron. The free-node
system is solved with a sparse direct solver (the paper names LU as one
option).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import direct, geometry, nearfield


def tet_gradients(nodes, tets):
    """Volumes |T| [T] and the gradients of the four barycentric coordinates
    of every tetrahedron [T, 4, 3]: with the edge matrix J = [x1-x0, x2-x0,
    x3-x0] (as columns), lambda_a = (J^{-1} (x - x0))_a for a = 1..3, so their
    gradients are the rows of J^{-1}; lambda_0 = 1 - the others."""
    P = np.asarray(nodes, dtype=np.float64)[tets]
    J = np.transpose(P[:, 1:, :] - P[:, :1, :], (0, 2, 1))
    vol = np.linalg.det(J) / 6.0
    Jinv = np.linalg.inv(J)
    G = np.concatenate([-Jinv.sum(axis=1, keepdims=True), Jinv], axis=1)
    return np.abs(vol), G


def stiffness(nodes, tets):
    """S_km = sum_T |T| grad lambda_m . grad lambda_k (CSR, N x N)."""
    vol, G = tet_gradients(nodes, tets)
    K = vol[:, None, None] * np.einsum("tai,tbi->tab", G, G)
    rows = np.repeat(tets, 4, axis=1).ravel()
    cols = np.tile(tets, (1, 4)).ravel()
    N = np.asarray(nodes).shape[0]
    return sp.coo_matrix((K.ravel(), (rows, cols)), shape=(N, N)).tocsr()


def load(nodes, tets, m_nodes):
    """b_k = sum_T |T| mbar_T . grad lambda_k, mbar_T the vertex mean of m."""
    vol, G = tet_gradients(nodes, tets)
    mbar = np.asarray(m_nodes, dtype=np.float64)[tets].mean(axis=1)
    contrib = vol[:, None] * np.einsum("ti,tai->ta", mbar, G)
    return np.bincount(tets.ravel(), weights=contrib.ravel(), minlength=np.asarray(nodes).shape[0])


def boundary_faces(nodes, tets):
    """Faces that belong to exactly one tetrahedron, oriented so that the
    cross product of their edge vectors points away from the tetrahedron's
    fourth vertex (outward). Returns (tris int32 [Mb, 3], owner tet [Mb]),
    ordered by the sorted vertex triple."""
    nodes = np.asarray(nodes, dtype=np.float64)
    T = tets.shape[0]
    faces = np.concatenate([tets[:, [1, 2, 3]], tets[:, [0, 2, 3]], tets[:, [0, 1, 3]],
                            tets[:, [0, 1, 2]]])
    opposite = np.concatenate([tets[:, 0], tets[:, 1], tets[:, 2], tets[:, 3]])
    owner = np.tile(np.arange(T), 4)
    key = np.sort(faces, axis=1)
    _, inv, counts = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    once = counts[inv.ravel()] == 1
    f, opp, own, k = faces[once], opposite[once], owner[once], key[once]
    n = np.cross(nodes[f[:, 1]] - nodes[f[:, 0]], nodes[f[:, 2]] - nodes[f[:, 0]])
    inward = np.einsum("ij,ij->i", n, nodes[opp] - nodes[f[:, 0]]) > 0
    f[inward] = f[inward][:, [0, 2, 1]]
    order = np.lexsort((k[:, 2], k[:, 1], k[:, 0]))
    return f[order].astype(np.int32), own[order]


def boundary_nodes(tets, nodes):
    tris, _ = boundary_faces(nodes, tets)
    flag = np.zeros(np.asarray(nodes).shape[0], dtype=bool)
    flag[tris.ravel()] = True
    return flag


def solve_dirichlet(S, b, bnd, values, method="direct"):
    """S(fn, fn) x(fn) = b(fn) - (S x_bn)(fn) (eq. poisson), x = values on the
    boundary nodes. method "direct": sparse LU; "cg": conjugate gradients with
    the diagonal preconditioner to a relative residual of 1e-13 (for meshes
    where the factorisation is too slow)."""
    x = np.zeros(S.shape[0])
    x[bnd] = values
    fn = np.nonzero(~bnd)[0]
    A = S[fn][:, fn].tocsr()
    rhs = b[fn] - S[fn][:, np.nonzero(bnd)[0]] @ x[bnd]
    if method == "direct":
        x[fn] = spla.spsolve(A.tocsc(), rhs)
    else:
        Minv = sp.diags(1.0 / A.diagonal())
        sol, info = spla.cg(A, rhs, rtol=1e-13, atol=0.0, maxiter=100000, M=Minv)
        if info != 0:
            raise RuntimeError(f"conjugate gradients did not converge (info {info})")
        x[fn] = sol
    return x


def solve_phi1(nodes, tets, m_nodes, method="direct"):
    """phi_1 at every node (zero on the boundary), eq. GR1 by eq. poisson."""
    S = stiffness(nodes, tets)
    b = load(nodes, tets, m_nodes)
    bnd = boundary_nodes(tets, nodes)
    return solve_dirichlet(S, b, bnd, 0.0, method)


def dphi1_dn(nodes, tets, phi1, tris, owner):
    """d phi_1 / dn on every boundary triangle: the (constant) gradient of the
    P1 function phi_1 in the tetrahedron owning the face, dotted with the face's
    outward unit normal."""
    nodes = np.asarray(nodes, dtype=np.float64)
    _, G = tet_gradients(nodes, tets[owner])
    grad = np.einsum("ta,tai->ti", np.asarray(phi1)[tets[owner]], G)
    n = np.cross(nodes[tris[:, 1]] - nodes[tris[:, 0]], nodes[tris[:, 2]] - nodes[tris[:, 0]])
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    return np.einsum("ti,ti->t", grad, n)


def stray_field_energy(nodes, tets, m_nodes, phi):
    """E = -(1/2) int_Omega m . H = (1/2) int_Omega m . grad phi with the stray
    field H = -grad phi (units of mu_0 Ms^2 times length^3): with m affine and
    grad phi constant on every tetrahedron, int_T m . grad phi = |T| mbar_T .
    grad phi_T exactly. The paper forms the field by mass lumping (Numerics
    section), which gives the same value for uniform m."""
    vol, G = tet_gradients(nodes, tets)
    grad = np.einsum("ta,tai->ti", np.asarray(phi)[tets], G)
    mbar = np.asarray(m_nodes, dtype=np.float64)[tets].mean(axis=1)
    return 0.5 * float(np.sum(vol * np.einsum("ti,ti->t", mbar, grad)))


def prism_demag_factor(a, b, c):
    """Demagnetising factor along the 2c edge of a uniformly magnetised
    rectangular prism 2a x 2b x 2c (closed form of Aharoni, J. Appl. Phys. 83,
    3432 (1998)); the stray-field energy of the prism magnetised along that
    edge is N V / 2 in units of mu_0 Ms^2."""
    r = np.sqrt(a * a + b * b + c * c)
    rab, rbc, rac = np.sqrt(a * a + b * b), np.sqrt(b * b + c * c), np.sqrt(a * a + c * c)
    t = ((b * b - c * c) / (2 * b * c) * np.log((r - a) / (r + a))
         + (a * a - c * c) / (2 * a * c) * np.log((r - b) / (r + b))
         + b / (2 * c) * np.log((rab + a) / (rab - a))
         + a / (2 * c) * np.log((rab + b) / (rab - b))
         + c / (2 * a) * np.log((rbc - b) / (rbc + b))
         + c / (2 * b) * np.log((rac - a) / (rac + a))
         + 2 * np.arctan(a * b / (c * r))
         + (a ** 3 + b ** 3 - 2 * c ** 3) / (3 * a * b * c)
         + (a * a + b * b - 2 * c * c) / (3 * a * b * c) * r
         + c / (a * b) * (rac + rbc)
         - (rab ** 3 + rbc ** 3 + rac ** 3) / (3 * a * b * c))
    return float(t / np.pi)


def scalar_potential(nodes, tets, m_nodes, grid, eps, alpha=2, es_h=0.2, es_r_lo=None,
                     es_r_hi=None, es_tol=1e-12, eta2=37.0, parts=False):
    """phi = phi_1 + phi_2 at every node (Alg. 1): phi_1 from eq. poisson, the
    element density g = mean(m.n) - d phi_1/dn on the boundary triangles,
    phi_2 = smooth part (R2 route) + near-field correction within eps."""
    nodes = np.asarray(nodes, dtype=np.float64)
    phi1 = solve_phi1(nodes, tets, m_nodes)
    tris, owner = boundary_faces(nodes, tets)
    dn = dphi1_dn(nodes, tets, phi1, tris, owner)
    dens = geometry.density_p1(nodes, tris, m_nodes, dn)
    prob = direct.prepare(nodes, tris, dens, grid, alpha, es_h, es_r_lo, es_r_hi, es_tol, eta2)
    phi2 = direct.phi_ndft(prob)
    if eps > 0:
        near, *_ = nearfield.phi_near(prob, nodes, tris, eps)
        phi2 = phi2 + near
    if parts:
        return phi1 + phi2, phi1, phi2, dn, tris
    return phi1 + phi2
