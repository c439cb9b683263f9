"""Host logic of the multigrid preconditioner (CPU only): the hierarchy of
SLP_PRECOND_AMG built from the free-node stiffness matrices of the oracle and
one cycle applied on the host with the device cycle's steps. The cycle must be
a symmetric positive definite operator (conjugate gradients require it) and
must make CG converge in a small, mesh-independent number of iterations."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import paper_1305_3162_amd as slp
from oracle import fem
from synth import ball_tets, cube_tets


def _free_stiffness(nodes, tets):
    S = fem.stiffness(nodes, tets)
    free = np.nonzero(~fem.boundary_nodes(tets, nodes))[0]
    return S[free][:, free].tocsr()


def _cycle(A):
    A = A.tocsr()
    A.sort_indices()

    def apply(r):
        z, _ = slp.amg_apply_host(A.indptr, A.indices, A.data, r)
        return z
    return apply


@pytest.mark.parametrize("mesh", ["cube12", "ball12"])
def test_cycle_is_symmetric_positive_definite(mesh):
    nodes, tets = cube_tets(12) if mesh == "cube12" else ball_tets(12, 1.0)
    A = _free_stiffness(nodes, tets)
    B = _cycle(A)
    rng = np.random.default_rng(11)
    _, nl = slp.amg_apply_host(A.indptr, A.indices, A.data, np.ones(A.shape[0]))
    assert nl >= 2
    for _ in range(5):
        x, y = rng.normal(size=(2, A.shape[0]))
        Bx, By = B(x), B(y)
        assert abs(x @ By - y @ Bx) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(By)
        assert x @ Bx > 0 and y @ By > 0
    # a linear operator: B(a x + y) = a B x + B y
    x, y = rng.normal(size=(2, A.shape[0]))
    assert np.allclose(B(2.5 * x + y), 2.5 * B(x) + B(y), rtol=1e-12, atol=1e-12 * np.abs(B(x)).max())


def _cg_iterations(A, M, b):
    it = [0]
    x, info = spla.cg(A, b, rtol=1e-10, atol=0.0, maxiter=2000, M=M,
                      callback=lambda xk: it.__setitem__(0, it[0] + 1))
    assert info == 0
    assert np.linalg.norm(b - A @ x) <= 1.01e-10 * np.linalg.norm(b)
    return it[0]


def test_cg_with_the_cycle_converges_in_few_iterations():
    """Jacobi-CG needs about twice the iterations when the mesh is refined
    twice; with the cycle the count stays small and nearly constant."""
    counts = {}
    for cells in (12, 24):
        nodes, tets = cube_tets(cells)
        A = _free_stiffness(nodes, tets)
        b = np.random.default_rng(3).normal(size=A.shape[0])
        counts[cells] = (_cg_iterations(A, sp.diags(1.0 / A.diagonal()), b),
                         _cg_iterations(A, spla.LinearOperator(A.shape, matvec=_cycle(A)), b))
    (j12, a12), (j24, a24) = counts[12], counts[24]
    assert a12 <= 20 and a24 <= 25 and a24 <= a12 + 6, counts
    assert j24 >= 1.6 * j12 and j24 >= 4 * a24, counts


def test_a_matrix_below_the_dense_limit_is_inverted_exactly():
    nodes, tets = cube_tets(6)                  # 125 free nodes: the coarsest level alone
    A = _free_stiffness(nodes, tets)
    r = np.random.default_rng(5).normal(size=A.shape[0])
    z, nl = slp.amg_apply_host(A.indptr, A.indices, A.data, r)
    assert nl == 1
    assert np.allclose(A @ z, r, rtol=1e-11, atol=1e-11 * np.abs(r).max())


def test_malformed_matrices_are_rejected():
    with pytest.raises(slp.SlpError, match="out of range"):
        slp.amg_apply_host(np.array([0, 1]), np.array([3]), np.array([1.0]), np.ones(1))
    A = sp.csr_matrix(np.array([[1.0, 0.0], [0.0, -1.0]]))
    with pytest.raises(slp.SlpError, match="positive"):
        slp.amg_apply_host(A.indptr, A.indices, A.data, np.ones(2))
