"""The library's FEM mesh analysis and stiffness assembly on the host
(slp_fem_assemble_host, the same code slp_fem_setup runs before its uploads)
against the oracle's assembly of eq. varu1 / poisson (CPU only): the free
nodes are the oracle's non-boundary nodes, and every entry of S(fn, fn)
matches (entries the library drops because their element contributions
cancel are zero in the oracle to the same rounding)."""
import numpy as np
import pytest

import paper_1305_3162_amd as slp
from oracle import fem
from synth import ball_tets, cube_tets


@pytest.mark.parametrize("mesh", ["cube6", "ball6", "cube10"])
def test_assembly_matches_oracle(mesh):
    nodes, tets = {"cube6": lambda: cube_tets(6), "ball6": lambda: ball_tets(6, 1.0),
                   "cube10": lambda: cube_tets(10)}[mesh]()
    rp, ci, v, fn = slp.fem_assemble_host(nodes, tets)
    free = np.nonzero(~fem.boundary_nodes(tets, nodes))[0]
    assert np.array_equal(fn, free)
    S = fem.stiffness(nodes, tets)[free][:, free].toarray()
    n = free.size
    A = np.zeros((n, n))
    for i in range(n):
        cols = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(cols) > 0)            # ascending, no duplicates
        A[i, cols] = v[rp[i]:rp[i + 1]]
    scale = np.abs(S).max()
    assert np.abs(A - S).max() <= 1e-13 * scale
    # what is not stored cancels in the oracle too
    dropped = (A == 0) & (S != 0)
    assert np.all(np.abs(S[dropped]) <= 1e-13 * scale)
    # symmetric, positive diagonal
    assert np.abs(A - A.T).max() <= 1e-14 * scale and np.all(np.diag(A) > 0)


def test_assembly_rejects_bad_meshes():
    nodes, tets = cube_tets(2)
    bad = tets.copy()
    bad[0, 0] = nodes.shape[0]
    with pytest.raises(slp.SlpError):
        slp.fem_assemble_host(nodes, bad)
    flat = tets.copy()
    flat[0] = [0, 1, 2, 2]
    with pytest.raises(slp.SlpError):
        slp.fem_assemble_host(nodes, flat)
