"""Pins of the oracle on P1..P3 triangles (perturbed split squares): the mass action on
a constant sums to the area, the Laplacian and Poisson operators annihilate constants,
the Laplacian of a linear field vanishes at interior nodes, and the operators are
symmetric."""
import numpy as np
import pytest

import oracle
from paper_1903_08243_amd import meshgen as mg


def _node_xy(mesh, space):
    k = space.degree
    alpha = mg.simplex_lattice(k, 2) / k
    X = mesh.coords[mesh.cell2vert]  # (ncells, 3, 2)
    pos = X[:, :1, :] + np.einsum("da,cae->cde", alpha, X[:, 1:, :] - X[:, :1, :])
    out = np.zeros((space.nnodes, 2))
    out[space.cell2node.ravel()] = pos.reshape(-1, 2)
    return out


@pytest.mark.parametrize("k", [1, 2, 3])
def test_tri_invariants(k):
    mesh = mg.tri_mesh(5, 0.2, config=0)
    space = mg.tri_space(mesh, k)
    one = np.ones(space.ndofs)
    c = np.exp(np.random.default_rng(k).normal(size=mesh.nverts))
    assert abs(oracle.OracleOp(space, oracle.OP_MASS).apply(one).sum() - 1.0) <= 1e-13
    for kind, coef in ((oracle.OP_LAPLACIAN, None), (oracle.OP_POISSON, c)):
        assert np.abs(oracle.OracleOp(space, kind, coef=coef).apply(one)).max() <= 1e-13
    # linear field: the Laplacian vanishes at interior nodes (exact quadrature)
    xy = _node_xy(mesh, space)
    u = 0.3 + 1.7 * xy[:, 0] - 0.9 * xy[:, 1]
    y = oracle.OracleOp(space, oracle.OP_LAPLACIAN).apply(u)
    interior = np.setdiff1d(np.arange(space.nnodes), space.boundary_nodes())
    assert np.abs(y[interior]).max() <= 1e-13
    assert np.abs(y[space.boundary_nodes()]).max() > 1e-3  # boundary rows carry the flux
    # symmetry
    H = oracle.OracleOp(space, oracle.OP_HELMHOLTZ)
    a, b = np.random.default_rng(1).uniform(-1, 1, (2, space.ndofs))
    assert abs(H.apply(a) @ b - a @ H.apply(b)) <= 1e-13 * abs(H.apply(a) @ b)
