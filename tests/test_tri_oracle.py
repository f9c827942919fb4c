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


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
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


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_tri_elasticity_invariants(k):
    """2D elasticity on perturbed triangles: rigid motions in the null space, the
    linear-field patch test (interior rows vanish) and its exact energy
    area * (lam tr(eps)^2 + 2 mu eps:eps), symmetry."""
    lam, mu = 0.7, 0.4
    mesh = mg.tri_mesh(5, 0.2, config=0)
    space = mg.tri_space(mesh, k, ncomp=2)
    op = oracle.OracleOp(space, oracle.OP_ELASTICITY, lam=lam, mu=mu)
    xy = _node_xy(mesh, space)
    X, Y = xy[:, 0], xy[:, 1]
    for ux, uy in ((np.ones_like(X), 0 * X), (0 * X, np.ones_like(X)), (-Y, X)):
        assert np.abs(op.apply(np.stack([ux, uy], axis=1).ravel())).max() <= 1e-12
    G = np.array([[0.3, -1.1], [0.7, 0.9]])
    u = np.stack([G[0, 0] * X + G[0, 1] * Y + 0.2, G[1, 0] * X + G[1, 1] * Y - 0.4], axis=1).ravel()
    y = op.apply(u).reshape(-1, 2)
    interior = np.setdiff1d(np.arange(space.nnodes), space.boundary_nodes())
    assert np.abs(y[interior]).max() <= 1e-12
    eps = (G + G.T) / 2
    assert abs(u @ y.ravel() - (lam * np.trace(eps) ** 2 + 2 * mu * (eps * eps).sum())) <= 1e-12
    a, b = np.random.default_rng(1).uniform(-1, 1, (2, space.ndofs))
    assert abs(op.apply(a) @ b - a @ op.apply(b)) <= 1e-13 * abs(op.apply(a) @ b)
