"""Pins of the oracle's St-Venant-Kirchhoff operators (supplementary operator list,
"hyperelasticity"): the tangent at u0 = 0 is linear elasticity, the tangent is the
derivative of the separately coded nonlinear residual (central differences, exact
after one Richardson step because the residual is a cubic polynomial along a line),
the tangent is symmetric (hyperelastic), and the residual vanishes for a rigid
rotation (E = 0)."""
import numpy as np
import pytest

import oracle
from paper_1903_08243_amd import meshgen as mg

LAM, MU = 1.0, 0.5


def _space(k, m=2, pert=0.2):
    mesh = mg.tet_mesh(m, pert, config=2, seed_k=k)
    return mesh, mg.tet_space(mesh, k, ncomp=3, config=2, seed_k=k)


def _node_coords(mesh, space):
    """Physical position of every node: the affine image of its reference position."""
    k = space.degree
    alpha = mg.simplex_lattice(k, 3) / k  # (D, 3)
    X = mesh.coords[mesh.cell2vert]  # (ncells, 4, 3)
    pos = X[:, :1, :] + np.einsum("da,cae->cde", alpha, X[:, 1:, :] - X[:, :1, :])
    out = np.zeros((space.nnodes, 3))
    out[space.cell2node.ravel()] = pos.reshape(-1, 3)
    return out


def _field(space, seed, amp):
    return amp * np.random.default_rng(seed).uniform(-1, 1, space.ndofs)


@pytest.mark.parametrize("k", [1, 2])
def test_tangent_at_zero_is_linear_elasticity(k):
    mesh, space = _space(k)
    x = _field(space, 1, 1.0)
    hyp = oracle.OracleOp(space, oracle.OP_HYPERELASTIC, lam=LAM, mu=MU, u0=np.zeros(space.ndofs))
    lin = oracle.OracleOp(space, oracle.OP_ELASTICITY, lam=LAM, mu=MU)
    y, ref = hyp.apply(x), lin.apply(x)
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("k", [1, 2])
def test_tangent_is_derivative_of_residual(k):
    mesh, space = _space(k)
    u0, w = _field(space, 2, 0.3), _field(space, 3, 1.0)
    K = oracle.OracleOp(space, oracle.OP_HYPERELASTIC, lam=LAM, mu=MU, u0=u0)
    R = oracle.OracleOp(space, oracle.OP_HYPER_RESIDUAL, lam=LAM, mu=MU)
    cd = lambda h: (R.apply(u0 + h * w) - R.apply(u0 - h * w)) / (2 * h)
    h = 1e-2
    d1, d2 = cd(h), cd(h / 2)
    rich = (4 * d2 - d1) / 3  # removes the h^2 term; the residual has no higher one
    Kw = K.apply(w)
    scale = np.abs(Kw).max()
    assert np.abs(rich - Kw).max() <= 1e-10 * scale
    # without extrapolation the difference is O(h^2) and nonzero: the pin can fail
    assert np.abs(d1 - Kw).max() > 1e-8 * scale


@pytest.mark.parametrize("k", [1, 2])
def test_tangent_is_symmetric(k):
    mesh, space = _space(k)
    u0 = _field(space, 4, 0.3)
    K = oracle.OracleOp(space, oracle.OP_HYPERELASTIC, lam=LAM, mu=MU, u0=u0)
    a, b = _field(space, 5, 1.0), _field(space, 6, 1.0)
    lhs, rhs = K.apply(a) @ b, a @ K.apply(b)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("k", [1, 2])
def test_residual_vanishes_for_rigid_rotation(k):
    mesh, space = _space(k)
    th = 0.7
    c, s = np.cos(th), np.sin(th)
    Rm = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]]) @ np.array(
        [[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])
    xn = _node_coords(mesh, space)
    u0 = (xn @ (Rm - np.eye(3)).T).ravel()
    R = oracle.OracleOp(space, oracle.OP_HYPER_RESIDUAL, lam=LAM, mu=MU)
    r = R.apply(u0)
    # a stretch of the same size does not vanish (the pin can fail)
    r_stretch = R.apply((xn * 0.3).ravel())
    assert np.abs(r).max() <= 1e-13 * np.abs(r_stretch).max()
    assert np.abs(r_stretch).max() > 1e-3
