"""Pins of the oracle's St-Venant-Kirchhoff operators (supplementary operator list,
"hyperelasticity") on P1/P2 tets and on Q1/Q2 trilinear hexes: the tangent at u0 = 0
is linear elasticity, the tangent is the derivative of the separately coded nonlinear
residual (central differences, exact after one Richardson step because the residual
is a cubic polynomial along a line for any fixed quadrature rule), the tangent is
symmetric (hyperelastic), and the residual vanishes for a rigid rotation (E = 0; the
rotation's displacement is linear, hence in the isoparametric space)."""
import numpy as np
import pytest

import oracle
from paper_1903_08243_amd import meshgen as mg

LAM, MU = 1.0, 0.5


CASES = [("tet", k) for k in range(1, 7)] + [("hex", 1), ("hex", 2)]


def _space(cell, k, m=2, pert=0.2):
    if cell == "hex":
        mesh = mg.hex_mesh(m, 0.15, config=1, seed_k=k)
        return mesh, mg.hex_space(mesh, k, ncomp=3, config=1)
    mesh = mg.tet_mesh(m, pert, config=2, seed_k=k)
    return mesh, mg.tet_space(mesh, k, ncomp=3, config=2, seed_k=k)


def _gll01(k):
    """GLL nodes on [0, 1]: the ends and the roots of P_k' (numpy Legendre series)."""
    inner = np.polynomial.legendre.Legendre.basis(k).deriv().roots() if k > 1 else np.zeros(0)
    return (np.concatenate([[-1.0], np.sort(inner.real), [1.0]]) + 1.0) / 2.0


def _node_coords(mesh, space):
    """Physical position of every node: the image of its reference position under the
    cell's affine (tet) or trilinear (hex, vertex v at (v&1, v>>1&1, v>>2&1)) map."""
    k = space.degree
    if mesh.cell_type == oracle.CELL_HEX:
        g = _gll01(k)
        n = k + 1
        ref = np.array([[g[i % n], g[(i // n) % n], g[i // (n * n)]] for i in range(n ** 3)])  # (D, 3)
        bits = np.array([[(v >> d) & 1 for d in range(3)] for v in range(8)])  # (8, 3)
        Nv = np.prod(np.where(bits[None, :, :] == 1, ref[:, None, :], 1.0 - ref[:, None, :]), axis=2)  # (D, 8)
        pos = np.einsum("dv,cve->cde", Nv, mesh.coords[mesh.cell2vert])
    else:
        alpha = mg.simplex_lattice(k, 3) / k  # (D, 3)
        X = mesh.coords[mesh.cell2vert]  # (ncells, 4, 3)
        pos = X[:, :1, :] + np.einsum("da,cae->cde", alpha, X[:, 1:, :] - X[:, :1, :])
    out = np.zeros((space.nnodes, 3))
    out[space.cell2node.ravel()] = pos.reshape(-1, 3)
    return out


def _field(space, seed, amp):
    return amp * np.random.default_rng(seed).uniform(-1, 1, space.ndofs)


@pytest.mark.parametrize("cell,k", CASES)
def test_tangent_at_zero_is_linear_elasticity(cell, k):
    mesh, space = _space(cell, k)
    x = _field(space, 1, 1.0)
    hyp = oracle.OracleOp(space, oracle.OP_HYPERELASTIC, lam=LAM, mu=MU, u0=np.zeros(space.ndofs))
    lin = oracle.OracleOp(space, oracle.OP_ELASTICITY, lam=LAM, mu=MU)
    y, ref = hyp.apply(x), lin.apply(x)
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("cell,k", CASES)
def test_tangent_is_derivative_of_residual(cell, k):
    mesh, space = _space(cell, k)
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


@pytest.mark.parametrize("cell,k", CASES)
def test_tangent_is_symmetric(cell, k):
    mesh, space = _space(cell, k)
    u0 = _field(space, 4, 0.3)
    K = oracle.OracleOp(space, oracle.OP_HYPERELASTIC, lam=LAM, mu=MU, u0=u0)
    a, b = _field(space, 5, 1.0), _field(space, 6, 1.0)
    lhs, rhs = K.apply(a) @ b, a @ K.apply(b)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("cell,k", CASES)
def test_residual_vanishes_for_rigid_rotation(cell, k):
    mesh, space = _space(cell, k)
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
