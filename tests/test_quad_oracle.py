"""Pins of the oracle on Q1..Q6 quadrilaterals (bilinear map, Gauss rule per direction).

* Q1 on the unit square: the textbook element mass and stiffness matrices.
* Q_k on an undistorted cell: mass = M1 (x) M1 and stiffness = K1 (x) M1 + M1 (x) K1,
  with the 1D matrices of the GLL Lagrange basis integrated exactly by a longer
  Gauss rule (GLL nodes from the roots of the Legendre derivative, not the oracle's
  tables).
* Perturbed meshes: the mass action on a constant sums to the area, the mass with a
  linear vertex coefficient integrates it exactly, the Laplacian and Poisson operators
  annihilate constants, the Laplacian of a linear field vanishes at interior nodes and
  its energy is |grad u|^2 times the area, and the operators are symmetric.
"""
import numpy as np
import pytest
from numpy.polynomial import legendre as L

import oracle
from paper_1903_08243_amd import meshgen as mg


def _gll01(k):
    """GLL nodes on [0, 1]: the ends and the roots of P_k'."""
    inner = L.legroots(L.legder([0] * k + [1])) if k >= 2 else np.zeros(0)
    return np.concatenate([[0.0], (np.sort(inner) + 1) / 2, [1.0]])


def _1d_matrices(k):
    """1D mass and stiffness of the Lagrange basis on the GLL nodes of [0, 1], by a
    Gauss-Legendre rule with k + 3 points (exact for the degree-2k products), the basis
    and its derivative evaluated by the product formula."""
    x = _gll01(k)
    t, w = L.leggauss(k + 3)
    t, w = (t + 1) / 2, w / 2
    n = k + 1
    V = np.ones((t.size, n))
    dV = np.zeros((t.size, n))
    for i in range(n):
        for m in range(n):
            if m == i:
                continue
            V[:, i] *= (t - x[m]) / (x[i] - x[m])
            term = np.full(t.size, 1.0 / (x[i] - x[m]))
            for r in range(n):
                if r != i and r != m:
                    term *= (t - x[r]) / (x[i] - x[r])
            dV[:, i] += term
    return V.T @ (w[:, None] * V), dV.T @ (w[:, None] * dV)


def _node_xy(mesh, space):
    """Physical position of every Q_k node: the bilinear map of the GLL lattice."""
    k = space.degree
    g = _gll01(k)
    i, j = np.meshgrid(np.arange(k + 1), np.arange(k + 1), indexing="xy")
    xi, eta = g[i.ravel()], g[j.ravel()]  # local node i + (k+1) j
    N = np.stack([(1 - xi) * (1 - eta), xi * (1 - eta), (1 - xi) * eta, xi * eta], axis=1)
    X = mesh.coords[mesh.cell2vert]  # (ncells, 4, 2)
    pos = np.einsum("dv,cva->cda", N, X)
    out = np.zeros((space.nnodes, 2))
    out[space.cell2node.ravel()] = pos.reshape(-1, 2)
    return out


def test_quad_q1_textbook():
    mesh = mg.quad_mesh(1)
    space = mg.quad_space(mesh, 1, renumber=False)
    Ke = oracle.OracleOp(space, oracle.OP_LAPLACIAN).element_matrices()[0]
    Me = oracle.OracleOp(space, oracle.OP_MASS).element_matrices()[0]
    # vertices (0,0), (1,0), (0,1), (1,1)
    K_ref = np.array([[4, -1, -1, -2], [-1, 4, -2, -1], [-1, -2, 4, -1], [-2, -1, -1, 4]]) / 6.0
    M_ref = np.array([[4, 2, 2, 1], [2, 4, 1, 2], [2, 1, 4, 2], [1, 2, 2, 4]]) / 36.0
    assert np.abs(Ke - K_ref).max() <= 1e-15
    assert np.abs(Me - M_ref).max() <= 1e-15


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_quad_tensor_structure(k):
    mesh = mg.quad_mesh(1)
    space = mg.quad_space(mesh, k, renumber=False)
    M1, K1 = _1d_matrices(k)
    Me = oracle.OracleOp(space, oracle.OP_MASS).element_matrices()[0]
    Ke = oracle.OracleOp(space, oracle.OP_LAPLACIAN).element_matrices()[0]
    He = oracle.OracleOp(space, oracle.OP_HELMHOLTZ).element_matrices()[0]
    # local node i + (k+1) j: kron(A_j, B_i)
    M = np.kron(M1, M1)
    K = np.kron(M1, K1) + np.kron(K1, M1)
    scale = np.abs(K).max()
    assert np.abs(Me - M).max() <= 1e-14
    assert np.abs(Ke - K).max() <= 1e-13 * scale
    assert np.abs(He - (K + M)).max() <= 1e-13 * scale


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_quad_invariants(k):
    mesh = mg.quad_mesh(4, 0.25, config=0)
    space = mg.quad_space(mesh, k)
    one = np.ones(space.ndofs)
    xy = _node_xy(mesh, space)
    vxy = mesh.coords
    assert abs(oracle.OracleOp(space, oracle.OP_MASS).apply(one).sum() - 1.0) <= 1e-13
    # a vertex coefficient linear in x, y is reproduced by the bilinear interpolation
    c = 0.5 + 0.8 * vxy[:, 0] + 0.3 * vxy[:, 1]
    s = oracle.OracleOp(space, oracle.OP_MASS, coef=c).apply(one).sum()
    assert abs(s - (0.5 + 0.4 + 0.15)) <= 1e-13
    kappa = np.exp(np.random.default_rng(k).normal(size=mesh.nverts))
    for kind, coef in ((oracle.OP_LAPLACIAN, None), (oracle.OP_POISSON, kappa)):
        assert np.abs(oracle.OracleOp(space, kind, coef=coef).apply(one)).max() <= 1e-12
    u = 0.3 + 1.7 * xy[:, 0] - 0.9 * xy[:, 1]
    A = oracle.OracleOp(space, oracle.OP_LAPLACIAN)
    y = A.apply(u)
    interior = np.setdiff1d(np.arange(space.nnodes), space.boundary_nodes())
    assert np.abs(y[interior]).max() <= 1e-12
    assert np.abs(y[space.boundary_nodes()]).max() > 1e-3
    assert abs(u @ y - (1.7 ** 2 + 0.9 ** 2)) <= 1e-12
    H = oracle.OracleOp(space, oracle.OP_HELMHOLTZ)
    a, b = np.random.default_rng(1).uniform(-1, 1, (2, space.ndofs))
    assert abs(H.apply(a) @ b - a @ H.apply(b)) <= 1e-13 * abs(H.apply(a) @ b)


def test_quad_detj_orientation():
    """The generated cells are positively oriented and tile the unit square."""
    mesh = mg.quad_mesh(6, 0.25, config=0)
    op = oracle.OracleOp(mg.quad_space(mesh, 2), oracle.OP_MASS)
    d = op.detj()
    assert d.min() > 0
    assert abs((d * op.qw[None, :]).sum() - 1.0) <= 1e-13


def _1d_cross(k):
    """A1[i, m] = int l_i' l_m over [0, 1] (first index differentiated)."""
    x = _gll01(k)
    t, w = L.leggauss(k + 3)
    t, w = (t + 1) / 2, w / 2
    n = k + 1
    V = np.ones((t.size, n))
    dV = np.zeros((t.size, n))
    for i in range(n):
        for m in range(n):
            if m == i:
                continue
            V[:, i] *= (t - x[m]) / (x[i] - x[m])
            term = np.full(t.size, 1.0 / (x[i] - x[m]))
            for r in range(n):
                if r != i and r != m:
                    term *= (t - x[r]) / (x[i] - x[r])
            dV[:, i] += term
    return dV.T @ (w[:, None] * V)


@pytest.mark.parametrize("k", [1, 2, 4, 6])
def test_quad_elasticity_tensor_structure(k):
    """Undistorted cell: block (c, c') of int sigma(u) : grad v is
    mu delta_cc' (T00 + T11) + mu T_c'c + lam T_cc', T_pq[d, d'] = int d_p phi_d d_q phi_d'."""
    lam, mu = 0.7, 0.4
    mesh = mg.quad_mesh(1)
    space = mg.quad_space(mesh, k, renumber=False, ncomp=2)
    Ae = oracle.OracleOp(space, oracle.OP_ELASTICITY, lam=lam, mu=mu).element_matrices()[0]
    M1, K1 = _1d_matrices(k)
    A1 = _1d_cross(k)
    T = {(0, 0): np.kron(M1, K1), (1, 1): np.kron(K1, M1), (0, 1): np.kron(A1.T, A1)}
    T[(1, 0)] = T[(0, 1)].T
    D = (k + 1) ** 2
    ref = np.zeros((2 * D, 2 * D))
    for c in range(2):
        for cp in range(2):
            blk = mu * T[(cp, c)] + lam * T[(c, cp)]
            if c == cp:
                blk = blk + mu * (T[(0, 0)] + T[(1, 1)])
            ref[c::2, cp::2] = blk  # dof = 2 node + component
    assert np.abs(Ae - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("k", [1, 3, 6])
def test_quad_elasticity_invariants(k):
    """Perturbed mesh: rigid motions in the null space, the linear-field patch test
    and its energy area * (lam tr(eps)^2 + 2 mu eps:eps)."""
    lam, mu = 1.0, 0.5
    mesh = mg.quad_mesh(4, 0.25, config=0)
    space = mg.quad_space(mesh, k, ncomp=2)
    op = oracle.OracleOp(space, oracle.OP_ELASTICITY, lam=lam, mu=mu)
    xy = _node_xy(mesh, space)
    X, Y = xy[:, 0], xy[:, 1]
    for ux, uy in ((np.ones_like(X), 0 * X), (0 * X, np.ones_like(X)), (-Y, X)):
        u = np.stack([ux, uy], axis=1).ravel()
        assert np.abs(op.apply(u)).max() <= 1e-12
    G = np.array([[0.3, -1.1], [0.7, 0.9]])  # u = G (x, y) + const
    u = np.stack([G[0, 0] * X + G[0, 1] * Y + 0.2, G[1, 0] * X + G[1, 1] * Y - 0.4], axis=1).ravel()
    y = op.apply(u).reshape(-1, 2)
    interior = np.setdiff1d(np.arange(space.nnodes), space.boundary_nodes())
    assert np.abs(y[interior]).max() <= 1e-12
    eps = (G + G.T) / 2
    energy = lam * np.trace(eps) ** 2 + 2 * mu * (eps * eps).sum()
    assert abs(u @ y.ravel() - energy) <= 1e-12


@pytest.mark.parametrize("kind", [0, 1, 2, 3, 4])
def test_quad_diagonal_is_assembled_diagonal(kind):
    """The oracle's diagonal on perturbed quads equals the diagonal of the matrix
    assembled from its element matrices (which the tensor-structure pins fix)."""
    mesh = mg.quad_mesh(3, 0.25, config=0)
    nc = 2 if kind == 4 else 1
    space = mg.quad_space(mesh, 3, ncomp=nc)
    c = np.exp(np.random.default_rng(3).normal(size=mesh.nverts)) if kind in (0, 3) else None
    op = oracle.OracleOp(space, kind, coef=c, lam=0.7, mu=0.4)
    d = np.diag(op.assemble_dense())
    assert np.abs(op.diagonal() - d).max() <= 1e-14 * np.abs(d).max()
