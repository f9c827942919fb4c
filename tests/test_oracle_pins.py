"""Pins of the CPU FP64 oracle against what the mathematics fixes.

Nothing here re-types an oracle formula: each check uses an independent route
(closed forms, exact polynomial integration with sympy/numpy polynomials,
invariants of the bilinear forms, or the linear-algebra identity between the
action and the assembled matrix).
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import sympy as sp

import oracle
from oracle import tables as T
from paper_1903_08243_amd import meshgen as mg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------- P1 quadrature
@pytest.mark.parametrize("n", range(1, 9))
def test_gauss_legendre_exactness(n):
    x, w = T.gauss_legendre01(n)
    for p in range(2 * n):
        assert abs(np.sum(w * x ** p) - 1.0 / (p + 1)) < 2e-15
    assert abs(np.sum(w * x ** (2 * n)) - 1.0 / (2 * n + 1)) > 1e-12


def test_gauss_legendre_closed_form_points():
    x, _ = T.gauss_legendre01(2)
    assert np.allclose(np.sort(2 * x - 1), [-1 / math.sqrt(3), 1 / math.sqrt(3)], atol=1e-15)
    x, w = T.gauss_legendre01(3)
    assert np.allclose(np.sort(2 * x - 1), [-math.sqrt(0.6), 0, math.sqrt(0.6)], atol=1e-15)
    assert np.allclose(2 * w[np.argsort(x)], [5 / 9, 8 / 9, 5 / 9], atol=1e-15)


# ----------------------------------------------------------------- P2 GLL nodes
def test_gll_closed_forms():
    s = math.sqrt
    closed = {
        1: [-1, 1],
        2: [-1, 0, 1],
        3: [-1, -1 / s(5), 1 / s(5), 1],
        4: [-1, -s(3 / 7), 0, s(3 / 7), 1],
        5: [-1, -s(1 / 3 + 2 * s(7) / 21), -s(1 / 3 - 2 * s(7) / 21),
            s(1 / 3 - 2 * s(7) / 21), s(1 / 3 + 2 * s(7) / 21), 1],
        6: [-1, -s((15 + 2 * s(15)) / 33), -s((15 - 2 * s(15)) / 33), 0,
            s((15 - 2 * s(15)) / 33), s((15 + 2 * s(15)) / 33), 1],
    }
    for k, ref in closed.items():
        got = 2 * T.gll_nodes01(k) - 1
        assert np.allclose(got, ref, atol=1e-14), k


# ----------------------------------------------------------------- P3 bases
@pytest.mark.parametrize("k", range(1, 7))
def test_lagrange1d_kronecker_and_partition(k):
    nodes = T.gll_nodes01(k)
    V, dV = T.lagrange1d(nodes, nodes)
    assert np.allclose(V, np.eye(k + 1), atol=1e-13)
    pts = np.linspace(0, 1, 17)
    V, dV = T.lagrange1d(nodes, pts)
    assert np.allclose(V.sum(1), 1.0, atol=1e-13)
    assert np.allclose(dV.sum(1), 0.0, atol=1e-11)
    # derivative against a central difference of the values
    e = 1e-6
    Vp, _ = T.lagrange1d(nodes, pts + e)
    Vm, _ = T.lagrange1d(nodes, pts - e)
    assert np.allclose((Vp - Vm) / (2 * e), dV, atol=1e-6)


@pytest.mark.parametrize("k,dim", [(k, d) for d in (2, 3) for k in range(1, 7)])
def test_simplex_lagrange_nodal_and_partition(k, dim):
    alpha = T.simplex_lattice(k, dim)
    pts = alpha / k
    phi, dphi = T.simplex_lagrange(k, dim, pts)
    assert np.allclose(phi, np.eye(len(alpha)), atol=1e-13)
    rnd = np.random.default_rng(0).dirichlet(np.ones(dim + 1), size=20)[:, 1:]
    phi, dphi = T.simplex_lagrange(k, dim, rnd)
    assert np.allclose(phi.sum(1), 1.0, atol=1e-13)
    assert np.allclose(dphi.sum(1), 0.0, atol=1e-11)
    e = 1e-6
    for d in range(dim):
        sh = np.zeros(dim)
        sh[d] = e
        fp, _ = T.simplex_lagrange(k, dim, rnd + sh)
        fm, _ = T.simplex_lagrange(k, dim, rnd - sh)
        assert np.allclose((fp - fm) / (2 * e), dphi[:, :, d], atol=1e-6)


@pytest.mark.parametrize("dim,deg", [(2, 3), (2, 5), (3, 2), (3, 4), (3, 5)])
def test_collapsed_rule_exact_on_monomials(dim, deg):
    """Closed form: int_ref xi^a = a! / (|a| + dim)! over the unit simplex."""
    pts, w = T.collapsed_rule(dim, deg)
    for a in np.ndindex(*([deg + 1] * dim)):
        if sum(a) > deg:
            continue
        exact = math.prod(math.factorial(ai) for ai in a) / math.factorial(sum(a) + dim)
        got = np.sum(w * np.prod(pts ** np.array(a), axis=1))
        assert abs(got - exact) < 1e-15, (a, got, exact)


# ----------------------------------------------------------------- P4 uniform hex = Kronecker form
_GLL_EXACT = {  # closed-form GLL points on [-1, 1]
    1: [-1, 1],
    2: [-1, 0, 1],
    3: [-1, -1 / sp.sqrt(5), 1 / sp.sqrt(5), 1],
    4: [-1, -sp.sqrt(sp.Rational(3, 7)), 0, sp.sqrt(sp.Rational(3, 7)), 1],
}


def _gll_1d_matrices(k):
    """1D element mass/stiffness on [0,1], exact (sympy, closed-form GLL points).

    Independent of the oracle: the Lagrange polynomials are built symbolically
    on the exact nodes and integrated exactly."""
    t = sp.symbols("t")
    nodes = [(sp.Integer(1) + sp.sympify(v)) / 2 for v in _GLL_EXACT[k]]
    n = k + 1
    polys = []
    for i in range(n):
        p = sp.Integer(1)
        for m in range(n):
            if m != i:
                p *= (t - nodes[m]) / (nodes[i] - nodes[m])
        polys.append(sp.expand(p))
    M = np.zeros((n, n))
    K = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            M[i, j] = float(sp.integrate(polys[i] * polys[j], (t, 0, 1)))
            K[i, j] = float(sp.integrate(sp.diff(polys[i], t) * sp.diff(polys[j], t), (t, 0, 1)))
    return M, K


@pytest.mark.parametrize("extra", [0, 1], ids=["q=k+1", "q=k+2"])
@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_uniform_hex_matches_kronecker_assembly(k, extra):
    """On the uniform mesh the integrands are polynomials of degree <= 2k per variable,
    so k+1 and k+2 Gauss points both integrate them exactly: the action equals the
    Kronecker form of the exact 1D matrices for either rule."""
    m = 2
    h = 1.0 / m
    mesh = mg.hex_mesh(m, 0.0)
    M1, K1 = _gll_1d_matrices(k)
    Me = h ** 3 * np.kron(np.kron(M1, M1), M1)  # local index i + n j + n^2 l -> kron(l, j, i)
    Ke = h * (np.kron(np.kron(M1, M1), K1) + np.kron(np.kron(M1, K1), M1) + np.kron(np.kron(K1, M1), M1))
    for ncomp, kind, Eloc in [(1, oracle.OP_MASS, Me), (1, oracle.OP_HELMHOLTZ, Me + Ke),
                              (3, oracle.OP_LAPLACIAN, Ke)]:
        sp_ = mg.hex_space(mesh, k, ncomp=ncomp, renumber=True, config=9)
        op = oracle.OracleOp(sp_, kind, nq1d=k + 1 + extra)
        A = np.zeros((op.ndofs, op.ndofs))
        for c2n in sp_.cell2node:
            for comp in range(ncomp):
                idx = c2n.astype(np.int64) * ncomp + comp
                A[np.ix_(idx, idx)] += Eloc
        x = np.random.default_rng(k).uniform(-1, 1, op.ndofs)
        y = op.apply(x)
        assert np.max(np.abs(y - A @ x)) <= 1e-13 * np.max(np.abs(A @ x))


def _read_stencils():
    out = {}
    with open(os.path.join(GOLDEN, "q1_hex_stencils.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            opname, where, coef, p = line.split()
            out[(opname, where)] = (float(Fraction(coef)), int(p))
    return out


def test_q1_interior_stencils_golden():
    m = 4
    h = 1.0 / m
    mesh = mg.hex_mesh(m, 0.0)
    sp_ = mg.hex_space(mesh, 1, renumber=False)
    st = _read_stencils()
    centre = 2 + 5 * (2 + 5 * 2)  # lattice node (2,2,2)
    offs = {"centre": (0, 0, 0), "face": (1, 0, 0), "edge": (1, 1, 0), "corner": (1, 1, 1)}
    for opname, kind in [("mass", oracle.OP_MASS), ("laplacian", oracle.OP_LAPLACIAN)]:
        op = oracle.OracleOp(sp_, kind)
        for where, o in offs.items():
            nb = (2 + o[0]) + 5 * ((2 + o[1]) + 5 * (2 + o[2]))
            e = np.zeros(op.ndofs)
            e[nb] = 1.0
            got = op.apply(e)[centre]
            coef, p = st[(opname, where)]
            assert abs(got - coef * h ** p) < 1e-15, (opname, where, got, coef * h ** p)


# ----------------------------------------------------------------- P5 volumes
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_hex_mass_volume_perturbed(k):
    mesh = mg.hex_mesh(3, 0.15, config=1, seed_k=k)
    sp_ = mg.hex_space(mesh, k)
    one = np.ones(sp_.ndofs)
    for kind in (oracle.OP_MASS, oracle.OP_HELMHOLTZ):
        op = oracle.OracleOp(sp_, kind)
        assert abs(one @ op.apply(one) - 1.0) < 1e-13


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_tet_mass_volume_perturbed(k):
    mesh = mg.tet_mesh(2, 0.2, config=2)
    sp_ = mg.tet_space(mesh, k, ncomp=1)
    op = oracle.OracleOp(sp_, oracle.OP_MASS)
    one = np.ones(sp_.ndofs)
    assert abs(one @ op.apply(one) - 1.0) < 1e-13


def test_tri_mass_coefficient_closed_form():
    """1^T M(c) 1 = int c = sum_T |T| (c_a + c_b + c_c) / 3 for P1 c."""
    mesh = mg.tri_mesh(6, 0.2, config=0)
    sp_ = mg.tri_p1_space(mesh, renumber=True)
    c = mg.uniform(mesh.nverts, 0.5, 1.5, 0, mg.PURPOSE_COEF)
    op = oracle.OracleOp(sp_, oracle.OP_MASS, coef=c)
    one = np.ones(sp_.ndofs)
    X = mesh.coords[mesh.cell2vert]
    area = 0.5 * np.abs((X[:, 1, 0] - X[:, 0, 0]) * (X[:, 2, 1] - X[:, 0, 1])
                        - (X[:, 2, 0] - X[:, 0, 0]) * (X[:, 1, 1] - X[:, 0, 1]))
    exact = np.sum(area * c[mesh.cell2vert].sum(1) / 3)
    assert abs(one @ op.apply(one) - exact) < 1e-14
    assert abs(area.sum() - 1.0) < 1e-14


# ----------------------------------------------------------------- P10 simplex closed forms
def test_tri_p1_mass_element_matrix_closed_form():
    """int_T lam_a lam_i lam_j = 2|T| a!b!c!/(a+b+c+2)!: 1/10, 1/30, 1/60 of |T|."""
    mesh = mg.tri_mesh(3, 0.2, config=0)
    sp_ = mg.tri_p1_space(mesh)
    c = mg.uniform(mesh.nverts, 0.5, 1.5, 0, mg.PURPOSE_COEF)
    op = oracle.OracleOp(sp_, oracle.OP_MASS, coef=c)
    Ae = op.element_matrices()
    X = mesh.coords[mesh.cell2vert]
    for K in range(mesh.ncells):
        area = 0.5 * abs((X[K, 1, 0] - X[K, 0, 0]) * (X[K, 2, 1] - X[K, 0, 1])
                         - (X[K, 2, 0] - X[K, 0, 0]) * (X[K, 1, 1] - X[K, 0, 1]))
        cv = c[mesh.cell2vert[K]]
        E = np.zeros((3, 3))
        for i in range(3):
            for j in range(3):
                for a in range(3):
                    cnt = [0, 0, 0]
                    for t in (a, i, j):
                        cnt[t] += 1
                    frac = 2 * math.prod(math.factorial(x) for x in cnt) / math.factorial(5)
                    E[i, j] += area * cv[a] * frac
        assert np.allclose(Ae[K], E, atol=1e-16, rtol=1e-14)


def _sympy_tet_stiffness_blocks(k):
    """S[a][b][i][j] = int_ref d_a phi_i d_b phi_j, exact rationals.

    The P_k basis is obtained by inverting the monomial Vandermonde matrix at the
    equispaced lattice points (an independent construction from the oracle's
    barycentric product formula)."""
    x, y, z = sp.symbols("x y z")
    alpha = T.simplex_lattice(k, 3)
    mons = [x ** p * y ** q * z ** r for p in range(k + 1) for q in range(k + 1)
            for r in range(k + 1) if p + q + r <= k]
    pts = [tuple(sp.Rational(int(a), k) for a in al) for al in alpha]
    V = sp.Matrix([[mm.subs({x: p[0], y: p[1], z: p[2]}) for mm in mons] for p in pts])
    C = V.inv()  # column i holds the monomial coefficients of phi_i
    phis = [sum(C[mi, i] * mons[mi] for mi in range(len(mons))) for i in range(len(pts))]
    grads = [[sp.diff(p, v) for v in (x, y, z)] for p in phis]

    def integ(f):
        # exact: int_ref x^p y^q z^r = p! q! r! / (p+q+r+3)!
        tot = sp.Rational(0)
        for (p, q, r), cf in sp.Poly(sp.expand(f), x, y, z).terms():
            tot += cf * sp.factorial(p) * sp.factorial(q) * sp.factorial(r) / sp.factorial(p + q + r + 3)
        return tot

    D = len(phis)
    S = np.zeros((3, 3, D, D))
    for a in range(3):
        for b in range(3):
            for i in range(D):
                for j in range(D):
                    S[a, b, i, j] = float(integ(grads[i][a] * grads[j][b]))
    return S


@pytest.mark.parametrize("k", [1, 2, 3])
def test_tet_elasticity_element_matrix_exact(k):
    """Element matrix of sigma(u):grad v against exact symbolic integration.

    With an affine map, grad phi = J^{-T} grad_ref phi, so
    A[(i,c),(j,d)] = |det J| sum_{a,b} Jinv[a,.]... expanded through the
    reference blocks S computed exactly by sympy."""
    lam, mu = 1.0, 0.5
    mesh = mg.tet_mesh(1, 0.2, config=2)
    sp_ = mg.tet_space(mesh, k, ncomp=3)
    op = oracle.OracleOp(sp_, oracle.OP_ELASTICITY, lam=lam, mu=mu)
    Ae = op.element_matrices()
    S = _sympy_tet_stiffness_blocks(k)
    D = S.shape[2]
    for K in range(mesh.ncells):
        X = mesh.coords[mesh.cell2vert[K]]
        J = np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], axis=1)  # J[a, b] = dx_a/dxi_b
        Kinv = np.linalg.inv(J)  # Kinv[b, a] = dxi_b/dx_a
        det = abs(np.linalg.det(J))
        # G[i][j][a][b] = int grad_a phi_i grad_b phi_j (physical)
        G = det * np.einsum("pa,qb,pqij->ijab", Kinv, Kinv, S)
        E = np.zeros((3 * D, 3 * D))
        for i in range(D):
            for j in range(D):
                for c in range(3):
                    for d in range(3):
                        # sigma(phi_j e_d) : grad(phi_i e_c)
                        val = lam * G[i, j, c, d] + mu * G[i, j, d, c]
                        if c == d:
                            val += mu * np.trace(G[i, j])
                        E[3 * i + c, 3 * j + d] = val
        assert np.allclose(Ae[K], E, rtol=1e-12, atol=1e-14 * np.abs(E).max())


# ----------------------------------------------------------------- P6 null spaces
@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_laplacian_kills_constants(k):
    mesh = mg.hex_mesh(3, 0.15, config=1, seed_k=k)
    for ncomp, kind, coef in [(1, oracle.OP_LAPLACIAN, None), (3, oracle.OP_LAPLACIAN, None),
                              (1, oracle.OP_POISSON, np.exp(np.random.default_rng(1).normal(size=mesh.nverts)))]:
        sp_ = mg.hex_space(mesh, k, ncomp=ncomp)
        op = oracle.OracleOp(sp_, kind, coef=coef)
        one = np.ones(sp_.ndofs)
        y = op.apply(one)
        scale = np.abs(op.apply(np.random.default_rng(0).uniform(-1, 1, sp_.ndofs))).max()
        assert np.abs(y).max() < 1e-13 * max(scale, 1.0)


def _tet_node_coords(mesh, sp_):
    k = sp_.degree
    alpha = T.simplex_lattice(k, 3) / k
    X = mesh.coords[mesh.cell2vert]  # (ncells, 4, 3)
    pos = X[:, None, 0, :] + np.einsum("da,cae->cde", alpha, X[:, 1:, :] - X[:, None, 0, :])
    out = np.zeros((sp_.nnodes, 3))
    out[sp_.cell2node.ravel()] = pos.reshape(-1, 3)
    return out


def _hex_node_coords(mesh, sp_):
    k = sp_.degree
    g = T.gll_nodes01(k)
    n = k + 1
    X = mesh.coords[mesh.cell2vert]  # (ncells, 8, 3)
    out = np.zeros((sp_.nnodes, 3))
    for l in range(n):
        for j in range(n):
            for i in range(n):
                xi = (g[i], g[j], g[l])
                p = np.zeros((mesh.ncells, 3))
                for v in range(8):
                    o = (v & 1, (v >> 1) & 1, (v >> 2) & 1)
                    wv = np.prod([xi[d] if o[d] else 1 - xi[d] for d in range(3)])
                    p += wv * X[:, v, :]
                out[sp_.cell2node[:, i + n * (j + n * l)]] = p
    return out


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_elasticity_kills_rigid_modes(k):
    mesh = mg.tet_mesh(2, 0.2, config=2)
    sp_ = mg.tet_space(mesh, k, ncomp=3)
    op = oracle.OracleOp(sp_, oracle.OP_ELASTICITY, lam=1.0, mu=0.5)
    xn = _tet_node_coords(mesh, sp_)
    scale = np.abs(op.apply(np.random.default_rng(0).uniform(-1, 1, sp_.ndofs))).max()
    modes = [np.eye(3)[c] + 0 * xn for c in range(3)]
    for axis in range(3):
        w = np.eye(3)[axis]
        modes.append(np.cross(w, xn))
    for u in modes:
        y = op.apply(u.ravel())
        assert np.abs(y).max() < 1e-12 * scale


# ----------------------------------------------------------------- P7 linear fields
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_hex_laplacian_of_linear_field_vanishes_inside(k):
    mesh = mg.hex_mesh(3, 0.15, config=1, seed_k=k)
    sp_ = mg.hex_space(mesh, k)
    op = oracle.OracleOp(sp_, oracle.OP_LAPLACIAN)
    xn = _hex_node_coords(mesh, sp_)
    g = np.array([0.3, -1.1, 0.7])
    y = op.apply(xn @ g)
    interior = np.ones(sp_.nnodes, bool)
    interior[sp_.boundary_nodes()] = False
    scale = np.abs(op.apply(np.random.default_rng(0).uniform(-1, 1, sp_.ndofs))).max()
    assert np.abs(y[interior]).max() < 1e-13 * scale
    assert np.abs(y[~interior]).max() > 1e-3 * scale  # boundary flux is not zero
    assert abs(y.sum()) < 1e-13 * scale


@pytest.mark.parametrize("k", [1, 2, 3])
def test_hex_elasticity_invariants(k):
    """Elasticity on perturbed trilinear hexes: the six rigid motions are in the null
    space, the linear-field patch test holds at interior nodes, and the energy of a
    linear field is lam tr(eps)^2 + 2 mu eps:eps (unit volume)."""
    lam, mu = 0.7, 0.4
    mesh = mg.hex_mesh(3, 0.15, config=1, seed_k=k)
    sp_ = mg.hex_space(mesh, k, ncomp=3)
    op = oracle.OracleOp(sp_, oracle.OP_ELASTICITY, lam=lam, mu=mu)
    xn = _hex_node_coords(mesh, sp_)
    X, Y, Z = xn[:, 0], xn[:, 1], xn[:, 2]
    one, zero = np.ones_like(X), np.zeros_like(X)
    scale = np.abs(op.apply(np.random.default_rng(0).uniform(-1, 1, sp_.ndofs))).max()
    for m in ((one, zero, zero), (zero, one, zero), (zero, zero, one), (-Y, X, zero), (zero, -Z, Y), (Z, zero, -X)):
        assert np.abs(op.apply(np.stack(m, axis=1).ravel())).max() < 1e-13 * scale
    G = np.array([[0.3, -1.1, 0.2], [0.7, 0.9, -0.4], [-0.5, 0.1, 0.6]])
    u = (xn @ G.T + np.array([0.2, -0.4, 0.1])).ravel()
    y = op.apply(u).reshape(-1, 3)
    interior = np.ones(sp_.nnodes, bool)
    interior[sp_.boundary_nodes()] = False
    assert np.abs(y[interior]).max() < 1e-13 * scale
    eps = (G + G.T) / 2
    assert abs(u @ y.ravel() - (lam * np.trace(eps) ** 2 + 2 * mu * (eps * eps).sum())) < 1e-12


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_tet_elasticity_patch_test(k):
    mesh = mg.tet_mesh(2, 0.2, config=2)
    sp_ = mg.tet_space(mesh, k, ncomp=3)
    op = oracle.OracleOp(sp_, oracle.OP_ELASTICITY, lam=1.0, mu=0.5)
    xn = _tet_node_coords(mesh, sp_)
    B = np.array([[0.3, -0.2, 0.5], [0.1, 0.4, -0.6], [-0.7, 0.2, 0.25]])
    u = xn @ B.T + np.array([0.1, 0.2, -0.3])
    y = op.apply(u.ravel()).reshape(-1, 3)
    interior = np.ones(sp_.nnodes, bool)
    interior[sp_.boundary_nodes()] = False
    scale = np.abs(op.apply(np.random.default_rng(0).uniform(-1, 1, sp_.ndofs))).max()
    assert np.abs(y[interior]).max() < 1e-12 * scale
    assert np.abs(y[~interior]).max() > 1e-3 * scale


# ----------------------------------------------------------------- P8 symmetry / sign, P9 assembly
def _small_ops():
    hexm = mg.hex_mesh(2, 0.15, config=1)
    tetm = mg.tet_mesh(1, 0.2, config=2)
    trim = mg.tri_mesh(4, 0.2, config=0)
    kap = np.exp(np.random.default_rng(3).normal(size=hexm.nverts))
    c = mg.uniform(trim.nverts, 0.5, 1.5, 0, mg.PURPOSE_COEF)
    return [
        ("hex-helm-2", oracle.OracleOp(mg.hex_space(hexm, 2), oracle.OP_HELMHOLTZ), True),
        ("hex-lap3-2", oracle.OracleOp(mg.hex_space(hexm, 2, ncomp=3), oracle.OP_LAPLACIAN), False),
        ("hex-pois-3", oracle.OracleOp(mg.hex_space(hexm, 3), oracle.OP_POISSON, coef=kap), False),
        ("hex-mass-1", oracle.OracleOp(mg.hex_space(hexm, 1), oracle.OP_MASS), True),
        ("tet-el-2", oracle.OracleOp(mg.tet_space(tetm, 2), oracle.OP_ELASTICITY), False),
        ("tet-el-3", oracle.OracleOp(mg.tet_space(tetm, 3), oracle.OP_ELASTICITY), False),
        ("tri-mass", oracle.OracleOp(mg.tri_p1_space(trim, True), oracle.OP_MASS, coef=c), True),
    ]


@pytest.mark.parametrize("name,op,definite", _small_ops(), ids=lambda v: v if isinstance(v, str) else "")
def test_symmetry_sign_and_assembly(name, op, definite):
    r = np.random.default_rng(11)
    x, z = r.uniform(-1, 1, op.ndofs), r.uniform(-1, 1, op.ndofs)
    Ax, Az = op.apply(x), op.apply(z)
    s = np.abs(Ax).max() * np.abs(z).sum()
    assert abs(Ax @ z - x @ Az) < 1e-14 * s
    if definite:
        assert x @ Ax > 0
    else:
        assert x @ Ax > -1e-14 * s
    A = op.assemble_dense()
    assert np.abs(A @ x - Ax).max() < 1e-14 * np.abs(Ax).max() * 10
    assert np.allclose(np.diag(A), op.diagonal(), rtol=1e-13, atol=1e-16)
    assert np.abs(A - A.T).max() < 1e-14 * np.abs(A).max() * 10
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev.min() > (1e-12 if definite else -1e-12) * ev.max()


def test_apply_range_is_partial_sum():
    """The paper's wrapper takes a cell range [start, end) and increments (Listing 3)."""
    mesh = mg.hex_mesh(3, 0.15)
    op = oracle.OracleOp(mg.hex_space(mesh, 2), oracle.OP_HELMHOLTZ)
    x = np.random.default_rng(0).uniform(-1, 1, op.ndofs)
    y = op.apply(x)
    y1 = op.apply(x, cells=(0, 10))
    y2 = op.apply(x, cells=(10, op.ncells))
    assert np.abs(y1 + y2 - y).max() < 1e-14 * np.abs(y).max()


# ----------------------------------------------------------------- P12 CG
def test_cg_matches_dense_solve():
    mesh = mg.hex_mesh(2, 0.15, config=1)
    op = oracle.OracleOp(mg.hex_space(mesh, 2), oracle.OP_HELMHOLTZ)
    A = op.assemble_dense()
    b = np.random.default_rng(4).uniform(-1, 1, op.ndofs)
    d = op.diagonal()
    x, it, rr = oracle.cg(op.apply, b, rtol=1e-12, precond=lambda r: r / d)
    xs = np.linalg.solve(A, b)
    assert rr <= 1e-12
    assert np.abs(x - xs).max() <= 1e-10 * np.abs(xs).max()
    x2, it2, rr2 = oracle.cg(op.apply, b, rtol=1e-12)
    assert np.abs(x2 - xs).max() <= 1e-10 * np.abs(xs).max()


# ----------------------------------------------------------------- mesh validity
def test_meshes_are_valid_and_oriented():
    for k in range(1, 4):
        mesh = mg.hex_mesh(4, 0.15, config=1, seed_k=k)
        op = oracle.OracleOp(mg.hex_space(mesh, k), oracle.OP_MASS)
        assert op.detj().min() > 0
    mesh = mg.tet_mesh(4, 0.2, config=2)
    op = oracle.OracleOp(mg.tet_space(mesh, 1, ncomp=1), oracle.OP_MASS)
    dj = op.detj()
    assert np.abs(dj).min() > 0
