"""Oracle tables: quadrature rules and densely tabulated basis functions.

TEST INFRASTRUCTURE. Only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the product library never does.

Everything here is the plain textbook definition, evaluated densely in FP64:

* Gauss-Legendre rules come from numpy's ``leggauss`` (a library primitive).
* Gauss-Lobatto-Legendre nodes of degree k are the end points and the roots of
  the derivative of the Legendre polynomial P_k (numpy polynomial roots).
* 1D Lagrange polynomials are products over the other nodes.
* Hex Q_k basis functions are products of 1D Lagrange polynomials, tabulated at
  every point of the tensor quadrature -- no sum factorisation.  The paper's
  element kernel likewise tabulates basis values and derivatives at quadrature
  points (Section 2.1, Listing 2: arrays of weights, basis values and basis
  derivatives shared by all elements).
* Simplex P_k Lagrange functions on the equispaced lattice use the barycentric
  product formula phi_alpha = prod_j prod_{m<alpha_j} (k*lambda_j - m)/(m+1).
* Simplex quadrature is the collapsed (Duffy) product of Gauss-Legendre rules,
  exact for polynomials of the requested degree.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import legendre as npleg


def gauss_legendre01(n: int):
    """n-point Gauss-Legendre rule on [0,1]: exact for degree <= 2n-1."""
    x, w = npleg.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def gll_nodes01(k: int) -> np.ndarray:
    """The k+1 Gauss-Lobatto-Legendre points on [0,1] (end points + roots of P_k')."""
    if k == 1:
        return np.array([0.0, 1.0])
    inner = npleg.Legendre.basis(k).deriv().roots()
    inner = np.sort(np.real(inner))
    return 0.5 * (np.concatenate([[-1.0], inner, [1.0]]) + 1.0)


def lagrange1d(nodes: np.ndarray, pts: np.ndarray):
    """Values V[q, i] = l_i(pts[q]) and derivatives dV[q, i] = l_i'(pts[q])."""
    n = len(nodes)
    V = np.ones((len(pts), n))
    dV = np.zeros((len(pts), n))
    for i in range(n):
        for m in range(n):
            if m != i:
                V[:, i] *= (pts - nodes[m]) / (nodes[i] - nodes[m])
        for j in range(n):
            if j == i:
                continue
            term = np.full(len(pts), 1.0 / (nodes[i] - nodes[j]))
            for m in range(n):
                if m != i and m != j:
                    term *= (pts - nodes[m]) / (nodes[i] - nodes[m])
            dV[:, i] += term
    return V, dV


def hex_tables(k: int, nq1d: int):
    """Dense tabulation of the Q_k (GLL) basis and the trilinear vertex basis.

    Returns (qw[nq], phi[nq, D], dphi[nq, D, 3], vN[nq, 8], vdN[nq, 8, 3]) with
    quadrature points (a, b, c) ordered a fastest and basis (i, j, l) i fastest.
    """
    g, w = gauss_legendre01(nq1d)
    V, dV = lagrange1d(gll_nodes01(k), g)
    n = k + 1
    nq, D = nq1d ** 3, n ** 3
    qw = np.zeros(nq)
    phi = np.zeros((nq, D))
    dphi = np.zeros((nq, D, 3))
    vN = np.zeros((nq, 8))
    vdN = np.zeros((nq, 8, 3))
    for c in range(nq1d):
        for b in range(nq1d):
            for a in range(nq1d):
                q = a + nq1d * (b + nq1d * c)
                qw[q] = w[a] * w[b] * w[c]
                xi = (g[a], g[b], g[c])
                for l in range(n):
                    for j in range(n):
                        for i in range(n):
                            d = i + n * (j + n * l)
                            phi[q, d] = V[a, i] * V[b, j] * V[c, l]
                            dphi[q, d, 0] = dV[a, i] * V[b, j] * V[c, l]
                            dphi[q, d, 1] = V[a, i] * dV[b, j] * V[c, l]
                            dphi[q, d, 2] = V[a, i] * V[b, j] * dV[c, l]
                for v in range(8):
                    o = ((v & 1), (v >> 1) & 1, (v >> 2) & 1)
                    f = [xi[dd] if o[dd] else 1.0 - xi[dd] for dd in range(3)]
                    df = [1.0 if o[dd] else -1.0 for dd in range(3)]
                    vN[q, v] = f[0] * f[1] * f[2]
                    vdN[q, v, 0] = df[0] * f[1] * f[2]
                    vdN[q, v, 1] = f[0] * df[1] * f[2]
                    vdN[q, v, 2] = f[0] * f[1] * df[2]
    return qw, phi, dphi, vN, vdN


def quad_tables(k: int, nq1d: int):
    """The 2D counterpart of hex_tables: Q_k (GLL) basis and the bilinear vertex basis.

    Returns (qw[nq], phi[nq, D], dphi[nq, D, 2], vN[nq, 4], vdN[nq, 4, 2]) with
    points (a, b) ordered a fastest, basis (i, j) i fastest, vertex v at (v & 1, v >> 1).
    """
    g, w = gauss_legendre01(nq1d)
    V, dV = lagrange1d(gll_nodes01(k), g)
    n = k + 1
    nq, D = nq1d ** 2, n ** 2
    qw = np.zeros(nq)
    phi = np.zeros((nq, D))
    dphi = np.zeros((nq, D, 2))
    vN = np.zeros((nq, 4))
    vdN = np.zeros((nq, 4, 2))
    for b in range(nq1d):
        for a in range(nq1d):
            q = a + nq1d * b
            qw[q] = w[a] * w[b]
            xi = (g[a], g[b])
            for j in range(n):
                for i in range(n):
                    d = i + n * j
                    phi[q, d] = V[a, i] * V[b, j]
                    dphi[q, d, 0] = dV[a, i] * V[b, j]
                    dphi[q, d, 1] = V[a, i] * dV[b, j]
            for v in range(4):
                o = (v & 1, v >> 1)
                f = [xi[dd] if o[dd] else 1.0 - xi[dd] for dd in range(2)]
                df = [1.0 if o[dd] else -1.0 for dd in range(2)]
                vN[q, v] = f[0] * f[1]
                vdN[q, v, 0] = df[0] * f[1]
                vdN[q, v, 1] = f[0] * df[1]
    return qw, phi, dphi, vN, vdN


def simplex_lattice(k: int, dim: int) -> np.ndarray:
    out = []
    if dim == 2:
        for a2 in range(k + 1):
            for a1 in range(k + 1 - a2):
                out.append((a1, a2))
    else:
        for a3 in range(k + 1):
            for a2 in range(k + 1 - a3):
                for a1 in range(k + 1 - a2 - a3):
                    out.append((a1, a2, a3))
    return np.array(out, dtype=np.int64)


def simplex_lagrange(k: int, dim: int, pts: np.ndarray):
    """Equispaced P_k Lagrange basis on the reference simplex.

    pts[q, :dim] are reference coordinates xi; lambda_0 = 1 - sum(xi),
    lambda_d = xi_d.  Returns phi[q, D], dphi[q, D, dim]."""
    alpha = simplex_lattice(k, dim)
    nq, D = pts.shape[0], alpha.shape[0]
    lam = np.concatenate([1.0 - pts.sum(axis=1, keepdims=True), pts], axis=1)  # (nq, dim+1)
    dlam = np.zeros((dim + 1, dim))
    dlam[0, :] = -1.0
    for d in range(dim):
        dlam[d + 1, d] = 1.0
    phi = np.zeros((nq, D))
    dphi = np.zeros((nq, D, dim))
    for i in range(D):
        full = np.concatenate([[k - alpha[i].sum()], alpha[i]])
        # factors: list of (barycentric index j, offset m)
        factors = [(j, m) for j in range(dim + 1) for m in range(full[j])]
        val = np.ones(nq)
        for (j, m) in factors:
            val *= (k * lam[:, j] - m) / (m + 1)
        phi[:, i] = val
        for f_idx, (j, m) in enumerate(factors):
            term = np.full(nq, k / (m + 1.0))
            for g_idx, (jj, mm) in enumerate(factors):
                if g_idx != f_idx:
                    term *= (k * lam[:, jj] - mm) / (mm + 1)
            dphi[:, i, :] += term[:, None] * dlam[j][None, :]
    return phi, dphi


def collapsed_rule(dim: int, degree: int):
    """Duffy-collapsed Gauss-Legendre rule on the reference simplex.

    tri: xi = (s, (1-s) t), weight (1-s);  tet: xi = (s, (1-s) t, (1-s)(1-t) r),
    weight (1-s)^2 (1-t).  n points per direction with 2n-1 >= degree + dim - 1
    make it exact for polynomials of total degree <= degree."""
    n = max(1, math.ceil((degree + dim) / 2))
    g, w = gauss_legendre01(n)
    pts, wts = [], []
    if dim == 2:
        for a in range(n):
            for b in range(n):
                s, t = g[a], g[b]
                pts.append((s, (1 - s) * t))
                wts.append(w[a] * w[b] * (1 - s))
    else:
        for a in range(n):
            for b in range(n):
                for c in range(n):
                    s, t, r = g[a], g[b], g[c]
                    pts.append((s, (1 - s) * t, (1 - s) * (1 - t) * r))
                    wts.append(w[a] * w[b] * w[c] * (1 - s) ** 2 * (1 - t))
    return np.array(pts), np.array(wts)


def simplex_tables(k: int, dim: int, degree: int):
    """Dense P_k basis and affine vertex basis at a collapsed rule of the given degree."""
    pts, qw = collapsed_rule(dim, degree)
    phi, dphi = simplex_lagrange(k, dim, pts)
    vN, vdN = simplex_lagrange(1, dim, pts)
    return qw, phi, dphi, vN, vdN
