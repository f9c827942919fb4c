"""Seeded synthetic inputs: meshes, cell-to-node maps, fields.

This module holds topology and random numbers only -- no quadrature, no basis
functions, no geometry of the finite element method. Both the CPU oracle and
the GPU library consume what it returns, so nothing here may compute a piece
of the operator action.

Conventions (shared by every consumer, stated once here):

* Hex cells: reference cell [0,1]^3, vertex v has reference position
  (v & 1, (v >> 1) & 1, (v >> 2) & 1).  Q_k nodes of a cell are ordered
  lexicographically, first coordinate fastest: local id = i + n*j + n*n*l with
  n = k+1.
* Tet cells: vertex list (v0, v1, v2, v3) maps to reference vertices (0,0,0),
  (1,0,0), (0,1,0), (0,0,1).  P_k nodes are the lattice points alpha/k with
  a1+a2+a3 <= k, ordered with a1 fastest, then a2, then a3.
* Tri cells: vertex list (v0, v1, v2) maps to (0,0), (1,0), (0,1); P1 nodes are
  the vertices.
* Vector fields are node-interleaved: dof = ncomp*node + component.

Random streams follow numpy ``default_rng([config, purpose, k])`` with purpose
0 perturbation, 1 permutation, 2 input vector, 3 coefficient, 4 right-hand
side, 5 random field.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from itertools import permutations

import numpy as np

CELL_TRI, CELL_TET, CELL_HEX, CELL_QUAD = 0, 1, 2, 3
PURPOSE_PERTURB, PURPOSE_PERM, PURPOSE_X, PURPOSE_COEF, PURPOSE_RHS, PURPOSE_GRF = range(6)


def rng(config: int, purpose: int, k: int = 0) -> np.random.Generator:
    return np.random.default_rng([int(config), int(purpose), int(k)])


@dataclass
class Mesh:
    cell_type: int
    coords: np.ndarray  # (nverts, gdim) float64
    cell2vert: np.ndarray  # (ncells, nv) int32
    lattice_m: int = 0  # cells per direction of the structured lattice
    vert_ijk: np.ndarray | None = None  # (nverts, gdim) int lattice index of each vertex

    @property
    def gdim(self) -> int:
        return self.coords.shape[1]

    @property
    def nverts(self) -> int:
        return self.coords.shape[0]

    @property
    def ncells(self) -> int:
        return self.cell2vert.shape[0]


@dataclass
class Space:
    mesh: Mesh
    degree: int
    ncomp: int
    cell2node: np.ndarray  # (ncells, D) int32, in user numbering
    nnodes: int
    node_ijk: np.ndarray | None = None  # (nnodes, gdim) lattice index of each node (user numbering)
    perm: np.ndarray | None = field(default=None)  # lattice id -> user node id

    @property
    def ndofs(self) -> int:
        return self.nnodes * self.ncomp

    def boundary_nodes(self) -> np.ndarray:
        """Nodes on the boundary of the unit cube/square, found from lattice indices."""
        mk = self.mesh.lattice_m * self.degree
        ijk = self.node_ijk
        return np.nonzero(np.any((ijk == 0) | (ijk == mk), axis=1))[0].astype(np.int32)


def _perturb(ijk: np.ndarray, m: int, amp: float, g: np.random.Generator) -> np.ndarray:
    """Lattice positions ijk/m moved by U(-amp*h, amp*h) per coordinate.

    A coordinate is moved only where its lattice index is interior, so boundary
    vertices slide tangentially and the domain stays the unit cube/square."""
    h = 1.0 / m
    x = ijk.astype(np.float64) * h
    if amp > 0:
        d = g.uniform(-amp * h, amp * h, size=x.shape)
        interior = (ijk > 0) & (ijk < m)
        x = x + np.where(interior, d, 0.0)
    return x


def _lattice(m: int, gdim: int) -> np.ndarray:
    """(m+1)^gdim lattice indices, first coordinate fastest."""
    n = m + 1
    idx = np.arange(n ** gdim, dtype=np.int64)
    cols = []
    for _ in range(gdim):
        cols.append(idx % n)
        idx = idx // n
    return np.stack(cols, axis=1)


def hex_mesh(m: int, perturb: float = 0.0, config: int = 1, seed_k: int = 0) -> Mesh:
    ijk = _lattice(m, 3)
    coords = _perturb(ijk, m, perturb, rng(config, PURPOSE_PERTURB, seed_k))
    c = np.arange(m)
    cz, cy, cx = np.meshgrid(c, c, c, indexing="ij")
    cx, cy, cz = cx.ravel(), cy.ravel(), cz.ravel()
    M = m + 1
    c2v = np.empty((m ** 3, 8), dtype=np.int32)
    for v in range(8):
        dx, dy, dz = v & 1, (v >> 1) & 1, (v >> 2) & 1
        c2v[:, v] = (cx + dx) + M * ((cy + dy) + M * (cz + dz))
    return Mesh(CELL_HEX, coords, c2v, m, ijk)


def hex_space(mesh: Mesh, k: int, ncomp: int = 1, renumber: bool = True,
              config: int = 1, seed_k: int | None = None) -> Space:
    m = mesh.lattice_m
    n = k + 1
    G = m * k + 1
    lat_ijk = _lattice(m * k, 3)
    c = np.arange(m)
    cz, cy, cx = np.meshgrid(c, c, c, indexing="ij")
    cx, cy, cz = cx.ravel(), cy.ravel(), cz.ravel()
    base = (cx * k) + G * ((cy * k) + G * (cz * k))
    loc = _lattice(k, 3)  # local node (i, j, l), i fastest
    off = loc[:, 0] + G * (loc[:, 1] + G * loc[:, 2])
    c2n = base[:, None] + off[None, :]
    nn = G ** 3
    perm = _permutation(nn, renumber, config, k if seed_k is None else seed_k)
    c2n = perm[c2n]
    node_ijk = np.empty_like(lat_ijk)
    node_ijk[perm] = lat_ijk
    return Space(mesh, k, ncomp, c2n.astype(np.int32), nn, node_ijk, perm)


def quad_mesh(m: int, perturb: float = 0.0, config: int = 0, seed_k: int = 0) -> Mesh:
    """Unit square, m x m bilinear quadrilaterals; vertex v of a cell at (v & 1, v >> 1)."""
    ij = _lattice(m, 2)
    coords = _perturb(ij, m, perturb, rng(config, PURPOSE_PERTURB, seed_k))
    c = np.arange(m)
    cy, cx = np.meshgrid(c, c, indexing="ij")
    cx, cy = cx.ravel(), cy.ravel()
    M = m + 1
    c2v = np.empty((m * m, 4), dtype=np.int32)
    for v in range(4):
        c2v[:, v] = (cx + (v & 1)) + M * (cy + (v >> 1))
    return Mesh(CELL_QUAD, coords, c2v, m, ij)


def quad_space(mesh: Mesh, k: int, renumber: bool = True, config: int = 0,
               seed_k: int | None = None, ncomp: int = 1) -> Space:
    """Q_k nodes: the k-refined lattice; local node (i, j), i fastest."""
    m = mesh.lattice_m
    G = m * k + 1
    c = np.arange(m)
    cy, cx = np.meshgrid(c, c, indexing="ij")
    base = cx.ravel() * k + G * (cy.ravel() * k)
    loc = _lattice(k, 2)
    c2n = base[:, None] + (loc[:, 0] + G * loc[:, 1])[None, :]
    nn = G * G
    perm = _permutation(nn, renumber, config, k if seed_k is None else seed_k)
    lat_ij = _lattice(m * k, 2)
    node_ij = np.empty_like(lat_ij)
    node_ij[perm] = lat_ij
    return Space(mesh, k, ncomp, perm[c2n].astype(np.int32), nn, node_ij, perm)


def _permutation(nn: int, renumber: bool, config: int, k: int) -> np.ndarray:
    if renumber:
        return rng(config, PURPOSE_PERM, k).permutation(nn).astype(np.int64)
    return np.arange(nn, dtype=np.int64)


# Kuhn (Freudenthal) split of the unit cube: one tet per permutation of the axes.
_KUHN = list(permutations(range(3)))


def tet_mesh(m: int, perturb: float = 0.0, config: int = 2, seed_k: int = 0) -> Mesh:
    ijk = _lattice(m, 3)
    coords = _perturb(ijk, m, perturb, rng(config, PURPOSE_PERTURB, seed_k))
    c = np.arange(m)
    cz, cy, cx = np.meshgrid(c, c, c, indexing="ij")
    base = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)
    M = m + 1
    cells = []
    for sigma in _KUHN:
        p = base.copy()
        vs = [p.copy()]
        for ax in sigma:
            p = p.copy()
            p[:, ax] += 1
            vs.append(p)
        cells.append(np.stack([v[:, 0] + M * (v[:, 1] + M * v[:, 2]) for v in vs], axis=1))
    c2v = np.stack(cells, axis=1).reshape(-1, 4).astype(np.int32)
    return Mesh(CELL_TET, coords, c2v, m, ijk)


def simplex_lattice(k: int, dim: int) -> np.ndarray:
    """Multi-indices alpha (|alpha| <= k) in the local node order of the conventions."""
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


def tet_space(mesh: Mesh, k: int, ncomp: int = 3, renumber: bool = True,
              config: int = 2, seed_k: int | None = None) -> Space:
    """P_k nodes of Kuhn tets are exactly the points of the k-refined lattice."""
    m = mesh.lattice_m
    G = m * k + 1
    vij = mesh.vert_ijk[mesh.cell2vert]  # (ncells, 4, 3)
    alpha = simplex_lattice(k, 3)  # (D, 3)
    # integer lattice position (refined) of each local node: k*v0 + sum_a alpha_a (v_a - v0)
    v0 = vij[:, 0, :]
    pos = k * v0[:, None, :] + np.einsum("da,cae->cde", alpha, vij[:, 1:, :] - v0[:, None, :])
    lat = pos[..., 0] + G * (pos[..., 1] + G * pos[..., 2])
    nn = G ** 3
    perm = _permutation(nn, renumber, config, k if seed_k is None else seed_k)
    lat_ijk = _lattice(m * k, 3)
    node_ijk = np.empty_like(lat_ijk)
    node_ijk[perm] = lat_ijk
    return Space(mesh, k, ncomp, perm[lat].astype(np.int32), nn, node_ijk, perm)


def tri_mesh(m: int, perturb: float = 0.0, config: int = 0) -> Mesh:
    """Unit square, m x m squares, each split along (i,j)->(i+1,j+1)."""
    ijk = _lattice(m, 2)
    coords = _perturb(ijk, m, perturb, rng(config, PURPOSE_PERTURB, 0))
    c = np.arange(m)
    cy, cx = np.meshgrid(c, c, indexing="ij")
    cx, cy = cx.ravel(), cy.ravel()
    M = m + 1
    v00 = cx + M * cy
    v10, v01, v11 = v00 + 1, v00 + M, v00 + M + 1
    t1 = np.stack([v00, v10, v11], axis=1)
    t2 = np.stack([v00, v11, v01], axis=1)
    c2v = np.stack([t1, t2], axis=1).reshape(-1, 3).astype(np.int32)
    return Mesh(CELL_TRI, coords, c2v, m, ijk)


def tri_p1_space(mesh: Mesh, renumber: bool = False, config: int = 0) -> Space:
    nn = mesh.nverts
    perm = _permutation(nn, renumber, config, 1)
    node_ijk = np.empty_like(mesh.vert_ijk)
    node_ijk[perm] = mesh.vert_ijk
    return Space(mesh, 1, 1, perm[mesh.cell2vert].astype(np.int32), nn, node_ijk, perm)


def tri_space(mesh: Mesh, k: int, renumber: bool = True, config: int = 0, seed_k: int | None = None,
              ncomp: int = 1) -> Space:
    """P_k nodes of the split squares are exactly the points of the k-refined lattice."""
    m = mesh.lattice_m
    G = m * k + 1
    vij = mesh.vert_ijk[mesh.cell2vert]  # (ncells, 3, 2)
    alpha = simplex_lattice(k, 2)  # (D, 2)
    v0 = vij[:, 0, :]
    pos = k * v0[:, None, :] + np.einsum("da,cae->cde", alpha, vij[:, 1:, :] - v0[:, None, :])
    lat = pos[..., 0] + G * pos[..., 1]
    nn = G ** 2
    perm = _permutation(nn, renumber, config, k if seed_k is None else seed_k)
    lat_ij = _lattice(m * k, 2)
    node_ijk = np.empty_like(lat_ij)
    node_ijk[perm] = lat_ij
    return Space(mesh, k, ncomp, perm[lat].astype(np.int32), nn, node_ijk, perm)


def uniform(n: int, lo: float, hi: float, config: int, purpose: int, k: int = 0) -> np.ndarray:
    return rng(config, purpose, k).uniform(lo, hi, size=n)


def gaussian_random_field(nverts_ijk: np.ndarray, m: int, ell: float = 0.1,
                          grid: int = 128, period: float = 1.5, config: int = 4) -> np.ndarray:
    """Smoothed Gaussian random field sampled at lattice vertices.

    White noise on a periodic grid^3 over [0, period)^3 is filtered in Fourier
    space to the squared-exponential covariance exp(-r^2 / (2 ell^2)), then
    normalised to sample mean 0 and standard deviation 1 over the grid.  The
    field is evaluated at the unit-cube lattice vertices ijk/m by trilinear
    interpolation of the grid."""
    g = rng(config, PURPOSE_GRF, 0)
    w = g.standard_normal((grid, grid, grid))
    h = period / grid
    f = np.fft.fftfreq(grid, d=h) * 2 * np.pi
    kx, ky, kz = np.meshgrid(f, f, f, indexing="ij")
    k2 = kx ** 2 + ky ** 2 + kz ** 2
    # spectral density of exp(-r^2/(2 l^2)) is proportional to exp(-l^2 k^2 / 2);
    # filtering white noise by its square root gives that covariance.
    filt = np.exp(-0.25 * ell ** 2 * k2)
    field = np.real(np.fft.ifftn(np.fft.fftn(w) * filt))
    field = (field - field.mean()) / field.std()
    p = nverts_ijk.astype(np.float64) / m / h  # grid coordinates
    i0 = np.floor(p).astype(np.int64)
    t = p - i0
    out = np.zeros(p.shape[0])
    for corner in range(8):
        o = np.array([(corner >> d) & 1 for d in range(3)])
        wgt = np.prod(np.where(o == 1, t, 1 - t), axis=1)
        idx = (i0 + o) % grid
        out += wgt * field[idx[:, 0], idx[:, 1], idx[:, 2]]
    return out
