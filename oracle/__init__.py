"""CPU FP64 oracle for the matrix-free finite element operator action.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. The GPU library
(``paper_1903_08243_amd``) never imports it, and it imports nothing from the
GPU library except the seeded input generators (``meshgen``), which contain
no arithmetic of the method.

Contents
--------
* ``tables``       quadrature rules and dense basis tabulations (numpy)
* ``oracle.c``     the cell loop: gather, local kernel at quadrature points,
                   scatter (plain C, OpenMP over cells with private outputs)
* ``OracleOp``     y = A x, diag(A), element matrices, dense assembly (tiny meshes)
* ``cg``           textbook (preconditioned) conjugate gradients in FP64
* ``conv``         direct conv3d forward / backward for the learned preconditioner

Every function cites the passage of the paper it follows. Parity of the FP32
GPU paths is checked only against this FP64 oracle (parity of FP32 otherwise
unpinned).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import tables

OP_MASS, OP_HELMHOLTZ, OP_LAPLACIAN, OP_POISSON, OP_ELASTICITY = range(5)
# St-Venant-Kirchhoff: tangent at a field u0 (bilinear in the trial field) and the
# nonlinear residual form itself (supplementary operator list, "hyperelasticity")
OP_HYPERELASTIC, OP_HYPER_RESIDUAL = 5, 6
CELL_TRI, CELL_TET, CELL_HEX, CELL_QUAD = 0, 1, 2, 3

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle's C cell loop with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               os.path.join(_HERE, "oracle.c"), "-o", _LIB_PATH, "-lm"])
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        _lib = ctypes.CDLL(_LIB_PATH)
        common = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                  ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                  ctypes.c_double, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
        _lib.oracle_apply.argtypes = common + [ctypes.c_long, ctypes.c_long, ctypes.c_long,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        _lib.oracle_diagonal.argtypes = common + [ctypes.c_long, ctypes.c_long, ctypes.c_void_p,
                                                  ctypes.c_int]
        _lib.oracle_element_matrices.argtypes = common + [ctypes.c_long, ctypes.c_void_p]
        _lib.oracle_detj.argtypes = common + [ctypes.c_long, ctypes.c_void_p]
        for f in (_lib.oracle_apply, _lib.oracle_diagonal, _lib.oracle_element_matrices,
                  _lib.oracle_detj):
            f.restype = ctypes.c_int
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


def simplex_quad_degree(kind: int, k: int, has_coef: bool) -> int:
    """Polynomial degree of the integrand on an affine simplex (so that the
    collapsed rule integrates it exactly and the result is rule-independent)."""
    c = 1 if has_coef else 0
    if kind in (OP_HYPERELASTIC, OP_HYPER_RESIDUAL):
        # grad u0 has degree k-1, S degree 2(k-1), dF S and F dS degree 3(k-1), times grad v
        return 4 * (k - 1)
    if kind == OP_MASS:
        return 2 * k + c
    if kind == OP_HELMHOLTZ:
        return 2 * k
    return max(0, 2 * k - 2) + (c if kind == OP_POISSON else 0)


class OracleOp:
    """Dense-tabulation FP64 operator (Section 2.1 local kernel, Section 2.2 loop).

    mesh/space come from ``paper_1903_08243_amd.meshgen``. ``coef`` is a
    per-vertex coefficient (mass: c, Poisson: kappa). Hex cells use the tensor
    Gauss rule with ``nq1d`` points per direction (default k+1); simplices use
    a collapsed Gauss rule exact for the integrand.
    """

    def __init__(self, space, kind, lam=1.0, mu=0.5, coef=None, nq1d=None, u0=None):
        mesh = space.mesh
        self.space, self.kind = space, kind
        if kind in (OP_HYPERELASTIC, OP_HYPER_RESIDUAL):
            assert mesh.cell_type in (CELL_TET, CELL_HEX) and space.ncomp == 3, "hyperelasticity: vector tets, hexes"
        if kind == OP_HYPERELASTIC:
            assert u0 is not None, "the tangent needs its linearisation point u0"
        self.lam, self.mu = float(lam), float(mu)
        k = space.degree
        if mesh.cell_type == CELL_HEX:
            qw, phi, dphi, vN, vdN = tables.hex_tables(k, nq1d or (k + 1))
        elif mesh.cell_type == CELL_QUAD:
            qw, phi, dphi, vN, vdN = tables.quad_tables(k, nq1d or (k + 1))
        else:
            dim = 2 if mesh.cell_type == CELL_TRI else 3
            qw, phi, dphi, vN, vdN = tables.simplex_tables(
                k, dim, simplex_quad_degree(kind, k, coef is not None))
        c = lambda a, t=np.float64: np.ascontiguousarray(a, dtype=t)
        self.qw, self.phi, self.dphi, self.vN, self.vdN = c(qw), c(phi), c(dphi), c(vN), c(vdN)
        self.coords = c(mesh.coords)
        self.c2v = c(mesh.cell2vert, np.int32)
        self.c2n = c(space.cell2node, np.int32)
        self.coef = None if coef is None else c(coef)
        self.u0 = None if u0 is None else c(u0)
        self.gdim, self.nvc = mesh.gdim, mesh.cell2vert.shape[1]
        self.D, self.ncomp = self.c2n.shape[1], space.ncomp
        self.nq = self.qw.shape[0]
        self.ncells = self.c2n.shape[0]
        self.ndofs = space.nnodes * space.ncomp

    def _common(self):
        return (self.gdim, self.nvc, _ptr(self.coords), _ptr(self.c2v), self.D, _ptr(self.c2n),
                self.ncomp, self.nq, _ptr(self.qw), _ptr(self.vN), _ptr(self.vdN), _ptr(self.phi),
                _ptr(self.dphi), self.kind, self.lam, self.mu, _ptr(self.coef), _ptr(self.u0))

    def apply(self, x, cells=None, nthreads=None):
        """y = A x (overwrites), optionally over the cell range [start, end) only. For
        OP_HYPER_RESIDUAL, y is the residual vector r(x; phi_i) (nonlinear in x)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        assert x.shape == (self.ndofs,)
        y = np.empty(self.ndofs)
        c0, c1 = (0, self.ncells) if cells is None else cells
        rc = _load().oracle_apply(*self._common(), c0, c1, self.ndofs, _ptr(x), _ptr(y),
                                  nthreads or default_threads())
        if rc != 0:
            raise MemoryError("oracle_apply failed")
        return y

    def diagonal(self, nthreads=None):
        d = np.empty(self.ndofs)
        rc = _load().oracle_diagonal(*self._common(), self.ncells, self.ndofs, _ptr(d),
                                     nthreads or default_threads())
        if rc != 0:
            raise MemoryError("oracle_diagonal failed")
        return d

    def element_matrices(self):
        n = self.D * self.ncomp
        out = np.empty((self.ncells, n, n))
        _load().oracle_element_matrices(*self._common(), self.ncells, _ptr(out))
        return out

    def detj(self):
        out = np.empty((self.ncells, self.nq))
        _load().oracle_detj(*self._common(), self.ncells, _ptr(out))
        return out

    def dof_map(self):
        """Cell-to-DoF map (ncells, D*ncomp): dof = ncomp*node + component."""
        nc = self.ncomp
        return (self.c2n[:, :, None].astype(np.int64) * nc + np.arange(nc)).reshape(self.ncells, -1)

    def assemble_dense(self):
        """Global matrix from element matrices (tiny meshes only)."""
        A = np.zeros((self.ndofs, self.ndofs))
        Ae = self.element_matrices()
        dm = self.dof_map()
        for K in range(self.ncells):
            A[np.ix_(dm[K], dm[K])] += Ae[K]
        return A


def cg(apply, b, x0=None, rtol=1e-10, maxit=10000, precond=None):
    """Textbook preconditioned conjugate gradients in FP64.

    Stops when ||b - A x||_2 / ||b||_2 <= rtol, measured on the recurrence
    residual and confirmed on the true residual. Returns (x, iterations,
    true relative residual)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply(x)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0, 0.0
    z = r if precond is None else precond(r)
    p = z.copy()
    rz = r @ z
    it = 0
    while it < maxit:
        if np.linalg.norm(r) / nb <= rtol:
            tr = np.linalg.norm(b - apply(x)) / nb
            if tr <= rtol:
                return x, it, tr
            r = b - apply(x)  # refresh drifted recurrence residual
            z = r if precond is None else precond(r)
            p = z.copy()
            rz = r @ z
        Ap = apply(p)
        alpha = rz / (p @ Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        z = r if precond is None else precond(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    return x, it, np.linalg.norm(b - apply(x)) / nb
