"""Assembled sparse matrix (CSR, user numbering) against the oracle: the pattern
bit-exact against its definition (an entry for every pair of dofs whose nodes share a
cell), the values against the oracle's dense assembly of its element matrices, and the
assembled matrix-vector product against the matrix-free action at a larger size."""
import numpy as np
import pytest

import oracle
from paper_1903_08243_amd import meshgen as mg

pytestmark = pytest.mark.gpu
TOL = {0: 1e-12, 1: 1e-5}
MASS, HELM, LAP, POIS, ELAS = 0, 1, 2, 3, 4


@pytest.fixture(scope="module")
def mf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1903_08243_amd as m
    m.load_library()
    return m


def _pattern(c2n, nnodes, nc):
    """CSR pattern by definition: sorted, duplicate-free columns per row."""
    rows = [set() for _ in range(nnodes)]
    for cell in c2n:
        for a in cell:
            rows[a].update(int(b) for b in cell)
    rowptr, col = [0], []
    for n in range(nnodes):
        cols = sorted(rows[n])
        for c in range(nc):
            col.extend(m * nc + d for m in cols for d in range(nc))
            rowptr.append(len(col))
    return np.array(rowptr, np.int64), np.array(col, np.int32)


def _dense(rowptr, col, vals, n):
    A = np.zeros((n, n))
    for r in range(n):
        A[r, col[rowptr[r]:rowptr[r + 1]]] = vals[rowptr[r]:rowptr[r + 1]]
    return A


def _tet(k, nc, m=3):
    mesh = mg.tet_mesh(m, 0.2, config=2, seed_k=k)  # 162 cells
    space = mg.tet_space(mesh, k, ncomp=nc, config=2, seed_k=k)
    return mesh, space


KINDS = ((MASS, False), (MASS, True), (HELM, False), (LAP, False), (POIS, True), (ELAS, False))
CASES = ([("tet", k, kind, coef) for k in (1, 2, 3) for kind, coef in KINDS]
         + [("tri", k, kind, coef) for k in (1, 2, 3) for kind, coef in KINDS]
         + [("quad", k, kind, coef) for k in (1, 2, 4) for kind, coef in KINDS]
         + [("hex", k, kind, coef) for k in (1, 2, 3) for kind, coef in KINDS])


def _space(cell, k, kind):
    if cell == "tet":
        return _tet(k, 3 if kind == ELAS else 1)
    if cell == "tri":
        mesh = mg.tri_mesh(9, 0.2, config=0)  # 162 cells
        if k == 1 and kind != ELAS:
            return mesh, mg.tri_p1_space(mesh, renumber=True)
        return mesh, mg.tri_space(mesh, k, seed_k=k, ncomp=2 if kind == ELAS else 1)
    if cell == "quad":
        mesh = mg.quad_mesh(5, 0.25, config=0)
        return mesh, mg.quad_space(mesh, k, ncomp=2 if kind == ELAS else 1)
    mesh = mg.hex_mesh(3, 0.15, config=1, seed_k=k)
    return mesh, mg.hex_space(mesh, k, ncomp=3 if kind == ELAS else 1, config=1)


@pytest.mark.parametrize("dirichlet", [False, True])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("cell,k,kind,coef", CASES)
def test_csr_matches_oracle_assembly(mf, cell, k, kind, coef, prec, dirichlet):
    print(f"csr {cell} k={k} kind={kind} coef={coef} prec={prec} dirichlet={dirichlet}", flush=True)
    mesh, space = _space(cell, k, kind)
    c = np.exp(np.random.default_rng(k).normal(size=mesh.nverts)) if coef else None
    mask = None
    bnd = np.zeros(0, np.int64)
    if dirichlet:
        bnd = space.boundary_nodes()
        mask = np.zeros(space.nnodes, np.uint8)
        mask[bnd] = 1
    op = mf.Operator(mf.Space.from_meshgen(space), kind, prec, vertex_coef=c, lam=1.0, mu=0.5, dirichlet=mask)
    rowptr, col, vals = op.csr()
    nc = space.ncomp
    rp_ref, col_ref = _pattern(np.asarray(space.cell2node), space.nnodes, nc)
    assert np.array_equal(rowptr, rp_ref) and np.array_equal(col, col_ref)
    A = _dense(rowptr, col, vals.double().cpu().numpy(), space.ndofs)
    ref = oracle.OracleOp(space, kind, lam=1.0, mu=0.5, coef=c).assemble_dense()
    if dirichlet:
        cd = (bnd[:, None] * nc + np.arange(nc)).ravel()
        ref[cd, :] = 0.0
        ref[:, cd] = 0.0
        ref[cd, cd] = 1.0
    assert np.abs(A - ref).max() <= TOL[prec] * np.abs(ref).max()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("k,kind,nc", [(2, ELAS, 3), (3, POIS, 1), (1, HELM, 1)])
def test_csr_matvec_equals_action(mf, k, kind, nc, prec):
    """At 12^3 x 6 tets (10368 cells) the assembled
    product A x equals the matrix-free action; the pattern is checked by definition."""
    import torch
    print(f"csr matvec k={k} kind={kind} prec={prec}", flush=True)
    mesh = mg.tet_mesh(12, 0.2, config=2, seed_k=k)
    space = mg.tet_space(mesh, k, ncomp=nc, config=2, seed_k=k)
    c = np.exp(np.random.default_rng(k).normal(size=mesh.nverts)) if kind == POIS else None
    op = mf.Operator(mf.Space.from_meshgen(space), kind, prec, vertex_coef=c, lam=1.0, mu=0.5)
    rowptr, col, vals = op.csr()
    rp_ref, col_ref = _pattern(np.asarray(space.cell2node), space.nnodes, nc)
    assert np.array_equal(rowptr, rp_ref) and np.array_equal(col, col_ref)
    x = mg.uniform(space.ndofs, -1, 1, 2, mg.PURPOSE_X, k)
    y = op.apply(torch.tensor(x, device="cuda", dtype=op.torch_dtype)).double().cpu().numpy()
    v = vals.double().cpu().numpy()
    rows = np.repeat(np.arange(space.ndofs), np.diff(rowptr))
    ax = np.bincount(rows, weights=v * x[col], minlength=space.ndofs)
    assert np.abs(ax - y).max() <= 4 * TOL[prec] * np.abs(y).max()


@pytest.mark.parametrize("prec", [0, 1])
def test_csr_matvec_equals_action_hex(mf, prec):
    """Q2 Helmholtz on 16^3 perturbed hexes with the paper's k+2 points: A x against the
    matrix-free action (coloured scatter)."""
    import torch
    mesh = mg.hex_mesh(16, 0.15, config=1, seed_k=2)
    space = mg.hex_space(mesh, 2, config=1)
    op = mf.Operator(mf.Space.from_meshgen(space), HELM, prec, nq1d=4)
    rowptr, col, vals = op.csr()
    x = mg.uniform(space.ndofs, -1, 1, 1, mg.PURPOSE_X, 2)
    y = op.apply(torch.tensor(x, device="cuda", dtype=op.torch_dtype)).double().cpu().numpy()
    v = vals.double().cpu().numpy()
    rows = np.repeat(np.arange(space.ndofs), np.diff(rowptr))
    ax = np.bincount(rows, weights=v * x[col], minlength=space.ndofs)
    assert np.abs(ax - y).max() <= 4 * TOL[prec] * np.abs(y).max()


def test_csr_unsupported_operators(mf):
    mesh = mg.hex_mesh(2, 0.1, config=3)
    op = mf.Operator(mf.Space.from_meshgen(mg.hex_space(mesh, 5, config=3)), HELM, 0)
    with pytest.raises(mf.MFError, match="assembly"):
        op.csr()
    tm = mg.tet_mesh(2, 0.2, config=2)
    ts = mg.tet_space(tm, 1, ncomp=3, config=2)
    u0 = 0.1 * mg.uniform(ts.ndofs, -1, 1, 2, mg.PURPOSE_COEF, 1)
    with pytest.raises(mf.MFError, match="assembly"):
        mf.Operator(mf.Space.from_meshgen(ts), mf.HYPERELASTIC, 0, u0=u0).csr()


def test_csr_rejects_another_space(mf):
    import ctypes
    mesh = mg.tet_mesh(2, 0.2, config=2)
    space = mg.tet_space(mesh, 1, ncomp=1, config=2)
    op = mf.Operator(mf.Space.from_meshgen(space), HELM, 0)
    other = mf.Space.from_meshgen(space)
    nnz = ctypes.c_int64()
    L = mf.load_library()
    assert L.mf_op_csr_pattern(op.handle, other.handle, None, None, ctypes.byref(nnz)) != 0
    assert "not created on this space" in L.mf_last_error().decode()
