"""GPU parity of the operators on Q1..Q6 quadrilaterals (mass with and without a vertex
coefficient, Helmholtz, Laplacian, Poisson, 2D elasticity) against the oracle, through
the C-ABI: both scatter modes, both precisions, k+1 and k+2 Gauss points per direction,
Dirichlet rows, range applies, a ragged cell count and sampled outputs at 1024^2 cells."""
import numpy as np
import pytest

import oracle
from paper_1903_08243_amd import meshgen as mg

pytestmark = pytest.mark.gpu
TOL = {0: 1e-12, 1: 1e-5}
MASS, HELM, LAP, POIS = 0, 1, 2, 3


@pytest.fixture(scope="module")
def mf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1903_08243_amd as m
    m.load_library()
    return m


def _relerr(y, ref):
    return np.abs(y - ref).max() / np.abs(ref).max()


def _case(k, m=11):
    # 121 cells: not a multiple of the 16 / 7 / 4 / 2 cells a workgroup holds
    mesh = mg.quad_mesh(m, 0.25, config=0)
    space = mg.quad_space(mesh, k, seed_k=k)
    x = mg.uniform(space.ndofs, -1, 1, 0, mg.PURPOSE_X, k)
    c = np.exp(np.random.default_rng(k).normal(size=mesh.nverts))
    return mesh, space, x, c


@pytest.mark.parametrize("scatter", [1, 2], ids=["atomic", "coloured"])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind,coef", [(MASS, False), (MASS, True), (HELM, False), (LAP, False), (POIS, True)],
                         ids=["mass", "mass-coef", "helmholtz", "laplacian", "poisson"])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_quad_action(mf, k, kind, coef, prec, scatter):
    import torch
    print(f"quad k={k} kind={kind} coef={coef} prec={prec} scatter={scatter}", flush=True)
    mesh, space, x, c = _case(k)
    c = c if coef else None
    ref = oracle.OracleOp(space, kind, coef=c).apply(x)
    op = mf.Operator(mf.Space.from_meshgen(space), kind, prec, vertex_coef=c, scatter=scatter)
    assert op.info["nqp"] == (k + 1) ** 2
    y = op.apply(torch.tensor(x, device="cuda", dtype=op.torch_dtype)).double().cpu().numpy()
    assert _relerr(y, ref) <= TOL[prec], _relerr(y, ref)


@pytest.mark.parametrize("k", [1, 3, 6])
def test_quad_paper_quadrature(mf, k):
    """The paper's k+2 Gauss points per direction (Q6: 8 x 8, every lane a point)."""
    import torch
    print(f"quad nq1d=k+2 k={k}", flush=True)
    mesh, space, x, c = _case(k)
    sp = mf.Space.from_meshgen(space)
    for kind, cf in ((HELM, None), (POIS, c)):
        ref = oracle.OracleOp(space, kind, coef=cf, nq1d=k + 2).apply(x)
        op = mf.Operator(sp, kind, mf.F64, nq1d=k + 2, vertex_coef=cf)
        assert op.info["nqp"] == (k + 2) ** 2
        y = op.apply(torch.tensor(x, device="cuda")).cpu().numpy()
        assert _relerr(y, ref) <= 1e-12, _relerr(y, ref)


@pytest.mark.parametrize("k", [2, 5])
def test_quad_dirichlet_range_errors(mf, k):
    import torch
    print(f"quad dirichlet/range k={k}", flush=True)
    mesh, space, x, c = _case(k)
    bnd = space.boundary_nodes()
    mask = np.zeros(space.nnodes, np.uint8)
    mask[bnd] = 1
    xm = x.copy()
    xm[bnd] = 0.0
    ref = oracle.OracleOp(space, HELM).apply(xm)
    ref[bnd] = x[bnd]
    sp = mf.Space.from_meshgen(space)
    xt = torch.tensor(x, device="cuda")
    for sc in (mf.SCATTER_ATOMIC, mf.SCATTER_COLOURED):
        op = mf.Operator(sp, HELM, mf.F64, dirichlet=mask, scatter=sc)
        assert _relerr(op.apply(xt).cpu().numpy(), ref) <= 1e-12
    lap = mf.Operator(sp, LAP, mf.F64)
    y = torch.zeros_like(xt)
    for a, b in ((0, 37), (37, 38), (38, mesh.ncells)):
        lap.apply_range(a, b, xt, y, accumulate=True)
    assert _relerr(y.cpu().numpy(), oracle.OracleOp(space, LAP).apply(x)) <= 1e-12
    # diagonal with constrained rows: 1 there
    d = mf.Operator(sp, HELM, mf.F64, dirichlet=mask).diagonal().cpu().numpy()
    dref = oracle.OracleOp(space, HELM).diagonal()
    dref[bnd] = 1.0
    assert _relerr(d, dref) <= 1e-12
    for bad in (k, k + 3):
        with pytest.raises(mf.MFError):
            mf.Operator(sp, LAP, mf.F64, nq1d=bad)
    with pytest.raises(mf.MFError):
        mf.Operator(sp, mf.ELASTICITY, mf.F64)  # one component


def test_quad_single_cell_and_tangled(mf):
    """One cell (a workgroup mostly idle) and the mesh check of a tangled cell."""
    import torch
    mesh = mg.quad_mesh(1)
    space = mg.quad_space(mesh, 3, renumber=False)
    x = mg.uniform(space.ndofs, -1, 1, 0, mg.PURPOSE_X, 3)
    ref = oracle.OracleOp(space, HELM).apply(x)
    op = mf.Operator(mf.Space.from_meshgen(space), HELM, mf.F64)
    assert _relerr(op.apply(torch.tensor(x, device="cuda")).cpu().numpy(), ref) <= 1e-12
    bad = mesh.cell2vert.copy()
    bad[0, [2, 3]] = bad[0, [3, 2]]  # bow-tie: det J changes sign inside the cell
    with pytest.raises(mf.MFError):
        mf.Mesh(mg.CELL_QUAD, mesh.coords, bad)


@pytest.mark.parametrize("k", [2, 6])
def test_quad_large_sampled(mf, k):
    """1024 x 1024 cells (Q6: 37.8 M dofs), Poisson, sampled outputs, both precisions."""
    import torch
    print(f"quad large k={k}", flush=True)
    mesh = mg.quad_mesh(1024, 0.25, config=0)
    space = mg.quad_space(mesh, k)
    x = mg.uniform(space.ndofs, -1, 1, 0, mg.PURPOSE_X, k)
    c = np.exp(np.random.default_rng(k).normal(size=mesh.nverts))
    rng = np.random.default_rng(0)
    nodes = rng.choice(space.nnodes, size=100, replace=False)
    touch = np.isin(space.cell2node, nodes).any(axis=1)
    sub = mg.Space(mg.Mesh(mesh.cell_type, mesh.coords, mesh.cell2vert[touch], mesh.lattice_m, mesh.vert_ijk),
                   k, 1, space.cell2node[touch], space.nnodes)
    ref = oracle.OracleOp(sub, POIS, coef=c).apply(x)
    sp = mf.Space.from_meshgen(space)
    for prec in (0, 1):
        op = mf.Operator(sp, POIS, prec, vertex_coef=c)
        y = op.apply(torch.tensor(x, device="cuda", dtype=op.torch_dtype)).double().cpu().numpy()
        assert np.abs(y[nodes] - ref[nodes]).max() / np.abs(ref[nodes]).max() <= TOL[prec]
        del op


@pytest.mark.parametrize("scatter", [1, 2], ids=["atomic", "coloured"])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_quad_elasticity(mf, k, prec, scatter):
    """2D linear elasticity (two node-interleaved components), lambda 0.7, mu 0.4."""
    import torch
    print(f"quad elasticity k={k} prec={prec} scatter={scatter}", flush=True)
    mesh = mg.quad_mesh(11, 0.25, config=0)
    space = mg.quad_space(mesh, k, seed_k=k, ncomp=2)
    x = mg.uniform(space.ndofs, -1, 1, 0, mg.PURPOSE_X, k)
    ref = oracle.OracleOp(space, oracle.OP_ELASTICITY, lam=0.7, mu=0.4).apply(x)
    op = mf.Operator(mf.Space.from_meshgen(space), mf.ELASTICITY, prec, lam=0.7, mu=0.4, scatter=scatter)
    y = op.apply(torch.tensor(x, device="cuda", dtype=op.torch_dtype)).double().cpu().numpy()
    assert _relerr(y, ref) <= TOL[prec], _relerr(y, ref)


@pytest.mark.parametrize("k", [2, 6])
def test_quad_elasticity_dirichlet_paper_rule(mf, k):
    """Clamped boundary (both components) with the paper's k+2 points, and a range apply."""
    import torch
    print(f"quad elasticity dirichlet k={k}", flush=True)
    mesh = mg.quad_mesh(11, 0.25, config=0)
    space = mg.quad_space(mesh, k, seed_k=k, ncomp=2)
    x = mg.uniform(space.ndofs, -1, 1, 0, mg.PURPOSE_X, k)
    bnd = space.boundary_nodes()
    mask = np.zeros(space.nnodes, np.uint8)
    mask[bnd] = 1
    bd = np.stack([2 * bnd, 2 * bnd + 1], axis=1).ravel()
    xm = x.copy()
    xm[bd] = 0.0
    ref = oracle.OracleOp(space, oracle.OP_ELASTICITY, nq1d=k + 2).apply(xm)
    ref[bd] = x[bd]
    sp = mf.Space.from_meshgen(space)
    xt = torch.tensor(x, device="cuda")
    op = mf.Operator(sp, mf.ELASTICITY, mf.F64, nq1d=k + 2, dirichlet=mask)
    assert _relerr(op.apply(xt).cpu().numpy(), ref) <= 1e-12
    op = mf.Operator(sp, mf.ELASTICITY, mf.F64)
    y = torch.zeros_like(xt)
    for a, b in ((0, 60), (60, mesh.ncells)):
        op.apply_range(a, b, xt, y, accumulate=True)
    assert _relerr(y.cpu().numpy(), oracle.OracleOp(space, oracle.OP_ELASTICITY).apply(x)) <= 1e-12


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind", [MASS, HELM, LAP, POIS, 4], ids=["mass", "helmholtz", "laplacian", "poisson",
                                                               "elasticity"])
@pytest.mark.parametrize("k", [1, 3, 6])
def test_quad_diagonal(mf, k, kind, prec):
    """diag(A) (the Jacobi preconditioner) against the oracle's, k+1 and k+2 points."""
    print(f"quad diagonal k={k} kind={kind} prec={prec}", flush=True)
    mesh = mg.quad_mesh(11, 0.25, config=0)
    nc = 2 if kind == 4 else 1
    space = mg.quad_space(mesh, k, seed_k=k, ncomp=nc)
    c = np.exp(np.random.default_rng(k).normal(size=mesh.nverts)) if kind in (MASS, POIS) else None
    sp = mf.Space.from_meshgen(space)
    for nq in (k + 1, k + 2):
        ref = oracle.OracleOp(space, kind, coef=c, nq1d=nq, lam=0.7, mu=0.4).diagonal()
        op = mf.Operator(sp, kind, prec, nq1d=nq, vertex_coef=c, lam=0.7, mu=0.4)
        d = op.diagonal().double().cpu().numpy()
        assert _relerr(d, ref) <= TOL[prec], _relerr(d, ref)


@pytest.mark.parametrize("kind", [HELM, 4], ids=["helmholtz", "elasticity"])
def test_quad_jacobi_cg(mf, kind):
    """Jacobi-preconditioned CG through the C-ABI on Q3 quads (Dirichlet boundary):
    the solution matches a dense solve of the oracle's assembled matrix."""
    import torch
    print(f"quad jacobi cg kind={kind}", flush=True)
    mesh = mg.quad_mesh(6, 0.25, config=0)
    nc = 2 if kind == 4 else 1
    space = mg.quad_space(mesh, 3, seed_k=3, ncomp=nc)
    bnd = space.boundary_nodes()
    mask = np.zeros(space.nnodes, np.uint8)
    mask[bnd] = 1
    bd = (bnd[:, None] * nc + np.arange(nc)).ravel()
    b = mg.uniform(space.ndofs, -1, 1, 0, mg.PURPOSE_RHS, 3)
    A = oracle.OracleOp(space, kind).assemble_dense()
    free = np.setdiff1d(np.arange(space.ndofs), bd)
    # constrained rows are the identity and constrained values leave the free rows
    xref = b.copy()
    xref[free] = np.linalg.solve(A[np.ix_(free, free)], b[free])
    sp = mf.Space.from_meshgen(space)
    op = mf.Operator(sp, kind, mf.F64, dirichlet=mask)
    x = torch.zeros(space.ndofs, dtype=torch.float64, device="cuda")
    bt = torch.tensor(b, device="cuda")
    info = mf.cg_solve(op, bt, x, precond=mf.JacobiPrecond(op), rtol=1e-12)
    assert info["rc"] == 0, info
    assert np.abs(x.cpu().numpy() - xref).max() <= 1e-8 * np.abs(xref).max()
