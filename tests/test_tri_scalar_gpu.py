"""GPU parity of the one-component operators on P1..P3 triangles (mass with and without
a vertex coefficient, Helmholtz, Laplacian, Poisson) against the oracle, through the
C-ABI. The P1 mass keeps its closed-form kernel; the other cases run the matrix-core
kernel (atomic, coloured and patch scatter); elasticity keeps the lane-per-cell kernel."""
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


def _case(k, m=9):
    mesh = mg.tri_mesh(m, 0.2, config=0)  # 162 cells: a ragged 64-cell batch
    space = mg.tri_space(mesh, k, seed_k=k)
    x = mg.uniform(space.ndofs, -1, 1, 0, mg.PURPOSE_X, k)
    c = np.exp(np.random.default_rng(k).normal(size=mesh.nverts))
    return mesh, space, x, c


@pytest.mark.parametrize("scatter", [1, 2], ids=["atomic", "coloured"])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind,coef", [(MASS, False), (MASS, True), (HELM, False), (LAP, False), (POIS, True)],
                         ids=["mass", "mass-coef", "helmholtz", "laplacian", "poisson"])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_tri_scalar_action(mf, k, kind, coef, prec, scatter):
    import torch
    print(f"tri scalar k={k} kind={kind} coef={coef} prec={prec} scatter={scatter}", flush=True)
    mesh, space, x, c = _case(k)
    c = c if coef else None
    ref = oracle.OracleOp(space, kind, coef=c).apply(x)
    op = mf.Operator(mf.Space.from_meshgen(space), kind, prec, vertex_coef=c, scatter=scatter)
    y = op.apply(torch.tensor(x, device="cuda", dtype=op.torch_dtype)).double().cpu().numpy()
    assert _relerr(y, ref) <= TOL[prec], _relerr(y, ref)


@pytest.mark.parametrize("k", [2, 3])
def test_tri_scalar_dirichlet_range_errors(mf, k):
    import torch
    mesh, space, x, c = _case(k)
    bnd = space.boundary_nodes()
    mask = np.zeros(space.nnodes, np.uint8)
    mask[bnd] = 1
    xm = x.copy()
    xm[bnd] = 0.0
    ref = oracle.OracleOp(space, HELM).apply(xm)
    ref[bnd] = x[bnd]
    sp = mf.Space.from_meshgen(space)
    op = mf.Operator(sp, HELM, mf.F64, dirichlet=mask)
    xt = torch.tensor(x, device="cuda")
    assert _relerr(op.apply(xt).cpu().numpy(), ref) <= 1e-12
    lap = mf.Operator(sp, LAP, mf.F64)
    y = torch.zeros_like(xt)
    for a, b in ((0, 50), (50, mesh.ncells)):
        lap.apply_range(a, b, xt, y, accumulate=True)
    assert _relerr(y.cpu().numpy(), oracle.OracleOp(space, LAP).apply(x)) <= 1e-12


# 40 x 40 x 2 = 3200 triangles: several patches of 2048, 1024, 512 or 256 cells, the
# last one ragged
@pytest.mark.parametrize("dirichlet", [False, True])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind,coef", [(MASS, True), (MASS, False), (HELM, False), (LAP, False), (POIS, True)],
                         ids=["mass-coef", "mass", "helmholtz", "laplacian", "poisson"])
@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_tri_scalar_patch(mf, k, kind, coef, prec, dirichlet):
    import torch
    if k == 1 and kind == MASS:
        pytest.skip("the P1 mass has its own closed-form patch kernel (test_simplex_patch_gpu)")
    print(f"tri scalar patch k={k} kind={kind} coef={coef} prec={prec} dirichlet={dirichlet}", flush=True)
    mesh, space, x, c = _case(k, m=40)
    c = c if coef else None
    bnd = space.boundary_nodes() if dirichlet else np.zeros(0, np.int64)
    mask = None
    if dirichlet:
        mask = np.zeros(space.nnodes, np.uint8)
        mask[bnd] = 1
    xm = x.copy()
    xm[bnd] = 0.0
    ref = oracle.OracleOp(space, kind, coef=c).apply(xm)
    ref[bnd] = x[bnd]
    op = mf.Operator(mf.Space.from_meshgen(space), kind, prec, vertex_coef=c, dirichlet=mask,
                     scatter=mf.SCATTER_PATCH)
    assert op.info["clears_output"] == 0 and op.info["scatter"] == mf.SCATTER_PATCH
    xt = torch.tensor(x, device="cuda", dtype=op.torch_dtype)
    y = op.apply(xt, torch.full_like(xt, float("nan"))).double().cpu().numpy()
    assert np.isfinite(y).all()
    assert _relerr(y, ref) <= TOL[prec], _relerr(y, ref)
    if not dirichlet:
        y0 = torch.tensor(mg.uniform(space.ndofs, -1, 1, 0, mg.PURPOSE_RHS, k), device="cuda", dtype=op.torch_dtype)
        yi = op.apply_internal(xt).double().cpu().numpy()
        yt = y0.clone()
        op.apply_range_internal(0, op.info["ncells"], xt, yt, accumulate=True)
        d = (yt.double() - y0.double()).cpu().numpy()
        assert np.abs(d - yi).max() <= 4 * TOL[prec] * (np.abs(yi).max() + 1.0)


def test_tri_scalar_large_sampled(mf):
    """512 x 512 x 2 triangles, P2 Poisson, sampled outputs."""
    import torch
    mesh = mg.tri_mesh(512, 0.2, config=0)
    space = mg.tri_space(mesh, 2)
    x = mg.uniform(space.ndofs, -1, 1, 0, mg.PURPOSE_X, 2)
    c = np.exp(np.random.default_rng(2).normal(size=mesh.nverts))
    rng = np.random.default_rng(0)
    nodes = rng.choice(space.nnodes, size=100, replace=False)
    touch = np.isin(space.cell2node, nodes).any(axis=1)
    sub = mg.Space(mg.Mesh(mesh.cell_type, mesh.coords, mesh.cell2vert[touch], mesh.lattice_m, mesh.vert_ijk),
                   2, 1, space.cell2node[touch], space.nnodes)
    ref = oracle.OracleOp(sub, POIS, coef=c).apply(x)
    sp = mf.Space.from_meshgen(space)
    for prec in (0, 1):
        op = mf.Operator(sp, POIS, prec, vertex_coef=c)
        y = op.apply(torch.tensor(x, device="cuda", dtype=op.torch_dtype)).double().cpu().numpy()
        assert np.abs(y[nodes] - ref[nodes]).max() / np.abs(ref[nodes]).max() <= TOL[prec]


@pytest.mark.parametrize("scatter", [1, 2], ids=["atomic", "coloured"])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_tri_elasticity(mf, k, prec, scatter):
    """2D linear elasticity (two node-interleaved components), lambda 0.7, mu 0.4."""
    import torch
    print(f"tri elasticity k={k} prec={prec} scatter={scatter}", flush=True)
    mesh = mg.tri_mesh(9, 0.2, config=0)
    space = mg.tri_space(mesh, k, seed_k=k, ncomp=2)
    x = mg.uniform(space.ndofs, -1, 1, 0, mg.PURPOSE_X, k)
    ref = oracle.OracleOp(space, oracle.OP_ELASTICITY, lam=0.7, mu=0.4).apply(x)
    op = mf.Operator(mf.Space.from_meshgen(space), mf.ELASTICITY, prec, lam=0.7, mu=0.4, scatter=scatter)
    y = op.apply(torch.tensor(x, device="cuda", dtype=op.torch_dtype)).double().cpu().numpy()
    assert _relerr(y, ref) <= TOL[prec], _relerr(y, ref)


@pytest.mark.parametrize("dirichlet", [False, True])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_tri_elasticity_patch(mf, k, prec, dirichlet):
    """Patch scatter of 2D elasticity on 40 x 40 x 2 triangles (several patches, the last
    ragged): every entry written, clamped rows, and the accumulating form."""
    import torch
    print(f"tri elasticity patch k={k} prec={prec} dirichlet={dirichlet}", flush=True)
    mesh = mg.tri_mesh(40, 0.2, config=0)
    space = mg.tri_space(mesh, k, seed_k=k, ncomp=2)
    x = mg.uniform(space.ndofs, -1, 1, 0, mg.PURPOSE_X, k)
    bnd = space.boundary_nodes() if dirichlet else np.zeros(0, np.int64)
    mask = None
    if dirichlet:
        mask = np.zeros(space.nnodes, np.uint8)
        mask[bnd] = 1
    bd = np.stack([2 * bnd, 2 * bnd + 1], axis=1).ravel()
    xm = x.copy()
    xm[bd] = 0.0
    ref = oracle.OracleOp(space, oracle.OP_ELASTICITY, lam=0.7, mu=0.4).apply(xm)
    ref[bd] = x[bd]
    op = mf.Operator(mf.Space.from_meshgen(space), mf.ELASTICITY, prec, lam=0.7, mu=0.4, dirichlet=mask,
                     scatter=mf.SCATTER_PATCH)
    assert op.info["clears_output"] == 0 and op.info["scatter"] == mf.SCATTER_PATCH
    xt = torch.tensor(x, device="cuda", dtype=op.torch_dtype)
    y = op.apply(xt, torch.full_like(xt, float("nan"))).double().cpu().numpy()
    assert np.isfinite(y).all()
    assert _relerr(y, ref) <= TOL[prec], _relerr(y, ref)
    if not dirichlet:
        y0 = torch.tensor(mg.uniform(space.ndofs, -1, 1, 0, mg.PURPOSE_RHS, k), device="cuda", dtype=op.torch_dtype)
        yi = op.apply_internal(xt).double().cpu().numpy()
        yt = y0.clone()
        op.apply_range_internal(0, op.info["ncells"], xt, yt, accumulate=True)
        d = (yt.double() - y0.double()).cpu().numpy()
        assert np.abs(d - yi).max() <= 4 * TOL[prec] * (np.abs(yi).max() + 1.0)


@pytest.mark.parametrize("k", [1, 3])
def test_tri_elasticity_dirichlet_range(mf, k):
    """Clamped boundary (both components) and a split range apply; one component is
    rejected."""
    import torch
    print(f"tri elasticity dirichlet k={k}", flush=True)
    mesh = mg.tri_mesh(9, 0.2, config=0)
    space = mg.tri_space(mesh, k, seed_k=k, ncomp=2)
    x = mg.uniform(space.ndofs, -1, 1, 0, mg.PURPOSE_X, k)
    bnd = space.boundary_nodes()
    mask = np.zeros(space.nnodes, np.uint8)
    mask[bnd] = 1
    bd = np.stack([2 * bnd, 2 * bnd + 1], axis=1).ravel()
    xm = x.copy()
    xm[bd] = 0.0
    ref = oracle.OracleOp(space, oracle.OP_ELASTICITY).apply(xm)
    ref[bd] = x[bd]
    sp = mf.Space.from_meshgen(space)
    xt = torch.tensor(x, device="cuda")
    op = mf.Operator(sp, mf.ELASTICITY, mf.F64, dirichlet=mask)
    assert _relerr(op.apply(xt).cpu().numpy(), ref) <= 1e-12
    op = mf.Operator(sp, mf.ELASTICITY, mf.F64)
    y = torch.zeros_like(xt)
    for a, b in ((0, 77), (77, mesh.ncells)):
        op.apply_range(a, b, xt, y, accumulate=True)
    assert _relerr(y.cpu().numpy(), oracle.OracleOp(space, oracle.OP_ELASTICITY).apply(x)) <= 1e-12
    with pytest.raises(mf.MFError):
        mf.Operator(mf.Space.from_meshgen(mg.tri_space(mesh, k)), mf.ELASTICITY, mf.F64)
