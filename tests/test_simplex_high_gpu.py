"""GPU parity of the degree 4-6 simplex operators (dense-tabulation kernel, triangles
and tetrahedra: mass with a vertex coefficient, Helmholtz, Laplacian, Poisson,
elasticity) against the oracle, through the C-ABI; their diagonals and CSR matrices."""
import numpy as np
import pytest

import oracle
from paper_1903_08243_amd import meshgen as mg

pytestmark = pytest.mark.gpu
TOL = {0: 1e-12, 1: 1e-5}
MASS, HELM, LAP, POIS, ELAS = 0, 1, 2, 3, 4
KINDS = ((MASS, True), (HELM, False), (LAP, False), (POIS, True), (ELAS, False))


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


def _case(cell, k, kind):
    if cell == "tet":
        mesh = mg.tet_mesh(2, 0.2, config=2, seed_k=k)  # 48 cells
        space = mg.tet_space(mesh, k, ncomp=3 if kind == ELAS else 1, config=2, seed_k=k)
    else:
        mesh = mg.tri_mesh(9, 0.2, config=0)  # 162 cells
        space = mg.tri_space(mesh, k, seed_k=k, ncomp=2 if kind == ELAS else 1)
    c = np.exp(np.random.default_rng(k).normal(size=mesh.nverts))
    x = mg.uniform(space.ndofs, -1, 1, 2, mg.PURPOSE_X, k)
    return mesh, space, c, x


@pytest.mark.parametrize("scatter", [1, 2], ids=["atomic", "coloured"])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind,coef", KINDS)
@pytest.mark.parametrize("cell,k", [(c, k) for c in ("tri", "tet") for k in (4, 5, 6)])
def test_high_degree_simplex_action(mf, cell, k, kind, coef, prec, scatter):
    import torch
    print(f"{cell} P{k} kind={kind} prec={prec} scatter={scatter}", flush=True)
    mesh, space, c, x = _case(cell, k, kind)
    c = c if coef else None
    ref = oracle.OracleOp(space, kind, lam=1.0, mu=0.5, coef=c).apply(x)
    op = mf.Operator(mf.Space.from_meshgen(space), kind, prec, vertex_coef=c, lam=1.0, mu=0.5, scatter=scatter)
    y = op.apply(torch.tensor(x, device="cuda", dtype=op.torch_dtype)).double().cpu().numpy()
    assert _relerr(y, ref) <= TOL[prec], _relerr(y, ref)


@pytest.mark.parametrize("cell,k,kind", [("tet", 5, POIS), ("tri", 6, ELAS), ("tet", 4, ELAS)])
def test_high_degree_simplex_dirichlet_and_range(mf, cell, k, kind):
    """Constrained boundary nodes (identity rows, zero columns) and range applies that
    add up to the full action."""
    import torch
    mesh, space, c, x = _case(cell, k, kind)
    c = c if kind == POIS else None
    nc = space.ncomp
    bnd = space.boundary_nodes()
    mask = np.zeros(space.nnodes, np.uint8)
    mask[bnd] = 1
    bd = (bnd[:, None] * nc + np.arange(nc)).ravel()
    xm = x.copy()
    xm[bd] = 0.0
    orc = oracle.OracleOp(space, kind, lam=1.0, mu=0.5, coef=c)
    ref = orc.apply(xm)
    ref[bd] = x[bd]
    sp = mf.Space.from_meshgen(space)
    op = mf.Operator(sp, kind, 0, vertex_coef=c, lam=1.0, mu=0.5, dirichlet=mask)
    xt = torch.tensor(x, device="cuda")
    assert _relerr(op.apply(xt).cpu().numpy(), ref) <= 1e-12
    op2 = mf.Operator(sp, kind, 0, vertex_coef=c, lam=1.0, mu=0.5)
    y = torch.zeros_like(xt)
    for a, b in ((0, 7), (7, mesh.ncells)):
        op2.apply_range(a, b, xt, y, accumulate=True)
    assert _relerr(y.cpu().numpy(), orc.apply(x)) <= 1e-12


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("cell,k,kind", [("tet", 4, HELM), ("tet", 6, ELAS), ("tri", 5, POIS), ("tri", 6, MASS)])
def test_high_degree_simplex_diagonal(mf, cell, k, kind, prec):
    mesh, space, c, _ = _case(cell, k, kind)
    c = c if kind in (MASS, POIS) else None
    op = mf.Operator(mf.Space.from_meshgen(space), kind, prec, vertex_coef=c, lam=1.0, mu=0.5)
    d = op.diagonal().double().cpu().numpy()
    ref = oracle.OracleOp(space, kind, lam=1.0, mu=0.5, coef=c).diagonal()
    assert _relerr(d, ref) <= TOL[prec]


@pytest.mark.parametrize("cell,k,kind", [("tet", 4, ELAS), ("tri", 6, HELM)])
def test_high_degree_simplex_csr(mf, cell, k, kind):
    mesh, space, c, _ = _case(cell, k, kind)
    op = mf.Operator(mf.Space.from_meshgen(space), kind, 0, lam=1.0, mu=0.5)
    rowptr, col, vals = op.csr()
    A = np.zeros((space.ndofs, space.ndofs))
    v = vals.cpu().numpy()
    for r in range(space.ndofs):
        A[r, col[rowptr[r]:rowptr[r + 1]]] = v[rowptr[r]:rowptr[r + 1]]
    ref = oracle.OracleOp(space, kind, lam=1.0, mu=0.5).assemble_dense()
    assert np.abs(A - ref).max() <= 1e-12 * np.abs(ref).max()


def test_high_degree_sampled_full_size(mf):
    """P4 tet elasticity on 24^3 x 6 cells (82,944; coloured scatter), sampled outputs
    against the oracle on the cells that touch them."""
    import torch
    mesh = mg.tet_mesh(24, 0.2, config=2, seed_k=4)
    space = mg.tet_space(mesh, 4, ncomp=3, config=2, seed_k=4)
    x = mg.uniform(space.ndofs, -1, 1, 2, mg.PURPOSE_X, 4)
    op = mf.Operator(mf.Space.from_meshgen(space), ELAS, 0, lam=1.0, mu=0.5)
    y = op.apply(torch.tensor(x, device="cuda")).cpu().numpy()
    nodes = np.random.default_rng(3).choice(space.nnodes, 60, replace=False)
    touch = np.isin(space.cell2node, nodes).any(axis=1)
    m = space.mesh
    sub = mg.Space(mg.Mesh(m.cell_type, m.coords, m.cell2vert[touch], m.lattice_m, m.vert_ijk), space.degree,
                   space.ncomp, space.cell2node[touch], space.nnodes)
    ref = oracle.OracleOp(sub, ELAS, lam=1.0, mu=0.5).apply(x)
    dofs = (nodes[:, None] * 3 + np.arange(3)).ravel()
    assert np.abs(y[dofs] - ref[dofs]).max() <= 1e-12 * np.abs(ref[dofs]).max()
