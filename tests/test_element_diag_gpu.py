"""Jacobi diagonals summed from element-matrix diagonals (one-component tet operators,
triangle operators of degree 1-3, hex elasticity, hex operators with the paper's k+2
points) against the oracle's diagonal, with and without constrained nodes."""
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


def _relerr(y, ref):
    return np.abs(y - ref).max() / np.abs(ref).max()


def _check(mf, space, kind, prec, coef=None, nq1d=None, dirichlet=False):
    mask = None
    bnd = np.zeros(0, np.int64)
    if dirichlet:
        bnd = space.boundary_nodes()
        mask = np.zeros(space.nnodes, np.uint8)
        mask[bnd] = 1
    op = mf.Operator(mf.Space.from_meshgen(space), kind, prec, vertex_coef=coef, lam=1.0, mu=0.5,
                     nq1d=nq1d or 0, dirichlet=mask)
    d = op.diagonal().double().cpu().numpy()
    ref = oracle.OracleOp(space, kind, lam=1.0, mu=0.5, coef=coef, nq1d=nq1d).diagonal()
    nc = space.ncomp
    ref[(bnd[:, None] * nc + np.arange(nc)).ravel()] = 1.0
    assert _relerr(d, ref) <= TOL[prec], _relerr(d, ref)


@pytest.mark.parametrize("dirichlet", [False, True])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("k,kind,coef", [(k, kind, coef) for k in (1, 2, 3) for kind, coef in
                                         ((MASS, True), (HELM, False), (LAP, False), (POIS, True))])
def test_tet_scalar_diagonal(mf, k, kind, coef, prec, dirichlet):
    print(f"tet diag k={k} kind={kind} prec={prec} dirichlet={dirichlet}", flush=True)
    mesh = mg.tet_mesh(3, 0.2, config=2, seed_k=k)  # 162 cells: ragged against 64-cell blocks
    space = mg.tet_space(mesh, k, ncomp=1, config=2, seed_k=k)
    c = np.exp(np.random.default_rng(k).normal(size=mesh.nverts)) if coef else None
    _check(mf, space, kind, prec, coef=c, dirichlet=dirichlet)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("k,kind,coef", [(k, kind, coef) for k in (1, 2, 3) for kind, coef in
                                         ((MASS, True), (HELM, False), (LAP, False), (POIS, True), (ELAS, False))]
                         + [(1, HELM, False)])
def test_tri_diagonal(mf, k, kind, coef, prec):
    print(f"tri diag k={k} kind={kind} prec={prec}", flush=True)
    mesh = mg.tri_mesh(9, 0.2, config=0)  # 162 cells
    space = mg.tri_space(mesh, k, seed_k=k, ncomp=2 if kind == ELAS else 1)
    c = np.exp(np.random.default_rng(k).normal(size=mesh.nverts)) if coef else None
    _check(mf, space, kind, prec, coef=c, dirichlet=(k == 2))


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("k,extra", [(1, 0), (2, 0), (3, 0), (4, 0), (1, 1), (2, 1), (3, 1)])
def test_hex_elasticity_diagonal(mf, k, extra, prec):
    print(f"hex elasticity diag k={k} q=k+1+{extra} prec={prec}", flush=True)
    mesh = mg.hex_mesh(3, 0.15, config=1, seed_k=k)
    space = mg.hex_space(mesh, k, ncomp=3)
    _check(mf, space, ELAS, prec, nq1d=k + 1 + extra, dirichlet=(k == 2))


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("kind,ncomp", [(HELM, 1), (LAP, 3), (MASS, 1), (POIS, 1)])
def test_hex_k_plus_2_diagonal(mf, k, kind, ncomp, prec):
    print(f"hex k+2 diag k={k} kind={kind} prec={prec}", flush=True)
    mesh = mg.hex_mesh(3, 0.15, config=1, seed_k=k)
    space = mg.hex_space(mesh, k, ncomp=ncomp, config=1)
    c = np.exp(np.random.default_rng(k).normal(size=mesh.nverts)) if kind in (MASS, POIS) else None
    _check(mf, space, kind, prec, coef=c, nq1d=k + 2, dirichlet=(k == 3))


def test_hyperelastic_diagonal_rejected(mf):
    mesh = mg.tet_mesh(2, 0.2, config=2)
    space = mg.tet_space(mesh, 1, ncomp=3, config=2)
    u0 = 0.1 * mg.uniform(space.ndofs, -1, 1, 2, mg.PURPOSE_COEF, 1)
    op = mf.Operator(mf.Space.from_meshgen(space), mf.HYPERELASTIC, mf.F64, u0=u0)
    with pytest.raises(mf.MFError, match="HYPERELASTIC"):
        op.diagonal()
