"""GPU parity of linear elasticity on Q1..Q6 trilinear hexahedra against the oracle,
through the C-ABI: both precisions and scatters, k+1 and k+2 Gauss points, Dirichlet
rows, range applies, and the user-numbering path with the fused gather."""
import numpy as np
import pytest

import oracle
from paper_1903_08243_amd import meshgen as mg

pytestmark = pytest.mark.gpu
TOL = {0: 1e-12, 1: 1e-5}


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


def _case(k, m=3):
    mesh = mg.hex_mesh(m, 0.15, config=1, seed_k=k)
    space = mg.hex_space(mesh, k, ncomp=3)  # renumbered nodes
    x = mg.uniform(space.ndofs, -1, 1, 1, mg.PURPOSE_X, k)
    return mesh, space, x


@pytest.mark.parametrize("scatter", [1, 2], ids=["atomic", "coloured"])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_hex_elasticity_action(mf, k, prec, scatter):
    import torch
    print(f"hex elasticity k={k} prec={prec} scatter={scatter}", flush=True)
    mesh, space, x = _case(k)
    ref = oracle.OracleOp(space, oracle.OP_ELASTICITY, lam=0.7, mu=0.4).apply(x)
    op = mf.Operator(mf.Space.from_meshgen(space), mf.ELASTICITY, prec, lam=0.7, mu=0.4, scatter=scatter)
    y = op.apply(torch.tensor(x, device="cuda", dtype=op.torch_dtype)).double().cpu().numpy()
    assert _relerr(y, ref) <= TOL[prec], _relerr(y, ref)


@pytest.mark.parametrize("k", [1, 3, 5, 6])
def test_hex_elasticity_paper_rule_dirichlet_range(mf, k):
    import torch
    print(f"hex elasticity k+2 / dirichlet / range k={k}", flush=True)
    mesh, space, x = _case(k)
    sp = mf.Space.from_meshgen(space)
    xt = torch.tensor(x, device="cuda")
    ref = oracle.OracleOp(space, oracle.OP_ELASTICITY, nq1d=k + 2).apply(x)
    op = mf.Operator(sp, mf.ELASTICITY, mf.F64, nq1d=k + 2)
    assert _relerr(op.apply(xt).cpu().numpy(), ref) <= 1e-12
    bnd = space.boundary_nodes()
    mask = np.zeros(space.nnodes, np.uint8)
    mask[bnd] = 1
    bd = (bnd[:, None] * 3 + np.arange(3)).ravel()
    xm = x.copy()
    xm[bd] = 0.0
    ref = oracle.OracleOp(space, oracle.OP_ELASTICITY).apply(xm)
    ref[bd] = x[bd]
    for sc in (mf.SCATTER_ATOMIC, mf.SCATTER_COLOURED):
        op = mf.Operator(sp, mf.ELASTICITY, mf.F64, dirichlet=mask, scatter=sc)
        assert _relerr(op.apply(xt).cpu().numpy(), ref) <= 1e-12
    op = mf.Operator(sp, mf.ELASTICITY, mf.F64)
    y = torch.zeros_like(xt)
    for a, b in ((0, 10), (10, 11), (11, mesh.ncells)):
        op.apply_range(a, b, xt, y, accumulate=True)
    assert _relerr(y.cpu().numpy(), oracle.OracleOp(space, oracle.OP_ELASTICITY).apply(x)) <= 1e-12
    with pytest.raises(mf.MFError):
        mf.Operator(sp, mf.ELASTICITY, mf.F64, nq1d=k + 3)


def test_hex_elasticity_errors(mf):
    mesh = mg.hex_mesh(2)
    with pytest.raises(mf.MFError):  # one component
        mf.Operator(mf.Space.from_meshgen(mg.hex_space(mesh, 2)), mf.ELASTICITY, mf.F64)
    with pytest.raises(mf.MFError):  # the patch scatter is Q1 scalar/vector Laplacian-type only
        mf.Operator(mf.Space.from_meshgen(mg.hex_space(mesh, 1, ncomp=3)), mf.ELASTICITY, mf.F64, scatter=3)
    with pytest.raises(mf.MFError):  # k+3 points
        mf.Operator(mf.Space.from_meshgen(mg.hex_space(mesh, 6, ncomp=3)), mf.ELASTICITY, mf.F64, nq1d=9)
