"""GPU parity of the St-Venant-Kirchhoff tangent (the paper's hyperelasticity operator
linearised at a displacement u0) against the oracle, through the C-ABI."""
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


def _case(k, m=None):
    m = m or (3 if k <= 3 else 2)  # 162 cells at m = 3: ragged batches; 48 at m = 2
    mesh = mg.tet_mesh(m, 0.2, config=2, seed_k=k)
    space = mg.tet_space(mesh, k, ncomp=3, config=2, seed_k=k)
    u0 = 0.3 * mg.uniform(space.ndofs, -1, 1, 2, mg.PURPOSE_COEF, k)
    x = mg.uniform(space.ndofs, -1, 1, 2, mg.PURPOSE_X, k)
    return mesh, space, u0, x


def _apply(mf, space, prec, u0, x, **kw):
    import torch
    op = mf.Operator(mf.Space.from_meshgen(space), mf.HYPERELASTIC, prec, lam=1.0, mu=0.5, u0=u0, **kw)
    xt = torch.tensor(x, device="cuda", dtype=op.torch_dtype)
    return op.apply(xt).double().cpu().numpy(), op


@pytest.mark.parametrize("scatter", [1, 2], ids=["atomic", "coloured"])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_tet_hyper_action(mf, k, prec, scatter):
    print(f"tet hyper k={k} prec={prec} scatter={scatter}", flush=True)
    mesh, space, u0, x = _case(k)
    ref = oracle.OracleOp(space, oracle.OP_HYPERELASTIC, lam=1.0, mu=0.5, u0=u0).apply(x)
    y, op = _apply(mf, space, prec, u0, x, scatter=scatter)
    assert op.info["nqp"] == {1: 1, 2: 14, 3: 125, 4: 343, 5: 729, 6: 1331}[k]
    assert _relerr(y, ref) <= TOL[prec], _relerr(y, ref)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_tet_hyper_dirichlet_rows(mf, k, prec):
    """Constrained boundary nodes: identity rows, zero columns; u0 still enters at
    the constrained nodes (it is a coefficient, gathered through an unflagged map)."""
    print(f"tet hyper dirichlet k={k} prec={prec}", flush=True)
    mesh, space, u0, x = _case(k)
    bnd = space.boundary_nodes()
    mask = np.zeros(space.nnodes, np.uint8)
    mask[bnd] = 1
    xm = x.reshape(-1, 3).copy()
    xm[bnd] = 0.0
    ref = oracle.OracleOp(space, oracle.OP_HYPERELASTIC, lam=1.0, mu=0.5, u0=u0).apply(xm.ravel()).reshape(-1, 3)
    ref[bnd] = x.reshape(-1, 3)[bnd]
    y, _ = _apply(mf, space, prec, u0, x, dirichlet=mask)
    assert _relerr(y, ref.ravel()) <= TOL[prec]


@pytest.mark.parametrize("k", [1, 2, 3, 4, 6])
def test_tet_hyper_at_zero_is_elasticity(mf, k):
    """At u0 = 0 the tangent is the linear elasticity operator (other quadrature rule,
    both exact)."""
    import torch
    mesh, space, _, x = _case(k)
    y, _ = _apply(mf, space, 0, np.zeros(space.ndofs), x)
    sp = mf.Space.from_meshgen(space)
    lin = mf.Operator(sp, mf.ELASTICITY, mf.F64, lam=1.0, mu=0.5)
    ref = lin.apply(torch.tensor(x, device="cuda")).cpu().numpy()
    assert _relerr(y, ref) <= 1e-12


def test_tet_hyper_errors(mf):
    mesh, space, u0, x = _case(2, m=2)
    sp = mf.Space.from_meshgen(space)
    with pytest.raises(mf.MFError):
        mf.Operator(sp, mf.HYPERELASTIC, mf.F64)  # no u0
    op = mf.Operator(sp, mf.HYPERELASTIC, mf.F64, u0=u0)
    with pytest.raises(mf.MFError):
        op.diagonal()


def test_tet_hyper_full_size_sampled(mf):
    """48^3 x 6 tets, P2 (the elasticity workload's mesh), on sampled outputs."""
    print("full tet hyper P2", flush=True)
    mesh = mg.tet_mesh(48, 0.2, config=2)
    space = mg.tet_space(mesh, 2, ncomp=3, config=2)
    u0 = 0.3 * mg.uniform(space.ndofs, -1, 1, 2, mg.PURPOSE_COEF, 2)
    x = mg.uniform(space.ndofs, -1, 1, 2, mg.PURPOSE_X, 2)
    rng = np.random.default_rng(0)
    nodes = rng.choice(space.nnodes, size=100, replace=False)
    touch = np.isin(space.cell2node, nodes).any(axis=1)
    sub = mg.Space(mg.Mesh(mesh.cell_type, mesh.coords, mesh.cell2vert[touch], mesh.lattice_m, mesh.vert_ijk),
                   2, 3, space.cell2node[touch], space.nnodes)
    ref = oracle.OracleOp(sub, oracle.OP_HYPERELASTIC, lam=1.0, mu=0.5, u0=u0).apply(x)
    dofs = (nodes[:, None] * 3 + np.arange(3)).ravel()
    for prec in (0, 1):
        y, _ = _apply(mf, space, prec, u0, x)
        err = np.abs(y[dofs] - ref[dofs]).max() / np.abs(ref[dofs]).max()
        assert err <= TOL[prec], (prec, err)


def _hex_case(k, m=3):
    mesh = mg.hex_mesh(m, 0.15, config=1, seed_k=k)  # 27 cells: ragged against 64 / q^3 cells per group
    space = mg.hex_space(mesh, k, ncomp=3, config=1)  # renumbered nodes
    u0 = 0.3 * mg.uniform(space.ndofs, -1, 1, 2, mg.PURPOSE_COEF, k)
    x = mg.uniform(space.ndofs, -1, 1, 2, mg.PURPOSE_X, k)
    return mesh, space, u0, x


@pytest.mark.parametrize("scatter", [1, 2], ids=["atomic", "coloured"])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("k,extra", [(k, 0) for k in range(1, 7)] + [(k, 1) for k in range(1, 7)])
def test_hex_hyper_action(mf, k, extra, prec, scatter):
    print(f"hex hyper k={k} q=k+1+{extra} prec={prec} scatter={scatter}", flush=True)
    mesh, space, u0, x = _hex_case(k)
    nq = k + 1 + extra
    ref = oracle.OracleOp(space, oracle.OP_HYPERELASTIC, lam=1.0, mu=0.5, u0=u0, nq1d=nq).apply(x)
    y, op = _apply(mf, space, prec, u0, x, scatter=scatter, nq1d=nq)
    assert op.info["nq1d"] == nq
    assert _relerr(y, ref) <= TOL[prec], _relerr(y, ref)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("k", [1, 3])
def test_hex_hyper_dirichlet_rows_and_range(mf, k, prec):
    """Constrained boundary nodes (u0 still enters there, through an unflagged map) and
    range applies that add up to the full action."""
    import torch
    print(f"hex hyper dirichlet k={k} prec={prec}", flush=True)
    mesh, space, u0, x = _hex_case(k)
    bnd = space.boundary_nodes()
    mask = np.zeros(space.nnodes, np.uint8)
    mask[bnd] = 1
    xm = x.reshape(-1, 3).copy()
    xm[bnd] = 0.0
    orc = oracle.OracleOp(space, oracle.OP_HYPERELASTIC, lam=1.0, mu=0.5, u0=u0)
    ref = orc.apply(xm.ravel()).reshape(-1, 3)
    ref[bnd] = x.reshape(-1, 3)[bnd]
    y, _ = _apply(mf, space, prec, u0, x, dirichlet=mask)
    assert _relerr(y, ref.ravel()) <= TOL[prec]
    _, op = _apply(mf, space, prec, u0, x)
    xt = torch.tensor(x, device="cuda", dtype=op.torch_dtype)
    yr = torch.zeros_like(xt)
    for a, b in ((0, 10), (10, mesh.ncells)):
        op.apply_range(a, b, xt, yr, accumulate=True)
    assert _relerr(yr.double().cpu().numpy(), orc.apply(x)) <= 4 * TOL[prec]


def test_hex_hyper_at_zero_is_elasticity(mf):
    import torch
    mesh, space, _, x = _hex_case(2)
    y, _ = _apply(mf, space, 0, np.zeros(space.ndofs), x)
    lin = mf.Operator(mf.Space.from_meshgen(space), mf.ELASTICITY, mf.F64, lam=1.0, mu=0.5)
    ref = lin.apply(torch.tensor(x, device="cuda")).cpu().numpy()
    assert _relerr(y, ref) <= 1e-12
