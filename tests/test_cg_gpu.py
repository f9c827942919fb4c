"""CG on the GPU: FP64 Jacobi-PCG and FP32-action iterative refinement vs dense solves."""
import numpy as np
import pytest

import oracle
from paper_1903_08243_amd import meshgen as mg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1903_08243_amd as mf
    mf.load_library()
    return mf


def _problem(kind=1, k=2, m=6, dirichlet=False):
    mesh = mg.hex_mesh(m, 0.15, config=3, seed_k=k)
    space = mg.hex_space(mesh, k, config=3)
    coef = np.exp(np.random.default_rng(7).normal(size=mesh.nverts)) if kind == 3 else None
    mask = None
    b = mg.uniform(space.ndofs, -1, 1, 3, mg.PURPOSE_RHS, k)
    orc = oracle.OracleOp(space, kind, coef=coef)
    A = orc.assemble_dense()
    if dirichlet:
        bnd = space.boundary_nodes()
        mask = np.zeros(space.nnodes, np.uint8)
        mask[bnd] = 1
        b[bnd] = 0.0
        keep = np.ones(space.ndofs, bool)
        keep[bnd] = False
        A = A[np.ix_(keep, keep)]
        xs = np.zeros(space.ndofs)
        xs[keep] = np.linalg.solve(A, b[keep])
    else:
        xs = np.linalg.solve(A, b)
    return space, coef, mask, b, xs


@pytest.mark.parametrize("refined", [False, True])
@pytest.mark.parametrize("kind,dirichlet", [(1, False), (3, True)], ids=["helmholtz", "poisson-dirichlet"])
def test_cg_matches_dense_solve(mf, refined, kind, dirichlet):
    import torch
    space, coef, mask, b, xs = _problem(kind=kind, dirichlet=dirichlet)
    sp = mf.Space.from_meshgen(space)
    A64 = mf.Operator(sp, kind, mf.F64, vertex_coef=coef, dirichlet=mask)
    A32 = mf.Operator(sp, kind, mf.F32, vertex_coef=coef, dirichlet=mask) if refined else None
    M = mf.JacobiPrecond(A64)
    bt = torch.tensor(b, device="cuda")
    x = torch.zeros_like(bt)
    info = mf.cg_solve(A64, bt, x, A32=A32, precond=M, rtol=1e-10)
    assert info["rc"] == 0
    assert info["rel_residual"] <= 1e-10
    xg = x.cpu().numpy()
    assert np.abs(xg - xs).max() <= 1e-8 * np.abs(xs).max()
    # the reported residual is the true FP64 residual
    if mask is None:
        r = b - oracle.OracleOp(space, kind, coef=coef).apply(xg)
        assert abs(np.linalg.norm(r) / np.linalg.norm(b) - info["rel_residual"]) <= 1e-11
    if refined:
        assert info["outer_iterations"] >= 2


@pytest.mark.parametrize("refined", [False, True])
@pytest.mark.parametrize("kind,dirichlet", [(1, False), (3, True)], ids=["helmholtz", "poisson-dirichlet"])
def test_cg_with_q1_patch_scatter(mf, refined, kind, dirichlet):
    """CG on Q1 operators that use the patch scatter (accumulating internal applies inside
    the captured iteration) against the dense solve."""
    import torch
    space, coef, mask, b, xs = _problem(kind=kind, k=1, m=8, dirichlet=dirichlet)
    sp = mf.Space.from_meshgen(space)
    P = mf.SCATTER_PATCH
    A64 = mf.Operator(sp, kind, mf.F64, vertex_coef=coef, dirichlet=mask, scatter=P)
    A32 = mf.Operator(sp, kind, mf.F32, vertex_coef=coef, dirichlet=mask, scatter=P) if refined else None
    M = mf.JacobiPrecond(A64)
    bt = torch.tensor(b, device="cuda")
    x = torch.zeros_like(bt)
    info = mf.cg_solve(A64, bt, x, A32=A32, precond=M, rtol=1e-10)
    assert info["rc"] == 0 and info["rel_residual"] <= 1e-10
    assert np.abs(x.cpu().numpy() - xs).max() <= 1e-8 * np.abs(xs).max()


def test_cg_nonzero_initial_guess_and_restart(mf):
    import torch
    space, coef, mask, b, xs = _problem(kind=1, k=3, m=4)
    sp = mf.Space.from_meshgen(space)
    A64 = mf.Operator(sp, 1, mf.F64)
    bt = torch.tensor(b, device="cuda")
    x = torch.tensor(xs + 1e-3 * np.random.default_rng(1).normal(size=xs.size), device="cuda")
    info = mf.cg_solve(A64, bt, x, rtol=1e-12)
    assert info["rc"] == 0 and info["rel_residual"] <= 1e-12
    assert np.abs(x.cpu().numpy() - xs).max() <= 1e-9 * np.abs(xs).max()


def test_cg_reports_not_converged(mf):
    import torch
    space, coef, mask, b, xs = _problem(kind=1, k=2, m=4)
    sp = mf.Space.from_meshgen(space)
    A64 = mf.Operator(sp, 1, mf.F64)
    bt = torch.tensor(b, device="cuda")
    x = torch.zeros_like(bt)
    info = mf.cg_solve(A64, bt, x, rtol=1e-12, maxit=3, raise_on_error=False)
    assert info["rc"] == -5  # MF_ENOTCONV
    assert info["inner_iterations"] <= 3 + 8  # stops within one graph chunk of the limit


def test_cg_detects_non_finite_input(mf):
    import torch
    space, coef, mask, b, xs = _problem(kind=1, k=2, m=4)
    sp = mf.Space.from_meshgen(space)
    A64 = mf.Operator(sp, 1, mf.F64)
    b = b.copy()
    b[3] = np.nan
    bt = torch.tensor(b, device="cuda")
    x = torch.zeros_like(bt)
    info = mf.cg_solve(A64, bt, x, rtol=1e-10, raise_on_error=False)
    assert info["rc"] == -6  # MF_EBREAKDOWN
