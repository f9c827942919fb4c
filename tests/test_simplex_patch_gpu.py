"""Patch scatter of the tet elasticity action (P2, P3), of the one-component P1-P5
tet operators and of the P1 triangle mass against the oracle.

A patch workgroup sums its cells' local results in LDS and writes each of its nodes
once (straight into y, or into a slot that the shared-node reduction sums), so an
overwrite apply writes every free entry without a clearing pass. Checked: the action
at 1e-12 (FP64) / 1e-5 (FP32) on meshes with several patches and a ragged last one,
a NaN-filled output fully written, Dirichlet rows, the accumulating form used inside
CG, and agreement with the coloured scatter (the LDS sums are atomics, so the order
of the additions, and the last bits, may change from run to run).
"""
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
        pytest.skip("no GPU")
    import paper_1903_08243_amd as mf
    mf.load_library()
    return mf


def _relerr(y, ref):
    return np.abs(y - ref).max() / np.abs(ref).max()


def _case(k, m, dirichlet):
    mesh = mg.tet_mesh(m, 0.2, config=2)
    space = mg.tet_space(mesh, k, ncomp=3, config=2)
    bnd = space.boundary_nodes() if dirichlet else np.zeros(0, np.int64)
    mask = None
    if dirichlet:
        mask = np.zeros(space.nnodes, np.uint8)
        mask[bnd] = 1
    x = mg.uniform(space.ndofs, -1, 1, 2, mg.PURPOSE_X, k)
    xm = x.reshape(-1, 3).copy()
    xm[bnd] = 0.0
    ref = oracle.OracleOp(space, oracle.OP_ELASTICITY, lam=1.0, mu=0.5).apply(xm.ravel()).reshape(-1, 3)
    ref[bnd] = x.reshape(-1, 3)[bnd]
    return space, mask, x, ref.ravel()


# 7^3 x 6 = 2058 cells: 5 patches of 512 (P2) or 9 of 256 (P3), the last one ragged
@pytest.mark.parametrize("dirichlet", [False, True])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("k", [2, 3])
def test_tet_patch_action_writes_every_entry(mf, k, prec, dirichlet):
    import torch
    print(f"tet patch k={k} prec={prec} dirichlet={dirichlet}", flush=True)
    space, mask, x, ref = _case(k, 7, dirichlet)
    op = mf.Operator(mf.Space.from_meshgen(space), mf.ELASTICITY, prec, lam=1.0, mu=0.5, dirichlet=mask,
                     scatter=mf.SCATTER_PATCH)
    assert op.info["clears_output"] == 0
    xt = torch.tensor(x, device="cuda", dtype=op.torch_dtype)
    y = op.apply(xt, torch.full_like(xt, float("nan"))).double().cpu().numpy()
    assert np.isfinite(y).all()
    assert _relerr(y, ref) <= TOL[prec], _relerr(y, ref)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("k", [2, 3])
def test_tet_patch_accumulates_and_repeats_bitwise(mf, k, prec):
    """The accumulating full apply (the form CG uses, internal numbering) adds the
    same values the overwrite apply writes."""
    import torch
    print(f"tet patch accumulate k={k} prec={prec}", flush=True)
    space, _, x, _ = _case(k, 7, False)
    op = mf.Operator(mf.Space.from_meshgen(space), mf.ELASTICITY, prec, lam=1.0, mu=0.5,
                     scatter=mf.SCATTER_PATCH)
    xt = torch.tensor(x, device="cuda", dtype=op.torch_dtype)
    y0 = torch.tensor(mg.uniform(space.ndofs, -1, 1, 2, mg.PURPOSE_RHS, k), device="cuda", dtype=op.torch_dtype)
    yi = op.apply_internal(xt).double().cpu().numpy()
    yt = y0.clone()
    op.apply_range_internal(0, op.info["ncells"], xt, yt, accumulate=True)
    d = (yt.double() - y0.double()).cpu().numpy()
    assert np.abs(d - yi).max() <= 4 * TOL[prec] * (np.abs(yi).max() + np.abs(y0.double().cpu().numpy()).max())


@pytest.mark.parametrize("k", [2, 3])
def test_tet_patch_matches_coloured_scatter(mf, k):
    """The patch scatter and the coloured launches sum the same cell results in
    different orders: FP64 agreement to rounding on a mesh of 13,182 cells."""
    import torch
    print(f"tet patch vs coloured k={k}", flush=True)
    mesh = mg.tet_mesh(13, 0.2, config=2)
    space = mg.tet_space(mesh, k, ncomp=3, config=2)
    sp = mf.Space.from_meshgen(space)
    x = torch.tensor(mg.uniform(space.ndofs, -1, 1, 2, mg.PURPOSE_X, k), device="cuda")
    a = mf.Operator(sp, mf.ELASTICITY, mf.F64, lam=1.0, mu=0.5, scatter=mf.SCATTER_PATCH).apply(x)
    b = mf.Operator(sp, mf.ELASTICITY, mf.F64, lam=1.0, mu=0.5, scatter=mf.SCATTER_COLOURED).apply(x)
    a, b = a.cpu().numpy(), b.cpu().numpy()
    assert _relerr(a, b) <= 1e-13


# one-component forms on 7^3 x 6 = 2058 tets: several patches (1024, 384, 256 or 128
# cells), the last one ragged; MASS and POISSON with a vertex coefficient, MASS also
# without
SCALAR = [(0, True), (0, False), (1, False), (2, False), (3, True)]


@pytest.mark.parametrize("dirichlet", [False, True])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind,coef", SCALAR)
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_tet_scalar_patch_action(mf, k, kind, coef, prec, dirichlet):
    import torch
    print(f"tet scalar patch k={k} kind={kind} coef={coef} prec={prec} dirichlet={dirichlet}", flush=True)
    mesh = mg.tet_mesh(7, 0.2, config=2, seed_k=k)
    space = mg.tet_space(mesh, k, ncomp=1, config=2, seed_k=k)
    c = np.exp(np.random.default_rng(k).normal(size=mesh.nverts)) if coef else None
    x = mg.uniform(space.ndofs, -1, 1, 2, mg.PURPOSE_X, k)
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
        # accumulating form (internal numbering), as inside CG
        y0 = torch.tensor(mg.uniform(space.ndofs, -1, 1, 2, mg.PURPOSE_RHS, k), device="cuda",
                          dtype=op.torch_dtype)
        yi = op.apply_internal(xt).double().cpu().numpy()
        yt = y0.clone()
        op.apply_range_internal(0, op.info["ncells"], xt, yt, accumulate=True)
        d = (yt.double() - y0.double()).cpu().numpy()
        assert np.abs(d - yi).max() <= 4 * TOL[prec] * (np.abs(yi).max() + 1.0)


def test_tet_patch_rejected_for_p1_elasticity(mf):
    mesh = mg.tet_mesh(2, 0.2, config=2)
    space = mg.tet_space(mesh, 1, ncomp=3, config=2)
    with pytest.raises(mf.MFError, match="patch scatter"):
        mf.Operator(mf.Space.from_meshgen(space), mf.ELASTICITY, mf.F64, lam=1.0, mu=0.5, scatter=mf.SCATTER_PATCH)


# 48 x 48 x 2 = 4608 triangles: three patches of 2048 cells, the last one ragged
@pytest.mark.parametrize("renumber", [False, True])
@pytest.mark.parametrize("prec", [0, 1])
def test_tri_mass_patch_writes_every_entry(mf, prec, renumber):
    import torch
    print(f"tri mass patch prec={prec} renumber={renumber}", flush=True)
    mesh = mg.tri_mesh(48, 0.2, config=0)
    space = mg.tri_p1_space(mesh, renumber=renumber)
    c = mg.uniform(mesh.nverts, 0.5, 1.5, 0, mg.PURPOSE_COEF)
    x = mg.uniform(space.ndofs, -1, 1, 0, mg.PURPOSE_X)
    ref = oracle.OracleOp(space, oracle.OP_MASS, coef=c).apply(x)
    op = mf.Operator(mf.Space.from_meshgen(space), mf.MASS, prec, vertex_coef=c, scatter=mf.SCATTER_PATCH)
    assert op.info["clears_output"] == 0
    xt = torch.tensor(x, device="cuda", dtype=op.torch_dtype)
    y = op.apply(xt, torch.full_like(xt, float("nan"))).double().cpu().numpy()
    assert np.isfinite(y).all()
    assert _relerr(y, ref) <= TOL[prec], _relerr(y, ref)
    # accumulating form, internal numbering
    y0 = torch.tensor(mg.uniform(space.ndofs, -1, 1, 0, mg.PURPOSE_RHS), device="cuda", dtype=op.torch_dtype)
    yi = op.apply_internal(xt).double().cpu().numpy()
    yt = y0.clone()
    op.apply_range_internal(0, op.info["ncells"], xt, yt, accumulate=True)
    d = (yt.double() - y0.double()).cpu().numpy()
    assert np.abs(d - yi).max() <= 4 * TOL[prec] * (np.abs(yi).max() + 1.0)
