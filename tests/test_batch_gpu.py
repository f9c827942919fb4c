"""Batched persistent-launch solves (many uneven hex operators) vs single solves."""
import os

import numpy as np
import pytest

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


def _systems(mf, sizes):
    import torch
    out = []
    for i, (m, k) in enumerate(sizes):
        mesh = mg.hex_mesh(m, 0.15, config=3, seed_k=10 + i)
        space = mg.hex_space(mesh, k, config=3, seed_k=10 + i)
        sp = mf.Space.from_meshgen(space)
        A64 = mf.Operator(sp, mf.HELMHOLTZ, mf.F64)
        A32 = mf.Operator(sp, mf.HELMHOLTZ, mf.F32)
        M = mf.JacobiPrecond(A64)
        b = torch.tensor(mg.uniform(space.ndofs, -1, 1, 3, mg.PURPOSE_RHS, 10 + i), device="cuda")
        out.append((sp, A64, A32, M, b))
    return out


@pytest.mark.parametrize("refined", [True, False])
def test_batch_solve_matches_single_solves(mf, refined):
    import torch
    sizes = [(3, 2), (5, 5), (4, 3), (6, 4), (2, 5), (7, 2), (3, 4)]  # uneven sizes and degrees
    sy = _systems(mf, sizes)
    xs = [torch.zeros_like(s[4]) for s in sy]
    B = mf.Batch([s[1] for s in sy], [s[4] for s in sy], xs, A32=[s[2] for s in sy] if refined else None,
                 M=[s[3] for s in sy])
    infos, rc = B.solve(rtol=1e-10)
    assert rc == 0
    for (sp, A64, A32, M, b), x, info in zip(sy, xs, infos):
        assert info["rel_residual"] <= 1e-10
        xr = torch.zeros_like(b)
        mf.cg_solve(A64, b, xr, precond=M, rtol=1e-12)
        ref = xr.cpu().numpy()
        assert np.abs(x.cpu().numpy() - ref).max() <= 1e-8 * np.abs(ref).max()
        # the reported residual is the true one
        r = (b - A64.apply(x)).norm() / b.norm()
        assert abs(float(r) - info["rel_residual"]) <= 1e-12


def test_batch_autotune_and_cache(mf, tmp_path):
    import torch
    sy = _systems(mf, [(4, 2), (5, 3), (3, 5)])
    xs = [torch.zeros_like(s[4]) for s in sy]
    B = mf.Batch([s[1] for s in sy], [s[4] for s in sy], xs, A32=[s[2] for s in sy], M=[s[3] for s in sy])
    cache = str(tmp_path / "tune.txt")
    t1 = B.autotune(cache)
    assert os.path.exists(cache) and open(cache).read().count("\n") == 1
    B.set_tuning(1, 64)
    t2 = B.autotune(cache)  # read back from the cache, not re-measured
    assert t2 == t1 and open(cache).read().count("\n") == 1
    infos, rc = B.solve(rtol=1e-10)
    assert rc == 0 and all(i["rel_residual"] <= 1e-10 for i in infos)
    # every work-list granularity gives the same batched solution
    ref = [x.clone() for x in xs]
    for per, grid in [(1, 37), (32, 2048), (1, -1)]:
        for x in xs:
            x.zero_()
        B.set_tuning(per, grid)
        infos, rc = B.solve(rtol=1e-10)
        assert rc == 0
        for x, r in zip(xs, ref):
            assert torch.allclose(x, r, rtol=0, atol=1e-9 * float(r.abs().max()))


@pytest.mark.parametrize("tuning", [(1, 0), (4, 512), (1, 37), (1, -1)])
def test_batched_action_matches_oracle(mf, tuning):
    """One batched launch over uneven systems (k = 2..5, ragged sizes, one 20^3 mesh)
    against the oracle's action, system by system: FP64 operators at 1e-12 and the
    FP32 inner operators at 1e-5 (relative max-norm), one wavefront per work item
    (grid 0), persistent grids with coarse and fine work lists, and each system's own
    kernels (grid -1)."""
    import torch
    import oracle
    sizes = [(3, 2), (5, 5), (4, 3), (20, 2), (6, 4), (2, 5), (7, 3), (9, 4)]
    spaces, A64, A32 = [], [], []
    for i, (m, k) in enumerate(sizes):
        mesh = mg.hex_mesh(m, 0.15, config=3, seed_k=30 + i)
        space = mg.hex_space(mesh, k, config=3, seed_k=30 + i)
        sp = mf.Space.from_meshgen(space)
        spaces.append(space)
        A64.append(mf.Operator(sp, mf.HELMHOLTZ, mf.F64))
        A32.append(mf.Operator(sp, mf.HELMHOLTZ, mf.F32))
    b = [torch.zeros(s.ndofs, dtype=torch.float64, device="cuda") for s in spaces]
    x = [torch.zeros_like(t) for t in b]
    B = mf.Batch(A64, b, x, A32=A32)
    B.set_tuning(*tuning)
    xs = [mg.uniform(s.ndofs, -1, 1, 3, mg.PURPOSE_X, 30 + i) for i, s in enumerate(spaces)]
    refs = [oracle.OracleOp(s, oracle.OP_HELMHOLTZ).apply(xv) for s, xv in zip(spaces, xs)]
    for inner, dt, tol in ((False, torch.float64, 1e-12), (True, torch.float32, 1e-5)):
        xd = [torch.tensor(xv, device="cuda", dtype=dt) for xv in xs]
        yd = [torch.full_like(t, float("nan")) for t in xd]
        B.apply_user(xd, yd, inner=inner)
        torch.cuda.synchronize()
        for i, (y, ref) in enumerate(zip(yd, refs)):
            err = np.abs(y.double().cpu().numpy() - ref).max() / np.abs(ref).max()
            assert err <= tol, (tuning, inner, sizes[i], err)
