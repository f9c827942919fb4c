"""CG without allocation (mf_cg_solve_noalloc) against mf_cg_solve.

Both entry points run the same kernels in the same order (the allocating one replays
them from captured graphs). The operators here use the coloured scatter (no
atomics), so every launch is deterministic and the two solves take the same
iterations to the same solution; the test allows 1e-12 relative max-norm, the FP64
action bar. (With atomic scatter the summation order, and so the rounding of the
FP32 inner action, changes from launch to launch.) Two calls in a row, the second on a
smaller system, check that the fixed device array is re-initialised between solves;
a system larger than the array is rejected before any device work.
"""
import ctypes

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


def _system(mf, m, k, refined, config=4):
    import torch
    mesh = mg.hex_mesh(m, 0.15, config=config, seed_k=k)
    space = mg.hex_space(mesh, k, config=config)
    sp = mf.Space.from_meshgen(space)
    A64 = mf.Operator(sp, mf.HELMHOLTZ, mf.F64, scatter=mf.SCATTER_COLOURED)
    A32 = mf.Operator(sp, mf.HELMHOLTZ, mf.F32, scatter=mf.SCATTER_COLOURED) if refined else None
    M = mf.JacobiPrecond(A64)
    b = torch.tensor(mg.uniform(space.ndofs, -1, 1, config, mg.PURPOSE_RHS, k), device="cuda")
    return sp, A64, A32, M, b


@pytest.mark.parametrize("refined", [False, True], ids=["fp64", "fp32-refined"])
def test_noalloc_matches_allocating_solve_twice(mf, refined):
    import torch
    for m, k in ((10, 3), (6, 2)):  # the second call: a smaller system
        sp, A64, A32, M, b = _system(mf, m, k, refined)
        x_ref = torch.zeros_like(b)
        x_na = torch.zeros_like(b)
        info_ref = mf.cg_solve(A64, b, x_ref, A32=A32, precond=M, rtol=1e-10)
        info_na = mf.cg_solve(A64, b, x_na, A32=A32, precond=M, rtol=1e-10, noalloc=True)
        torch.cuda.synchronize()
        print(f"noalloc m={m} k={k} refined={refined}: {info_na} vs {info_ref}", flush=True)
        assert info_ref["rc"] == 0 and info_na["rc"] == 0
        assert info_na["rel_residual"] <= 1e-10
        assert info_na["inner_iterations"] == info_ref["inner_iterations"]
        assert info_na["outer_iterations"] == info_ref["outer_iterations"]
        xr, xn = x_ref.cpu().numpy(), x_na.cpu().numpy()
        assert np.abs(xn - xr).max() <= 1e-12 * np.abs(xr).max()


def test_noalloc_unpreconditioned_and_initial_guess(mf):
    import torch
    sp, A64, _, _, b = _system(mf, 7, 2, False, config=3)
    x0 = torch.tensor(mg.uniform(A64.ndofs, -1, 1, 3, mg.PURPOSE_X, 2), device="cuda")
    x_ref, x_na = x0.clone(), x0.clone()
    info_ref = mf.cg_solve(A64, b, x_ref, precond=None, rtol=1e-10)
    info_na = mf.cg_solve(A64, b, x_na, precond=None, rtol=1e-10, noalloc=True)
    assert info_ref["rc"] == 0 and info_na["rc"] == 0
    assert info_na["inner_iterations"] == info_ref["inner_iterations"]
    xr, xn = x_ref.cpu().numpy(), x_na.cpu().numpy()
    assert np.abs(xn - xr).max() <= 1e-12 * np.abs(xr).max()


def test_noalloc_rejects_systems_beyond_the_array(mf):
    import torch
    # Q4 on 32^3 cells: 2,146,689 DoFs need 3 x 8 B x n + 16 B x n (renumbered) > 64 MiB
    mesh = mg.hex_mesh(32, 0.15, config=1, seed_k=4)
    space = mg.hex_space(mesh, 4, config=1)
    A64 = mf.Operator(mf.Space.from_meshgen(space), mf.HELMHOLTZ, mf.F64)
    b = torch.ones(space.ndofs, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    info = mf.cg_solve(A64, b, x, rtol=1e-10, noalloc=True, raise_on_error=False)
    assert info["rc"] == -1  # MF_EINVAL
    msg = mf.load_library().mf_last_error().decode()
    assert "more than the" in msg and str(64 << 20) in msg
    assert float(x.abs().max()) == 0.0  # nothing ran
