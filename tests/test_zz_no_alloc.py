"""The allocation-free projection (kvs_project_noalloc) against the context
path (kvs_project) on the same inputs: same iteration count, phi and f_S to
the FP64 bar, two calls in a row with the second on a smaller grid (the
shared scratch array keeps the first call's contents), a warm start from a
guess with a non-zero outer layer, an oversize grid rejected with a message,
and no change of the device's free memory across a call."""
import numpy as np
import pytest

from oracle.analysis import rel_l2
from workloads import gaussian_push

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2607_28414_amd import kvs as k
    k.lib()
    return k, torch


def say(*a):
    print(*a, flush=True)


def force_of(grid, seed):
    nx, ny, nz = grid[:3]
    rng = np.random.default_rng(seed)
    return gaussian_push(grid, 1.0e-3, 2.0e-3, 1e4) + 300.0 * rng.standard_normal((3, nz, ny, nx))


def context_projection(kvs, grid, F, **opts):
    shp = (grid[2], grid[1], grid[0])
    ctx = kvs.kvs_create(grid, precision=kvs.KVS_FP64)
    try:
        kvs.kvs_set_force(ctx, F)
        rep = kvs.kvs_project(ctx, **opts)
        return rep, kvs.kvs_get_phi(ctx, shp), kvs.kvs_get_projected_force(ctx, shp)
    finally:
        kvs.kvs_destroy(ctx)


def noalloc_projection(kvs, torch, grid, F, phi0=None, **opts):
    shp = (grid[2], grid[1], grid[0])
    Fd = torch.from_numpy(np.ascontiguousarray(F)).to("cuda")
    phid = torch.full(shp, np.nan, dtype=torch.float64, device="cuda") if phi0 is None else \
        torch.from_numpy(np.ascontiguousarray(phi0)).to("cuda")
    FSd = torch.full((3,) + shp, np.nan, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    rep = kvs.kvs_project_noalloc(grid, Fd.data_ptr(), phid.data_ptr(), FSd.data_ptr(), **opts)
    torch.cuda.synchronize()
    return rep, phid.cpu().numpy(), FSd.cpu().numpy()


GRID_A = (70, 45, 53, 0.25e-3, 0.3e-3, 0.2e-3)
GRID_B = (33, 29, 17, 0.25e-3, 0.25e-3, 0.25e-3)


@pytest.mark.parametrize("precond", [0, 1])
def test_noalloc_matches_context_projection_twice(env, precond):
    kvs, torch = env
    for grid, seed in ((GRID_A, 1), (GRID_B, 2)):  # the second call on a smaller grid
        say(f"case noalloc precond {precond} grid {grid[:3]}")
        F = force_of(grid, seed)
        opts = dict(tol=1e-10, max_iter=5000, precond=precond)
        rep_c, phi_c, FS_c = context_projection(kvs, grid, F, **opts)
        rep_n, phi_n, FS_n = noalloc_projection(kvs, torch, grid, F, **opts)
        say(f"iterations {rep_c['iters']} / {rep_n['iters']}, true residual {rep_c['relres_true']:.3e} / "
            f"{rep_n['relres_true']:.3e}")
        assert rep_n["status"] == 0 and rep_n["iters"] == rep_c["iters"] > 0
        assert rep_n["relres_true"] == pytest.approx(rep_c["relres_true"], rel=1e-9)
        assert rel_l2(phi_n, phi_c) <= 1e-12
        assert rel_l2(FS_n, FS_c) <= 1e-12
        # the outer layers are written (the outputs started as NaN)
        assert np.all(np.isfinite(phi_n)) and np.all(np.isfinite(FS_n))
        assert not FS_n[:, 0].any() and not FS_n[:, :, :, -1].any() and not phi_n[:, -1].any()


def test_noalloc_warm_start_and_fixed_iterations(env):
    kvs, torch = env
    grid = GRID_B
    shp = (grid[2], grid[1], grid[0])
    F1, F2 = force_of(grid, 3), force_of(grid, 4)
    say("case noalloc warm start")
    # context path: project F1, then F2 from F1's phi
    ctx = kvs.kvs_create(grid, precision=kvs.KVS_FP64)
    try:
        kvs.kvs_set_force(ctx, F1)
        kvs.kvs_project(ctx, tol=1e-10)
        phi1 = kvs.kvs_get_phi(ctx, shp)
        kvs.kvs_set_force(ctx, F2)
        rep_c = kvs.kvs_project(ctx, tol=1e-10, warm_start=True)
        phi_c, FS_c = kvs.kvs_get_phi(ctx, shp), kvs.kvs_get_projected_force(ctx, shp)
    finally:
        kvs.kvs_destroy(ctx)
    guess = phi1.copy()
    guess[0], guess[:, :, -1] = 7.0, -3.0  # the outer layer of a guess is cleared first
    rep_n, phi_n, FS_n = noalloc_projection(kvs, torch, grid, F2, phi0=guess, tol=1e-10, warm_start=True)
    assert rep_n["iters"] == rep_c["iters"]
    assert rel_l2(phi_n, phi_c) <= 1e-12 and rel_l2(FS_n, FS_c) <= 1e-12
    # parity mode: exactly the requested iterations
    rep_f, _, _ = noalloc_projection(kvs, torch, grid, F1, fixed_iters=17, precond=kvs.KVS_PC_NONE)
    assert rep_f["iters"] == 17


def test_noalloc_rejects_oversize_and_unet(env):
    kvs, torch = env
    say("case noalloc errors")
    big = (130, 130, 130, 1e-3, 1e-3, 1e-3)
    with pytest.raises(kvs.KvsError) as e:
        kvs.kvs_project_noalloc(big, 1, 1, 1)  # rejected before any pointer is used
    assert e.value.status == kvs.KVS_EINVAL and "too large" in str(e.value)
    with pytest.raises(kvs.KvsError) as e:
        kvs.kvs_project_noalloc(GRID_B, 1, 1, 1, precond=kvs.KVS_PC_UNET)
    assert e.value.status == kvs.KVS_EINVAL


def test_noalloc_leaves_free_device_memory_unchanged(env):
    kvs, torch = env
    say("case noalloc free memory")
    grid = GRID_A
    shp = (grid[2], grid[1], grid[0])
    Fd = torch.from_numpy(force_of(grid, 5)).to("cuda")
    phid = torch.empty(shp, dtype=torch.float64, device="cuda")
    FSd = torch.empty((3,) + shp, dtype=torch.float64, device="cuda")
    kvs.kvs_project_noalloc(grid, Fd.data_ptr(), phid.data_ptr(), FSd.data_ptr(), tol=1e-8)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        rep = kvs.kvs_project_noalloc(grid, Fd.data_ptr(), phid.data_ptr(), FSd.data_ptr(), tol=1e-8)
        assert rep["status"] == 0
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
