"""The projection's CG with its search direction stored in FP32 (the default
of FP32 contexts; r and phi stay FP64 and are updated with the stored
direction) against the oracle's FP64 true residual and against the same
solve with FP64 directions, and the switch between the two on one context."""
import numpy as np
import pytest

import oracle
from workloads import cfg2_inclusions_fp32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kvs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2607_28414_amd import kvs as k
    k.lib()
    return k


def say(*a):
    print(*a, flush=True)


def solve(kvs, w, direction=None, ctx=None):
    """Jacobi-PCG to 1e-8 of the workload's force on an FP32 context (a new
    one unless ctx is given); returns (report, phi)."""
    own = ctx is None
    if own:
        ctx = kvs.kvs_create(w.grid, precision=kvs.KVS_FP32)
    try:
        if own:
            kvs.kvs_set_material(ctx, w.G, w.rho, w.eta)
            kvs.kvs_set_force(ctx, w.F)
        if direction is not None:
            kvs.kvs_set_direction_precision(ctx, direction)
        rep = kvs.kvs_project(ctx, tol=1e-8, precond=kvs.KVS_PC_JACOBI)
        return rep, kvs.kvs_get_phi(ctx, (w.grid[2], w.grid[1], w.grid[0]))
    finally:
        if own:
            kvs.kvs_destroy(ctx)


@pytest.mark.parametrize("n", [64, 97])
def test_fp32_direction_reaches_the_tolerance(kvs, n):
    """The inclusion workload shrunk to n^3 (97^3: ragged tiles): with FP32
    directions (the default) and with FP64 ones, iteration counts within 3 %
    of each other (measured: 223 / 218 at 64^3, 253 / 248 at 97^3, 904 / 894
    at 256^3), the oracle's FP64 true residual of each phi below 1e-8, and the
    two phi within 1e-4 of each other in relative L2: each is within
    kappa * 1e-8 of the exact solution, kappa < 4 n^2 / pi^2 < 4e3 for the
    Jacobi-scaled 7-point Laplacian here."""
    w = cfg2_inclusions_fp32(n)
    b = oracle.divergence(w.grid, w.F)
    say(f"case cg direction fp32 {n}^3")
    rep32, phi32 = solve(kvs, w)
    say(f"case cg direction fp64 {n}^3")
    rep64, phi64 = solve(kvs, w, kvs.KVS_FP64)
    t32 = oracle.true_relres(w.grid, b, phi32)
    t64 = oracle.true_relres(w.grid, b, phi64)
    d = np.linalg.norm(phi32 - phi64) / np.linalg.norm(phi64)
    say(f"{n}^3: iterations {rep32['iters']} (fp32) / {rep64['iters']} (fp64), true residuals {t32:.3e} / "
        f"{t64:.3e}, phi difference {d:.2e}")
    assert rep32["status"] == 0 and rep64["status"] == 0
    assert abs(rep32["iters"] - rep64["iters"]) <= 0.03 * rep64["iters"]
    assert t32 < 1e-8 and t64 < 1e-8
    assert t32 == pytest.approx(rep32["relres_true"], rel=1e-6)
    assert d < 1e-4


def test_switching_direction_precision_on_one_context(kvs):
    """FP32 -> FP64 -> FP32 directions on one context give bitwise the phi
    of new contexts with each setting: a switch clears both direction buffers,
    whose outer planes the sweeps read as zeros (the other width's view would
    find the last solve's values there)."""
    w = cfg2_inclusions_fp32(48)
    say("case cg direction switch 48^3")
    ref = {d: solve(kvs, w, d)[1] for d in (kvs.KVS_FP32, kvs.KVS_FP64)}
    assert not np.array_equal(ref[kvs.KVS_FP32], ref[kvs.KVS_FP64])
    ctx = kvs.kvs_create(w.grid, precision=kvs.KVS_FP32)
    try:
        kvs.kvs_set_material(ctx, w.G, w.rho, w.eta)
        kvs.kvs_set_force(ctx, w.F)
        for d in (kvs.KVS_FP32, kvs.KVS_FP64, kvs.KVS_FP32, kvs.KVS_FP64):
            _, phi = solve(kvs, w, d, ctx=ctx)
            assert np.array_equal(phi, ref[d]), d
        with pytest.raises(Exception):
            kvs.kvs_set_direction_precision(ctx, 7)
    finally:
        kvs.kvs_destroy(ctx)
