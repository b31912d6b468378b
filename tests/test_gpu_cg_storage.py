"""The projection's CG with FP32 storage (the default of FP32 contexts):
the search direction in FP32 (r and phi FP64, updated with the stored
direction) and the residual in FP32 as well (reliable updates from the FP64
phi, the true residual confirmed), against the oracle's FP64 true residual
and the same solve in FP64 storage, and the switch between the settings on
one context."""
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


def solve(kvs, w, storage=None, ctx=None):
    """Jacobi-PCG to 1e-8 of the workload's force on an FP32 context (a new
    one unless ctx is given), storage = (direction, residual) precision or
    None for the defaults; returns (report, phi)."""
    own = ctx is None
    if own:
        ctx = kvs.kvs_create(w.grid, precision=kvs.KVS_FP32)
    try:
        if own:
            kvs.kvs_set_material(ctx, w.G, w.rho, w.eta)
            kvs.kvs_set_force(ctx, w.F)
        if storage is not None:
            kvs.kvs_set_direction_precision(ctx, storage[0])
            kvs.kvs_set_residual_precision(ctx, storage[1])
        rep = kvs.kvs_project(ctx, tol=1e-8, precond=kvs.KVS_PC_JACOBI)
        return rep, kvs.kvs_get_phi(ctx, (w.grid[2], w.grid[1], w.grid[0]))
    finally:
        if own:
            kvs.kvs_destroy(ctx)


@pytest.mark.parametrize("n", [64, 97])
def test_fp32_storage_reaches_the_tolerance(kvs, n):
    """The inclusion workload shrunk to n^3 (97^3: ragged tiles), solved with
    FP32 direction and residual (the default), FP32 direction only, and FP64
    storage: iteration counts within 5 % of the FP64 one, the oracle's FP64
    true residual of every phi below 1e-8 (and equal to the reported one),
    and the phi within 1e-4 of each other in relative L2: each is within
    kappa * 1e-8 of the exact solution, kappa < 4 n^2 / pi^2 < 4e3 for the
    Jacobi-scaled 7-point Laplacian here."""
    w = cfg2_inclusions_fp32(n)
    b = oracle.divergence(w.grid, w.F)
    runs = {}
    for name, st in (("fp32", None), ("fp32 direction", (kvs.KVS_FP32, kvs.KVS_FP64)),
                     ("fp64", (kvs.KVS_FP64, kvs.KVS_FP64))):
        say(f"case cg storage {name} {n}^3")
        rep, phi = solve(kvs, w, st)
        t = oracle.true_relres(w.grid, b, phi)
        runs[name] = (rep, phi, t)
        say(f"{n}^3 {name}: {rep['iters']} iterations, true residual {t:.3e}")
    rep64, phi64, _ = runs["fp64"]
    for name, (rep, phi, t) in runs.items():
        d = np.linalg.norm(phi - phi64) / np.linalg.norm(phi64)
        say(f"{n}^3 {name}: phi against fp64 {d:.2e}")
        assert rep["status"] == 0
        assert abs(rep["iters"] - rep64["iters"]) <= 0.05 * rep64["iters"]
        assert t < 1e-8
        assert t == pytest.approx(rep["relres_true"], rel=1e-6)
        assert d < 1e-4


def test_switching_storage_on_one_context(kvs):
    """Every change of direction and residual storage on one context gives
    bitwise the phi of a new context with that setting: a change clears the
    buffers whose outer planes the sweeps read as zeros (the other width's
    view would find the last solve's values there)."""
    w = cfg2_inclusions_fp32(48)
    say("case cg storage switch 48^3")
    F32, F64 = kvs.KVS_FP32, kvs.KVS_FP64
    order = [(F32, F32), (F64, F64), (F32, F64), (F64, F32), (F32, F32), (F64, F64)]
    ref = {st: solve(kvs, w, st)[1] for st in set(order)}
    assert not np.array_equal(ref[(F32, F32)], ref[(F64, F64)])
    ctx = kvs.kvs_create(w.grid, precision=kvs.KVS_FP32)
    try:
        kvs.kvs_set_material(ctx, w.G, w.rho, w.eta)
        kvs.kvs_set_force(ctx, w.F)
        for st in order:
            _, phi = solve(kvs, w, st, ctx=ctx)
            assert np.array_equal(phi, ref[st]), st
        with pytest.raises(Exception):
            kvs.kvs_set_direction_precision(ctx, 7)
        with pytest.raises(Exception):
            kvs.kvs_set_residual_precision(ctx, -1)
    finally:
        kvs.kvs_destroy(ctx)
