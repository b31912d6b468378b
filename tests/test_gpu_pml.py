"""The absorbing layer (C-PML, oracle/pml.py) on the GPU, through the C ABI:
parity with the oracle (FP64 1e-12, FP32 2e-5) on ragged heterogeneous
viscous grids with a force, memory reset with the state, absorption at a
larger size against a reference domain, and the error paths."""
import numpy as np
import pytest

import oracle
from oracle import pml
from oracle.analysis import rel_l2
from workloads import curl_wavespeed_case, gaussian_push, spherical_inclusions

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


def hetero(shape, seed):
    nx, ny, nz = shape
    h = 0.25e-3
    grid = (nx, ny, nz, h, h * 1.1, h * 0.9)
    rng = np.random.default_rng(seed)
    G, rho, eta, _ = spherical_inclusions(grid, rng, 4, (2e3, 1000.0, 0.5), (0.8e-3, 2e-3), (1e3, 1e4),
                                          (1000.0, 1100.0), (0.0, 1.5), 1)
    F = gaussian_push(grid, 0.8e-3, 2e-3, 1e4) + 50.0 * rng.standard_normal((3, nz, ny, nx))
    return grid, G, rho, eta, F


@pytest.mark.parametrize("shape,L", [((29, 23, 31), 4), ((70, 13, 17), 5), ((11, 11, 11), 4)])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_pml_matches_oracle(kvs, shape, L, precision):
    say(f"case pml {shape} L {L} precision {precision}")
    grid, G, rho, eta, F = hetero(shape, 3)
    dt = 0.4 * oracle.stable_dt(grid, G, rho, eta)
    FS, _, _ = oracle.project(grid, F, tol=1e-11)
    env = np.array([1.0, 1.0, 0.5, 0.0, 2.0])
    nsteps = 90
    probes = np.array([[i, shape[1] // 2, shape[2] // 2] for i in range(shape[0])]
                      + [[shape[0] // 2, j, 2] for j in range(shape[1])])
    _, _, tr_o = pml.run_pml(grid, G, rho, eta, dt, nsteps, L, FS=FS, env=env, probes=probes, comp=3)
    ctx = kvs.kvs_create(grid, precision=precision)
    try:
        kvs.kvs_set_material(ctx, G, rho, eta)
        kvs.kvs_set_dt(ctx, dt)
        kvs.kvs_set_pml(ctx, L)
        kvs.kvs_set_projected_force(ctx, FS)
        kvs.kvs_set_envelope(ctx, env)
        kvs.kvs_set_probes(ctx, probes, 3)
        kvs.kvs_step(ctx, nsteps)
        tr = kvs.kvs_read_traces(ctx, len(probes), 3)
        # the layer's memory is part of the state: a reset and the same run again
        kvs.kvs_reset_state(ctx)
        kvs.kvs_step(ctx, nsteps)
        tr2 = kvs.kvs_read_traces(ctx, len(probes), 3)
    finally:
        kvs.kvs_destroy(ctx)
    assert rel_l2(tr, tr_o) < (1e-12 if precision == 0 else 2e-5)
    assert np.array_equal(tr2, tr)


def test_pml_uniform_medium_curl_state(kvs):
    """Uniform viscous medium (scalar material path) from the curl state."""
    w = curl_wavespeed_case(n=40, h=0.5e-3, sigma=1.5e-3, offsets_mm=(2.0, 4.0))
    G, rho, eta = 4e3, 1000.0, 0.3
    dt = 0.4 * oracle.stable_dt(w["grid"], G, rho, eta)
    u0, w0 = oracle.curl_state(w["grid"], w["A"], dt)
    _, _, tr_o = pml.run_pml(w["grid"], G, rho, eta, dt, 120, 6, R=1e-4, alpha_max=500.0, u=u0, w=w0,
                             probes=w["probes"], comp=2)
    ctx = kvs.kvs_create(w["grid"], precision=kvs.KVS_FP64)
    try:
        kvs.kvs_set_material_uniform(ctx, G, rho, eta)
        kvs.kvs_set_dt(ctx, dt)
        kvs.kvs_set_pml(ctx, 6, R=1e-4, alpha_max=500.0)
        kvs.kvs_set_state_curl(ctx, w["A"])
        kvs.kvs_set_probes(ctx, w["probes"], 2)
        kvs.kvs_step(ctx, 120)
        tr = kvs.kvs_read_traces(ctx, len(w["probes"]), 1)
    finally:
        kvs.kvs_destroy(ctx)
    assert rel_l2(tr, tr_o) < 1e-12


def test_pml_absorbs_at_scale(kvs):
    """128^3 curl source with a 12-cell layer against the same source on 256^3
    (no reflection reaches the sensors within the window), FP32: the layer's
    trace error is below 1e-3 of the Dirichlet wall's."""
    h, G, rho, eta = 0.25e-3, 4e3, 1000.0, 0.2
    say("case pml absorption 128^3 vs 256^3")

    def run(n, L):
        w = curl_wavespeed_case(n=n, h=h, sigma=1.0e-3, offsets_mm=(3.0, 6.0, 9.0))
        ctx = kvs.kvs_create(w["grid"], precision=kvs.KVS_FP32)
        try:
            kvs.kvs_set_material_uniform(ctx, G, rho, eta)
            dt = 0.4 * kvs.kvs_stable_dt(ctx)
            kvs.kvs_set_dt(ctx, dt)
            if L:
                kvs.kvs_set_pml(ctx, L)
            kvs.kvs_set_state_curl(ctx, w["A"])
            kvs.kvs_set_probes(ctx, w["probes"], 2)
            kvs.kvs_step(ctx, int(14e-3 / dt))
            return kvs.kvs_read_traces(ctx, len(w["probes"]), 1)
        finally:
            kvs.kvs_destroy(ctx)

    ref = run(256, 0)
    e_wall = rel_l2(run(128, 0), ref)
    e_pml = rel_l2(run(128, 12), ref)
    say(f"pml: wall {e_wall:.3e}, layer {e_pml:.3e}")
    assert e_wall > 0.05 and e_pml < 1e-3 * e_wall


def test_pml_full_size_256_matches_oracle(kvs):
    """The absorbing layer's benchmark configuration: the 256^3 inclusion
    medium, no sponge, a 10-cell layer, the autotuned tile shape, FP32 state.
    Two steps from a white-noise state (zero on the Dirichlet layer; every
    layer cell and face active, the memory variables non-zero after the
    first step) against the FP64
    oracle on the whole grid: w within 1e-5 of max|w|, u within that plus
    one FP32 rounding of max|u|."""
    from oracle.pml import run_pml
    from workloads import cfg2_inclusions_fp32
    wl = cfg2_inclusions_fp32(256)
    grid = wl.grid
    shp = (3, grid[2], grid[1], grid[0])
    rng = np.random.default_rng(77)
    u0 = (rng.standard_normal(shp) * 1e-6).astype(np.float32).astype(np.float64)
    w0 = (rng.standard_normal(shp) * 1e-8).astype(np.float32).astype(np.float64)
    for a in (u0, w0):  # the Dirichlet layer holds zeros (kvs_set_state enforces it)
        a[:, [0, -1], :, :] = 0.0
        a[:, :, [0, -1], :] = 0.0
        a[:, :, :, [0, -1]] = 0.0
    say("case pml full size 256^3, 10 cells, 2 steps from noise")
    ctx = kvs.kvs_create(grid, precision=kvs.KVS_FP32)
    try:
        kvs.kvs_set_material(ctx, wl.G, wl.rho, wl.eta)
        dt = wl.dt_factor * kvs.kvs_stable_dt(ctx)
        kvs.kvs_set_dt(ctx, dt)
        kvs.kvs_set_pml(ctx, 10)
        variant, _ = kvs.kvs_autotune_step(ctx, 10)
        kvs.kvs_set_state(ctx, u0, w0, 0)
        kvs.kvs_step(ctx, 2)
        u, w, step = kvs.kvs_get_state(ctx, shp[1:])
    finally:
        kvs.kvs_destroy(ctx)
    say(f"pml full size: variant {variant}, oracle running")
    u_o, w_o, _ = run_pml(grid, wl.G, wl.rho, wl.eta, dt, 2, 10, u=u0, w=w0)
    ew = np.abs(w - w_o).max() / np.abs(w_o).max()
    eu = np.abs(u - u_o).max()
    say(f"pml full size: max |w - w_o| / max|w_o| {ew:.2e}, max |u - u_o| {eu:.2e} (max|u| {np.abs(u_o).max():.2e})")
    assert step == 2
    assert ew < 1e-5
    assert eu < 1e-5 * np.abs(w_o).max() + 2.0 ** -23 * np.abs(u_o).max()


def test_pml_errors(kvs):
    grid = (20, 20, 20, 1e-3, 1e-3, 1e-3)
    ctx = kvs.kvs_create(grid, sponge_cells=4)
    try:
        with pytest.raises(kvs.KvsError) as e:
            kvs.kvs_set_pml(ctx, 4)
        assert e.value.status == kvs.KVS_EINVAL
    finally:
        kvs.kvs_destroy(ctx)
    ctx = kvs.kvs_create(grid)
    try:
        for cells, R in ((9, 1e-5), (-1, 1e-5), (4, 0.0), (4, 1.5)):
            with pytest.raises(kvs.KvsError) as e:
                kvs.kvs_set_pml(ctx, cells, R=R)
            assert e.value.status == kvs.KVS_EINVAL, (cells, R)
        kvs.kvs_set_pml(ctx, 8)
        kvs.kvs_set_pml(ctx, 0)
    finally:
        kvs.kvs_destroy(ctx)
    b = kvs.kvs_batch_create([grid], precision=kvs.KVS_FP32)
    try:
        c0 = kvs.kvs_batch_instance(b, 0)
        kvs.kvs_set_material_uniform(c0, 2e3, 1000.0, 0.1)
        kvs.kvs_set_dt(c0, 0.4 * kvs.kvs_stable_dt(c0))
        kvs.kvs_set_pml(c0, 4)
        with pytest.raises(kvs.KvsError) as e:
            kvs.kvs_batch_step(b, 1)
        assert e.value.status == kvs.KVS_ESTATE
    finally:
        kvs.kvs_batch_destroy(b)
