"""Batched sweeps: many homogeneous instances advanced by one launch per step
(replayed as a hipGraph), checked instance by instance against the oracle
and against single-context stepping."""
import numpy as np
import pytest

import oracle
from oracle.analysis import rel_l2
from workloads import gaussian_push, x_line_probes

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


H = 0.25e-3
CASES = [  # (edge or (nx, ny, nz), G, eta)
    ((24, 24, 24), 2e3, 0.0),
    ((30, 28, 26), 5e3, 0.7),
    ((32, 32, 32), 1e3, 1.5),
    ((32, 32, 32), 8e3, 0.2),
    ((40, 22, 34), 3e3, 0.0),
]
L_SPONGE = 4
NSTEPS = 90


def setup_instance(kvs, ctx, grid, G, eta, F, FS=None):
    """Uniform medium, dt = 0.4 x limit, 30 us push; the projected force is
    the given FS (the oracle's, so that only stepping is compared), else the
    GPU projection of F."""
    kvs.kvs_set_material_uniform(ctx, G, 1000.0, eta)
    dt = 0.4 * kvs.kvs_stable_dt(ctx)
    kvs.kvs_set_dt(ctx, dt)
    env = np.ones(max(1, int(round(30e-6 / dt))))
    kvs.kvs_set_envelope(ctx, env)
    if FS is not None:
        kvs.kvs_set_projected_force(ctx, FS)
    else:
        kvs.kvs_set_force(ctx, F)
        kvs.kvs_project(ctx, tol=1e-12)
    return dt, env


def make_batch(kvs, precision):
    grids = [tuple(s) + (H, H, H) for s, _, _ in CASES]
    b = kvs.kvs_batch_create(grids, precision=precision, sponge_cells=L_SPONGE, sponge_sigma_max=800.0)
    info = []
    for i, ((shape), G, eta) in enumerate(CASES):
        grid = grids[i]
        ctx = kvs.kvs_batch_instance(b, i)
        F = gaussian_push(grid, 0.75e-3, 1.5e-3, 1e4)
        FS_o, _, _ = oracle.project(grid, F, tol=1e-12)
        dt, env = setup_instance(kvs, ctx, grid, G, eta, F, FS=FS_o)
        probes = x_line_probes(grid)
        kvs.kvs_batch_set_probes(b, i, probes)
        info.append((grid, G, eta, FS_o, dt, env, probes))
    kvs.kvs_batch_set_component(b, 2)
    return b, info


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_instances_match_oracle(kvs, precision):
    say(f"case batch vs oracle precision {precision}")
    b, info = make_batch(kvs, precision)
    try:
        kvs.kvs_batch_step(b, NSTEPS)
        traces = [kvs.kvs_batch_read_traces(b, i, len(info[i][6])) for i in range(len(info))]
    finally:
        kvs.kvs_batch_destroy(b)
    for i, (grid, G, eta, FS_o, dt, env, probes) in enumerate(info):
        _, _, tr_o = oracle.run(grid, G, 1000.0, eta, dt, NSTEPS, FS=FS_o, env=env, probes=probes, comp=2,
                                sponge_cells=L_SPONGE, sigma_max=800.0)
        err = rel_l2(traces[i], tr_o[:, :, 0])
        say(f"instance {i}: rel L2 {err:.2e}")
        assert err < (1e-12 if precision == 0 else 2e-5), (i, err)


def test_batch_equals_single_context_bitwise_and_replays(kvs):
    """FP32: the batched step computes exactly what the single-context step
    (same tile shape) computes; a replayed graph after reset and a run split
    at an odd step give identical traces."""
    say("case batch bitwise / replay / odd split")
    b, info = make_batch(kvs, 1)
    try:
        kvs.kvs_batch_step(b, NSTEPS)
        first = [kvs.kvs_batch_read_traces(b, i, len(info[i][6])) for i in range(len(info))]
        kvs.kvs_batch_reset(b)
        kvs.kvs_batch_step(b, NSTEPS)  # same start, steps, trace slot: graph replay
        second = [kvs.kvs_batch_read_traces(b, i, len(info[i][6])) for i in range(len(info))]
        kvs.kvs_batch_reset(b)
        kvs.kvs_batch_step(b, 37)
        kvs.kvs_batch_step(b, NSTEPS - 37)
        split = [kvs.kvs_batch_read_traces(b, i, len(info[i][6])) for i in range(len(info))]
        shp = [(g[2], g[1], g[0]) for g, *_ in info]
        states = [kvs.kvs_get_state(kvs.kvs_batch_instance(b, i), shp[i]) for i in range(len(info))]
    finally:
        kvs.kvs_batch_destroy(b)
    for i in range(len(info)):
        assert np.array_equal(first[i], second[i]) and np.array_equal(first[i], split[i])
        assert states[i][2] == NSTEPS
    # single contexts, tile shape of the batch (64 x 8, one cell per lane)
    for i, (grid, G, eta, FS_o, dt, env, probes) in enumerate(info):
        ctx = kvs.kvs_create(grid, precision=1, sponge_cells=L_SPONGE, sponge_sigma_max=800.0)
        try:
            setup_instance(kvs, ctx, grid, G, eta, None, FS=FS_o)
            kvs.kvs_set_probes(ctx, probes, 2)
            kvs.kvs_set_step_variant(ctx, 1)
            kvs.kvs_step(ctx, NSTEPS)
            tr = kvs.kvs_read_traces(ctx, len(probes), 1)[:, :, 0]
        finally:
            kvs.kvs_destroy(ctx)
        assert np.array_equal(tr, first[i]), i


WIDE = [  # (nx, ny, nz), G, eta: x rows that take each row-fitted tile width
    ((40, 30, 20), 2e3, 0.0),     # 64 x 8
    ((100, 20, 18), 5e3, 0.7),    # 128 x 8 (FP64: 128 x 4)
    ((150, 16, 20), 1e3, 1.5),    # 192 x 4 (FP64: 128 x 4, two per row)
    ((210, 14, 12), 8e3, 0.2),    # 256 x 4 (FP64: 128 x 4, two per row)
    ((300, 10, 10), 3e3, 0.0),    # two 256 x 4 tiles per row (FP64: three 128 x 4)
]


@pytest.mark.parametrize("precision", [0, 1])
def test_row_fitted_batch_tiles_match_oracle_and_single_contexts(kvs, precision):
    """The row-fitted batch tiling (one launch per tile width per step) on
    instances whose x rows take every width, a ragged last tile and two
    tiles per row: traces against the oracle (FP64 1e-12, FP32 2e-5) and,
    in FP32, bitwise against each instance stepped alone with the same tile
    shape."""
    say(f"case row-fitted batch tiles precision {precision}")
    grids = [tuple(sh) + (H, H, H) for sh, _, _ in WIDE]
    b = kvs.kvs_batch_create(grids, precision=precision, sponge_cells=L_SPONGE, sponge_sigma_max=800.0)
    info = []
    try:
        for i, (sh, G, eta) in enumerate(WIDE):
            grid = grids[i]
            F = gaussian_push(grid, 0.75e-3, 1.5e-3, 1e4)
            FS_o, _, _ = oracle.project(grid, F, tol=1e-12)
            dt, env = setup_instance(kvs, kvs.kvs_batch_instance(b, i), grid, G, eta, F, FS=FS_o)
            probes = x_line_probes(grid)
            kvs.kvs_batch_set_probes(b, i, probes)
            info.append((grid, G, eta, FS_o, dt, env, probes))
        kvs.kvs_batch_set_component(b, 2)
        kvs.kvs_batch_set_tuning(b, kvs.KVS_BATCH_FIT_ROWS, 16)
        kvs.kvs_batch_step(b, NSTEPS)
        traces = [kvs.kvs_batch_read_traces(b, i, len(info[i][6])) for i in range(len(info))]
    finally:
        kvs.kvs_batch_destroy(b)
    for i, (grid, G, eta, FS_o, dt, env, probes) in enumerate(info):
        _, _, tr_o = oracle.run(grid, G, 1000.0, eta, dt, NSTEPS, FS=FS_o, env=env, probes=probes, comp=2,
                                sponge_cells=L_SPONGE, sigma_max=800.0)
        err = rel_l2(traces[i], tr_o[:, :, 0])
        say(f"instance {i} nx {grid[0]}: rel L2 {err:.2e}")
        assert err < (1e-12 if precision == 0 else 2e-5), (i, err)
    if precision == 1:
        # single-context variants of the same tile shapes (64 x 8, 128 x 8,
        # 256 x 4); the 192 x 4 tile has no single-context variant
        same_shape = {0: 1, 1: 6, 3: 7, 4: 7}
        for i, v in same_shape.items():
            grid, G, eta, FS_o, dt, env, probes = info[i]
            ctx = kvs.kvs_create(grid, precision=1, sponge_cells=L_SPONGE, sponge_sigma_max=800.0)
            try:
                setup_instance(kvs, ctx, grid, G, eta, None, FS=FS_o)
                kvs.kvs_set_probes(ctx, probes, 2)
                kvs.kvs_set_step_tuning(ctx, v, 16, 1)
                kvs.kvs_step(ctx, NSTEPS)
                tr = kvs.kvs_read_traces(ctx, len(probes), 1)[:, :, 0]
            finally:
                kvs.kvs_destroy(ctx)
            assert np.array_equal(tr, traces[i]), i


def test_batch_shared_projection_and_call_order(kvs):
    say("case batch share projection / call order")
    grid = (32, 32, 32, H, H, H)
    b = kvs.kvs_batch_create([grid, grid], precision=1, sponge_cells=L_SPONGE)
    try:
        F = gaussian_push(grid, 0.75e-3, 1.5e-3, 1e4)
        c0, c1 = kvs.kvs_batch_instance(b, 0), kvs.kvs_batch_instance(b, 1)
        setup_instance(kvs, c0, grid, 2e3, 0.3, F)
        kvs.kvs_set_material_uniform(c1, 6e3, 1000.0, 0.9)
        kvs.kvs_set_dt(c1, 0.4 * kvs.kvs_stable_dt(c1))
        kvs.kvs_set_envelope(c1, [1.0, 1.0])
        with pytest.raises(kvs.KvsError) as e:
            kvs.kvs_batch_step(b, 3)  # instance 1 has no projection
        assert e.value.status == kvs.KVS_ESTATE
        kvs.kvs_batch_share_projection(b, 0, 1)
        shp = (32, 32, 32)
        assert np.array_equal(kvs.kvs_get_projected_force(c0, shp), kvs.kvs_get_projected_force(c1, shp))
        kvs.kvs_batch_step(b, 3)
        kvs.kvs_step(c1, 1)  # outside the batch
        with pytest.raises(kvs.KvsError) as e:
            kvs.kvs_batch_step(b, 1)
        assert e.value.status == kvs.KVS_ESTATE
    finally:
        kvs.kvs_batch_destroy(b)


def test_every_batch_tile_shape_matches_oracle(kvs):
    """Each batch tile shape and a short z chunk give the oracle's traces
    (FP32 bar), and autotuning leaves the state untouched."""
    b, info = make_batch(kvs, 1)
    try:
        v0, z0, ms = kvs.kvs_batch_autotune(b, 2)
        assert len(ms) == kvs.kvs_num_step_variants() + 1 and np.all(ms > 0)
        assert (v0 == kvs.KVS_BATCH_FIT_ROWS or 0 <= v0 < len(ms) - 1) and z0 in (16, 32, 64)
        for i in range(len(info)):
            u, w, s = kvs.kvs_get_state(kvs.kvs_batch_instance(b, i), (info[i][0][2], info[i][0][1], info[i][0][0]))
            assert s == 0 and not u.any() and not w.any()
        results = {}
        for v in list(range(kvs.kvs_num_step_variants())) + [kvs.KVS_BATCH_FIT_ROWS]:
            say(f"case batch shape {v}")
            kvs.kvs_batch_reset(b)
            kvs.kvs_batch_set_tuning(b, v, 16)
            kvs.kvs_batch_step(b, NSTEPS)
            results[v] = [kvs.kvs_batch_read_traces(b, i, len(info[i][6])) for i in range(len(info))]
    finally:
        kvs.kvs_batch_destroy(b)
    for i, (grid, G, eta, FS_o, dt, env, probes) in enumerate(info):
        _, _, tr_o = oracle.run(grid, G, 1000.0, eta, dt, NSTEPS, FS=FS_o, env=env, probes=probes, comp=2,
                                sponge_cells=L_SPONGE, sigma_max=800.0)
        for v, tr in results.items():
            assert rel_l2(tr[i], tr_o[:, :, 0]) < 2e-5, (v, i)


def test_batch_rerun_with_changed_envelope_matches_oracle(kvs):
    """A run, a reset, a longer push on one instance and a run of the same
    length from the same step: the second run must not replay the graph of
    the first (its steps past the old push read no force), so every
    instance matches the oracle with its new envelope (FP32 bar); a third
    run with the envelope switched off entirely matches too."""
    say("case batch rerun with a changed envelope")
    b, info = make_batch(kvs, 1)
    try:
        kvs.kvs_batch_step(b, NSTEPS)
        kvs.kvs_batch_reset(b)
        grid, G, eta, FS_o, dt, env, probes = info[1]
        long_env = np.ones(len(env) + 25)
        kvs.kvs_set_envelope(kvs.kvs_batch_instance(b, 1), long_env)
        kvs.kvs_batch_step(b, NSTEPS)
        second = [kvs.kvs_batch_read_traces(b, i, len(info[i][6])) for i in range(len(info))]
        kvs.kvs_batch_reset(b)
        for i in range(len(info)):
            kvs.kvs_set_envelope(kvs.kvs_batch_instance(b, i), [])
        kvs.kvs_batch_step(b, NSTEPS)
        third = [kvs.kvs_batch_read_traces(b, i, len(info[i][6])) for i in range(len(info))]
    finally:
        kvs.kvs_batch_destroy(b)
    for i, (grid, G, eta, FS_o, dt, env, probes) in enumerate(info):
        e = long_env if i == 1 else env
        _, _, tr_o = oracle.run(grid, G, 1000.0, eta, dt, NSTEPS, FS=FS_o, env=e, probes=probes, comp=2,
                                sponge_cells=L_SPONGE, sigma_max=800.0)
        err = rel_l2(second[i], tr_o[:, :, 0])
        say(f"instance {i}: rel L2 {err:.2e} (push {len(e)} steps)")
        assert err < 2e-5, (i, err)
        assert not third[i].any(), i


def test_batch_sweep_edges_96_and_160_match_oracle(kvs):
    """Instances of the 64-instance sweep's shape with edges that are not
    multiples of the tile width (96 and 160 cells: several x tiles with a
    partial last one), in the sweep's launch configuration (autotuned tile
    shape and z chunk, 8-cell sponge of default strength, 100 us push, dt =
    0.4 x the stable limit): lateral-line u_z traces over 200 steps against
    the oracle's run from the oracle's own projection, relative L2 within
    2e-5 per instance."""
    say("case batch edges 96 and 160")
    h = 0.25e-3
    draws = [(96, 10 ** (3 + 4 / 9), 0.7), (160, 10 ** (3 + 7 / 9), 1.2)]
    grids = [(e, e, e, h, h, h) for e, _, _ in draws]
    nsteps = 200
    b = kvs.kvs_batch_create(grids, precision=1, sponge_cells=8, sponge_sigma_max=-1.0)
    info = []
    try:
        for i, ((e, G, eta), grid) in enumerate(zip(draws, grids)):
            ctx = kvs.kvs_batch_instance(b, i)
            kvs.kvs_set_material_uniform(ctx, G, 1000.0, eta)
            dt = 0.4 * kvs.kvs_stable_dt(ctx)
            kvs.kvs_set_dt(ctx, dt)
            env = np.ones(int(round(100e-6 / dt)))
            kvs.kvs_set_envelope(ctx, env)
            F = gaussian_push(grid, 1e-3, 4e-3, 1e4)
            FS_o, _, rep_o = oracle.project(grid, F, tol=1e-8, jacobi=True)
            kvs.kvs_set_projected_force(ctx, FS_o)
            probes = x_line_probes(grid)
            kvs.kvs_batch_set_probes(b, i, probes)
            smax = kvs.kvs_sponge_sigma_max(ctx)
            info.append((grid, G, eta, dt, env, FS_o, probes, smax))
        kvs.kvs_batch_set_component(b, 2)
        v, z, _ = kvs.kvs_batch_autotune(b, 3)
        kvs.kvs_batch_step(b, nsteps)
        traces = [kvs.kvs_batch_read_traces(b, i, len(info[i][6])) for i in range(len(info))]
    finally:
        kvs.kvs_batch_destroy(b)
    for i, (grid, G, eta, dt, env, FS_o, probes, smax) in enumerate(info):
        assert smax == pytest.approx(oracle.default_sigma_max(grid, G, 1000.0, 8), rel=1e-13)
        _, _, tr_o = oracle.run(grid, G, 1000.0, eta, dt, nsteps, FS=FS_o, env=env, probes=probes, comp=2,
                                sponge_cells=8, sigma_max=smax)
        err = rel_l2(traces[i], tr_o[:, :, 0])
        say(f"edge {grid[0]}: tile variant {v}, z {z}, rel L2 {err:.2e}")
        assert err < 2e-5, (grid[0], err)


SMALL = [  # (nx, ny, nz), G, eta: every state fits one workgroup's LDS (FP64: 48 B per node, <= 3200 nodes)
    ((13, 14, 15), 2e3, 0.0),
    ((12, 18, 9), 5e3, 0.7),
    ((17, 11, 13), 1e3, 1.5),
    ((9, 9, 9), 8e3, 0.2),
]


def make_small_batch(kvs, precision, cases=SMALL, L=2):
    grids = [tuple(s) + (H, H, H) for s, _, _ in cases]
    b = kvs.kvs_batch_create(grids, precision=precision, sponge_cells=L, sponge_sigma_max=800.0)
    info = []
    for i, (_, G, eta) in enumerate(cases):
        grid = grids[i]
        ctx = kvs.kvs_batch_instance(b, i)
        F = gaussian_push(grid, 0.5e-3, 1.0e-3, 1e4) + 30.0 * np.random.default_rng(i).standard_normal(
            (3, grid[2], grid[1], grid[0]))
        FS_o, _, _ = oracle.project(grid, F, tol=1e-12)
        dt, env = setup_instance(kvs, ctx, grid, G, eta, F, FS=FS_o)
        env = np.concatenate([env, [0.0, 0.5, 0.0, 1.0]])  # switches on and off
        kvs.kvs_set_envelope(ctx, env)
        probes = np.array([[ii, grid[1] // 2, grid[2] // 2] for ii in range(grid[0])])
        kvs.kvs_batch_set_probes(b, i, probes)
        info.append((grid, G, eta, FS_o, dt, env, probes))
    kvs.kvs_batch_set_component(b, 1)
    return b, info


@pytest.mark.parametrize("precision", [0, 1])
def test_persistent_small_batch_matches_oracle(kvs, precision):
    """Small instances take the persistent path (one launch for the whole run,
    state in LDS): traces of the y component against the oracle (FP64 1e-12,
    FP32 2e-5) over a run split at an odd step, the final state equal to the
    oracle's; the per-step path gives the same traces to the bar."""
    say(f"case persistent small batch precision {precision}")
    b, info = make_small_batch(kvs, precision)
    try:
        assert kvs.kvs_batch_uses_persistent(b)
        kvs.kvs_batch_step(b, 37)
        kvs.kvs_batch_step(b, 53)
        traces = [kvs.kvs_batch_read_traces(b, i, len(info[i][6])) for i in range(len(info))]
        states = [kvs.kvs_get_state(kvs.kvs_batch_instance(b, i), (g[2], g[1], g[0])) for i, (g, *_) in
                  enumerate(info)]
        kvs.kvs_batch_reset(b)
        kvs.kvs_batch_set_persistent(b, False)
        assert not kvs.kvs_batch_uses_persistent(b)
        kvs.kvs_batch_step(b, 90)
        tiled = [kvs.kvs_batch_read_traces(b, i, len(info[i][6])) for i in range(len(info))]
    finally:
        kvs.kvs_batch_destroy(b)
    bar = 1e-12 if precision == 0 else 2e-5
    for i, (grid, G, eta, FS_o, dt, env, probes) in enumerate(info):
        u_o, w_o, tr_o = oracle.run(grid, G, 1000.0, eta, dt, 90, FS=FS_o, env=env, probes=probes, comp=1,
                                    sponge_cells=2, sigma_max=800.0)
        err = rel_l2(traces[i], tr_o[:, :, 0])
        say(f"instance {i} {grid[:3]}: persistent rel L2 {err:.2e}, per-step {rel_l2(tiled[i], tr_o[:, :, 0]):.2e}")
        assert err < bar and rel_l2(tiled[i], tr_o[:, :, 0]) < bar, (i, err)
        u, w, step = states[i]
        assert step == 90
        assert rel_l2(u, u_o) < bar and rel_l2(w, w_o) < bar


def test_persistent_path_needs_every_instance_to_fit(kvs):
    """One instance too large for a workgroup's LDS sends the whole batch to
    the per-step launches; the small instances still match the oracle."""
    say("case persistent fallback")
    cases = SMALL[:2] + [((30, 28, 26), 5e3, 0.7)]
    b, info = make_small_batch(kvs, 1, cases=cases)
    try:
        assert not kvs.kvs_batch_uses_persistent(b)
        kvs.kvs_batch_step(b, 40)
        traces = [kvs.kvs_batch_read_traces(b, i, len(info[i][6])) for i in range(len(info))]
    finally:
        kvs.kvs_batch_destroy(b)
    for i, (grid, G, eta, FS_o, dt, env, probes) in enumerate(info):
        _, _, tr_o = oracle.run(grid, G, 1000.0, eta, dt, 40, FS=FS_o, env=env, probes=probes, comp=1,
                                sponge_cells=2, sigma_max=800.0)
        assert rel_l2(traces[i], tr_o[:, :, 0]) < 2e-5
