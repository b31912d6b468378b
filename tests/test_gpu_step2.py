"""Two-step launches (temporal blocking of the Sec. 3.1 update): the state
and the probe traces after any number of steps are bitwise those of one-step
launches, on ragged grids, with several z segments, with force steps and odd
step counts mixed in; the contexts where the two-step kernel does not apply
fall back to one-step launches; kernel timing counts steps; and the FP32
traces stay within 2e-5 of the FP64 oracle."""
import numpy as np
import pytest

import oracle
from oracle.analysis import rel_l2
from workloads import cfg2_inclusions_fp32, spherical_inclusions

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


def medium(grid, seed):
    """Background plus six spheres of 2-6 cells radius (h = 0.25 mm)."""
    rng = np.random.default_rng(seed)
    G, rho, eta, _ = spherical_inclusions(grid, rng, 6, (3e3, 1000.0, 0.5), (0.5e-3, 1.5e-3), (1e3, 2e4),
                                          (950.0, 1100.0), (0.1, 2.0), 1)
    return G, rho, eta


def probe_set(grid, seed):
    """A lateral line, then random distinct cells (boundary rows included) off
    the planes k = 0, nz - 1."""
    nx, ny, nz = grid[:3]
    rng = np.random.default_rng(seed)
    cells = [(i, ny // 2, nz // 2) for i in range(nx)]
    seen = set(cells)
    while len(cells) < min(nx + 40, nx * ny * (nz - 2)):
        c = (int(rng.integers(0, nx)), int(rng.integers(0, ny)), int(rng.integers(1, nz - 1)))
        if c not in seen:
            seen.add(c)
            cells.append(c)
    return np.array(cells, dtype=np.int64)


def run(kvs, grid, mat, F, env, probes, comp, calls, blocking, zchunk=0, variant=None):
    ctx = kvs.kvs_create(grid, precision=kvs.KVS_FP32, sponge_cells=4, sponge_sigma_max=-1.0)
    try:
        if np.isscalar(mat[0]):
            kvs.kvs_set_material_uniform(ctx, *mat)
        else:
            kvs.kvs_set_material(ctx, *mat)
        kvs.kvs_set_dt(ctx, 0.5 * kvs.kvs_stable_dt(ctx))
        kvs.kvs_set_force(ctx, F)
        kvs.kvs_project(ctx, tol=1e-8, precond=kvs.KVS_PC_JACOBI)
        kvs.kvs_set_envelope(ctx, env)
        kvs.kvs_set_probes(ctx, probes, comp)
        if variant is not None or zchunk:
            kvs.kvs_set_step_tuning(ctx, variant or 0, zchunk)
        kvs.kvs_set_step_blocking(ctx, blocking)
        applies = kvs.kvs_step_blocking_applies(ctx)
        for n in calls:
            kvs.kvs_step(ctx, n)
        tr = kvs.kvs_read_traces(ctx, len(probes), 3 if comp == 3 else 1)
        shp = (grid[2], grid[1], grid[0])
        u, w, step = kvs.kvs_get_state(ctx, shp)
    finally:
        kvs.kvs_destroy(ctx)
    return applies, tr, u, w, step


@pytest.mark.parametrize("nx,ny,nz,zchunk,comp,het", [
    (70, 41, 36, 0, 2, True),     # 128-wide tiles, odd row count
    (70, 41, 36, 5, 3, True),     # seven z segments, the last ragged; all components
    (200, 30, 40, 0, 0, True),    # 256-wide tiles
    (256, 24, 19, 4, 1, True),    # full-width rows, ragged z segments
    (5, 3, 3, 0, 2, True),        # one interior cell
    (96, 35, 30, 7, 2, False),    # homogeneous medium
    (230, 17, 22, 0, 3, False),   # homogeneous, 256-wide tiles
])
def test_two_step_launches_match_one_step_bitwise(kvs, nx, ny, nz, zchunk, comp, het):
    h = 0.25e-3
    grid = (nx, ny, nz, h, h, h)
    say(f"case two-step bitwise {nx}x{ny}x{nz} zchunk {zchunk} comp {comp} heterogeneous {het}")
    mat = medium(grid, nx + ny + nz) if het else (4e3, 1050.0, 0.9)
    rng = np.random.default_rng(7)
    F = rng.standard_normal((3, nz, ny, nx))
    env = np.r_[np.ones(7), 0.0, 0.0, 1.0]  # force on steps 0..6 and 9
    probes = probe_set(grid, 3)
    calls = (1, 10, 6, 14)  # 31 steps: odd counts, force steps at odd and even offsets
    ref = run(kvs, grid, mat, F, env, probes, comp, calls, blocking=1, zchunk=zchunk)
    got = run(kvs, grid, mat, F, env, probes, comp, calls, blocking=2, zchunk=zchunk)
    assert not ref[0] or got[0]
    assert got[0], "the two-step kernel should apply to this context"
    assert ref[4] == got[4] == sum(calls)
    assert ref[1].shape == got[1].shape == (sum(calls), len(probes), 3 if comp == 3 else 1)
    for name, a, b in zip(("traces", "u", "w"), ref[1:4], got[1:4]):
        diff = np.max(np.abs(a - b)) / max(np.max(np.abs(a)), 1e-300)
        say(f"  {name}: max |diff| / max |ref| = {diff:.3e}")
        assert np.array_equal(a, b), name
    assert np.max(np.abs(ref[2])) > 0.0


def test_where_two_step_launches_apply(kvs):
    h = 0.25e-3
    grid = (40, 20, 12, h, h, h)
    mat = medium(grid, 1)

    def applies(precision=None, material=mat, pml=0, peak=False, probes=None, nx=40):
        g = (nx,) + grid[1:]
        ctx = kvs.kvs_create(g, precision=kvs.KVS_FP32 if precision is None else precision, sponge_cells=0)
        try:
            if np.isscalar(material[0]):
                kvs.kvs_set_material_uniform(ctx, *material)
            elif nx != 40:
                kvs.kvs_set_material(ctx, *medium(g, 1))
            else:
                kvs.kvs_set_material(ctx, *material)
            kvs.kvs_set_dt(ctx, 0.5 * kvs.kvs_stable_dt(ctx))
            if pml:
                kvs.kvs_set_pml(ctx, pml)
            if peak:
                kvs.kvs_set_peak_planes(ctx, [(2, 6)])
            if probes is not None:
                kvs.kvs_set_probes(ctx, probes, 2)
            return kvs.kvs_step_blocking_applies(ctx)
        finally:
            kvs.kvs_destroy(ctx)

    assert applies()
    assert applies(probes=[[3, 4, 5], [4, 4, 5]])
    assert not applies(precision=kvs.KVS_FP64)
    assert applies(material=(3e3, 1000.0, 0.5))  # homogeneous viscous
    assert not applies(material=(3e3, 1000.0, 0.0))  # homogeneous elastic
    zero_eta = (mat[0], mat[1], np.zeros_like(mat[2]))
    assert not applies(material=zero_eta)  # elastic
    assert not applies(pml=4)
    assert not applies(peak=True)
    assert not applies(probes=[[3, 4, 5], [3, 4, 5]])  # the same cell twice
    assert not applies(probes=[[3, 4, 0]])  # on the plane k = 0
    assert not applies(probes=[[3, 4, 11]])  # on the plane k = nz - 1
    assert not applies(nx=257)
    ctx = kvs.kvs_create(grid, precision=kvs.KVS_FP32)
    try:
        for bad in (0, 3, -1):
            with pytest.raises(kvs.KvsError) as e:
                kvs.kvs_set_step_blocking(ctx, bad)
            assert e.value.status == kvs.KVS_EINVAL
    finally:
        kvs.kvs_destroy(ctx)


def test_fallback_contexts_give_the_one_step_result(kvs):
    """Where the two-step kernel does not apply (an absorbing layer here),
    blocking 2 leaves the result bitwise unchanged."""
    h = 0.25e-3
    grid = (48, 30, 26, h, h, h)
    say("case two-step fallback with a layer")
    mat = medium(grid, 11)
    out = []
    for blocking in (1, 2):
        ctx = kvs.kvs_create(grid, precision=kvs.KVS_FP32, sponge_cells=0)
        try:
            kvs.kvs_set_material(ctx, *mat)
            kvs.kvs_set_dt(ctx, 0.5 * kvs.kvs_stable_dt(ctx))
            kvs.kvs_set_pml(ctx, 6)
            kvs.kvs_set_step_blocking(ctx, blocking)
            assert not kvs.kvs_step_blocking_applies(ctx)
            rng = np.random.default_rng(2)
            u0 = rng.standard_normal((3, 26, 30, 48)) * 1e-6
            kvs.kvs_set_state(ctx, u0, np.zeros_like(u0), 0)
            kvs.kvs_step(ctx, 9)
            out.append(kvs.kvs_get_state(ctx, (26, 30, 48))[0])
        finally:
            kvs.kvs_destroy(ctx)
    assert np.array_equal(out[0], out[1])


def test_kernel_timing_counts_steps_of_two_step_launches(kvs):
    h = 0.25e-3
    grid = (64, 32, 30, h, h, h)
    say("case two-step timing")
    ctx = kvs.kvs_create(grid, precision=kvs.KVS_FP32, sponge_cells=4)
    try:
        kvs.kvs_set_material(ctx, *medium(grid, 4))
        kvs.kvs_set_dt(ctx, 0.5 * kvs.kvs_stable_dt(ctx))
        kvs.kvs_set_step_blocking(ctx, 2)
        kvs.kvs_enable_kernel_timing(ctx, True)
        kvs.kvs_step(ctx, 17)  # eight two-step launches and one one-step launch
        ms, n = kvs.kvs_kernel_time(ctx)
        assert n == 17 and ms > 0.0, (n, ms)
        (ms1, n1), (ms2, n2) = kvs.kvs_kernel_time_split(ctx)
        assert (n1, n2) == (1, 8), (n1, n2)
        assert ms1 > 0.0 and ms2 > 0.0 and abs(ms1 + ms2 - ms) <= 1e-9 * ms
    finally:
        kvs.kvs_destroy(ctx)


def test_two_step_fp32_traces_within_2e5_of_oracle(kvs):
    """Inclusion workload physics at 64^3 with two-step launches: FP32 state
    (FP64 projection) against the FP64 oracle, 1500 steps, relative L2 of the
    lateral-line traces within 2e-5."""
    w = cfg2_inclusions_fp32(n=64)
    say("case two-step fp32 inclusions 64^3 against the oracle")
    dt = w.dt_factor * oracle.stable_dt(w.grid, w.G, w.rho, w.eta)
    env = w.envelope_for(dt)
    smax = oracle.default_sigma_max(w.grid, w.G, w.rho, w.sponge_cells)
    FS_o, _, rep_o = oracle.project(w.grid, w.F, tol=w.tol, jacobi=True)
    nsteps = 1500
    _, _, tr_o = oracle.run(w.grid, w.G, w.rho, w.eta, dt, nsteps, FS=FS_o, env=env, probes=w.probes, comp=2,
                            sponge_cells=w.sponge_cells, sigma_max=smax)
    ctx = kvs.kvs_create(w.grid, precision=kvs.KVS_FP32, sponge_cells=w.sponge_cells, sponge_sigma_max=smax)
    try:
        kvs.kvs_set_material(ctx, w.G, w.rho, w.eta)
        kvs.kvs_set_dt(ctx, dt)
        kvs.kvs_set_force(ctx, w.F)
        kvs.kvs_project(ctx, tol=w.tol, fixed_iters=rep_o["iters"], precond=kvs.KVS_PC_JACOBI)
        kvs.kvs_set_envelope(ctx, env)
        kvs.kvs_set_probes(ctx, w.probes, 2)
        kvs.kvs_set_step_blocking(ctx, 2)
        assert kvs.kvs_step_blocking_applies(ctx)
        kvs.kvs_step(ctx, nsteps)
        tr = kvs.kvs_read_traces(ctx, len(w.probes), 1)
    finally:
        kvs.kvs_destroy(ctx)
    err = rel_l2(tr, tr_o)
    say(f"two-step fp32 trace rel L2 {err:.3e}")
    assert err <= 2e-5


BATCH_CASES = [  # (nx, ny, nz), G, eta: 128-, 192- and 256-wide tiles, one elastic instance
    ((70, 41, 36), 3e3, 0.5),
    ((96, 30, 40), 8e3, 1.2),
    ((130, 33, 29), 2e3, 0.0),
    ((200, 26, 31), 5e3, 0.3),
    ((64, 20, 18), 1e3, 0.8),
]


def run_batch(kvs, blocking, calls):
    h = 0.25e-3
    grids = [s + (h, h, h) for s, _, _ in BATCH_CASES]
    b = kvs.kvs_batch_create(grids, precision=kvs.KVS_FP32, sponge_cells=4, sponge_sigma_max=800.0)
    try:
        kvs.kvs_batch_set_persistent(b, False)
        probes = []
        for i, (shape, G, eta) in enumerate(BATCH_CASES):
            c = kvs.kvs_batch_instance(b, i)
            kvs.kvs_set_material_uniform(c, G, 1000.0, eta)
            kvs.kvs_set_dt(c, 0.4 * kvs.kvs_stable_dt(c))
            rng = np.random.default_rng(20 + i)
            kvs.kvs_set_projected_force(c, rng.standard_normal((3, shape[2], shape[1], shape[0])) * 1e-3)
            kvs.kvs_set_envelope(c, np.r_[np.ones(5 + i), 0.0, 0.0, 1.0])  # push steps at odd and even offsets
            p = probe_set(grids[i], 30 + i)
            kvs.kvs_batch_set_probes(b, i, p)
            probes.append(p)
        kvs.kvs_batch_set_component(b, 2)
        kvs.kvs_batch_set_step_blocking(b, blocking)
        applies = kvs.kvs_batch_step_blocking_applies(b)
        for n in calls:
            kvs.kvs_batch_step(b, n)
        traces = [kvs.kvs_batch_read_traces(b, i, len(probes[i])) for i in range(len(BATCH_CASES))]
        states = [kvs.kvs_get_state(kvs.kvs_batch_instance(b, i), (s[2], s[1], s[0]))[:2]
                  for i, (s, _, _) in enumerate(BATCH_CASES)]
    finally:
        kvs.kvs_batch_destroy(b)
    return applies, traces, states


def test_batch_two_step_launches_match_one_step_bitwise(kvs):
    """A batch of homogeneous instances of five widths (one elastic) advanced
    with two steps per launch: the traces and states of every instance are
    bitwise those of one step per launch, over calls of odd step counts with
    push steps mixed in, and a replayed graph gives the same again."""
    say("case batch two-step bitwise")
    calls = (1, 10, 6, 14)
    _, ref_tr, ref_st = run_batch(kvs, 1, calls)
    applies, tr, st = run_batch(kvs, 2, calls)
    assert applies
    for i in range(len(BATCH_CASES)):
        assert ref_tr[i].shape == (sum(calls), len(probe_set(BATCH_CASES[i][0] + (1, 1, 1), 30 + i)))
        assert np.array_equal(tr[i], ref_tr[i]), i
        assert np.array_equal(st[i][0], ref_st[i][0]) and np.array_equal(st[i][1], ref_st[i][1]), i
    assert max(np.max(np.abs(t)) for t in ref_tr) > 0.0


def test_batch_two_step_applies_only_where_supported(kvs):
    h = 0.25e-3
    grids = [(40, 20, 12, h, h, h), (300, 10, 8, h, h, h)]
    for wide, eta in ((False, 0.5), (False, 0.0), (True, 0.5)):
        b = kvs.kvs_batch_create(grids if wide else grids[:1], precision=kvs.KVS_FP32)
        try:
            for i in range(2 if wide else 1):
                c = kvs.kvs_batch_instance(b, i)
                kvs.kvs_set_material_uniform(c, 3e3, 1000.0, eta)
                kvs.kvs_set_dt(c, 0.4 * kvs.kvs_stable_dt(c))
            assert kvs.kvs_batch_step_blocking_applies(b) == (eta > 0 and not wide)
            if eta > 0 and not wide:
                kvs.kvs_batch_set_probes(b, 0, [[3, 4, 0]])  # on the plane k = 0
                assert not kvs.kvs_batch_step_blocking_applies(b)
            with pytest.raises(kvs.KvsError):
                kvs.kvs_batch_set_step_blocking(b, 3)
        finally:
            kvs.kvs_batch_destroy(b)


def test_two_step_resume_from_saved_state_is_bitwise(kvs):
    """Stop after an odd number of steps (the pairing of the steps changes),
    save the state, restore it into a new context and go on: the state and the
    traces of the continued run are bitwise those of an uninterrupted run."""
    h = 0.25e-3
    grid = (90, 33, 28, h, h, h)
    say("case two-step resume")
    mat = medium(grid, 9)
    probes = probe_set(grid, 4)
    shp = (grid[2], grid[1], grid[0])

    def new_ctx():
        ctx = kvs.kvs_create(grid, precision=kvs.KVS_FP32, sponge_cells=4, sponge_sigma_max=-1.0)
        kvs.kvs_set_material(ctx, *mat)
        kvs.kvs_set_dt(ctx, 0.5 * kvs.kvs_stable_dt(ctx))
        kvs.kvs_set_probes(ctx, probes, 2)
        return ctx

    rng = np.random.default_rng(6)
    u0 = rng.standard_normal((3,) + shp) * 1e-6
    w0 = rng.standard_normal((3,) + shp) * 1e-8
    ctx = new_ctx()
    try:
        kvs.kvs_set_state(ctx, u0, w0, 0)
        kvs.kvs_step(ctx, 40)
        ref_tr = kvs.kvs_read_traces(ctx, len(probes), 1)
        ref_u, ref_w, ref_n = kvs.kvs_get_state(ctx, shp)
    finally:
        kvs.kvs_destroy(ctx)
    ctx = new_ctx()
    try:
        kvs.kvs_set_state(ctx, u0, w0, 0)
        kvs.kvs_step(ctx, 13)
        tr1 = kvs.kvs_read_traces(ctx, len(probes), 1)
        u, w, n = kvs.kvs_get_state(ctx, shp)
    finally:
        kvs.kvs_destroy(ctx)
    ctx = new_ctx()
    try:
        assert kvs.kvs_step_blocking_applies(ctx)
        kvs.kvs_set_state(ctx, u, w, n)
        kvs.kvs_step(ctx, 27)
        tr2 = kvs.kvs_read_traces(ctx, len(probes), 1)
        got_u, got_w, got_n = kvs.kvs_get_state(ctx, shp)
    finally:
        kvs.kvs_destroy(ctx)
    assert n == 13 and got_n == ref_n == 40
    assert np.array_equal(np.concatenate([tr1, tr2]), ref_tr)
    assert np.array_equal(got_u, ref_u) and np.array_equal(got_w, ref_w)
