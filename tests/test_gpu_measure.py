"""Measurement entry points: the per-dispatch step-kernel timing and the
streaming reference kernels that the benchmark's roofline lines use."""
import time

import numpy as np
import pytest

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


def test_kernel_timing_counts_every_step_launch(kvs):
    """With timing on, every step launch is timed once; the summed kernel
    time is positive and below the wall time of the calls; switched off, the
    totals stay as they were and later steps are not counted; switched on
    again, they restart from zero; the state is the same as without timing
    (bitwise)."""
    say("case kernel timing")
    h = 0.25e-3
    grid = (70, 40, 36, h, h, h)
    results = []
    for timed in (False, True):
        ctx = kvs.kvs_create(grid, precision=kvs.KVS_FP32, sponge_cells=4)
        try:
            kvs.kvs_set_material_uniform(ctx, 3e3, 1000.0, 0.4)
            kvs.kvs_set_dt(ctx, 0.4 * kvs.kvs_stable_dt(ctx))
            rng = np.random.default_rng(5)
            u0 = rng.standard_normal((3, 36, 40, 70)) * 1e-6
            kvs.kvs_set_state(ctx, u0, np.zeros_like(u0), 0)
            kvs.kvs_enable_kernel_timing(ctx, timed)
            t0 = time.perf_counter()
            kvs.kvs_step(ctx, 17)
            u, _, _ = kvs.kvs_get_state(ctx, (36, 40, 70))
            wall_ms = (time.perf_counter() - t0) * 1e3
            ms, n = kvs.kvs_kernel_time(ctx)
            if timed:
                assert n == 17 and 0.0 < ms < wall_ms, (n, ms, wall_ms)
                kvs.kvs_enable_kernel_timing(ctx, False)
                kvs.kvs_step(ctx, 3)
                assert kvs.kvs_kernel_time(ctx) == (ms, 17)
                kvs.kvs_enable_kernel_timing(ctx, True)
                assert kvs.kvs_kernel_time(ctx) == (0.0, 0)
                kvs.kvs_step(ctx, 2)
                ms3, n3 = kvs.kvs_kernel_time(ctx)
                assert n3 == 2 and ms3 > 0.0, (n3, ms3)
            else:
                assert n == 0
            results.append(u)  # both compared after the same 17 steps
        finally:
            kvs.kvs_destroy(ctx)
    assert np.array_equal(results[0], results[1])


@pytest.mark.parametrize("reads,writes", [(9, 6), (6, 6)])
def test_stream_reference_is_a_plausible_bandwidth(kvs, reads, writes):
    """The streaming reference over 16 M elements reports a bandwidth between
    1 TB/s and the 8 TB/s HBM peak (it moves 4 (reads + writes) bytes per
    element)."""
    say(f"case stream reference {reads} reads + {writes} writes")
    gbs = kvs.kvs_measure_stream(1 << 24, 3, reads=reads, writes=writes)
    say(f"{gbs:.0f} GB/s")
    assert 1000.0 < gbs < 8000.0, gbs


def test_stream_reference_rejects_bad_arguments(kvs):
    for bad in (dict(n=100), dict(n=1 << 20, reps=0), dict(n=1 << 20, reads=5), dict(n=1 << 20, reads=9, writes=5)):
        args = dict(n=1 << 20, reps=1, reads=6, writes=6)
        args.update(bad)
        with pytest.raises(kvs.KvsError) as e:
            kvs.kvs_measure_stream(args["n"], args["reps"], reads=args["reads"], writes=args["writes"])
        assert e.value.status == kvs.KVS_EINVAL
