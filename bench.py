"""Benchmark of the shear solver's hot path on one MI355X.

Default workload (--workload inclusions): one benchmark step is one whole
simulation of the 256^3 heterogeneous inclusion workload (FP32 stencil
state, FP64 projection): return the medium to rest, take the force pattern
from device memory, project it (divergence, Jacobi-PCG to 1e-8, gradient
subtraction), advance 4000 FDTD steps with the push envelope and the
lateral-line probe traces, and read the traces back.  The material, force
pattern and probes are resident in HBM before timing.

--workload kvline: the 1-D harmonic Kelvin-Voigt sweep (16 viscosities as
one batch of line instances, one persistent launch), time of the whole
sweep; pml, arf and fpcg: the cost legs of the absorbing layer, the
radiation-force generator and the learned preconditioner.

--workload batch: one benchmark step is the 64-instance homogeneous sweep
(edges 96..192, G and eta from the sweep values): all instances to rest, one
projection per distinct grid shared by its instances, 2000 steps of every
instance as one replayed hipGraph (one launch per step and tile width over
all instances), lateral-line traces read back.

value = interior cell-updates of the timed steps / timed wall time
        (whole job, projection included), in Gcell-updates/s.
roofline: the dominant FDTD kernel over its HIP-event-timed launches,
          algorithmic bytes per interior cell-update (48 B of FP32 u, w read +
          written, 12 B of G, eta, dt^2/rho, and 12 B of f_S on push steps) x
          the cell-updates one launch processes, over its mean launch
          duration, against 8 TB/s.  By default that kernel is the two-step
          kernel (two cell-updates per cell and launch; it moves 60 B per two
          updates and is limited by vector-ALU issue: limited_by, and alu =
          its algorithmic FP32 flop rate, 147 flop per cell-update, against
          the 78.6 TFLOP/s FMA peak without packed FP32); the one-step push
          launches are listed beside it.  With --step-blocking 1 it is the
          one-step kernel.  stream_gbs / frac_of_stream: a stream with the
          one-step kernel's 9 reads and 6 writes per cell and no stencil,
          measured in the same run (the ceiling of any one-step kernel);
          copy_gbs / frac_of_copy: a plain device-to-device copy.
          traffic: HBM bytes per launch from the rocprofv3 counter runs of
          the same kernel source (null when the source differs).
one_step_kernel: the one-step kernel alone after the timed region (200
          launches without force): us per launch, fraction of 8 TB/s,
          traffic.
cpu_baseline: the FP64 CPU oracle on a bounded sample of the same workload
              (all host threads; steps and projection iterations, scaled to
              the whole job), its host's CPU model, and a shorter sample on
              one thread.
The same line carries the other configurations as legs (config1, batch,
kvline, time_varying, shell, arf), each with its own oracle timing, and
projection_learned (outside the timed region): projection time to a true
1e-8 of the learned flexible PCG vs Jacobi-PCG on the time-varying
workload's 384 x 384 x 512 grid, after training the network by the committed
recipe (training time reported separately).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM traffic of the FDTD step kernel from rocprofv3 counter runs of this
# benchmark (256^3 inclusion workload, one launch without force): FETCH_SIZE
# and WRITE_SIZE in KiB per dispatch, per tile-shape variant, taken on the
# step-kernel sources (STEP_SOURCES) whose SHA-256 is STEP_SOURCE_SHA.  Each counter is
# scaled by what it reads for a plain copy of known size (--copy-calibration):
# FETCH_SIZE reports half of the bytes a copy reads, WRITE_SIZE all of the
# bytes it writes.  A changed source voids the figures (traffic -> null).
STEP_SOURCE_SHA = "f26c91bb5db918abca9fc803284f993aa0fe815a66b95bb68a2d2f50a855e0e9"
STEP_COUNTERS_KIB = {  # variant -> (FETCH_SIZE, WRITE_SIZE), mean of 6 dispatches
    0: (423983.2, 390146.0),
    1: (400448.2, 390146.0),
    2: (322676.2, 390146.0),
    3: (302672.6, 390146.3),
    4: (361179.7, 390146.0),
    5: (331166.7, 390146.0),
    6: (304537.1, 390146.4),
    7: (304696.8, 390146.7),
}
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0
# The same counters for the two-step kernel (step2_kernel, one launch = two
# steps without force), taken on STEP2_SOURCES with SHA-256 STEP2_SOURCE_SHA.
STEP2_SOURCE_SHA = "8a13c07d6ffc431d3d458ff01837be9fa8a7ec2b08a1f5cfc443e77c110124c7"
STEP2_COUNTERS_KIB = (329607.6, 390148.0)  # (FETCH_SIZE, WRITE_SIZE), mean of 6 dispatches
# Algorithmic FP32 arithmetic of one heterogeneous viscous cell-update of the
# summed-form leapfrog (Sec. 3.1), an FMA counted as two: six harmonic face
# moduli 2 G G' / (G + G') / h^2 (5 each, 30); the sponge factors s,
# (1 - s) / (1 + s), (dt^2 / rho) / (1 + s) and eta / dt (6); per component
# the flux divergence of G grad u (6 differences, 6 products, 5 sums: 17), the
# Laplacian of w (4 per axis and 2 sums: 14), acc += (eta / dt) lap w (2),
# w' = a1 w + a2 acc (3) and u' = u + w' (1): 37 x 3 = 111.  Total 147.
# storage of the projection's CG on the FP32 contexts of every leg (the library's default there)
CG_STORAGE = ("FP32 search direction and residual (residual recomputed from phi whenever r.r has fallen 1e4-fold), "
              "FP64 potential, inner products and norms; flexible PCG: also z in FP32")
FLOP_PER_CELL_UPDATE = 147
# FP32 vector peak of the MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz x 2
# (FMA) = 78.6 TFLOP/s without packed FP32 instructions (which this build does
# not emit), 157.3 TFLOP/s with them (the published figure).
FP32_PEAK_TFLOPS, FP32_PACKED_PEAK_TFLOPS = 78.6, 157.3
METRIC = "FDTD Gcell-updates/s (% HBM roofline); projection time, learned-FPCG vs PCG @1e-8"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["inclusions", "batch", "fpcg", "arf", "pml", "kvline"], default="inclusions",
                    help="fpcg: profiling aid, flexible-PCG iterations on the 384 x 384 x 512 grid; "
                         "arf: the ARF accumulation leg alone; pml: cost of the absorbing layer")
    ap.add_argument("--grid", type=int, default=256, help="cubic grid edge of the inclusion workload")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the CPU oracle leg (profiling runs)")
    ap.add_argument("--cpu-sample-steps", type=int, default=100)
    ap.add_argument("--step-variant", type=int, default=-1,
                    help="pin the step-kernel tile shape (default: autotune); used by the counter runs")
    ap.add_argument("--step-blocking", type=int, default=2, choices=[1, 2],
                    help="FDTD steps per launch in the main and batched legs (2: the two-step kernels)")
    ap.add_argument("--train-rounds", type=int, default=4,
                    help="training rounds on the network's own flexible-PCG residuals")
    ap.add_argument("--train-grid", type=int, default=64, help="edge of the cubic unit training grids")
    ap.add_argument("--unet-bottleneck", type=int, default=4,
                    help="convolutions in the network's quarter-resolution bottleneck (in, dilated 64->64 ones, out)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-preconditioner projection comparison")
    ap.add_argument("--learned-epochs", type=int, default=4,
                    help="projections of the time-varying workload timed per method")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the full-size time-varying and shell workload legs")
    ap.add_argument("--tv-epochs", type=int, default=4, help="epochs of the time-varying workload window")
    ap.add_argument("--shell-steps", type=int, default=300, help="steps of the shell workload window")
    ap.add_argument("--arf-repeats", type=int, default=8, help="accumulate launches of the ARF leg")
    ap.add_argument("--batch-steps", type=int, default=2, help="timed sweeps of the batched leg in the default run")
    ap.add_argument("--batch-warmup", type=int, default=1, help="untimed sweeps of the batched leg in the default run")
    ap.add_argument("--no-extra-legs", action="store_true",
                    help="skip the 48^3 FP64, batched-sweep, KV-line and streaming-reference legs")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (HBM counter calibration)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


STEP_SOURCES = ("kvs_step_tile.hpp", "kvs_step.hip", "kvs_tiling.hpp")
STEP2_SOURCES = ("kvs_step2.hip", "kvs_step2_tile.hpp", "kvs_step_tile.hpp", "kvs_tiling.hpp")


def step_source_sha(names=STEP_SOURCES):
    """SHA-256 over a step kernel's sources (tile code, kernel and launch
    shapes, tile order), in the order given."""
    import hashlib
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_2607_28414_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def step2_traffic():
    """Measured HBM bytes per two-step launch, or None when the counters are
    not for this source."""
    if STEP2_COUNTERS_KIB is None or step_source_sha(STEP2_SOURCES) != STEP2_SOURCE_SHA:
        return None
    fetch, write = STEP2_COUNTERS_KIB
    return (fetch * FETCH_SCALE + write * WRITE_SCALE) * 1024.0


def step_traffic(variant):
    """Measured HBM bytes per step-kernel launch, or None when the counters
    are not for this source or this tile shape."""
    if STEP_SOURCE_SHA is None or variant not in STEP_COUNTERS_KIB or step_source_sha() != STEP_SOURCE_SHA:
        return None
    fetch, write = STEP_COUNTERS_KIB[variant]
    return (fetch * FETCH_SCALE + write * WRITE_SCALE) * 1024.0


def copy_calibration(mib):
    """A plain device-to-device copy of `mib` MiB (the HIP runtime's copy
    kernel behind a same-type tensor copy), five launches: the reference for
    the HBM byte counters."""
    import torch
    n = mib * 1024 * 1024 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 4, "copy_calibration_bytes_written": n * 4}), flush=True)


def measured_copy_gbs(mib=1024, reps=10):
    """Bandwidth of a plain device-to-device copy on this GPU (the HIP
    runtime's copy kernel behind a same-type tensor copy of `mib` MiB), read
    plus write bytes over the median of `reps` HIP-event-timed copies: the
    practical streaming ceiling next to the 8 TB/s peak."""
    import numpy as np
    import torch
    n = mib * 1024 * 1024 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    del a, b
    return 2.0 * n * 4 / (float(np.median(ms)) * 1e-3) / 1e9


def learned_projection(args, net):
    """Projection time to 1e-8, learned flexible PCG vs Jacobi-PCG, on the
    time-varying workload's grid (384 x 384 x 512, h = 0.2 mm): the network
    `net` is trained first by the committed recipe (timed separately), then each
    method projects the pushes of `learned_epochs` re-projection epochs
    (moving focus, redrawn modulation phases) from phi = 0, and again
    warm-started from the previous epoch's phi.  Times are HIP events around
    divergence + solve + gradient subtraction."""
    import numpy as np
    import torch

    from paper_2607_28414_amd import kvs, train
    from workloads import focal_modulated_params

    nx, ny, nz, h = 384, 384, 512, 0.2e-3
    grid = (nx, ny, nz, h, h, h)
    log(f"bench: training the preconditioner ({args.train_grid}^3 unit grids, {args.train_rounds} rounds on its own "
        "residuals)")
    ctx = None
    try:
        tr = train.train_default(net, n=args.train_grid, seed=0, rounds=args.train_rounds)
        ctx = kvs.kvs_create(grid, precision=kvs.KVS_FP32, stream=torch.cuda.current_stream().cuda_stream)
        kvs.kvs_set_preconditioner(ctx, net)
        res = {"jacobi": {"iters": [], "ms": [], "relres_true": []},
               "fpcg": {"iters": [], "ms": [], "fallbacks": [], "relres_true": []},
               "jacobi_warm": {"iters": [], "ms": [], "relres_true": []},
               "fpcg_warm": {"iters": [], "ms": [], "relres_true": []}}
        for e in range(args.learned_epochs):
            push = focal_modulated_params(grid, epoch=e)
            for name, pc in (("jacobi", kvs.KVS_PC_JACOBI), ("fpcg", kvs.KVS_PC_UNET)):
                kvs.kvs_set_force_pattern(ctx, **push)  # generated on the device
                # both methods stop only when the FP64 true residual is below 1e-8
                rep = kvs.kvs_project(ctx, tol=1e-8, max_iter=20000, precond=pc, confirm_true=True)
                res[name]["iters"].append(rep["iters"])
                res[name]["ms"].append(rep["ms"])
                res[name]["relres_true"].append(rep["relres_true"])
                if pc == kvs.KVS_PC_UNET:
                    res[name]["fallbacks"].append(kvs.kvs_last_fallbacks(ctx))
                assert rep["status"] == 0 and rep["relres_true"] < 1e-8, rep
            log(f"bench: epoch {e}: jacobi {res['jacobi']['iters'][-1]} it {res['jacobi']['ms'][-1]:.0f} ms, "
                f"fpcg {res['fpcg']['iters'][-1]} it {res['fpcg']['ms'][-1]:.0f} ms")
        # warm-started: consecutive epochs, phi kept from the previous solve of the same method
        for name, pc in (("jacobi_warm", kvs.KVS_PC_JACOBI), ("fpcg_warm", kvs.KVS_PC_UNET)):
            for e in range(args.learned_epochs):
                kvs.kvs_set_force_pattern(ctx, **focal_modulated_params(grid, epoch=e))
                rep = kvs.kvs_project(ctx, tol=1e-8, max_iter=20000, precond=pc, warm_start=e > 0,
                                      confirm_true=True)
                assert rep["status"] == 0 and rep["relres_true"] < 1e-8, rep
                if e > 0:
                    res[name]["iters"].append(rep["iters"])
                    res[name]["ms"].append(rep["ms"])
                    res[name]["relres_true"].append(rep["relres_true"])
    finally:
        if ctx is not None:
            kvs.kvs_destroy(ctx)
    jm, fm = float(np.mean(res["jacobi"]["ms"])), float(np.mean(res["fpcg"]["ms"]))
    out = {
        "workload": f"{nx}x{ny}x{nz}, h 0.2 mm, focal push (1 mm / 4 mm) x random-phase modulation, focus moving "
                    f"1 mm per 20 us, epochs 0-{args.learned_epochs - 1} (10 steps of 1.75 us each)",
        "tol": 1e-8,
        "jacobi_ms": jm, "fpcg_ms": fm, "speedup": jm / fm,
        "jacobi_iters": res["jacobi"]["iters"], "fpcg_iters": res["fpcg"]["iters"],
        "fpcg_fallbacks": res["fpcg"]["fallbacks"],
        "jacobi_relres_true": res["jacobi"]["relres_true"], "fpcg_relres_true": res["fpcg"]["relres_true"],
        "stop_rule": "FP64 true residual ||-b - A phi|| / ||b|| < 1e-8 for both methods (restart from the true "
                     "residual when the recursive one met the tolerance first)",
        "cg_storage": CG_STORAGE,
        "warm_start": {"jacobi_ms": float(np.mean(res["jacobi_warm"]["ms"])) if res["jacobi_warm"]["ms"] else None,
                       "fpcg_ms": float(np.mean(res["fpcg_warm"]["ms"])) if res["fpcg_warm"]["ms"] else None,
                       "jacobi_iters": res["jacobi_warm"]["iters"], "fpcg_iters": res["fpcg_warm"]["iters"],
                       "jacobi_relres_true": res["jacobi_warm"]["relres_true"],
                       "fpcg_relres_true": res["fpcg_warm"]["relres_true"]},
        "network": "3-level linear U-Net 16/32/64 channels, 4 bottleneck convs, BF16 MFMA, FP32 accumulation",
        "train_seconds": tr.train_seconds,
        "train_samples": len(tr.samples),
    }
    ws = out["warm_start"]
    if ws["jacobi_ms"] and ws["fpcg_ms"]:
        ws["speedup"] = ws["jacobi_ms"] / ws["fpcg_ms"]
    return out


def time_varying_window(args, net):
    """The time-varying-source workload in full (384 x 384 x 512, G and eta
    from random fields, F_S always on), over a window of `tv_epochs`
    re-projection epochs: per epoch the focal push of that epoch, a warm-
    started learned-FPCG projection to 1e-8, then 10 FDTD steps.  Step-kernel
    launches are timed with HIP events (72 algorithmic bytes per cell-update:
    state 48, material 12, F_S 12); epochs are timed whole."""
    import numpy as np
    import torch

    from paper_2607_28414_amd import kvs
    from workloads import cfg4_grf_material, focal_modulated_params

    log("bench: time-varying workload 384x384x512 (random medium, F_S always on)")
    grid, G, rho, eta = cfg4_grf_material()
    cells = (grid[0] - 2) * (grid[1] - 2) * (grid[2] - 2)
    stream = torch.cuda.current_stream()
    ctx = kvs.kvs_create(grid, precision=kvs.KVS_FP32, sponge_cells=8, sponge_sigma_max=-1.0,
                         stream=stream.cuda_stream)
    try:
        kvs.kvs_set_material(ctx, G, rho, eta)
        dt = 0.4 * kvs.kvs_stable_dt(ctx)
        kvs.kvs_set_dt(ctx, dt)
        kvs.kvs_set_envelope(ctx, np.ones(3000))
        kvs.kvs_set_preconditioner(ctx, net)
        variant, _ = kvs.kvs_autotune_step(ctx, 10)
        iters, pms, fbs, ems, rts = [], [], [], [], []
        kvs.kvs_enable_kernel_timing(ctx, True)
        for e in range(args.tv_epochs):
            # the epoch's force (standing in for the acoustic solver's output) is
            # generated by the library's pattern kernel inside the epoch
            push = focal_modulated_params(grid, epoch=e, dt=dt)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            kvs.kvs_set_force_pattern(ctx, **push)
            rep = kvs.kvs_project(ctx, tol=1e-8, max_iter=20000, precond=kvs.KVS_PC_UNET, warm_start=e > 0,
                                  confirm_true=True)
            kvs.kvs_step(ctx, 10)
            torch.cuda.synchronize()
            ems.append((time.perf_counter() - t0) * 1e3)
            if (e + 1) % 50 == 0:
                log(f"bench: time-varying epoch {e + 1} of {args.tv_epochs}")
            assert rep["status"] == 0 and rep["relres_true"] < 1e-8, rep
            iters.append(rep["iters"])
            pms.append(rep["ms"])
            rts.append(rep["relres_true"])
            fbs.append(kvs.kvs_last_fallbacks(ctx))
        k_ms, k_launches = kvs.kvs_kernel_time(ctx)
        kvs.kvs_enable_kernel_timing(ctx, False)
        u, _, step = kvs.kvs_get_state(ctx, (grid[2], grid[1], grid[0]))
        assert np.all(np.isfinite(u)) and step == 10 * args.tv_epochs
    finally:
        kvs.kvs_destroy(ctx)
    per = k_ms / k_launches
    achieved = cells * 72 / (per * 1e-3) / 1e9
    cpu = None
    if not args.no_cpu_baseline:
        from workloads import force_from_params
        log("bench: oracle window of the time-varying workload")
        cpu = oracle_window(grid, G, rho, eta, dt, force_from_params(grid, focal_modulated_params(grid, epoch=0, dt=dt)),
                            3, 10, 8, proj_iters=1593)
    del G, eta
    return {
        "workload": f"384x384x512, h 0.2 mm, G = 10^(3 + Phi(xi)) Pa and eta = 1.5 Phi(xi') Pa s (3 mm random "
                    f"fields), rho 1000, 8-cell sponge, dt {dt:.3e} s (0.4 x stable limit), epochs 0-"
                    f"{args.tv_epochs - 1}: focal push re-projected by warm-started learned FPCG, then 10 steps",
        "fdtd_kernel_ms_avg": per, "fdtd_kernel_gcells": cells / (per * 1e-3) / 1e9,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_cell_update": 72, "launches": k_launches, "variant": variant},
        "projection_iters": iters, "projection_ms": pms, "fallbacks": fbs, "projection_relres_true": rts,
        "epoch_ms": ems, "epoch_ms_mean_after_first": float(np.mean(ems[1:])) if len(ems) > 1 else None,
        "cpu_baseline": cpu,
    }


def arf_workload(args):
    """Acoustic radiation force accumulation on the 512 x 512 x 640 grid of the
    transcranial workload: Poynting form, FP32 samples of a synthetic focused
    1 MHz tone burst (8 samples per launch, the same 8 samples folded in
    `arf_repeats` times), then the force pattern with a uniform alpha and c.
    Each accumulate launch is timed with HIP events on the context's stream;
    algorithmic bytes per launch = (8 x 16 + 2 x 24) B per cell (the samples
    read once, the three FP64 sums read and written once)."""
    import torch

    from paper_2607_28414_amd import kvs
    from workloads.gpu import beam_samples_device

    grid = (512, 512, 640, 0.2e-3, 0.2e-3, 0.2e-3)
    N = 512 * 512 * 640
    ns = 8
    log("bench: ARF accumulation 512x512x640")
    # synthetic samples standing in for an acoustic solver's output, drawn on
    # the device by the input generator's kernel
    p, v = beam_samples_device(grid, ns, per=8, cycles=2, focus=(0.0, 0.0, 0.03))
    torch.cuda.synchronize()
    ctx = kvs.kvs_create(grid, precision=kvs.KVS_FP32)
    try:
        lib_stream = torch.cuda.ExternalStream(kvs.kvs_stream(ctx))
        kvs.kvs_arf_begin(ctx, kvs.KVS_ARF_POYNTING)
        kvs.kvs_arf_accumulate_device(ctx, p.data_ptr(), v.data_ptr(), ns, 1)  # warm-up
        kvs.kvs_arf_begin(ctx, kvs.KVS_ARF_POYNTING)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.arf_repeats)]
        for e0, e1 in ev:
            e0.record(lib_stream)
            kvs.kvs_arf_accumulate_device(ctx, p.data_ptr(), v.data_ptr(), ns, 1)
            e1.record(lib_stream)
        f0 = torch.cuda.Event(enable_timing=True)
        f1 = torch.cuda.Event(enable_timing=True)
        f0.record(lib_stream)
        kvs.kvs_arf_set_force(ctx, 5.8, 1540.0, 8 * 2, mask=None)
        f1.record(lib_stream)
        # peak acoustic strain maps from the same pressure samples
        kvs.kvs_strain_begin(ctx, 1000.0 * 1540.0 ** 2)
        kvs.kvs_strain_accumulate_device(ctx, p.data_ptr(), ns, 1)  # warm-up
        kvs.kvs_strain_begin(ctx, 1000.0 * 1540.0 ** 2)
        sev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.arf_repeats)]
        for e0, e1 in sev:
            e0.record(lib_stream)
            kvs.kvs_strain_accumulate_device(ctx, p.data_ptr(), ns, 1)
            e1.record(lib_stream)
        torch.cuda.synchronize()
        ms = [a.elapsed_time(b) for a, b in ev]
        strain_ms = [a.elapsed_time(b) for a, b in sev]
        force_ms = f0.elapsed_time(f1)
    finally:
        kvs.kvs_destroy(ctx)
        del p, v
        torch.cuda.empty_cache()
    per = sum(ms) / len(ms)
    achieved = N * (ns * 16 + 2 * 24) / (per * 1e-3) / 1e9
    sper = sum(strain_ms) / len(strain_ms)
    s_achieved = N * (ns * 4 + 2 * 16) / (sper * 1e-3) / 1e9
    return {
        "workload": "512x512x640 grid, Poynting form, FP32 samples of a focused 1 MHz tone burst (8 per launch), "
                    f"{args.arf_repeats} launches, then the force pattern (uniform alpha 5.8 Np/m, c 1540 m/s)",
        "samples": ns * args.arf_repeats,
        "accumulate_ms_avg": per,
        "gcell_samples_per_s": N * ns / (per * 1e-3) / 1e9,
        "set_force_ms": force_ms,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_cell": "8 x 16 (samples) + 48 (sums read and written) per launch"},
        "strain": {"accumulate_ms_avg": sper, "gcell_samples_per_s": N * ns / (sper * 1e-3) / 1e9,
                   "achieved_GBs": s_achieved, "frac_of_hbm_peak": s_achieved / HBM_PEAK_GBS,
                   "algorithmic_bytes_per_cell": "8 x 4 (pressure samples) + 32 (two FP64 peak maps read and "
                                                 "written) per launch; one FP64 division, 7 cached p reads per cell and sample"},
    }


def run_pml_bench(args):
    """Cost of the absorbing layer: the 256^3 inclusion medium, push projected
    by Jacobi-PCG, 500 steps without sponge, once with the Dirichlet walls
    alone and once with a 10-cell C-PML; HIP events on the context's stream
    around the steps (step kernel, probe gather, and the layer's passes)."""
    import torch

    from paper_2607_28414_amd import kvs
    from workloads import cfg2_inclusions_fp32

    w = cfg2_inclusions_fp32(n=256)
    out = {}
    for L in (0, 10):
        ctx = kvs.kvs_create(w.grid, precision=kvs.KVS_FP32)
        try:
            kvs.kvs_set_material(ctx, w.G, w.rho, w.eta)
            dt = w.dt_factor * kvs.kvs_stable_dt(ctx)
            kvs.kvs_set_dt(ctx, dt)
            kvs.kvs_set_envelope(ctx, w.envelope_for(dt))
            kvs.kvs_set_probes(ctx, w.probes, w.comp)
            if L:
                kvs.kvs_set_pml(ctx, L)
            kvs.kvs_set_force(ctx, w.F)
            kvs.kvs_project(ctx, tol=w.tol, max_iter=20000)
            variant, _ = kvs.kvs_autotune_step(ctx, 10)
            kvs.kvs_step(ctx, 20)
            kvs.kvs_reset_state(ctx)
            stream = torch.cuda.ExternalStream(kvs.kvs_stream(ctx))
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            kvs.kvs_step(ctx, 500)
            e1.record(stream)
            torch.cuda.synchronize()
            out[L] = e0.elapsed_time(e1) / 500
        finally:
            kvs.kvs_destroy(ctx)
    n = 256
    band = (n - 2) ** 3 - (n - 2 - 20) ** 3
    return {"workload": "256^3 inclusions, 500 steps, no sponge: Dirichlet walls vs a 10-cell C-PML",
            "ms_per_step_walls": out[0], "ms_per_step_pml": out[10],
            "pml_overhead_ms": out[10] - out[0], "layer_cells": band,
            "layer_fraction": band / (n - 2) ** 3}


def shell_workload(args, net):
    """The transcranial-like workload in full (512 x 512 x 640, curved stiff
    shell, 6000-step run window of `shell_steps` steps): one projection of
    the separable push by learned FPCG and by Jacobi-PCG (both from phi = 0
    to 1e-8), then stepping with the 90-step push and the peak-|u| maps on
    the three planes through the push.  The step kernel is timed with HIP
    events; the whole stepping (step kernel, probe gather and peak update)
    with events around it."""
    import numpy as np
    import torch

    from paper_2607_28414_amd import kvs
    from workloads import cfg5_shell

    log("bench: shell workload 512x512x640")
    w = cfg5_shell()
    cells = w.interior_cells
    stream = torch.cuda.current_stream()
    ctx = kvs.kvs_create(w.grid, precision=kvs.KVS_FP32, sponge_cells=w.sponge_cells, sponge_sigma_max=-1.0,
                         stream=stream.cuda_stream)
    try:
        kvs.kvs_set_material(ctx, w.G, w.rho, w.eta)
        dt = w.dt_factor * kvs.kvs_stable_dt(ctx)
        kvs.kvs_set_dt(ctx, dt)
        env = w.envelope_for(dt)
        kvs.kvs_set_envelope(ctx, env)
        variant, _ = kvs.kvs_autotune_step(ctx, 10)
        kvs.kvs_set_force(ctx, w.F)
        kvs.kvs_set_preconditioner(ctx, net)
        rj = kvs.kvs_project(ctx, tol=1e-8, max_iter=20000, precond=kvs.KVS_PC_JACOBI, confirm_true=True)
        rf = kvs.kvs_project(ctx, tol=1e-8, max_iter=20000, precond=kvs.KVS_PC_UNET, confirm_true=True)
        assert rj["status"] == 0 and rj["relres_true"] < 1e-8, rj
        assert rf["status"] == 0 and rf["relres_true"] < 1e-8, rf
        fb = kvs.kvs_last_fallbacks(ctx)
        log(f"bench: shell projection jacobi {rj['iters']} it {rj['ms']:.0f} ms, fpcg {rf['iters']} it "
            f"{rf['ms']:.0f} ms")
        planes = w.meta["peak_planes"]
        kvs.kvs_set_peak_planes(ctx, planes)
        kvs.kvs_set_probes(ctx, w.probes, 2)
        kvs.kvs_step(ctx, 5)  # warm-up launches
        kvs.kvs_reset_state(ctx)
        kvs.kvs_enable_kernel_timing(ctx, True)
        # events on the context's own stream (the library makes one when the
        # caller's stream is the null stream)
        lib_stream = torch.cuda.ExternalStream(kvs.kvs_stream(ctx))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(lib_stream)
        kvs.kvs_step(ctx, args.shell_steps)
        e1.record(lib_stream)
        torch.cuda.synchronize()
        k_ms, k_launches = kvs.kvs_kernel_time(ctx)
        kvs.kvs_enable_kernel_timing(ctx, False)
        all_ms = e0.elapsed_time(e1)
        peak = {f"axis{a}_index{i}": float(kvs.kvs_peak_map(ctx, a, i, w.grid).max()) for a, i in planes}
    finally:
        kvs.kvs_destroy(ctx)
    per = k_ms / k_launches
    n_push = min(len(env), args.shell_steps)
    bytes_total = cells * (60 * args.shell_steps + 12 * n_push)
    achieved = bytes_total / (k_ms * 1e-3) / 1e9
    cpu = None
    if not args.no_cpu_baseline:
        log("bench: oracle window of the shell workload")
        cpu = oracle_window(w.grid, w.G, w.rho, w.eta, dt, w.F, 2, 8, w.sponge_cells, proj_iters=rj["iters"])
    w.G = w.rho = w.eta = w.F = None
    return {
        "workload": f"512x512x640, h 0.2 mm, curved shell 5-8 mm (100 kPa, 1900, 2 Pa s) over soft tissue "
                    f"(1.5 kPa, 1040, 0.8 Pa s), 8-cell sponge, push 20 mm below the shell (1 mm / 5 mm, 5e4 "
                    f"N/m^3, {len(env)} steps), dt {dt:.3e} s, first {args.shell_steps} of 6000 steps, peak |u| "
                    f"maps on 3 planes",
        "projection": {"tol": 1e-8, "jacobi_iters": rj["iters"], "jacobi_ms": rj["ms"], "fpcg_iters": rf["iters"],
                       "fpcg_ms": rf["ms"], "speedup": rj["ms"] / rf["ms"], "fpcg_fallbacks": fb,
                       "jacobi_relres_true": rj["relres_true"], "fpcg_relres_true": rf["relres_true"],
                       "cg_storage": CG_STORAGE},
        "fdtd_kernel_ms_avg": per, "fdtd_kernel_gcells": cells * args.shell_steps / (k_ms * 1e-3) / 1e9,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_cell_update": "60 (+12 on push steps)", "launches": k_launches,
                     "variant": variant},
        "stepping_ms_per_step": all_ms / args.shell_steps,
        "sensor_overhead_ms_per_step": all_ms / args.shell_steps - per,
        "peak_u_m": peak,
        "cpu_baseline": cpu,
    }


def run_fpcg_profile(args):
    """Profiling aid for the learned preconditioner's kernels: two flexible-
    PCG solves of 10 fixed iterations on the 384 x 384 x 512 grid with the
    time-varying workload's epoch-0 force and a network with random weights
    (the kernels' work does not depend on the weights).  Not a benchmark
    result: prints the solve times only."""
    import numpy as np
    import torch

    from paper_2607_28414_amd import kvs, train
    from workloads import focal_modulated_params

    g = (384, 384, 512, 0.2e-3, 0.2e-3, 0.2e-3)
    net = kvs.kvs_unet_create((16, 32, 64), 4)
    ctx = None
    try:
        train.init_weights(net, np.random.default_rng(0))
        ctx = kvs.kvs_create(g, precision=kvs.KVS_FP32, stream=torch.cuda.current_stream().cuda_stream)
        kvs.kvs_set_force_pattern(ctx, **focal_modulated_params(g, epoch=0))
        kvs.kvs_set_preconditioner(ctx, net)
        ms = [kvs.kvs_project(ctx, tol=1e-8, precond=kvs.KVS_PC_UNET, fixed_iters=10)["ms"] for _ in range(2)]
    finally:
        if ctx is not None:
            kvs.kvs_destroy(ctx)
        kvs.kvs_unet_destroy(net)
    return {"profiling_aid": "flexible PCG, 10 fixed iterations, 384x384x512, untrained network", "solve_ms": ms}


def cpu_baseline(w, dt, smax, FS_host, nsteps, proj_iters, cg_sample=40):
    """The FP64 oracle, as it stands, on a bounded sample of the whole
    workload, timed on the host cores: `nsteps` FDTD steps (from rest, push
    on) and `cg_sample` Jacobi-PCG iterations of the projection (with its
    divergence and gradient subtraction).  value = the whole job (the
    projection's `proj_iters` iterations and the workload's steps) at the
    sampled per-step and per-iteration times, in the metric's unit."""
    import numpy as np

    import oracle
    env = w.envelope_for(dt)
    oracle.lib()
    t0 = time.perf_counter()
    oracle.run(w.grid, w.G, w.rho, w.eta, dt, nsteps, FS=FS_host, env=env, probes=w.probes, comp=2,
               sponge_cells=w.sponge_cells, sigma_max=smax)
    el = time.perf_counter() - t0
    t1 = time.perf_counter()
    oracle.project(w.grid, w.F, fixed_iters=cg_sample, jacobi=True)
    el_cg = time.perf_counter() - t1
    t_step, t_iter = el / nsteps, el_cg / cg_sample
    t_job = proj_iters * t_iter + w.nsteps * t_step
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # the same oracle on one thread (OpenMP's runtime shared with the oracle's library)
    import ctypes
    one = None
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
        gomp.omp_set_num_threads(1)
        n1 = 4
        t2 = time.perf_counter()
        oracle.run(w.grid, w.G, w.rho, w.eta, dt, n1, FS=FS_host, env=env, probes=w.probes, comp=2,
                   sponge_cells=w.sponge_cells, sigma_max=smax)
        one = w.interior_cells * n1 / (time.perf_counter() - t2) / 1e9
        gomp.omp_set_num_threads(cores)
    except OSError:
        pass
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
    except OSError:
        pass
    return {"value": w.interior_cells * w.nsteps / t_job / 1e9, "unit": "Gcell-updates/s", "cores": cores,
            "kind": "oracle", "cpu_model": model, "host_cpus": os.cpu_count(),
            "fdtd_only": w.interior_cells * nsteps / el / 1e9, "s_per_step": t_step, "s_per_cg_iteration": t_iter,
            "whole_job_s": t_job, "value_one_thread_fdtd": one,
            "sample": f"{nsteps} FDTD steps of the same {w.grid[0]}^3 workload from rest with the push on ({el:.1f} s) "
                      f"and {cg_sample} Jacobi-PCG iterations of its projection with divergence and gradient "
                      f"subtraction ({el_cg:.1f} s), FP64 C oracle, OpenMP; value = the whole job ({proj_iters} "
                      f"iterations + {w.nsteps} steps) at the sampled rates; value_one_thread_fdtd: 4 steps on one "
                      f"thread"}


def oracle_window(grid, G, rho, eta, dt, F, nsteps, cg_iters, sponge_cells, proj_iters=None):
    """The FP64 oracle, as it stands, on a stated window of a full-size
    workload (the whole run would take hours on the host): `nsteps` FDTD steps
    from rest with the force on (the force itself in place of its projection:
    a step's cost does not depend on the values) and one Jacobi-PCG
    projection of `cg_iters` fixed iterations with its divergence and
    gradient subtraction, timed on the host cores.  Reports Gcell-updates/s of
    the steps and seconds per CG iteration; with proj_iters, the seconds one
    projection at that iteration count would take at the sampled rate."""
    import oracle
    oracle.lib()
    cells = (grid[0] - 2) * (grid[1] - 2) * (grid[2] - 2)
    smax = oracle.default_sigma_max(grid, G, rho, sponge_cells)
    t0 = time.perf_counter()
    oracle.run(grid, G, rho, eta, dt, nsteps, FS=F, env=[1.0] * nsteps, sponge_cells=sponge_cells, sigma_max=smax)
    el = time.perf_counter() - t0
    t1 = time.perf_counter()
    oracle.project(grid, F, fixed_iters=cg_iters, jacobi=True)
    el_cg = time.perf_counter() - t1
    out = {"value": cells * nsteps / el / 1e9, "unit": "Gcell-updates/s", "kind": "oracle",
           "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
           "s_per_step": el / nsteps, "s_per_cg_iteration": el_cg / cg_iters,
           "sample": f"{nsteps} FDTD steps from rest with the force on ({el:.1f} s) and one Jacobi-PCG projection "
                     f"of {cg_iters} fixed iterations with divergence and gradient subtraction ({el_cg:.1f} s), "
                     f"FP64 C oracle, OpenMP"}
    if proj_iters:
        out["s_per_projection_at_gpu_iters"] = proj_iters * el_cg / cg_iters
        out["gpu_projection_iters"] = proj_iters
    return out


def run_config1(args):
    """The plain method at CPU size (48^3 FP64 homogeneous, Jacobi-PCG to
    1e-10, 200 steps, u_z on the lateral line): the whole simulation on the
    GPU (force resident in HBM, timed over repeats) and the oracle's whole
    run on the host cores; both traces compared."""
    import numpy as np
    import torch

    import oracle
    from oracle.analysis import rel_l2
    from paper_2607_28414_amd import kvs
    from workloads import cfg1_homogeneous_fp64

    w = cfg1_homogeneous_fp64()
    log("bench: 48^3 FP64 workload")
    stream = torch.cuda.current_stream()
    ctx = kvs.kvs_create(w.grid, precision=kvs.KVS_FP64, sponge_cells=w.sponge_cells, sponge_sigma_max=-1.0,
                         stream=stream.cuda_stream)
    try:
        kvs.kvs_set_material_uniform(ctx, w.G, w.rho, w.eta)
        kvs.kvs_set_dt(ctx, w.dt)
        kvs.kvs_set_envelope(ctx, w.env)
        kvs.kvs_set_probes(ctx, w.probes, w.comp)
        kvs.kvs_autotune_step(ctx, 5)
        F_dev = torch.from_numpy(np.ascontiguousarray(w.F)).to("cuda")

        def sim():
            kvs.kvs_reset_state(ctx)
            kvs.kvs_set_force_device(ctx, F_dev.data_ptr(), 0)
            rep = kvs.kvs_project(ctx, tol=w.tol, precond=kvs.KVS_PC_JACOBI)
            kvs.kvs_step(ctx, w.nsteps)
            return rep, kvs.kvs_read_traces(ctx, len(w.probes), 1)

        sim()
        torch.cuda.synchronize()
        reps = 10
        t0 = time.perf_counter()
        for _ in range(reps):
            rep, tr = sim()
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        smax = kvs.kvs_sponge_sigma_max(ctx)
    finally:
        kvs.kvs_destroy(ctx)
    cells = w.interior_cells
    out = {"workload": "homogeneous 48^3 FP64, h 0.5 mm, G 3 kPa, 8-cell sponge, Gaussian push 100 us, Jacobi-PCG "
                       "to 1e-10, dt 5e-5 s, 200 steps, u_z on the lateral line (cache-resident: no roofline)",
           "value": cells * w.nsteps / el / 1e9, "unit": "Gcell-updates/s", "ms_per_simulation": el * 1e3,
           "projection_iters": rep["iters"], "cpu_baseline": None}
    if not args.no_cpu_baseline:
        oracle.lib()
        t1 = time.perf_counter()
        FS_o, _, rep_o = oracle.project(w.grid, w.F, tol=w.tol, jacobi=True)
        _, _, tr_o = oracle.run(w.grid, w.G, w.rho, w.eta, w.dt, w.nsteps, FS=FS_o, env=w.env, probes=w.probes,
                                comp=w.comp, sponge_cells=w.sponge_cells, sigma_max=smax)
        el_o = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": cells * w.nsteps / el_o / 1e9, "unit": "Gcell-updates/s",
                               "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
                               "kind": "oracle", "sample": f"the whole simulation (projection {rep_o['iters']} "
                                                           f"iterations + 200 steps), {el_o:.2f} s"}
        out["trace_rel_l2_vs_oracle"] = rel_l2(tr, tr_o)
    return out


def run_batch(args, steps=None, warmup=None):
    """The 64-instance batched sweep; returns the result line (steps and
    warmup default to the command line's)."""
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    import numpy as np
    import torch

    from paper_2607_28414_amd import kvs
    from workloads import cfg3_batch_draws, gaussian_push, x_line_probes

    torch.cuda.set_device(0)
    h = 0.25e-3
    draws = cfg3_batch_draws(64)
    grids = [(e, e, e, h, h, h) for e, _, _, _ in draws]
    log(f"bench: building 64-instance batch ({sum(e ** 3 for e, *_ in draws) / 1e6:.0f} M cells)")
    b = kvs.kvs_batch_create(grids, precision=kvs.KVS_FP32, sponge_cells=8, sponge_sigma_max=-1.0,
                             stream=torch.cuda.current_stream().cuda_stream)
    nsteps = 2000
    try:
        first_of = {}
        F_dev = {}
        n_push = []
        for i, (e, G, rho, eta) in enumerate(draws):
            ctx = kvs.kvs_batch_instance(b, i)
            kvs.kvs_set_material_uniform(ctx, G, rho, eta)
            dt = 0.4 * kvs.kvs_stable_dt(ctx)
            kvs.kvs_set_dt(ctx, dt)
            env = np.ones(int(round(100e-6 / dt)))
            n_push.append(min(len(env), nsteps))
            kvs.kvs_set_envelope(ctx, env)
            kvs.kvs_batch_set_probes(b, i, x_line_probes(grids[i]))
            if e not in first_of:
                first_of[e] = i
                F_dev[e] = torch.from_numpy(gaussian_push(grids[i], 1e-3, 4e-3, 1e4)).to("cuda")
        kvs.kvs_batch_set_component(b, 2)
        bv, bz, bms = kvs.kvs_batch_autotune(b, 5)
        kvs.kvs_batch_set_step_blocking(b, args.step_blocking)
        two = args.step_blocking == 2 and kvs.kvs_batch_step_blocking_applies(b)
        log(f"bench: batch tile variant {bv}, z planes {bz} ({', '.join(f'{m:.2f}' for m in bms)} ms per step)")
        cells = [(e - 2) ** 3 for e, *_ in draws]

        def one_step():
            kvs.kvs_batch_reset(b)
            reps = {}
            for e, i in first_of.items():
                ctx = kvs.kvs_batch_instance(b, i)
                kvs.kvs_set_force_device(ctx, F_dev[e].data_ptr(), 0)
                reps[e] = kvs.kvs_project(ctx, tol=1e-8, precond=kvs.KVS_PC_JACOBI)
            for i, (e, *_) in enumerate(draws):
                if first_of[e] != i:
                    kvs.kvs_batch_share_projection(b, first_of[e], i)
            kvs.kvs_batch_step(b, nsteps)
            tr = [kvs.kvs_batch_read_traces(b, i, grids[i][0]) for i in range(len(draws))]
            return reps, tr

        for q in range(warmup):
            log(f"bench: warmup step {q} (graph capture)")
            one_step()
        torch.cuda.synchronize()
        log(f"bench: timing {steps} steps")
        t0 = time.perf_counter()
        for q in range(steps):
            reps, tr = one_step()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        # stepping alone: one replayed graph, between two device synchronisations
        kvs.kvs_batch_reset(b)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kvs.kvs_batch_step(b, nsteps)
        torch.cuda.synchronize()
        step_ms = (time.perf_counter() - t1) * 1e3
        assert all(np.all(np.isfinite(t)) for t in tr), "non-finite traces"
    finally:
        kvs.kvs_batch_destroy(b)
    total = sum(cells) * nsteps
    value = steps * total / el / 1e9
    bytes_total = 48.0 * total + 12.0 * sum(c * p for c, p in zip(cells, n_push))
    achieved = bytes_total / (step_ms * 1e-3) / 1e9
    # the homogeneous step's own read/write mix (6 + 6 FP32 per cell) streamed
    # over the same cell count: the practical ceiling for this kernel
    stream_gbs = kvs.kvs_measure_stream(sum(cells), 5, reads=6, writes=6)
    return {
        "metric": METRIC, "value": value, "unit": "Gcell-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": el / steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched sweep: 64 homogeneous instances, edges 96-192 (cubic), G 1-10 kPa, "
                               "eta 0-1.5 Pa s, rho 1000, dx 0.25 mm, 8-cell sponge, Gaussian push 100 us, "
                               "projection per distinct grid shared, 2000 steps each as one hipGraph, FP32",
                   "instances": 64, "total_cells": sum(e ** 3 for e, *_ in draws), "fdtd_steps": nsteps,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": ("batch_step2_kernel (two steps per launch over all instances, one launch per "
                                "tile width; push steps one per launch)" if two else
                                "batch_step_kernel (one launch per step over all instances)")
                               + "; graph time incl. probe gathers",
                     "steps_per_launch": 2 if two else 1,
                     "algorithmic_bytes_per_cell_update": "48 (+12 on push steps)", "graph_ms": step_ms,
                     "variant": bv, "zchunk": bz, "stream_gbs": stream_gbs,
                     "frac_of_stream": achieved / stream_gbs,
                     "stream_note": "kvs_measure_stream_rw(6, 6): the homogeneous step's 6 FP32 reads + 6 writes "
                                    "per cell (48 B) with no stencil, over the interior cell count"},
        "projection": {"precond": "jacobi", "tol": 1e-8,
                       "per_grid": {str(e): {"iters": r["iters"], "ms": r["ms"]} for e, r in reps.items()}},
        "cpu_baseline": batch_cpu_window(draws, {e: r["iters"] for e, r in reps.items()}, nsteps)
        if not args.no_cpu_baseline else None,
    }


def batch_cpu_window(draws, proj_iters, nsteps, steps_sample=6, cg_sample=20):
    """The FP64 oracle on a window of the batched sweep: for each distinct
    edge, `steps_sample` steps of one of its instances (from rest, push on)
    and `cg_sample` Jacobi-PCG iterations of its grid's projection; value =
    the whole sweep (every instance's `nsteps` steps and one projection per
    distinct grid at the GPU's iteration counts) at the sampled rates."""
    import numpy as np

    import oracle
    from workloads import gaussian_push, x_line_probes
    h = 0.25e-3
    oracle.lib()
    t_step, t_iter, spent = {}, {}, 0.0
    for e in sorted(proj_iters):
        _, G, rho, eta = next(d for d in draws if d[0] == e)
        grid = (e, e, e, h, h, h)
        F = gaussian_push(grid, 1e-3, 4e-3, 1e4)
        t0 = time.perf_counter()
        FS, _, _ = oracle.project(grid, F, fixed_iters=cg_sample, jacobi=True)
        t_iter[e] = (time.perf_counter() - t0) / cg_sample
        dt = 0.4 * oracle.stable_dt(grid, G, rho, eta)
        smax = oracle.default_sigma_max(grid, G, rho, 8)
        t1 = time.perf_counter()
        oracle.run(grid, G, rho, eta, dt, steps_sample, FS=FS, env=np.ones(steps_sample), probes=x_line_probes(grid),
                   comp=2, sponge_cells=8, sigma_max=smax)
        t_step[e] = (time.perf_counter() - t1) / steps_sample
        spent += time.perf_counter() - t0
    t_job = sum(nsteps * t_step[d[0]] for d in draws) + sum(proj_iters[e] * t_iter[e] for e in proj_iters)
    updates = nsteps * sum((d[0] - 2) ** 3 for d in draws)
    return {"value": updates / t_job / 1e9, "unit": "Gcell-updates/s",
            "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)), "kind": "oracle",
            "whole_sweep_s": t_job,
            "sample": f"per distinct edge ({', '.join(str(e) for e in sorted(proj_iters))}): {steps_sample} steps of "
                      f"one instance and {cg_sample} Jacobi-PCG iterations of its projection, {spent:.1f} s in all; "
                      f"value = the whole 64-instance sweep at the sampled rates"}


def run_kvline_bench(args):
    """The 1-D harmonic Kelvin-Voigt sweep (Sec. 4.3): the 16 viscosities as
    one FP32 batch of 301 x 3 x 3 line instances (transverse spacings 1e6 m),
    a common dt = 0.3 x the most viscous instance's limit, 16 ms of harmonic
    drive (16071 steps) replayed as one hipGraph; HIP events on the batch's
    stream around the replay.  The oracle runs the same sweep on the host for
    the CPU baseline."""
    import numpy as np
    import torch

    from paper_2607_28414_amd import kvs
    from workloads import KV_LINE_ETAS, kv_line_case, kv_line_grid

    torch.cuda.set_device(0)
    G, rho = 4e3, 1000.0
    grid = kv_line_grid()
    n = len(KV_LINE_ETAS)
    stream = torch.cuda.current_stream()
    b = kvs.kvs_batch_create([grid] * n, precision=kvs.KVS_FP32, sponge_cells=0, stream=stream.cuda_stream)
    try:
        dts = []
        for i, eta in enumerate(KV_LINE_ETAS):
            ctx = kvs.kvs_batch_instance(b, i)
            kvs.kvs_set_material_uniform(ctx, G, rho, eta)
            dts.append(kvs.kvs_stable_dt(ctx))
        dt = 0.3 * min(dts)
        nsteps = int(round(16e-3 / dt))
        cases = []
        for i, eta in enumerate(KV_LINE_ETAS):
            ctx = kvs.kvs_batch_instance(b, i)
            kvs.kvs_set_dt(ctx, dt)
            # sensor placement from the expected wave is irrelevant to the cost:
            # the elastic wavelength and no attenuation for every instance
            case = kv_line_case(grid, eta, dt, nsteps, 0.0, 2.0)
            kvs.kvs_set_envelope(ctx, case["env"])
            kvs.kvs_set_projected_force(ctx, case["FS"])
            kvs.kvs_batch_set_probes(b, i, case["probes"])
            cases.append(case)
        kvs.kvs_batch_set_component(b, 2)
        persistent = kvs.kvs_batch_uses_persistent(b)
        log(f"bench: kv line sweep, {n} instances, {nsteps} steps ("
            + ("one persistent launch" if persistent else "graph capture") + ")")
        kvs.kvs_batch_step(b, nsteps)
        # events on the batch's own stream (the library makes one when it is
        # handed the null stream)
        lib_stream = torch.cuda.ExternalStream(kvs.kvs_stream(kvs.kvs_batch_instance(b, 0)))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ms = []
        for _ in range(max(1, args.steps)):
            kvs.kvs_batch_reset(b)
            torch.cuda.synchronize()
            e0.record(lib_stream)
            kvs.kvs_batch_step(b, nsteps)
            e1.record(lib_stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        tr = kvs.kvs_batch_read_traces(b, n - 1, len(cases[-1]["probes"]))
        assert np.all(np.isfinite(tr)), "non-finite traces"
    finally:
        kvs.kvs_batch_destroy(b)
    gpu_ms = float(np.median(ms))
    res = {"workload": f"1-D harmonic Kelvin-Voigt sweep: {n} viscosities (0-1.5 Pa s) as one FP32 batch of "
                       f"{grid[0]}x3x3 lines, h 0.1 mm, {nsteps} steps (16 ms), "
                       + ("one persistent launch (state in LDS, one workgroup per line)" if persistent
                          else "one hipGraph of per-step launches"),
           "ms_per_sweep": gpu_ms, "us_per_step": 1e3 * gpu_ms / nsteps, "instances": n, "fdtd_steps": nsteps,
           "cpu_baseline": None}
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        for eta, case in zip(KV_LINE_ETAS, cases):
            oracle.run(grid, G, rho, eta, dt, nsteps, FS=case["FS"], env=case["env"], probes=case["probes"],
                       comp=2)
        cpu_ms = (time.perf_counter() - t0) * 1e3
        # the oracle splits its loops over z planes: a line has one interior plane
        res["cpu_baseline"] = {"value": cpu_ms, "unit": "ms per sweep", "cores": 1, "kind": "oracle",
                               "sample": "the whole sweep, FP64, one thread (one interior z plane)"}
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the solver has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.workload == "batch":
        print(json.dumps(run_batch(args)), flush=True)
        return
    if args.workload == "fpcg":
        print(json.dumps(run_fpcg_profile(args)), flush=True)
        return
    if args.workload == "arf":
        print(json.dumps(arf_workload(args)), flush=True)
        return
    if args.workload == "pml":
        print(json.dumps(run_pml_bench(args)), flush=True)
        return
    if args.workload == "kvline":
        print(json.dumps(run_kvline_bench(args)), flush=True)
        return
    import numpy as np
    import torch

    from paper_2607_28414_amd import kvs
    from workloads import cfg2_inclusions_fp32

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    n = args.grid
    log(f"bench: building inclusion workload {n}^3")
    w = cfg2_inclusions_fp32(n=n)
    ctx = kvs.kvs_create(w.grid, precision=kvs.KVS_FP32, sponge_cells=w.sponge_cells, sponge_sigma_max=-1.0,
                         stream=stream.cuda_stream)
    try:
        kvs.kvs_set_material(ctx, w.G, w.rho, w.eta)
        dt = w.dt_factor * kvs.kvs_stable_dt(ctx)
        kvs.kvs_set_dt(ctx, dt)
        env = w.envelope_for(dt)
        kvs.kvs_set_envelope(ctx, env)
        kvs.kvs_set_probes(ctx, w.probes, w.comp)
        F_dev = torch.from_numpy(np.ascontiguousarray(w.F)).to("cuda")
        if args.step_variant >= 0:
            variant = args.step_variant
            kvs.kvs_set_step_variant(ctx, variant)
            log(f"bench: step-kernel variant {variant} (pinned)")
        else:
            variant, variant_ms = kvs.kvs_autotune_step(ctx, 20)
            log(f"bench: step-kernel variant {variant} ({', '.join(f'{m * 1e3:.1f}' for m in variant_ms)} us)")
        kvs.kvs_set_step_blocking(ctx, args.step_blocking)
        log(f"bench: {args.step_blocking} step(s) per launch (two-step kernel applies: "
            f"{kvs.kvs_step_blocking_applies(ctx)})")
        torch.cuda.synchronize()
        nsteps = w.nsteps
        cells = w.interior_cells
        n_push = min(len(env), nsteps)

        def one_step():
            kvs.kvs_reset_state(ctx)
            kvs.kvs_set_force_device(ctx, F_dev.data_ptr(), 0)
            rep = kvs.kvs_project(ctx, tol=w.tol, max_iter=20000, precond=kvs.KVS_PC_JACOBI)
            kvs.kvs_step(ctx, nsteps)
            tr = kvs.kvs_read_traces(ctx, len(w.probes), 1)
            return rep, tr

        for q in range(args.warmup):
            log(f"bench: warmup step {q}")
            rep, _ = one_step()
        torch.cuda.synchronize()
        kvs.kvs_enable_kernel_timing(ctx, True)
        log(f"bench: timing {args.steps} steps")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        proj_ms = []
        for q in range(args.steps):
            rep, tr = one_step()
            proj_ms.append(rep["ms"])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        k_ms, k_launches = kvs.kvs_kernel_time(ctx)
        (ms1, n1), (ms2, n2) = kvs.kvs_kernel_time_split(ctx)
        kvs.kvs_enable_kernel_timing(ctx, False)
        assert np.all(np.isfinite(tr)), "non-finite traces"
        # after the timed region: the same simulation with the force handed over
        # from host memory (FP64, pageable) across PCIe
        F_host = np.ascontiguousarray(w.F)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kvs.kvs_reset_state(ctx)
        kvs.kvs_set_force(ctx, F_host)
        kvs.kvs_project(ctx, tol=w.tol, max_iter=20000, precond=kvs.KVS_PC_JACOBI)
        kvs.kvs_step(ctx, nsteps)
        kvs.kvs_read_traces(ctx, len(w.probes), 1)
        torch.cuda.synchronize()
        pcie_ms = (time.perf_counter() - t1) * 1e3
        FS_host = kvs.kvs_get_projected_force(ctx, w.shape) if not args.no_cpu_baseline else None
        smax = kvs.kvs_sponge_sigma_max(ctx)
        # reference: the one-step kernel alone on the same medium (200 launches
        # without force, continuing from the state above)
        kvs.kvs_set_envelope(ctx, [])
        kvs.kvs_set_step_blocking(ctx, 1)
        kvs.kvs_enable_kernel_timing(ctx, True)
        kvs.kvs_step(ctx, 200)
        one_ms, one_n = kvs.kvs_kernel_time(ctx)
        kvs.kvs_enable_kernel_timing(ctx, False)
    finally:
        kvs.kvs_destroy(ctx)

    total_updates = args.steps * nsteps * cells
    value = total_updates / el / 1e9
    # algorithmic bytes of the step launches over the timed launches (the
    # one-step model: 60 B per cell-update, 72 B on push steps)
    bytes_total = args.steps * (nsteps * cells * 60 + n_push * cells * 12)
    achieved = bytes_total / (k_ms * 1e-3) / 1e9
    copy_gbs = measured_copy_gbs()  # after the timed region
    stream_gbs = kvs.kvs_measure_stream(cells, 10) if not args.no_extra_legs else None
    one_us = one_ms / one_n * 1e3
    one_gbs = cells * 60 / (one_us * 1e-6) / 1e9
    one_step = {"kernel": "step_kernel (one step per launch, no force)", "us_per_launch": one_us,
                "launches": one_n, "variant": variant, "achieved_GBs": one_gbs,
                "frac_of_hbm_peak": one_gbs / HBM_PEAK_GBS, "traffic": step_traffic(variant),
                "frac_of_stream": one_gbs / stream_gbs if stream_gbs else None,
                "note": "reference run of the one-step kernel after the timed region, 60 B per cell-update"}
    if n2 > 0:
        # dominant kernel: two steps per launch, bound by vector-ALU issue
        t2 = ms2 / n2  # ms per two-step launch
        tflops = FLOP_PER_CELL_UPDATE * 2 * cells / (t2 * 1e-3) / 1e12
        hbm_eq = 60 * 2 * cells / (t2 * 1e-3) / 1e9
        traffic2 = step2_traffic()
        roofline = {
            "bound": "hbm",
            "achieved": hbm_eq,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": hbm_eq / HBM_PEAK_GBS,
            "traffic": traffic2,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "algorithmic_bytes_per_launch": 60 * 2 * cells,
            "traffic_over_algorithmic": traffic2 / (60 * 2 * cells) if traffic2 else None,
            "kernel": "step2_kernel (two FDTD steps per launch)",
            "algorithmic_bytes_per_cell_update": 60,
            "units_per_launch": "2 x interior cells (cell-updates)",
            "limited_by": "vector-ALU issue (79-83 % VALU busy in the counter runs); the kernel moves 60 B per "
                          "two cell-updates, about 0.55x the one-step algorithmic bytes",
            "alu": {"achieved": tflops, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": tflops / FP32_PEAK_TFLOPS, "flop_per_cell_update": FLOP_PER_CELL_UPDATE,
                    "peak_note": "FP32 FMA peak without packed FP32 (256 CUs x 4 SIMDs x 16 lanes x 2 x 2.4 GHz)",
                    "frac_of_packed_fp32_peak": tflops / FP32_PACKED_PEAK_TFLOPS},
            "kernel_ms_avg": t2,
            "launches": n2,
            "steps_per_launch": 2,
            "us_per_step": t2 / 2 * 1e3,
            "copy_gbs": copy_gbs,
            "frac_of_copy": hbm_eq / copy_gbs,
            "stream_gbs": stream_gbs,
            "frac_of_stream": hbm_eq / stream_gbs if stream_gbs else None,
            "stream_note": "kvs_measure_stream: the one-step pattern, 9 FP32 reads + 6 writes per cell (60 B) with "
                           "no stencil, over the interior cell count: the ceiling of any one-step kernel",
            "one_step_launches": {"launches": n1, "ms_avg": ms1 / n1 if n1 else None,
                                  "note": "push steps (with force) and an odd last step, one step each"},
        }
    else:
        traffic = step_traffic(variant)
        roofline = {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "traffic_over_algorithmic": traffic / (cells * 60) if traffic else None,
            "kernel": "step_kernel (FDTD step)",
            "algorithmic_bytes_per_cell_update": "60 (+12 on push steps)",
            "kernel_ms_avg": k_ms / max(k_launches, 1),
            "launches": k_launches,
            "variant": variant,
            "copy_gbs": copy_gbs,
            "frac_of_copy": achieved / copy_gbs,
            "stream_gbs": stream_gbs,
            "frac_of_stream": achieved / stream_gbs if stream_gbs else None,
            "stream_note": "kvs_measure_stream: the step's 9 FP32 reads + 6 writes per cell (60 B) with no stencil, "
                           "over the interior cell count",
        }
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"heterogeneous inclusions {n}^3, dx 0.25 mm, 12 spheres, Gaussian push 100 us, "
                        f"dt 0.4 x stable limit, {nsteps} FDTD steps, FP32 state + Jacobi-PCG projection to 1e-8 (FP64 potential, inner products and true residual; FP32 search direction and recursive residual with reliable updates)",
            "grid": [n, n, n],
            "fdtd_steps": nsteps,
            "interior_cells": cells,
            "parallelism": "single GPU",
        },
        "roofline": roofline,
        "one_step_kernel": one_step,
        "step_blocking": args.step_blocking,
        "fdtd_kernel_gcells": args.steps * nsteps * cells / (k_ms * 1e-3) / 1e9,
        "pcie_inclusive": {"value": nsteps * cells / (pcie_ms * 1e-3) / 1e9, "unit": "Gcell-updates/s",
                           "ms_per_step": pcie_ms, "host_force_bytes": int(F_host.nbytes),
                           "note": "one simulation with the force copied from pageable host memory (FP64) "
                                   "instead of device memory; traces to the host as in the timed steps"},
        "projection": {"precond": "jacobi", "tol": w.tol, "iters": rep["iters"],
                       "relres_true": rep["relres_true"], "ms": float(np.mean(proj_ms)), "cg_storage": CG_STORAGE},
    }
    if not args.no_cpu_baseline:
        log(f"bench: CPU oracle sample ({args.cpu_sample_steps} steps, then 4 on one thread)")
        res["cpu_baseline"] = cpu_baseline(w, dt, smax, FS_host, args.cpu_sample_steps, rep["iters"])
    else:
        res["cpu_baseline"] = None
    res["config1"] = res["batch"] = res["kvline"] = None
    if not args.no_extra_legs:
        res["config1"] = run_config1(args)
        res["batch"] = run_batch(args, steps=args.batch_steps, warmup=args.batch_warmup)
        res["kvline"] = run_kvline_bench(args)
    res["projection_learned"] = res["time_varying"] = res["shell"] = res["arf"] = None
    if not args.no_learned:
        net = kvs.kvs_unet_create((16, 32, 64), args.unet_bottleneck)
        try:
            res["projection_learned"] = learned_projection(args, net)
            if not args.no_workloads:
                res["time_varying"] = time_varying_window(args, net)
                res["shell"] = shell_workload(args, net)
                res["arf"] = arf_workload(args)
        finally:
            kvs.kvs_unet_destroy(net)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
