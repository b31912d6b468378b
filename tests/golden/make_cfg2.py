"""Writes cfg2_256_traces.npz: the oracle's own end-to-end run of the 256^3
inclusion workload (workloads.cfg2_inclusions_fp32(), the benchmark's
workload): dt = 0.4 x the stable limit, the default sponge strength, the
Jacobi-PCG projection of the Gaussian push to 1e-8 (Sec. 3.2.3) and 4000
steps of the summed-form update (Sec. 3.1, 3.3) in FP64, with the u_z
traces of 32 of the 256 lateral-line probes (x = 2, 10, ..., 250 on the line
through the push) after every step.  Calls only the oracle and the input
generator.

    python tests/golden/make_cfg2.py          # about 25 min on 8 cores
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import cfg2_inclusions_fp32  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg2_256_traces.npz")
KEEP = np.arange(2, 256, 8)  # probe indices along the x line


def main():
    w = cfg2_inclusions_fp32(n=256)
    t0 = time.time()
    dt = w.dt_factor * oracle.stable_dt(w.grid, w.G, w.rho, w.eta)
    smax = oracle.default_sigma_max(w.grid, w.G, w.rho, w.sponge_cells)
    env = w.envelope_for(dt)
    FS, _, rep = oracle.project(w.grid, w.F, tol=w.tol, max_iter=20000, jacobi=True)
    print(f"projection {rep} ({time.time() - t0:.0f} s)", flush=True)
    assert rep["status"] == 0
    probes = w.probes[KEEP]
    u = w_ = None
    chunks = []
    done = 0
    while done < w.nsteps:
        n = min(250, w.nsteps - done)
        u, w_, tr = oracle.run(w.grid, w.G, w.rho, w.eta, dt, n, FS=FS, env=env, u=u, w=w_, step0=done,
                               probes=probes, comp=w.comp, sponge_cells=w.sponge_cells, sigma_max=smax)
        chunks.append(tr[:, :, 0])
        done += n
        print(f"step {done} / {w.nsteps} ({time.time() - t0:.0f} s)", flush=True)
    np.savez_compressed(OUT, traces=np.concatenate(chunks), probes=probes, dt=dt, sigma_max=smax,
                        n_push=len(env), projection_iters=rep["iters"], relres_true=rep["relres_true"])
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
