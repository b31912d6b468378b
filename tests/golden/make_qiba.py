"""Writes qiba_240x200x200.txt: the oracle's results for the QIBA-like
phantoms of Sec. 4.4 (workloads.qiba_phantoms() defaults): per phantom the
time step, the group speed from cross-correlation of the axial velocity
traces at 4-14 mm lateral offsets, the lags, and the axial displacement
traces of three sensors (4, 9 and 14 mm).  One Jacobi-PCG projection to 1e-8
serves all phantoms (same grid and force); 8-cell sponge with the default
strength; dt = 0.4 x the stable limit.  Calls only the oracle and the input
generator.

    python tests/golden/make_qiba.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle.analysis import centred_velocity, group_speed_xcorr  # noqa: E402
import workloads  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "qiba_240x200x200.txt")
SPONGE = 8
KEEP = (0, 10, 20)  # sensors stored in full: 4, 9 and 14 mm


def main():
    w = workloads.qiba_phantoms()
    grid = w["grid"]
    FS, _, rep = oracle.project(grid, w["F"], tol=1e-8, jacobi=True)
    print("projection", rep, flush=True)
    lines = ["# Oracle (FP64) results of the QIBA-like phantoms (Sec. 4.4), written by tests/golden/make_qiba.py",
             f"# projection_iters {rep['iters']}",
             "# offsets_m " + " ".join(repr(float(o)) for o in w["offsets"]),
             "# kept_sensors " + " ".join(str(k) for k in KEEP)]
    for G in w["G"]:
        dt = w["dt_factor"] * oracle.stable_dt(grid, G, w["rho"], w["eta"])
        smax = oracle.default_sigma_max(grid, G, w["rho"], SPONGE)
        env = np.ones(max(1, int(round(w["push_time"] / dt))))
        _, _, tr = oracle.run(grid, G, w["rho"], w["eta"], dt, w["nsteps"], FS=FS, env=env, probes=w["probes"],
                              comp=w["comp"], sponge_cells=SPONGE, sigma_max=smax)
        tr = tr[:, :, 0]
        speed, lags = group_speed_xcorr(centred_velocity(tr, dt), w["offsets"], dt)
        print(f"G {G}: dt {dt} speed {speed} (cs {np.sqrt(G / w['rho'])})", flush=True)
        lines.append(f"# phantom G {G!r} dt {dt!r} sigma_max {smax!r} n_push {len(env)} speed {speed!r}")
        lines.append("# lags " + " ".join(repr(float(v)) for v in lags))
        for row in tr[:, KEEP]:
            lines.append(" ".join(f"{v:.17e}" for v in row))
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
