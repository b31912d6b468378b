"""Writes curl_wavespeed_180.txt: the oracle's u_z traces of the non-viscous
wavespeed validation (Sec. 4.1) at the four depth sensors, 180^3 grid, curl
initial state, 360 steps.  Calls only the oracle and the input generator.

    python tests/golden/make_curl_wavespeed.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "curl_wavespeed_180.txt")


def main():
    w = workloads.curl_wavespeed_case()
    dt = w["dt_factor"] * oracle.stable_dt(w["grid"], w["G"], w["rho"], w["eta"])
    u, ww = oracle.curl_state(w["grid"], w["A"], dt)
    _, _, tr = oracle.run(w["grid"], w["G"], w["rho"], w["eta"], dt, w["nsteps"], u=u, w=ww, probes=w["probes"],
                          comp=2)
    with open(OUT, "w") as f:
        f.write("# Oracle (FP64) u_z traces of the Sec. 4.1 wavespeed validation: workloads.curl_wavespeed_case()\n")
        f.write("# defaults, curl initial state, written by tests/golden/make_curl_wavespeed.py.\n")
        f.write(f"# dt {dt!r}\n")
        f.write("# offsets_m " + " ".join(repr(float(o)) for o in w["offsets"]) + "\n")
        f.write("# one row per step (u_z after the step), one column per sensor\n")
        for row in tr[:, :, 0]:
            f.write(" ".join(f"{v:.17e}" for v in row) + "\n")


if __name__ == "__main__":
    main()
