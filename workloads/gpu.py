"""Device-side input drawing for benchmarks and tests: synthetic acoustic
samples (the focused tone burst of ``acoustic_beam_samples``) written by a
small HIP kernel into torch-allocated device buffers, instead of being
computed by torch or on the host.  Holds none of the solver's arithmetic;
the solver library does not use it."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "beam.hip")
LIB = os.path.join(HERE, "libworkloads.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

_lib = None


def build(verbose: bool = False) -> str:
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError(f"{LIB} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB)
        d, i = C.c_double, C.c_int
        L.wl_beam_samples.argtypes = [i, i, i, d, d, d, d, d, d, d, d, d, d, d, d, i, i, C.c_longlong, i, i,
                                      C.c_void_p, C.c_void_p, C.c_void_p]
        L.wl_beam_samples.restype = i
        _lib = L
    return _lib


def beam_samples_device(grid, samples, f0=1.0e6, c=1540.0, rho=1000.0, alpha=5.8, p0=1.5e6, w0=1.5e-3,
                        focus=(0.0, 0.0, 0.0), per=20, cycles=10, s0=0, dtype="float32", with_v=True, stream=None):
    """(p, v) as torch device tensors, [samples][nz][ny][nx] and
    [samples][3][nz][ny][nx] (v None when with_v is False), with the
    parameters and meaning of workloads.acoustic_beam_samples."""
    import torch
    nx, ny, nz, hx, hy, hz = grid
    tdt = torch.float32 if dtype in ("float32", np.float32, torch.float32) else torch.float64
    p = torch.empty((samples, nz, ny, nx), dtype=tdt, device="cuda")
    v = torch.empty((samples, 3, nz, ny, nx), dtype=tdt, device="cuda") if with_v else None
    st = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    err = lib().wl_beam_samples(int(nx), int(ny), int(nz), float(hx), float(hy), float(hz), float(focus[0]),
                                float(focus[1]), float(focus[2]), float(f0), float(c), float(rho), float(alpha),
                                float(p0), float(w0), int(per), int(cycles), int(s0), int(samples),
                                1 if tdt == torch.float32 else 0, p.data_ptr(), v.data_ptr() if v is not None else None,
                                st or None)
    if err != 0:
        raise RuntimeError(f"wl_beam_samples failed with HIP error {err}")
    return p, v
