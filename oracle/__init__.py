"""Plain FP64 CPU oracle of the reduced Kelvin-Voigt shear solver.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``.  The GPU library never imports,
links or calls anything here, and nothing here imports the GPU library.

The arithmetic lives in ``kvs_oracle.c`` (plain loops, FP64, OpenMP on the
outer loop); this module only marshals numpy arrays into it.  Arrays use the
layout [nz][ny][nx] (x fastest) for scalars and [3][nz][ny][nx] for vectors.
A grid is the tuple ``(nx, ny, nz, hx, hy, hz)``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kvs_oracle.c")
LIB = os.path.join(HERE, "libkvs_oracle.so")

OK, EINVAL, ENOMEM, ENOTCONV, EBREAKDOWN = 0, 1, 2, 4, 5


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11", "-Wall", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


class _Grid(C.Structure):
    _fields_ = [("nx", C.c_long), ("ny", C.c_long), ("nz", C.c_long),
                ("hx", C.c_double), ("hy", C.c_double), ("hz", C.c_double)]


class _Report(C.Structure):
    _fields_ = [("iters", C.c_long), ("relres_recursive", C.c_double),
                ("relres_true", C.c_double), ("status", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        lp = C.POINTER(C.c_long)
        gp = C.POINTER(_Grid)
        L.ora_laplacian.argtypes = [gp, dp, dp]
        L.ora_elastic.argtypes = [gp, dp, dp, dp]
        L.ora_divergence.argtypes = [gp, dp, dp]
        L.ora_true_relres.argtypes = [gp, dp, dp]
        L.ora_true_relres.restype = C.c_double
        L.ora_cg.argtypes = [gp, dp, dp, C.c_double, C.c_long, C.c_long, C.c_int, C.POINTER(_Report)]
        L.ora_grad_subtract.argtypes = [gp, dp, dp, dp]
        L.ora_project.argtypes = [gp, dp, dp, dp, C.c_double, C.c_long, C.c_long, C.c_int, C.POINTER(_Report)]
        L.ora_sponge_sigma.argtypes = [gp, C.c_long, C.c_long, C.c_long, C.c_int, C.c_double]
        L.ora_sponge_sigma.restype = C.c_double
        L.ora_default_sigma_max.argtypes = [gp, dp, dp, C.c_int]
        L.ora_default_sigma_max.restype = C.c_double
        L.ora_stable_dt.argtypes = [gp, dp, dp, dp]
        L.ora_stable_dt.restype = C.c_double
        L.ora_run.argtypes = [gp, dp, dp, dp, C.c_int, C.c_double, C.c_double, dp, dp, C.c_long,
                              dp, dp, C.c_long, C.c_long, lp, C.c_long, C.c_int, dp]
        L.ora_step_cells.argtypes = [gp, dp, dp, dp, C.c_int, C.c_double, C.c_double, dp, C.c_double,
                                     dp, dp, lp, C.c_long, dp, dp]
        _lib = L
    return _lib


def _g(grid):
    nx, ny, nz, hx, hy, hz = grid
    return C.byref(_Grid(int(nx), int(ny), int(nz), float(hx), float(hy), float(hz)))


def _d(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _shape(grid):
    nx, ny, nz = (int(v) for v in grid[:3])
    return (nz, ny, nx)


def _field(grid, v):
    """Scalar material argument: broadcast a number to a full field."""
    if np.isscalar(v):
        return np.full(_shape(grid), float(v))
    return _f64(v).reshape(_shape(grid))


def laplacian(grid, q):
    q = _f64(q)
    out = np.empty_like(q)
    lib().ora_laplacian(_g(grid), _d(q), _d(out))
    return out


def elastic(grid, G, q):
    G = _field(grid, G)
    q = _f64(q)
    out = np.empty_like(q)
    lib().ora_elastic(_g(grid), _d(G), _d(q), _d(out))
    return out


def divergence(grid, F):
    F = _f64(F)
    b = np.empty(_shape(grid))
    lib().ora_divergence(_g(grid), _d(F), _d(b))
    return b


def true_relres(grid, b, phi):
    return lib().ora_true_relres(_g(grid), _d(_f64(b)), _d(_f64(phi)))


def cg(grid, rhs, tol=1e-10, max_iter=10000, fixed_iters=0, jacobi=False):
    """Solve (-lap_h) phi = rhs on the interior; returns (phi, report dict)."""
    rhs = _f64(rhs)
    phi = np.zeros_like(rhs)
    rep = _Report()
    lib().ora_cg(_g(grid), _d(rhs), _d(phi), tol, int(max_iter), int(fixed_iters), int(bool(jacobi)), C.byref(rep))
    return phi, _rep(rep)


def _rep(rep):
    return dict(iters=rep.iters, relres_recursive=rep.relres_recursive,
                relres_true=rep.relres_true, status=rep.status)


def grad_subtract(grid, F, phi):
    F = _f64(F)
    FS = np.empty_like(F)
    lib().ora_grad_subtract(_g(grid), _d(F), _d(_f64(phi)), _d(FS))
    return FS


def project(grid, F, tol=1e-10, max_iter=10000, fixed_iters=0, jacobi=False):
    """Separable-source pre-computation: returns (FS, phi, report dict)."""
    F = _f64(F)
    FS = np.empty_like(F)
    phi = np.empty(_shape(grid))
    rep = _Report()
    lib().ora_project(_g(grid), _d(F), _d(FS), _d(phi), tol, int(max_iter), int(fixed_iters),
                      int(bool(jacobi)), C.byref(rep))
    return FS, phi, _rep(rep)


def sponge_sigma(grid, i, j, k, cells, sigma_max):
    return lib().ora_sponge_sigma(_g(grid), int(i), int(j), int(k), int(cells), float(sigma_max))


def default_sigma_max(grid, G, rho, cells):
    return lib().ora_default_sigma_max(_g(grid), _d(_field(grid, G)), _d(_field(grid, rho)), int(cells))


def stable_dt(grid, G, rho, eta):
    return lib().ora_stable_dt(_g(grid), _d(_field(grid, G)), _d(_field(grid, rho)), _d(_field(grid, eta)))


def run(grid, G, rho, eta, dt, nsteps, FS=None, env=None, u=None, w=None, step0=0,
        probes=None, comp=2, sponge_cells=0, sigma_max=0.0):
    """Advance the state by nsteps.  Returns (u, w, traces) with traces of
    shape [nsteps][nprobes][ncomp] (ncomp = 3 if comp == 3 else 1)."""
    shp = _shape(grid)
    G, rho, eta = _field(grid, G), _field(grid, rho), _field(grid, eta)
    u = np.zeros((3,) + shp) if u is None else _f64(u).copy()
    w = np.zeros((3,) + shp) if w is None else _f64(w).copy()
    probes = np.zeros((0, 3), dtype=np.int64) if probes is None else np.ascontiguousarray(probes, dtype=np.int64)
    ncomp = 3 if comp == 3 else 1
    traces = np.zeros((int(nsteps), len(probes), ncomp))
    FSa = None if FS is None else _f64(FS)
    enva = None if env is None else _f64(env)
    st = lib().ora_run(_g(grid), _d(G), _d(rho), _d(eta), int(sponge_cells), float(sigma_max), float(dt),
                       _d(FSa) if FSa is not None else None, _d(enva) if enva is not None else None,
                       0 if enva is None else len(enva), _d(u), _d(w), int(step0), int(nsteps),
                       probes.ctypes.data_as(C.POINTER(C.c_long)), len(probes), int(comp), _d(traces))
    if st != OK:
        raise RuntimeError(f"ora_run failed with status {st}")
    return u, w, traces


def step_cells(grid, G, rho, eta, dt, u, w, cells, FS=None, gn=0.0, sponge_cells=0, sigma_max=0.0):
    """One step evaluated at the listed flat interior cell indices only.
    Returns (u_new, w_new), each [ncells][3]."""
    G, rho, eta = _field(grid, G), _field(grid, rho), _field(grid, eta)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    uo = np.zeros((len(cells), 3))
    wo = np.zeros((len(cells), 3))
    FSa = None if FS is None else _f64(FS)
    st = lib().ora_step_cells(_g(grid), _d(G), _d(rho), _d(eta), int(sponge_cells), float(sigma_max), float(dt),
                              _d(FSa) if FSa is not None else None, float(gn), _d(_f64(u)), _d(_f64(w)),
                              cells.ctypes.data_as(C.POINTER(C.c_long)), len(cells), _d(uo), _d(wo))
    if st != OK:
        raise RuntimeError(f"ora_step_cells failed with status {st}")
    return uo, wo


def plane_view(a, axis, index):
    """Slice [..][nz][ny][nx] arrays on a grid plane: axis 0 -> [nz][ny],
    axis 1 -> [nz][nx], axis 2 -> [ny][nx]."""
    return {0: lambda: a[..., :, :, index], 1: lambda: a[..., :, index, :], 2: lambda: a[..., index, :, :]}[axis]()


def peak_maps(grid, G, rho, eta, dt, nsteps, planes, FS=None, env=None, u=None, w=None, step0=0,
              sponge_cells=0, sigma_max=0.0):
    """Running peak of the displacement magnitude |u| on grid planes (the
    |u| slices and peak displacement of the transcranial demonstration,
    Sec. 5.1): the maps start at |u| of the given state and after every step
    take the larger of themselves and |u^{n+1}|.  planes = [(axis, index)].
    Returns (maps, u, w)."""
    shp = _shape(grid)
    u = np.zeros((3,) + shp) if u is None else _f64(u).copy()
    w = np.zeros((3,) + shp) if w is None else _f64(w).copy()

    def mag(a, axis, index):
        v = plane_view(a, axis, index)
        return np.sqrt(v[0] ** 2 + v[1] ** 2 + v[2] ** 2)

    maps = [mag(u, a, i) for a, i in planes]
    for n in range(int(nsteps)):
        u, w, _ = run(grid, G, rho, eta, dt, 1, FS=FS, env=env, u=u, w=w, step0=step0 + n,
                      sponge_cells=sponge_cells, sigma_max=sigma_max)
        maps = [np.maximum(m, mag(u, a, i)) for m, (a, i) in zip(maps, planes)]
    return maps, u, w


def curl(grid, A):
    """Centred curl of a vector potential A ([3][nz][ny][nx]) on the interior
    nodes, zero on the outer layer: the curl-based initialisation of Sec. 3.5
    (a divergence-free field built from a vector potential), with the centred
    first differences (f(+a) - f(-a)) / (2 h_a) of the grid."""
    nx, ny, nz, hx, hy, hz = grid
    A = _f64(A).reshape((3,) + _shape(grid))

    def dx(f):
        return (f[1:-1, 1:-1, 2:] - f[1:-1, 1:-1, :-2]) / (2 * hx)

    def dy(f):
        return (f[1:-1, 2:, 1:-1] - f[1:-1, :-2, 1:-1]) / (2 * hy)

    def dz(f):
        return (f[2:, 1:-1, 1:-1] - f[:-2, 1:-1, 1:-1]) / (2 * hz)

    Ax, Ay, Az = A
    out = np.zeros_like(A)
    out[0, 1:-1, 1:-1, 1:-1] = dy(Az) - dz(Ay)
    out[1, 1:-1, 1:-1, 1:-1] = dz(Ax) - dx(Az)
    out[2, 1:-1, 1:-1, 1:-1] = dx(Ay) - dy(Ax)
    return out


def curl_state(grid, A, dt):
    """Initial state (u, w) of the summed form for an initial velocity equal
    to the curl of A: u = 0 and w = u^0 - u^{-1} = dt * curl(A)."""
    v = curl(grid, A)
    return np.zeros_like(v), dt * v
