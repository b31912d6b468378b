"""ctypes binding of libkvs.so (declared in include/kvs.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Functions keep the C names; a ``kvs_status`` other than KVS_OK
raises :class:`KvsError` carrying the status and the context's last error.
There is no fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libkvs.so")

KVS_OK, KVS_EINVAL, KVS_ENOMEM, KVS_EDEVICE, KVS_ENOTCONV, KVS_EBREAKDOWN, KVS_EUNSTABLE, KVS_ESTATE = range(8)
KVS_FP64, KVS_FP32 = 0, 1
KVS_PC_NONE, KVS_PC_JACOBI, KVS_PC_UNET = 0, 1, 2
KVS_ARF_PLANE, KVS_ARF_POYNTING = 1, 2
STATUS_NAMES = {0: "KVS_OK", 1: "KVS_EINVAL", 2: "KVS_ENOMEM", 3: "KVS_EDEVICE", 4: "KVS_ENOTCONV",
                5: "KVS_EBREAKDOWN", 6: "KVS_EUNSTABLE", 7: "KVS_ESTATE"}


class KvsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class kvs_grid(C.Structure):
    _fields_ = [("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64),
                ("hx", C.c_double), ("hy", C.c_double), ("hz", C.c_double)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class kvs_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("sponge_cells", C.c_int32), ("sponge_sigma_max", C.c_double),
                ("device", C.c_int32), ("stream", C.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN),
                ("alloc_user", C.c_void_p)]


class TorchAllocator:
    """kvs_opts allocator callbacks backed by torch's caching allocator on
    one device and stream (the stream the context runs on, so that the
    allocator's stream ordering matches the library's).  Counts the calls
    and the bytes in use."""

    def __init__(self, device, stream):
        import torch
        self._torch = torch
        self.device, self.stream = int(device), int(stream or 0)
        self.allocs = self.frees = self.live_bytes = 0
        self._sizes = {}
        self.alloc_fn = ALLOC_FN(self._alloc)
        self.free_fn = FREE_FN(self._free)

    def _alloc(self, nbytes, _user):
        ptr = self._torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
        self.allocs += 1
        self.live_bytes += int(nbytes)
        self._sizes[ptr] = int(nbytes)
        return ptr

    def _free(self, ptr, _user):
        self._torch.cuda.caching_allocator_delete(ptr)
        self.frees += 1
        self.live_bytes -= self._sizes.pop(ptr, 0)


# allocators in use, kept alive while their context or batch lives
_ALLOCATORS = {}


def _opts(precision, sponge_cells, sponge_sigma_max, device, stream, allocator):
    o = kvs_opts(int(precision), int(sponge_cells), float(sponge_sigma_max), int(device), stream or None)
    if allocator is not None:
        o.alloc, o.free = allocator.alloc_fn, allocator.free_fn
    return o


KVS_MAX_FORCE_MODES = 16


class kvs_force_pattern(C.Structure):
    _fields_ = [("axis", C.c_int32), ("F0", C.c_double), ("centre", C.c_double * 3),
                ("sigma_lateral", C.c_double), ("sigma_axial", C.c_double), ("box_lateral", C.c_double),
                ("box_axial", C.c_double), ("n_modes", C.c_int32), ("mod_amp", C.c_double),
                ("k", (C.c_double * 3) * KVS_MAX_FORCE_MODES), ("phase", C.c_double * KVS_MAX_FORCE_MODES)]


class kvs_solve_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int64), ("precond", C.c_int32),
                ("fixed_iters", C.c_int64), ("warm_start", C.c_int32), ("confirm_true", C.c_int32)]


class kvs_solve_report(C.Structure):
    _fields_ = [("iters", C.c_int64), ("relres_recursive", C.c_double), ("relres_true", C.c_double),
                ("ms", C.c_double), ("status", C.c_int32)]


_lib = None

_P = C.c_void_p
_D = C.POINTER(C.c_double)
_I64 = C.POINTER(C.c_int64)

# name -> (argtypes, restype)
SIGNATURES = {
    "kvs_create": ([C.POINTER(kvs_grid), C.POINTER(kvs_opts), C.POINTER(C.c_void_p)], C.c_int),
    "kvs_destroy": ([_P], None),
    "kvs_status_string": ([C.c_int], C.c_char_p),
    "kvs_last_error": ([_P], C.c_char_p),
    "kvs_synchronize": ([_P], C.c_int),
    "kvs_get_grid": ([_P, C.POINTER(kvs_grid)], C.c_int),
    "kvs_stream": ([_P], C.c_void_p),
    "kvs_set_material": ([_P, _D, _D, _D], C.c_int),
    "kvs_set_material_uniform": ([_P, C.c_double, C.c_double, C.c_double], C.c_int),
    "kvs_stable_dt": ([_P, _D], C.c_int),
    "kvs_sponge_sigma_max": ([_P, _D], C.c_int),
    "kvs_set_dt": ([_P, C.c_double], C.c_int),
    "kvs_set_force": ([_P, _D], C.c_int),
    "kvs_set_force_device": ([_P, C.c_void_p, C.c_int32], C.c_int),
    "kvs_set_force_pattern": ([_P, C.POINTER(kvs_force_pattern)], C.c_int),
    "kvs_get_force": ([_P, _D], C.c_int),
    "kvs_set_envelope": ([_P, _D, C.c_int64], C.c_int),
    "kvs_project": ([_P, C.POINTER(kvs_solve_opts), C.POINTER(kvs_solve_report)], C.c_int),
    "kvs_project_noalloc": ([C.POINTER(kvs_grid), C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(kvs_solve_opts),
                             C.c_int32, C.c_void_p, C.POINTER(kvs_solve_report)], C.c_int),
    "kvs_noalloc_last_error": ([], C.c_char_p),
    "kvs_set_projected_force": ([_P, _D], C.c_int),
    "kvs_set_preconditioner": ([_P, _P], C.c_int),
    "kvs_last_fallbacks": ([_P, _I64], C.c_int),
    "kvs_get_projected_force": ([_P, _D], C.c_int),
    "kvs_get_phi": ([_P, _D], C.c_int),
    "kvs_set_probes": ([_P, _I64, C.c_int64, C.c_int32], C.c_int),
    "kvs_step": ([_P, C.c_int64], C.c_int),
    "kvs_trace_count": ([_P, _I64], C.c_int),
    "kvs_read_traces": ([_P, _D, C.c_int64, _I64], C.c_int),
    "kvs_clear_traces": ([_P], C.c_int),
    "kvs_get_state": ([_P, _D, _D, _I64], C.c_int),
    "kvs_set_state": ([_P, _D, _D, C.c_int64], C.c_int),
    "kvs_reset_state": ([_P], C.c_int),
    "kvs_set_state_curl": ([_P, _D, C.c_int64], C.c_int),
    "kvs_set_pml": ([_P, C.c_int32, C.c_double, C.c_double], C.c_int),
    "kvs_set_peak_planes": ([_P, C.POINTER(C.c_int32), _I64, C.c_int32], C.c_int),
    "kvs_peak_map": ([_P, C.c_int32, C.c_int64, _D], C.c_int),
    "kvs_enable_kernel_timing": ([_P, C.c_int32], C.c_int),
    "kvs_num_step_variants": ([], C.c_int32),
    "kvs_batch_create": ([C.POINTER(kvs_grid), C.c_int32, C.POINTER(kvs_opts), C.POINTER(C.c_void_p)], C.c_int),
    "kvs_batch_destroy": ([_P], None),
    "kvs_batch_last_error": ([_P], C.c_char_p),
    "kvs_batch_instance": ([_P, C.c_int32], C.c_void_p),
    "kvs_batch_share_projection": ([_P, C.c_int32, C.c_int32], C.c_int),
    "kvs_batch_set_probes": ([_P, C.c_int32, _I64, C.c_int64], C.c_int),
    "kvs_batch_set_component": ([_P, C.c_int32], C.c_int),
    "kvs_batch_step": ([_P, C.c_int64], C.c_int),
    "kvs_batch_reset": ([_P], C.c_int),
    "kvs_batch_trace_count": ([_P, _I64], C.c_int),
    "kvs_batch_read_traces": ([_P, C.c_int32, _D, C.c_int64, _I64], C.c_int),
    "kvs_batch_set_tuning": ([_P, C.c_int32, C.c_int32], C.c_int),
    "kvs_batch_set_persistent": ([_P, C.c_int32], C.c_int),
    "kvs_batch_uses_persistent": ([_P, C.POINTER(C.c_int32)], C.c_int),
    "kvs_unet_create": ([C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_void_p)], C.c_int),
    "kvs_unet_destroy": ([_P], None),
    "kvs_unet_last_error": ([_P], C.c_char_p),
    "kvs_unet_num_weights": ([_P], C.c_int64),
    "kvs_unet_set_weights": ([_P, C.POINTER(C.c_float), C.c_int64], C.c_int),
    "kvs_unet_get_weights": ([_P, C.POINTER(C.c_float), C.c_int64], C.c_int),
    "kvs_unet_forward": ([_P, C.c_void_p, C.c_double, C.c_double, C.c_void_p, C.c_int64, C.c_int64, C.c_int64,
                          C.c_void_p], C.c_int),
    "kvs_unet_conv_kpad": ([C.c_int32], C.c_int64),
    "kvs_unet_backward": ([_P, C.c_void_p, C.c_double, C.c_void_p, C.c_double, C.c_int64, C.c_int64, C.c_int64,
                           C.c_int32, C.c_void_p], C.c_int),
    "kvs_unet_get_grad": ([_P, C.POINTER(C.c_float), C.c_int64], C.c_int),
    "kvs_unet_train_sample": ([_P, C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.c_int32,
                               C.POINTER(C.c_double), C.c_void_p], C.c_int),
    "kvs_unet_adam_step": ([_P, C.c_double, C.c_int32, C.c_void_p], C.c_int),
    "kvs_unet_num_layers": ([_P], C.c_int32),
    "kvs_unet_layer": ([_P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                        C.POINTER(C.c_int32)], C.c_int),
    "kvs_unet_sample_from_x": ([C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.POINTER(C.c_double),
                                C.c_void_p], C.c_int),
    "kvs_unet_make_sample": ([_P, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)], C.c_int),
    "kvs_unet_conv_check": ([C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_uint16), C.POINTER(C.c_uint16), C.c_int64,
                             C.c_int64, C.c_int64, C.POINTER(C.c_uint16), C.POINTER(C.c_uint16)], C.c_int),
    "kvs_batch_autotune": ([_P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32), _D, C.c_int32], C.c_int),
    "kvs_set_step_variant": ([_P, C.c_int32], C.c_int),
    "kvs_set_step_tuning": ([_P, C.c_int32, C.c_int32, C.c_int32], C.c_int),
    "kvs_autotune_step": ([_P, C.c_int32, C.POINTER(C.c_int32), _D, C.c_int32], C.c_int),
    "kvs_set_step_blocking": ([_P, C.c_int32], C.c_int),
    "kvs_set_direction_precision": ([_P, C.c_int32], C.c_int),
    "kvs_set_residual_precision": ([_P, C.c_int32], C.c_int),
    "kvs_kernel_time_split": ([_P, _D, C.POINTER(C.c_int64)], C.c_int),
    "kvs_batch_set_step_blocking": ([_P, C.c_int32], C.c_int),
    "kvs_batch_step_blocking_applies": ([_P], C.c_int32),
    "kvs_step_blocking_applies": ([_P], C.c_int32),
    "kvs_kernel_time": ([_P, _D, _I64], C.c_int),
    "kvs_measure_stream": ([C.c_int32, C.c_int64, C.c_int32, _D], C.c_int),
    "kvs_measure_stream_rw": ([C.c_int32, C.c_int64, C.c_int32, C.c_int32, C.c_int32, _D], C.c_int),
    "kvs_arf_begin": ([_P, C.c_int32], C.c_int),
    "kvs_strain_begin": ([_P, _D, C.c_int64], C.c_int),
    "kvs_strain_accumulate_device": ([_P, C.c_void_p, C.c_int64, C.c_int32], C.c_int),
    "kvs_strain_get": ([_P, _D, _D, _I64], C.c_int),
    "kvs_arf_accumulate_device": ([_P, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32], C.c_int),
    "kvs_arf_accumulate": ([_P, _D, _D, C.c_int64], C.c_int),
    "kvs_arf_get_sums": ([_P, _D, _I64], C.c_int),
    "kvs_arf_set_force": ([_P, _D, C.c_int64, _D, C.c_int64, _D, C.c_int64, C.POINTER(C.c_uint8), C.c_double,
                           _D], C.c_int),
}


def lib():
    """Load libkvs.so from the package directory; raise when it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(status, ctx=None):
    if status != KVS_OK:
        msg = lib().kvs_last_error(ctx)
        raise KvsError(status, msg.decode() if msg else "")
    return status


def _dptr(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---- thin wrappers with the C names ------------------------------------

def kvs_get_grid(ctx):
    g = kvs_grid()
    _check(lib().kvs_get_grid(ctx, C.byref(g)), ctx)
    return (g.nx, g.ny, g.nz, g.hx, g.hy, g.hz)


def _cells(ctx):
    nx, ny, nz = kvs_get_grid(ctx)[:3]
    return nx * ny * nz


def _host(ctx, a, ncomp, broadcast=False):
    """FP64 C-contiguous copy of a host argument of ncomp * N values; a
    number is broadcast when `broadcast`.  A wrong size raises before the
    library reads the buffer."""
    n = ncomp * _cells(ctx)
    if broadcast and np.isscalar(a):
        return np.full(n, float(a))
    a = _f64(a)
    if a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def _out_shape(ctx, shape):
    if int(np.prod(shape)) != _cells(ctx):
        raise ValueError(f"shape {tuple(shape)} does not match the grid")
    return tuple(shape)


def kvs_create(grid, precision=KVS_FP64, sponge_cells=0, sponge_sigma_max=-1.0, device=0, stream=None,
               allocator=None):
    """allocator: None (hipMalloc inside the library) or a TorchAllocator for
    this device (best built for the same `stream`: the library synchronises
    its stream before it hands a buffer back, so any stream is safe)."""
    nx, ny, nz, hx, hy, hz = grid
    g = kvs_grid(int(nx), int(ny), int(nz), float(hx), float(hy), float(hz))
    o = _opts(precision, sponge_cells, sponge_sigma_max, device, stream, allocator)
    out = C.c_void_p()
    _check(lib().kvs_create(C.byref(g), C.byref(o), C.byref(out)))
    if allocator is not None:
        _ALLOCATORS[out.value] = allocator
    return out


def kvs_destroy(ctx):
    lib().kvs_destroy(ctx)
    _ALLOCATORS.pop(ctx.value if isinstance(ctx, C.c_void_p) else ctx, None)


def kvs_synchronize(ctx):
    _check(lib().kvs_synchronize(ctx), ctx)


def kvs_stream(ctx):
    return lib().kvs_stream(ctx)


def kvs_set_material(ctx, G, rho, eta):
    """Arrays of N values each; a number stands for a uniform field."""
    G, rho, eta = (_host(ctx, v, 1, broadcast=True) for v in (G, rho, eta))
    _check(lib().kvs_set_material(ctx, _dptr(G), _dptr(rho), _dptr(eta)), ctx)


def kvs_set_material_uniform(ctx, G, rho, eta):
    _check(lib().kvs_set_material_uniform(ctx, float(G), float(rho), float(eta)), ctx)


def kvs_stable_dt(ctx):
    v = C.c_double()
    _check(lib().kvs_stable_dt(ctx, C.byref(v)), ctx)
    return v.value


def kvs_sponge_sigma_max(ctx):
    v = C.c_double()
    _check(lib().kvs_sponge_sigma_max(ctx, C.byref(v)), ctx)
    return v.value


def kvs_set_dt(ctx, dt):
    _check(lib().kvs_set_dt(ctx, float(dt)), ctx)


def kvs_set_force(ctx, F):
    F = _host(ctx, F, 3)
    _check(lib().kvs_set_force(ctx, _dptr(F)), ctx)


def kvs_measure_stream(n, reps=10, device=0, reads=9, writes=6):
    """GB/s of the streaming reference kernel over n cells: the
    heterogeneous FDTD step's 9-read / 6-write FP32 pattern, or with
    reads=6 the homogeneous batched step's 6 / 6."""
    out = C.c_double()
    if (reads, writes) == (9, 6):
        _check(lib().kvs_measure_stream(int(device), int(n), int(reps), C.byref(out)))
    else:
        _check(lib().kvs_measure_stream_rw(int(device), int(n), int(reads), int(writes), int(reps), C.byref(out)))
    return out.value


def kvs_set_force_pattern(ctx, axis, F0, centre, sigma_lateral, sigma_axial, box_lateral=-1.0, box_axial=-1.0,
                          k=(), phase=(), mod_amp=0.0):
    """Closed-form force pattern generated by the library (marshalling only):
    the parameters of workloads' pattern dicts."""
    k = np.asarray(k, dtype=np.float64).reshape(-1, 3)
    phase = np.asarray(phase, dtype=np.float64).reshape(-1)
    if len(k) != len(phase) or len(k) > KVS_MAX_FORCE_MODES:
        raise ValueError("k and phase need the same number of modes, at most KVS_MAX_FORCE_MODES")
    p = kvs_force_pattern()
    p.axis, p.F0 = int(axis), float(F0)
    for d in range(3):
        p.centre[d] = float(centre[d])
    p.sigma_lateral, p.sigma_axial = float(sigma_lateral), float(sigma_axial)
    p.box_lateral, p.box_axial = float(box_lateral), float(box_axial)
    p.n_modes, p.mod_amp = len(k), float(mod_amp)
    for m in range(len(k)):
        for d in range(3):
            p.k[m][d] = float(k[m, d])
        p.phase[m] = float(phase[m])
    _check(lib().kvs_set_force_pattern(ctx, C.byref(p)), ctx)


def kvs_set_force_device(ctx, ptr, dtype):
    _check(lib().kvs_set_force_device(ctx, C.c_void_p(ptr), int(dtype)), ctx)


def kvs_get_force(ctx, shape):
    out = np.empty((3,) + _out_shape(ctx, shape))
    _check(lib().kvs_get_force(ctx, _dptr(out)), ctx)
    return out


def kvs_set_envelope(ctx, g):
    g = _f64(g if g is not None else [])
    _check(lib().kvs_set_envelope(ctx, _dptr(g) if len(g) else None, len(g)), ctx)


def kvs_project(ctx, tol=1e-8, max_iter=10000, precond=KVS_PC_JACOBI, fixed_iters=0, warm_start=False,
                raise_on_status=True, confirm_true=False):
    o = kvs_solve_opts(float(tol), int(max_iter), int(precond), int(fixed_iters), int(bool(warm_start)),
                       int(bool(confirm_true)))
    rep = kvs_solve_report()
    st = lib().kvs_project(ctx, C.byref(o), C.byref(rep))
    if raise_on_status:
        _check(st, ctx)
    return dict(iters=rep.iters, relres_recursive=rep.relres_recursive, relres_true=rep.relres_true,
                ms=rep.ms, status=rep.status, return_status=st)


def kvs_project_noalloc(grid, F_ptr, phi_ptr, FS_ptr, tol=1e-8, max_iter=10000, precond=KVS_PC_JACOBI,
                        fixed_iters=0, warm_start=False, confirm_true=False, device=0, stream=None,
                        raise_on_status=True):
    """Projection on caller-owned device buffers with the library's fixed
    scratch array (no allocation): F (3N doubles) read, phi (N doubles) and
    FS (3N doubles) written; addresses as integers (e.g. tensor.data_ptr())."""
    nx, ny, nz, hx, hy, hz = grid
    g = kvs_grid(int(nx), int(ny), int(nz), float(hx), float(hy), float(hz))
    o = kvs_solve_opts(float(tol), int(max_iter), int(precond), int(fixed_iters), int(bool(warm_start)),
                       int(bool(confirm_true)))
    rep = kvs_solve_report()
    st = lib().kvs_project_noalloc(C.byref(g), F_ptr, phi_ptr, FS_ptr, C.byref(o), int(device), stream or None,
                                   C.byref(rep))
    if raise_on_status and st != KVS_OK:
        msg = lib().kvs_noalloc_last_error()
        raise KvsError(st, msg.decode() if msg else "")
    return dict(iters=rep.iters, relres_recursive=rep.relres_recursive, relres_true=rep.relres_true,
                ms=rep.ms, status=rep.status, return_status=st)


KVS_NOALLOC_SCRATCH_BYTES = 66 << 20


def kvs_set_projected_force(ctx, FS):
    FS = _host(ctx, FS, 3)
    _check(lib().kvs_set_projected_force(ctx, _dptr(FS)), ctx)


def kvs_get_projected_force(ctx, shape):
    out = np.empty((3,) + _out_shape(ctx, shape))
    _check(lib().kvs_get_projected_force(ctx, _dptr(out)), ctx)
    return out


def kvs_get_phi(ctx, shape):
    out = np.empty(_out_shape(ctx, shape))
    _check(lib().kvs_get_phi(ctx, _dptr(out)), ctx)
    return out


def kvs_set_probes(ctx, ijk, comp):
    a = np.ascontiguousarray(np.asarray(ijk, dtype=np.int64).reshape(-1, 3))
    _check(lib().kvs_set_probes(ctx, a.ctypes.data_as(_I64) if len(a) else None, len(a), int(comp)), ctx)


def kvs_step(ctx, nsteps):
    _check(lib().kvs_step(ctx, int(nsteps)), ctx)


def kvs_trace_count(ctx):
    v = C.c_int64()
    _check(lib().kvs_trace_count(ctx, C.byref(v)), ctx)
    return v.value


def kvs_read_traces(ctx, nprobes, ncomp):
    n = kvs_trace_count(ctx)
    out = np.empty((n, nprobes, ncomp))
    nw = C.c_int64()
    _check(lib().kvs_read_traces(ctx, _dptr(out), out.size, C.byref(nw)), ctx)
    assert nw.value == out.size
    return out


def kvs_clear_traces(ctx):
    _check(lib().kvs_clear_traces(ctx), ctx)


def kvs_get_state(ctx, shape):
    shape = _out_shape(ctx, shape)
    u = np.empty((3,) + shape)
    w = np.empty((3,) + tuple(shape))
    step = C.c_int64()
    _check(lib().kvs_get_state(ctx, _dptr(u), _dptr(w), C.byref(step)), ctx)
    return u, w, step.value


def kvs_set_state(ctx, u, w, step):
    u, w = _host(ctx, u, 3), _host(ctx, w, 3)
    _check(lib().kvs_set_state(ctx, _dptr(u), _dptr(w), int(step)), ctx)


def kvs_set_pml(ctx, cells, R=1e-5, alpha_max=-1.0):
    _check(lib().kvs_set_pml(ctx, int(cells), float(R), float(alpha_max)), ctx)


def kvs_set_state_curl(ctx, A, step=0):
    A = _host(ctx, A, 3)
    _check(lib().kvs_set_state_curl(ctx, _dptr(A), int(step)), ctx)


def kvs_reset_state(ctx):
    _check(lib().kvs_reset_state(ctx), ctx)


def kvs_set_peak_planes(ctx, planes):
    """planes: sequence of (axis, index) pairs; [] switches the maps off."""
    planes = list(planes)
    ax = np.ascontiguousarray([p[0] for p in planes], dtype=np.int32)
    ix = np.ascontiguousarray([p[1] for p in planes], dtype=np.int64)
    n = len(planes)
    _check(lib().kvs_set_peak_planes(ctx, ax.ctypes.data_as(C.POINTER(C.c_int32)) if n else None,
                                     ix.ctypes.data_as(_I64) if n else None, n), ctx)


def kvs_peak_map(ctx, axis, index, grid):
    """Running peak of |u| on a registered plane of `grid` (nx, ny, nz, ...):
    [nz][ny] for axis 0, [nz][nx] for axis 1, [ny][nx] for axis 2."""
    nx, ny, nz = (int(v) for v in grid[:3])
    shape = {0: (nz, ny), 1: (nz, nx), 2: (ny, nx)}[int(axis)]
    out = np.empty(shape)
    _check(lib().kvs_peak_map(ctx, int(axis), int(index), _dptr(out)), ctx)
    return out


def kvs_enable_kernel_timing(ctx, on):
    _check(lib().kvs_enable_kernel_timing(ctx, int(bool(on))), ctx)


def kvs_kernel_time(ctx):
    """(summed kernel ms, steps the timed launches advanced)."""
    ms = C.c_double()
    n = C.c_int64()
    _check(lib().kvs_kernel_time(ctx, C.byref(ms), C.byref(n)), ctx)
    return ms.value, n.value


def kvs_kernel_time_split(ctx):
    """((ms, launches) of one-step launches, (ms, launches) of two-step launches)."""
    ms = np.zeros(2)
    n = (C.c_int64 * 2)()
    _check(lib().kvs_kernel_time_split(ctx, _dptr(ms), n), ctx)
    return (float(ms[0]), int(n[0])), (float(ms[1]), int(n[1]))


def kvs_num_step_variants():
    return lib().kvs_num_step_variants()


def kvs_set_step_variant(ctx, v):
    _check(lib().kvs_set_step_variant(ctx, int(v)), ctx)


def kvs_autotune_step(ctx, trial_steps=20):
    n = kvs_num_step_variants()
    ms = np.zeros(n)
    chosen = C.c_int32()
    _check(lib().kvs_autotune_step(ctx, int(trial_steps), C.byref(chosen), _dptr(ms), n), ctx)
    return chosen.value, ms


def kvs_set_step_tuning(ctx, v, zchunk=0, remap=True):
    _check(lib().kvs_set_step_tuning(ctx, int(v), int(zchunk), int(bool(remap))), ctx)


def kvs_set_step_blocking(ctx, steps):
    _check(lib().kvs_set_step_blocking(ctx, int(steps)), ctx)


def kvs_set_direction_precision(ctx, precision):
    """Storage of the projection's CG search direction (KVS_FP64 or KVS_FP32)."""
    _check(lib().kvs_set_direction_precision(ctx, int(precision)), ctx)


def kvs_set_residual_precision(ctx, precision):
    """Storage of the projection CG's residual (KVS_FP64 or KVS_FP32, reliable updates)."""
    _check(lib().kvs_set_residual_precision(ctx, int(precision)), ctx)


def kvs_step_blocking_applies(ctx):
    return bool(lib().kvs_step_blocking_applies(ctx))


# ---- batches ----------------------------------------------------------------

def _bcheck(status, b):
    if status != KVS_OK:
        msg = lib().kvs_batch_last_error(b)
        raise KvsError(status, msg.decode() if msg else "")


def kvs_batch_create(grids, precision=KVS_FP32, sponge_cells=0, sponge_sigma_max=-1.0, device=0, stream=None,
                     allocator=None):
    arr = (kvs_grid * len(grids))(*[kvs_grid(int(g[0]), int(g[1]), int(g[2]), float(g[3]), float(g[4]), float(g[5]))
                                    for g in grids])
    o = _opts(precision, sponge_cells, sponge_sigma_max, device, stream, allocator)
    out = C.c_void_p()
    _bcheck(lib().kvs_batch_create(arr, len(grids), C.byref(o), C.byref(out)), None)
    if allocator is not None:
        _ALLOCATORS[out.value] = allocator
    return out


def kvs_batch_set_persistent(b, on):
    _bcheck(lib().kvs_batch_set_persistent(b, int(bool(on))), b)


def kvs_batch_set_step_blocking(b, steps):
    _bcheck(lib().kvs_batch_set_step_blocking(b, int(steps)), b)


def kvs_batch_step_blocking_applies(b):
    return bool(lib().kvs_batch_step_blocking_applies(b))


def kvs_batch_uses_persistent(b):
    out = C.c_int32()
    _bcheck(lib().kvs_batch_uses_persistent(b, C.byref(out)), b)
    return bool(out.value)


def kvs_batch_destroy(b):
    lib().kvs_batch_destroy(b)
    _ALLOCATORS.pop(b.value if isinstance(b, C.c_void_p) else b, None)


def kvs_batch_instance(b, i):
    p = lib().kvs_batch_instance(b, int(i))
    if not p:
        raise KvsError(KVS_EINVAL, f"no instance {i}")
    return C.c_void_p(p)


def kvs_batch_share_projection(b, src, dst):
    _bcheck(lib().kvs_batch_share_projection(b, int(src), int(dst)), b)


def kvs_batch_set_probes(b, i, ijk):
    a = np.ascontiguousarray(np.asarray(ijk, dtype=np.int64).reshape(-1, 3))
    _bcheck(lib().kvs_batch_set_probes(b, int(i), a.ctypes.data_as(_I64) if len(a) else None, len(a)), b)


def kvs_batch_set_component(b, comp):
    _bcheck(lib().kvs_batch_set_component(b, int(comp)), b)


def kvs_batch_step(b, nsteps):
    _bcheck(lib().kvs_batch_step(b, int(nsteps)), b)


def kvs_batch_reset(b):
    _bcheck(lib().kvs_batch_reset(b), b)


def kvs_batch_trace_count(b):
    v = C.c_int64()
    _bcheck(lib().kvs_batch_trace_count(b, C.byref(v)), b)
    return v.value


def kvs_batch_read_traces(b, i, nprobes):
    n = kvs_batch_trace_count(b)
    out = np.empty((n, nprobes))
    nw = C.c_int64()
    _bcheck(lib().kvs_batch_read_traces(b, int(i), _dptr(out), out.size, C.byref(nw)), b)
    assert nw.value == out.size
    return out


def kvs_batch_set_tuning(b, variant, zchunk):
    _bcheck(lib().kvs_batch_set_tuning(b, int(variant), int(zchunk)), b)


KVS_BATCH_FIT_ROWS = -1


def kvs_batch_autotune(b, trial_steps=5):
    """Returns (variant, z planes, ms per launch of each candidate: the
    variants, then the row-fitted tiling); variant may be KVS_BATCH_FIT_ROWS."""
    n = kvs_num_step_variants() + 1
    ms = np.zeros(n)
    v, z = C.c_int32(), C.c_int32()
    _bcheck(lib().kvs_batch_autotune(b, int(trial_steps), C.byref(v), C.byref(z), _dptr(ms), n), b)
    return v.value, z.value, ms


# ---- learned preconditioner -------------------------------------------------

def _ucheck(status, net):
    if status != KVS_OK:
        msg = lib().kvs_unet_last_error(net)
        raise KvsError(status, msg.decode() if msg else "")


def kvs_unet_create(channels=(16, 32, 64), n_bottleneck=4):
    ch = (C.c_int32 * 3)(*channels)
    out = C.c_void_p()
    _ucheck(lib().kvs_unet_create(ch, int(n_bottleneck), C.byref(out)), None)
    return out


def kvs_unet_destroy(net):
    lib().kvs_unet_destroy(net)


def kvs_unet_num_weights(net):
    return lib().kvs_unet_num_weights(net)


def kvs_unet_set_weights(net, w):
    w = np.ascontiguousarray(w, dtype=np.float32)
    _ucheck(lib().kvs_unet_set_weights(net, w.ctypes.data_as(C.POINTER(C.c_float)), w.size), net)


def kvs_unet_get_weights(net):
    w = np.empty(kvs_unet_num_weights(net), dtype=np.float32)
    _ucheck(lib().kvs_unet_get_weights(net, w.ctypes.data_as(C.POINTER(C.c_float)), w.size), net)
    return w


def kvs_unet_forward(net, r_ptr, in_scale, out_scale, z_ptr, dims, stream=None):
    nx, ny, nz = dims
    _ucheck(lib().kvs_unet_forward(net, C.c_void_p(r_ptr), float(in_scale), float(out_scale), C.c_void_p(z_ptr),
                                   int(nx), int(ny), int(nz), stream or None), net)


def kvs_unet_conv_kpad(ci):
    return lib().kvs_unet_conv_kpad(int(ci))


def kvs_unet_conv_check(ci, co, dil, A_bits, B_bits, dims, W_bits):
    nx, ny, nz = dims
    A = np.ascontiguousarray(A_bits, dtype=np.uint16)
    W = np.ascontiguousarray(W_bits, dtype=np.uint16)
    B = None if B_bits is None else np.ascontiguousarray(B_bits, dtype=np.uint16)
    out = np.empty(nx * ny * nz * co, dtype=np.uint16)
    u16 = C.POINTER(C.c_uint16)
    _ucheck(lib().kvs_unet_conv_check(int(ci), int(co), int(dil), A.ctypes.data_as(u16),
                                      B.ctypes.data_as(u16) if B is not None else None, int(nx), int(ny), int(nz),
                                      W.ctypes.data_as(u16), out.ctypes.data_as(u16)), None)
    return out


def kvs_unet_backward(net, r_ptr, in_scale, dz_ptr, dz_scale, dims, accumulate=False, stream=None):
    nx, ny, nz = dims
    _ucheck(lib().kvs_unet_backward(net, C.c_void_p(r_ptr), float(in_scale), C.c_void_p(dz_ptr), float(dz_scale),
                                    int(nx), int(ny), int(nz), int(bool(accumulate)), stream or None), net)


def kvs_unet_get_grad(net):
    g = np.empty(kvs_unet_num_weights(net), dtype=np.float32)
    _ucheck(lib().kvs_unet_get_grad(net, g.ctypes.data_as(C.POINTER(C.c_float)), g.size), net)
    return g


def kvs_unet_train_sample(net, b_ptr, x_ptr, dims, accumulate=False, stream=None):
    nx, ny, nz = dims
    loss = C.c_double()
    _ucheck(lib().kvs_unet_train_sample(net, C.c_void_p(b_ptr), C.c_void_p(x_ptr), int(nx), int(ny), int(nz),
                                        int(bool(accumulate)), C.byref(loss), stream or None), net)
    return loss.value


def kvs_unet_adam_step(net, lr, n_samples=1, stream=None):
    _ucheck(lib().kvs_unet_adam_step(net, float(lr), int(n_samples), stream or None), net)


def kvs_unet_layers(net):
    """[(ci, co, dil, taps)] of every layer in network order."""
    out = []
    for l in range(lib().kvs_unet_num_layers(net)):
        v = [C.c_int32() for _ in range(4)]
        _ucheck(lib().kvs_unet_layer(net, l, *[C.byref(a) for a in v]), net)
        out.append(tuple(a.value for a in v))
    return out


def kvs_unet_sample_from_x(x_ptr, b_ptr, dims, stream=None):
    rms = C.c_double()
    nx, ny, nz = dims
    _ucheck(lib().kvs_unet_sample_from_x(C.c_void_p(x_ptr), C.c_void_p(b_ptr), int(nx), int(ny), int(nz),
                                         C.byref(rms), stream or None), None)
    return rms.value


def kvs_unet_make_sample(ctx, k_snapshot, b_ptr, x_ptr, precond=KVS_PC_JACOBI):
    rms = C.c_double()
    _check(lib().kvs_unet_make_sample(ctx, int(k_snapshot), int(precond), C.c_void_p(b_ptr), C.c_void_p(x_ptr),
                                      C.byref(rms)), ctx)
    return rms.value


def kvs_set_preconditioner(ctx, net):
    _check(lib().kvs_set_preconditioner(ctx, net), ctx)


def kvs_last_fallbacks(ctx):
    v = C.c_int64()
    _check(lib().kvs_last_fallbacks(ctx, C.byref(v)), ctx)
    return v.value


# ---- acoustic radiation force ---------------------------------------------

def kvs_arf_begin(ctx, mode):
    _check(lib().kvs_arf_begin(ctx, int(mode)), ctx)


def kvs_arf_accumulate_device(ctx, p_ptr, v_ptr, nsamp, dtype):
    """Device pointers (ints, e.g. a tensor's data_ptr()); v_ptr None in the
    plane-wave form."""
    _check(lib().kvs_arf_accumulate_device(ctx, C.c_void_p(p_ptr), C.c_void_p(v_ptr) if v_ptr else None,
                                           int(nsamp), int(dtype)), ctx)


def kvs_arf_accumulate(ctx, p, v=None):
    """Host samples: p [nsamp][N...], v [nsamp][3][N...] or None."""
    n = _cells(ctx)
    p = _f64(p)
    if p.size % n:
        raise ValueError(f"p holds {p.size} values, not a whole number of samples of {n}")
    nsamp = p.size // n
    if v is not None:
        v = _f64(v)
        if v.size != 3 * n * nsamp:
            raise ValueError(f"v holds {v.size} values, expected {3 * n * nsamp}")
    _check(lib().kvs_arf_accumulate(ctx, _dptr(p), _dptr(v) if v is not None else None, nsamp), ctx)


def kvs_arf_get_sums(ctx, shape, mode):
    """(sums, nsamp): sums [nz][ny][nx] (plane-wave form) or [3][nz][ny][nx]."""
    shape = _out_shape(ctx, shape)
    out = np.empty(shape if mode == KVS_ARF_PLANE else (3,) + shape)
    ns = C.c_int64()
    _check(lib().kvs_arf_get_sums(ctx, _dptr(out), C.byref(ns)), ctx)
    return out, ns.value


def _coef(ctx, a):
    """A number (uniform) or a per-cell map: (array, count)."""
    if np.isscalar(a):
        return np.array([float(a)]), 1
    a = _host(ctx, a, 1)
    return a, a.size


def kvs_arf_set_force(ctx, alpha, c, n_pulse, rho=None, mask=None, beam_dir=None):
    A, na = _coef(ctx, alpha)
    Cs, nc = _coef(ctx, c)
    R, nr = _coef(ctx, rho) if rho is not None else (None, 0)
    M = None
    if mask is not None:
        M = np.ascontiguousarray(np.asarray(mask).reshape(-1) != 0, dtype=np.uint8)
        if M.size != _cells(ctx):
            raise ValueError("mask needs N values")
    d = _f64(beam_dir) if beam_dir is not None else None
    if d is not None and d.size != 3:
        raise ValueError("beam_dir needs 3 values")
    _check(lib().kvs_arf_set_force(ctx, _dptr(A), na, _dptr(Cs), nc, _dptr(R) if R is not None else None, nr,
                                   M.ctypes.data_as(C.POINTER(C.c_uint8)) if M is not None else None,
                                   float(n_pulse), _dptr(d) if d is not None else None), ctx)


# ---- acoustic strain ----------------------------------------------------------

def kvs_strain_begin(ctx, K):
    A, n = _coef(ctx, K)
    _check(lib().kvs_strain_begin(ctx, _dptr(A), n), ctx)


def kvs_strain_accumulate_device(ctx, p_ptr, nsamp, dtype):
    _check(lib().kvs_strain_accumulate_device(ctx, C.c_void_p(p_ptr), int(nsamp), int(dtype)), ctx)


def kvs_strain_get(ctx, shape):
    """(peak |eps|, peak |grad eps|, nsamp) as [nz][ny][nx] arrays."""
    shape = _out_shape(ctx, shape)
    pe, pg = np.empty(shape), np.empty(shape)
    ns = C.c_int64()
    _check(lib().kvs_strain_get(ctx, _dptr(pe), _dptr(pg), C.byref(ns)), ctx)
    return pe, pg, ns.value
