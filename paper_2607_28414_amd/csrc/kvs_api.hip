// C ABI of the shear solver (declarations and contracts in include/kvs.h).
// Host code only: argument checking, buffer ownership, call ordering, and
// the launch sequence of the kernels in kvs_step.hip and kvs_cg.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "kvs_internal.hpp"

namespace {

thread_local std::string g_create_err;

kvs_status fail(kvs_ctx* c, kvs_status s, const std::string& msg) {
    if (c)
        c->err = msg;
    else
        g_create_err = msg;
    return s;
}

#define API_HIP(c, call)                                                                                 \
    do {                                                                                                 \
        hipError_t e_ = (call);                                                                          \
        if (e_ != hipSuccess) return fail(c, KVS_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

size_t tsize(const kvs_ctx* c) { return c->prec == KVS_FP32 ? sizeof(float) : sizeof(double); }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Closed-form stability bound of a homogeneous medium (every face modulus is G).
double uniform_dt_max(const kvs_grid& g, double G, double rho, double eta) {
    const double S = 1.0 / (g.hx * g.hx) + 1.0 / (g.hy * g.hy) + 1.0 / (g.hz * g.hz);
    const double qa = G / rho * S, qb = 2.0 * eta / rho * S;
    return (-qb + std::sqrt(qb * qb + 4.0 * qa)) / (2.0 * qa);
}

void resolve_sigma(kvs_ctx* c, double cmax) {
    c->cmax = cmax;
    c->pml_dirty = true;
    if (c->sponge_cells <= 0) {
        c->sigma_max = 0.0;
        return;
    }
    if (c->sigma_user >= 0.0) {
        c->sigma_max = c->sigma_user;
        return;
    }
    const double hmin = std::min(c->grid.hx, std::min(c->grid.hy, c->grid.hz));
    c->sigma_max = 6.0 * std::log(10.0) * cmax / ((double)c->sponge_cells * hmin);
}

template <typename P>
void dfree(const KvsMem& m, P*& p) {
    m.put((void*)p);
    p = nullptr;
}

void release(kvs_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (int b = 0; b < 2; ++b) {
        dfree(c->mem, c->u[b]);
        dfree(c->mem, c->w[b]);
        dfree(c->mem, c->p[b]);
    }
    dfree(c->mem, c->G);
    dfree(c->mem, c->eta);
    dfree(c->mem, c->rho_t);
    dfree(c->mem, c->crho);
    dfree(c->mem, c->F);
    dfree(c->mem, c->FS);
    dfree(c->mem, c->phi);
    dfree(c->mem, c->r);
    dfree(c->mem, c->r2);
    dfree(c->mem, c->Ap);
    dfree(c->mem, c->partials);
    dfree(c->mem, c->cgs);
    dfree(c->mem, c->probe_cells);
    dfree(c->mem, c->probe_rowtab);
    dfree(c->mem, c->probe_ptab);
    dfree(c->mem, c->traces);
    dfree(c->mem, c->peak);
    dfree(c->mem, c->arf_sum);
    dfree(c->mem, c->strain_K);
    dfree(c->mem, c->strain_peak);
    dfree(c->mem, c->pml_tab);
    dfree(c->mem, c->pml_mem);
    if (c->cgs_host) (void)hipHostFree(c->cgs_host);
    c->cgs_host = nullptr;
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    c->ev_pool.clear();
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    c->stream = nullptr;
}

kvs_status need_material(kvs_ctx* c) {
    if (!c) return KVS_EINVAL;
    if (!c->have_material) return fail(c, KVS_ESTATE, "no material set");
    return KVS_OK;
}

kvs_status ensure_trace_capacity(kvs_ctx* c, int64_t more) {
    if (c->nprobes == 0) return KVS_OK;
    const int64_t need = c->trace_steps + more;
    if (need <= c->trace_cap) return KVS_OK;
    int64_t cap = std::max<int64_t>(need, std::max<int64_t>(2 * c->trace_cap, 1024));
    const int64_t per = c->nprobes * ncomp_of(c->probe_comp);
    double* nb = nullptr;
    API_HIP(c, c->mem.get(&nb, sizeof(double) * per * cap));
    if (c->traces && c->trace_steps > 0)
        API_HIP(c, hipMemcpyAsync(nb, c->traces, sizeof(double) * per * c->trace_steps, hipMemcpyDeviceToDevice,
                                  c->stream));
    API_HIP(c, hipStreamSynchronize(c->stream));
    dfree(c->mem, c->traces);
    c->traces = nb;
    c->trace_cap = cap;
    return KVS_OK;
}

// Accumulate the durations of the recorded event pairs and recycle them.
kvs_status flush_timing(kvs_ctx* c) {
    if (c->ev_used == 0) return KVS_OK;
    API_HIP(c, hipEventSynchronize(c->ev_pool[2 * c->ev_used - 1]));
    for (int64_t q = 0; q < c->ev_used; ++q) {
        float ms = 0.f;
        API_HIP(c, hipEventElapsedTime(&ms, c->ev_pool[2 * q], c->ev_pool[2 * q + 1]));
        const int adv = c->ev_steps[(size_t)q];
        c->timed_ms += ms;
        c->timed_launches += adv;
        c->timed_ms_kind[adv - 1] += ms;
        c->timed_n_kind[adv - 1] += 1;
    }
    c->ev_used = 0;
    return KVS_OK;
}

kvs_status next_event_pair(kvs_ctx* c, hipEvent_t* a, hipEvent_t* b) {
    const int64_t cap_pairs = 1 << 14;
    if (c->ev_used >= cap_pairs) {
        kvs_status s = flush_timing(c);
        if (s != KVS_OK) return s;
    }
    while ((int64_t)c->ev_pool.size() < 2 * (c->ev_used + 1)) {
        hipEvent_t e;
        API_HIP(c, hipEventCreate(&e));
        c->ev_pool.push_back(e);
    }
    if ((int64_t)c->ev_steps.size() < c->ev_used + 1) c->ev_steps.resize((size_t)c->ev_used + 1);
    c->ev_steps[(size_t)c->ev_used] = 1;
    *a = c->ev_pool[2 * c->ev_used];
    *b = c->ev_pool[2 * c->ev_used + 1];
    c->ev_used += 1;
    return KVS_OK;
}

}  // namespace

extern "C" {

const char* kvs_status_string(kvs_status s) {
    switch (s) {
        case KVS_OK: return "ok";
        case KVS_EINVAL: return "invalid argument";
        case KVS_ENOMEM: return "out of memory";
        case KVS_EDEVICE: return "device error";
        case KVS_ENOTCONV: return "not converged";
        case KVS_EBREAKDOWN: return "CG breakdown";
        case KVS_EUNSTABLE: return "time step above the stability limit";
        case KVS_ESTATE: return "call order / missing state";
    }
    return "unknown status";
}

const char* kvs_last_error(const kvs_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

void* kvs_stream(const kvs_ctx* c) { return c ? (void*)c->stream : nullptr; }

kvs_status kvs_create(const kvs_grid* grid, const kvs_opts* opts, kvs_ctx** out) {
    if (!out) return fail(nullptr, KVS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!grid) return fail(nullptr, KVS_EINVAL, "grid is NULL");
    const kvs_grid g = *grid;
    if (g.nx < 3 || g.ny < 3 || g.nz < 3) return fail(nullptr, KVS_EINVAL, "every axis needs >= 3 nodes");
    if (!finite_pos(g.hx) || !finite_pos(g.hy) || !finite_pos(g.hz))
        return fail(nullptr, KVS_EINVAL, "spacings must be finite and > 0");
    const double Nd = (double)g.nx * (double)g.ny * (double)g.nz;
    if (Nd > 2.0e9) return fail(nullptr, KVS_EINVAL, "grid above 2e9 nodes (32-bit in-plane indexing)");
    kvs_opts o{};
    o.precision = KVS_FP64;
    o.sponge_cells = 0;
    o.sponge_sigma_max = -1.0;
    if (opts) o = *opts;
    if (o.precision != KVS_FP64 && o.precision != KVS_FP32) return fail(nullptr, KVS_EINVAL, "unknown precision");
    if (o.sponge_cells < 0) return fail(nullptr, KVS_EINVAL, "sponge_cells < 0");
    if (std::isnan(o.sponge_sigma_max)) return fail(nullptr, KVS_EINVAL, "sponge_sigma_max is NaN");
    if ((o.alloc == nullptr) != (o.free == nullptr))
        return fail(nullptr, KVS_EINVAL, "alloc and free must be given together");

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(nullptr, KVS_EDEVICE, "no HIP device");
    if (o.device < 0 || o.device >= ndev) return fail(nullptr, KVS_EINVAL, "device ordinal out of range");
    if (hipSetDevice(o.device) != hipSuccess) return fail(nullptr, KVS_EDEVICE, "hipSetDevice failed");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, o.device) != hipSuccess)
        return fail(nullptr, KVS_EDEVICE, "hipGetDeviceProperties failed");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(nullptr, KVS_EDEVICE, std::string("library built for gfx950, device is ") + prop.gcnArchName);

    kvs_ctx* c = new (std::nothrow) kvs_ctx();
    if (!c) return fail(nullptr, KVS_ENOMEM, "host allocation failed");
    c->grid = g;
    c->N = g.nx * g.ny * g.nz;
    c->prec = o.precision;
    c->dir_prec = o.precision;
    c->res_prec = o.precision;
    c->device = o.device;
    c->sponge_cells = o.sponge_cells;
    c->sigma_user = o.sponge_sigma_max;
    if (o.stream) {
        c->stream = (hipStream_t)o.stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return fail(nullptr, KVS_EDEVICE, "hipStreamCreate failed");
        }
        c->own_stream = true;
    }
    c->mem.alloc = o.alloc;
    c->mem.release = o.free;
    c->mem.user = o.alloc_user;
    c->mem.stream = c->stream;
    const size_t ts = tsize(c);
    const size_t N = (size_t)c->N;
    c->npart = kvs_cg_partials_needed(g);
    bool ok = true;
    for (int b = 0; b < 2 && ok; ++b) {
        ok = ok && c->mem.get(&c->u[b], 3 * N * ts) == hipSuccess;
        ok = ok && c->mem.get(&c->w[b], 3 * N * ts) == hipSuccess;
        ok = ok && c->mem.get(&c->p[b], N * sizeof(double)) == hipSuccess;
    }
    ok = ok && c->mem.get(&c->F, 3 * N * sizeof(double)) == hipSuccess;
    ok = ok && c->mem.get(&c->FS, 3 * N * ts) == hipSuccess;
    ok = ok && c->mem.get(&c->phi, N * sizeof(double)) == hipSuccess;
    ok = ok && c->mem.get(&c->r, N * sizeof(double)) == hipSuccess;
    ok = ok && c->mem.get(&c->Ap, N * sizeof(double)) == hipSuccess;
    ok = ok && c->mem.get(&c->partials, 3 * (size_t)std::max<int64_t>(c->npart, 2048) * sizeof(double)) == hipSuccess;
    ok = ok && c->mem.get(&c->cgs, sizeof(CgState)) == hipSuccess;
    ok = ok && hipHostMalloc(&c->cgs_host, sizeof(CgState), hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        release(c);
        delete c;
        return fail(nullptr, KVS_ENOMEM, "device allocation failed");
    }
    bool z = true;
    for (int b = 0; b < 2; ++b) {
        z = z && hipMemsetAsync(c->u[b], 0, 3 * N * ts, c->stream) == hipSuccess;
        z = z && hipMemsetAsync(c->w[b], 0, 3 * N * ts, c->stream) == hipSuccess;
        z = z && hipMemsetAsync(c->p[b], 0, N * sizeof(double), c->stream) == hipSuccess;
    }
    z = z && hipMemsetAsync(c->F, 0, 3 * N * sizeof(double), c->stream) == hipSuccess;
    z = z && hipMemsetAsync(c->FS, 0, 3 * N * ts, c->stream) == hipSuccess;
    z = z && hipMemsetAsync(c->phi, 0, N * sizeof(double), c->stream) == hipSuccess;
    z = z && hipMemsetAsync(c->r, 0, N * sizeof(double), c->stream) == hipSuccess;
    z = z && hipMemsetAsync(c->Ap, 0, N * sizeof(double), c->stream) == hipSuccess;
    z = z && hipStreamSynchronize(c->stream) == hipSuccess;
    if (!z) {
        release(c);
        delete c;
        return fail(nullptr, KVS_EDEVICE, "initial zero fill failed");
    }
    *out = c;
    return KVS_OK;
}

void kvs_destroy(kvs_ctx* c) {
    if (!c) return;
    release(c);
    delete c;
}

kvs_status kvs_synchronize(kvs_ctx* c) {
    if (!c) return KVS_EINVAL;
    API_HIP(c, hipStreamSynchronize(c->stream));
    return KVS_OK;
}

kvs_status kvs_set_material(kvs_ctx* c, const double* G, const double* rho, const double* eta) {
    if (!c) return KVS_EINVAL;
    if (!G || !rho || !eta) return fail(c, KVS_EINVAL, "material pointer is NULL");
    const int64_t N = c->N;
    bool visc = false;
    for (int64_t q = 0; q < N; ++q) {
        if (!finite_pos(G[q]) || !finite_pos(rho[q]) || !std::isfinite(eta[q]) || eta[q] < 0.0)
            return fail(c, KVS_EINVAL, "material must have finite G > 0, rho > 0, eta >= 0 (cell " +
                                           std::to_string(q) + ")");
        visc = visc || eta[q] > 0.0;
    }
    API_HIP(c, hipSetDevice(c->device));
    const size_t ts = tsize(c);
    if (!c->G) API_HIP(c, c->mem.get(&c->G, N * ts));
    if (!c->eta) API_HIP(c, c->mem.get(&c->eta, N * ts));
    if (!c->rho_t) API_HIP(c, c->mem.get(&c->rho_t, N * ts));
    if (!c->crho) API_HIP(c, c->mem.get(&c->crho, N * ts));
    double* tmp = nullptr;
    const int64_t npart = 2 * 1024;
    API_HIP(c, c->mem.get(&tmp, sizeof(double) * (3 * N + npart + 2)));
    double* dG = tmp;
    double* drho = tmp + N;
    double* deta = tmp + 2 * N;
    double* part = tmp + 3 * N;
    double* res = part + npart;
    kvs_status st = KVS_OK;
    double host_res[2] = {0, 0};
    do {
        hipError_t e = hipMemcpyAsync(dG, G, sizeof(double) * N, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(drho, rho, sizeof(double) * N, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(deta, eta, sizeof(double) * N, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = kvs_launch_stable_dt(c, dG, drho, deta, part, npart, res);
        if (e == hipSuccess) e = kvs_launch_cast_material(c, dG, drho, deta);
        if (e == hipSuccess) e = hipMemcpyAsync(host_res, res, sizeof(host_res), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) st = fail(c, KVS_EDEVICE, std::string("set_material: ") + hipGetErrorString(e));
    } while (false);
    c->mem.put(tmp);
    if (st != KVS_OK) return st;
    c->hetero = true;
    c->viscous = visc;
    c->have_material = true;
    c->dt_max = host_res[0];
    resolve_sigma(c, host_res[1]);
    if (c->have_dt) {
        if (c->dt > c->dt_max * (1.0 + 1e-12)) {
            c->have_dt = false;
        } else {
            API_HIP(c, kvs_launch_crho(c));
        }
    }
    return KVS_OK;
}

kvs_status kvs_set_material_uniform(kvs_ctx* c, double G, double rho, double eta) {
    if (!c) return KVS_EINVAL;
    if (!finite_pos(G) || !finite_pos(rho) || !std::isfinite(eta) || eta < 0.0)
        return fail(c, KVS_EINVAL, "material must have finite G > 0, rho > 0, eta >= 0");
    c->hetero = false;
    c->viscous = eta > 0.0;
    c->G0 = G;
    c->rho0 = rho;
    c->eta0 = eta;
    c->have_material = true;
    c->dt_max = uniform_dt_max(c->grid, G, rho, eta);
    resolve_sigma(c, std::sqrt(G / rho));
    if (c->have_dt && c->dt > c->dt_max * (1.0 + 1e-12)) c->have_dt = false;
    return KVS_OK;
}

kvs_status kvs_get_grid(const kvs_ctx* c, kvs_grid* out) {
    if (!c || !out) return KVS_EINVAL;
    *out = c->grid;
    return KVS_OK;
}

kvs_status kvs_stable_dt(const kvs_ctx* cc, double* dt_max) {
    kvs_ctx* c = const_cast<kvs_ctx*>(cc);
    kvs_status s = need_material(c);
    if (s != KVS_OK) return s;
    if (!dt_max) return fail(c, KVS_EINVAL, "dt_max is NULL");
    *dt_max = c->dt_max;
    return KVS_OK;
}

kvs_status kvs_sponge_sigma_max(const kvs_ctx* cc, double* sigma_max) {
    kvs_ctx* c = const_cast<kvs_ctx*>(cc);
    kvs_status s = need_material(c);
    if (s != KVS_OK) return s;
    if (!sigma_max) return fail(c, KVS_EINVAL, "sigma_max is NULL");
    *sigma_max = c->sigma_max;
    return KVS_OK;
}

kvs_status kvs_set_dt(kvs_ctx* c, double dt) {
    kvs_status s = need_material(c);
    if (s != KVS_OK) return s;
    if (!finite_pos(dt)) return fail(c, KVS_EINVAL, "dt must be finite and > 0");
    if (dt > c->dt_max * (1.0 + 1e-12))
        return fail(c, KVS_EUNSTABLE, "dt " + std::to_string(dt) + " above the stability limit " +
                                          std::to_string(c->dt_max));
    c->dt = dt;
    c->have_dt = true;
    c->pml_dirty = true;
    API_HIP(c, kvs_launch_crho(c));
    return KVS_OK;
}

kvs_status kvs_set_force(kvs_ctx* c, const double* F) {
    if (!c) return KVS_EINVAL;
    if (!F) return fail(c, KVS_EINVAL, "F is NULL");
    API_HIP(c, hipMemcpyAsync(c->F, F, sizeof(double) * 3 * c->N, hipMemcpyHostToDevice, c->stream));
    API_HIP(c, hipStreamSynchronize(c->stream));
    c->have_force = true;
    c->fs_current = false;
    return KVS_OK;
}

kvs_status kvs_set_force_pattern(kvs_ctx* c, const kvs_force_pattern* p) {
    if (!c) return KVS_EINVAL;
    if (!p) return fail(c, KVS_EINVAL, "pattern is NULL");
    if (p->axis < 0 || p->axis > 2) return fail(c, KVS_EINVAL, "axis must be 0..2");
    if (!finite_pos(p->sigma_lateral) || !finite_pos(p->sigma_axial))
        return fail(c, KVS_EINVAL, "sigmas must be finite and > 0");
    if (p->n_modes < 0 || p->n_modes > KVS_MAX_FORCE_MODES) return fail(c, KVS_EINVAL, "n_modes out of range");
    bool ok = std::isfinite(p->F0) && std::isfinite(p->box_lateral) && std::isfinite(p->box_axial) &&
              std::isfinite(p->mod_amp);
    for (int d = 0; d < 3; ++d) ok = ok && std::isfinite(p->centre[d]);
    for (int m = 0; m < p->n_modes; ++m)
        ok = ok && std::isfinite(p->k[m][0]) && std::isfinite(p->k[m][1]) && std::isfinite(p->k[m][2]) &&
             std::isfinite(p->phase[m]);
    if (!ok) return fail(c, KVS_EINVAL, "pattern value not finite");
    API_HIP(c, hipSetDevice(c->device));
    API_HIP(c, kvs_launch_force_pattern(c, p));
    c->have_force = true;
    c->fs_current = false;
    return KVS_OK;
}

kvs_status kvs_set_force_device(kvs_ctx* c, const void* F, int32_t dtype) {
    if (!c) return KVS_EINVAL;
    if (!F) return fail(c, KVS_EINVAL, "F is NULL");
    if (dtype == 0) {
        API_HIP(c, hipMemcpyAsync(c->F, F, sizeof(double) * 3 * c->N, hipMemcpyDeviceToDevice, c->stream));
    } else if (dtype == 1) {
        API_HIP(c, kvs_launch_f32_to_f64(c, static_cast<const float*>(F), c->F, 3 * c->N));
    } else {
        return fail(c, KVS_EINVAL, "dtype must be 0 (double) or 1 (float)");
    }
    c->have_force = true;
    c->fs_current = false;
    return KVS_OK;
}

kvs_status kvs_get_force(const kvs_ctx* cc, double* F) {
    kvs_ctx* c = const_cast<kvs_ctx*>(cc);
    if (!c) return KVS_EINVAL;
    if (!F) return fail(c, KVS_EINVAL, "F is NULL");
    if (!c->have_force) return fail(c, KVS_ESTATE, "no force set");
    API_HIP(c, hipSetDevice(c->device));
    API_HIP(c, hipMemcpyAsync(F, c->F, sizeof(double) * 3 * c->N, hipMemcpyDeviceToHost, c->stream));
    API_HIP(c, hipStreamSynchronize(c->stream));
    return KVS_OK;
}

kvs_status kvs_set_envelope(kvs_ctx* c, const double* g, int64_t n) {
    if (!c) return KVS_EINVAL;
    if (n < 0 || (n > 0 && !g)) return fail(c, KVS_EINVAL, "bad envelope");
    for (int64_t q = 0; q < n; ++q)
        if (!std::isfinite(g[q])) return fail(c, KVS_EINVAL, "envelope value not finite");
    c->env.assign(g, g + n);
    return KVS_OK;
}

kvs_status kvs_project(kvs_ctx* c, const kvs_solve_opts* opts, kvs_solve_report* rep) {
    if (!c) return KVS_EINVAL;
    if (!c->have_force) return fail(c, KVS_ESTATE, "no force set");
    kvs_solve_opts o{};
    o.tol = 1e-8;
    o.max_iter = 10000;
    o.precond = KVS_PC_JACOBI;
    if (opts) o = *opts;
    if (o.fixed_iters < 0) return fail(c, KVS_EINVAL, "fixed_iters < 0");
    if (o.fixed_iters == 0 && !(o.tol > 0.0 && std::isfinite(o.tol))) return fail(c, KVS_EINVAL, "tol must be > 0");
    if (o.max_iter <= 0) return fail(c, KVS_EINVAL, "max_iter must be > 0");
    if (o.precond != KVS_PC_NONE && o.precond != KVS_PC_JACOBI && o.precond != KVS_PC_UNET)
        return fail(c, KVS_EINVAL, "unknown preconditioner");
    if (o.precond == KVS_PC_UNET) {
        if (!c->net) return fail(c, KVS_ESTATE, "no network set (kvs_set_preconditioner)");
        const kvs_grid& g = c->grid;
        if (std::fabs(g.hx - g.hy) > 1e-12 * g.hx || std::fabs(g.hx - g.hz) > 1e-12 * g.hx)
            return fail(c, KVS_EINVAL, "the network preconditioner needs equal spacings");
    }
    API_HIP(c, hipSetDevice(c->device));
    return kvs_run_projection(c, &o, rep);
}

kvs_status kvs_set_preconditioner(kvs_ctx* c, kvs_unet* net) {
    if (!c) return KVS_EINVAL;
    c->net = net;
    return KVS_OK;
}

kvs_status kvs_last_fallbacks(const kvs_ctx* c, int64_t* n) {
    if (!c || !n) return KVS_EINVAL;
    *n = c->last_fallbacks;
    return KVS_OK;
}

kvs_status kvs_set_projected_force(kvs_ctx* c, const double* FS) {
    if (!c) return KVS_EINVAL;
    if (!FS) return fail(c, KVS_EINVAL, "FS is NULL");
    const size_t bytes = sizeof(double) * 3 * c->N;
    if (c->prec == KVS_FP64) {
        API_HIP(c, hipMemcpyAsync(c->FS, FS, bytes, hipMemcpyHostToDevice, c->stream));
        API_HIP(c, hipStreamSynchronize(c->stream));
    } else {
        double* tmp = nullptr;
        API_HIP(c, c->mem.get(&tmp, bytes));
        hipError_t e = hipMemcpyAsync(tmp, FS, bytes, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = kvs_launch_cast(c, tmp, c->FS, 3 * c->N);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        c->mem.put(tmp);
        if (e != hipSuccess) return fail(c, KVS_EDEVICE, std::string("set_projected_force: ") + hipGetErrorString(e));
    }
    c->fs_current = true;
    return KVS_OK;
}

kvs_status kvs_get_projected_force(const kvs_ctx* cc, double* FS) {
    kvs_ctx* c = const_cast<kvs_ctx*>(cc);
    if (!c) return KVS_EINVAL;
    if (!FS) return fail(c, KVS_EINVAL, "FS is NULL");
    const size_t bytes = sizeof(double) * 3 * c->N;
    if (c->prec == KVS_FP64) {
        API_HIP(c, hipMemcpyAsync(FS, c->FS, bytes, hipMemcpyDeviceToHost, c->stream));
        API_HIP(c, hipStreamSynchronize(c->stream));
        return KVS_OK;
    }
    double* tmp = nullptr;
    API_HIP(c, c->mem.get(&tmp, bytes));
    hipError_t e = kvs_launch_widen(c, c->FS, tmp, 3 * c->N);
    if (e == hipSuccess) e = hipMemcpyAsync(FS, tmp, bytes, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    c->mem.put(tmp);
    if (e != hipSuccess) return fail(c, KVS_EDEVICE, std::string("get_projected_force: ") + hipGetErrorString(e));
    return KVS_OK;
}

kvs_status kvs_get_phi(const kvs_ctx* cc, double* phi) {
    kvs_ctx* c = const_cast<kvs_ctx*>(cc);
    if (!c) return KVS_EINVAL;
    if (!phi) return fail(c, KVS_EINVAL, "phi is NULL");
    API_HIP(c, hipMemcpyAsync(phi, c->phi, sizeof(double) * c->N, hipMemcpyDeviceToHost, c->stream));
    API_HIP(c, hipStreamSynchronize(c->stream));
    return KVS_OK;
}

kvs_status kvs_set_probes(kvs_ctx* c, const int64_t* ijk, int64_t n, int32_t comp) {
    if (!c) return KVS_EINVAL;
    if (n < 0 || (n > 0 && !ijk)) return fail(c, KVS_EINVAL, "bad probe list");
    if (comp < 0 || comp > 3) return fail(c, KVS_EINVAL, "comp must be 0..3");
    std::vector<int64_t> flat((size_t)n);
    const kvs_grid& g = c->grid;
    for (int64_t p = 0; p < n; ++p) {
        const int64_t i = ijk[3 * p], j = ijk[3 * p + 1], k = ijk[3 * p + 2];
        if (i < 0 || i >= g.nx || j < 0 || j >= g.ny || k < 0 || k >= g.nz)
            return fail(c, KVS_EINVAL, "probe " + std::to_string(p) + " outside the grid");
        flat[(size_t)p] = i + g.nx * (j + g.ny * k);
    }
    // row tables for the two-step kernel: each probed grid row (j, k) gets nx
    // entries holding the probe index of each of its cells (or -1)
    std::vector<int> rowtab, ptab;
    bool rows_ok = n > 0 && n < (int64_t)1 << 30;
    if (rows_ok) {
        rowtab.assign((size_t)(g.ny * g.nz), -1);
        for (int64_t p = 0; p < n && rows_ok; ++p) {
            const int64_t i = ijk[3 * p], j = ijk[3 * p + 1], k = ijk[3 * p + 2];
            if (k == 0 || k == g.nz - 1) {
                rows_ok = false;  // never formed by the two-step kernel (Dirichlet planes)
                break;
            }
            int& off = rowtab[(size_t)(j + g.ny * k)];
            if (off < 0) {
                if (ptab.size() + (size_t)g.nx > (size_t)INT_MAX) {
                    rows_ok = false;  // offsets are 32-bit on the device
                    break;
                }
                off = (int)ptab.size();
                ptab.resize(ptab.size() + (size_t)g.nx, -1);
            }
            int& slot = ptab[(size_t)off + (size_t)i];
            if (slot >= 0) rows_ok = false;  // the same cell twice
            slot = (int)p;
        }
    }
    if (rows_ok) {
        // one entry per 64-cell segment of each row: the row's offset where
        // the segment holds a probe, else -1
        const int64_t nseg = (g.nx + 63) / 64;
        std::vector<int> segtab((size_t)(g.ny * g.nz * nseg), -1);
        for (int64_t r = 0; r < g.ny * g.nz; ++r) {
            const int off = rowtab[(size_t)r];
            if (off < 0) continue;
            for (int64_t i = 0; i < g.nx; ++i)
                if (ptab[(size_t)off + (size_t)i] >= 0) segtab[(size_t)(r * nseg + i / 64)] = off;
        }
        rowtab.swap(segtab);
    }
    API_HIP(c, hipStreamSynchronize(c->stream));
    dfree(c->mem, c->probe_cells);
    dfree(c->mem, c->probe_rowtab);
    dfree(c->mem, c->probe_ptab);
    dfree(c->mem, c->traces);
    c->trace_cap = 0;
    c->trace_steps = 0;
    c->nprobes = n;
    c->probe_comp = comp;
    c->probe_rows_ok = n == 0 || rows_ok;
    if (n > 0) {
        API_HIP(c, c->mem.get(&c->probe_cells, sizeof(int64_t) * n));
        API_HIP(c, hipMemcpyAsync(c->probe_cells, flat.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, c->stream));
        if (rows_ok) {
            API_HIP(c, c->mem.get(&c->probe_rowtab, sizeof(int) * rowtab.size()));
            API_HIP(c, c->mem.get(&c->probe_ptab, sizeof(int) * ptab.size()));
            API_HIP(c, hipMemcpyAsync(c->probe_rowtab, rowtab.data(), sizeof(int) * rowtab.size(),
                                      hipMemcpyHostToDevice, c->stream));
            API_HIP(c, hipMemcpyAsync(c->probe_ptab, ptab.data(), sizeof(int) * ptab.size(), hipMemcpyHostToDevice,
                                      c->stream));
        }
        API_HIP(c, hipStreamSynchronize(c->stream));
    }
    return KVS_OK;
}

kvs_status kvs_step(kvs_ctx* c, int64_t nsteps) {
    kvs_status s = need_material(c);
    if (s != KVS_OK) return s;
    if (nsteps < 0) return fail(c, KVS_EINVAL, "nsteps < 0");
    if (!c->have_dt) return fail(c, KVS_ESTATE, "no time step set");
    const int64_t n_env = (int64_t)c->env.size();
    for (int64_t n = c->step; n < std::min(c->step + nsteps, n_env); ++n)
        if (c->env[(size_t)n] != 0.0 && !c->fs_current)
            return fail(c, KVS_ESTATE, "the envelope is non-zero but the projected force is not current");
    s = ensure_trace_capacity(c, nsteps);
    if (s != KVS_OK) return s;
    API_HIP(c, hipSetDevice(c->device));
    if (c->pml_cells > 0 && c->pml_dirty) {
        API_HIP(c, kvs_pml_build(c));
        c->pml_dirty = false;
    }
    // The probe values of a step's result are recorded by extra blocks of the
    // next step's launch, which read that launch's input state: one launch
    // per step (or per pair of steps, where the two-step kernel applies: it
    // records the intermediate state itself), and one gather after the last
    // step of the call.
    const int64_t per_slot = c->nprobes * ncomp_of(c->probe_comp);
    for (int64_t q = 0; q < nsteps;) {
        const int64_t n = c->step;
        const double gn = n < n_env ? c->env[(size_t)n] : 0.0;
        const double gn1 = n + 1 < n_env ? c->env[(size_t)(n + 1)] : 0.0;
        const int adv = c->step_block == 2 && q + 1 < nsteps && gn == 0.0 && gn1 == 0.0 && kvs_step2_supported(c) ? 2 : 1;
        if (c->nprobes > 0 && q > 0) c->probe_fused_out = c->traces + (c->trace_steps - 1) * per_slot;
        if (c->nprobes > 0 && adv == 2) c->probe_mid_out = c->traces + c->trace_steps * per_slot;
        if (c->timing) {
            hipEvent_t ea = nullptr, eb = nullptr;
            s = next_event_pair(c, &ea, &eb);
            if (s != KVS_OK) return s;
            c->ev_steps[(size_t)(c->ev_used - 1)] = adv;
            c->launch_ev[0] = ea;
            c->launch_ev[1] = eb;
        }
        const hipError_t le = adv == 2 ? kvs_launch_step2(c) : kvs_launch_step(c, gn);
        c->launch_ev[0] = c->launch_ev[1] = nullptr;
        c->probe_fused_out = nullptr;
        c->probe_mid_out = nullptr;
        API_HIP(c, le);
        if (c->pml_cells > 0) API_HIP(c, kvs_launch_pml(c, gn));
        c->cur = 1 - c->cur;
        if (c->nprobes > 0) c->trace_steps += adv;  // last slot filled by the next launch or the gather below
        if (c->npeak > 0) API_HIP(c, kvs_launch_peak_update(c, c->u[c->cur]));
        c->step += adv;
        q += adv;
    }
    if (c->nprobes > 0 && nsteps > 0) API_HIP(c, kvs_launch_probe_gather(c, c->u[c->cur], c->trace_steps - 1));
    return KVS_OK;
}

kvs_status kvs_trace_count(const kvs_ctx* c, int64_t* n) {
    if (!c || !n) return KVS_EINVAL;
    *n = c->trace_steps;
    return KVS_OK;
}

kvs_status kvs_read_traces(const kvs_ctx* cc, double* out, int64_t cap, int64_t* n_written) {
    kvs_ctx* c = const_cast<kvs_ctx*>(cc);
    if (!c) return KVS_EINVAL;
    if (cap < 0 || (cap > 0 && !out)) return fail(c, KVS_EINVAL, "bad output buffer");
    const int64_t total = c->trace_steps * c->nprobes * ncomp_of(c->probe_comp);
    const int64_t n = std::min(cap, total);
    if (n > 0) {
        API_HIP(c, hipMemcpyAsync(out, c->traces, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    }
    API_HIP(c, hipStreamSynchronize(c->stream));
    if (n_written) *n_written = n;
    return KVS_OK;
}

kvs_status kvs_clear_traces(kvs_ctx* c) {
    if (!c) return KVS_EINVAL;
    c->trace_steps = 0;
    return KVS_OK;
}

kvs_status kvs_get_state(const kvs_ctx* cc, double* u, double* w, int64_t* step) {
    kvs_ctx* c = const_cast<kvs_ctx*>(cc);
    if (!c) return KVS_EINVAL;
    const size_t bytes = sizeof(double) * 3 * c->N;
    double* tmp = nullptr;
    if (c->prec == KVS_FP32) API_HIP(c, c->mem.get(&tmp, bytes));
    hipError_t e = hipSuccess;
    void* src[2] = {c->u[c->cur], c->w[c->cur]};
    double* dst[2] = {u, w};
    for (int q = 0; q < 2 && e == hipSuccess; ++q) {
        if (!dst[q]) continue;
        if (c->prec == KVS_FP64) {
            e = hipMemcpyAsync(dst[q], src[q], bytes, hipMemcpyDeviceToHost, c->stream);
        } else {
            e = kvs_launch_widen(c, src[q], tmp, 3 * c->N);
            if (e == hipSuccess) e = hipMemcpyAsync(dst[q], tmp, bytes, hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (tmp) c->mem.put(tmp);
    if (e != hipSuccess) return fail(c, KVS_EDEVICE, std::string("get_state: ") + hipGetErrorString(e));
    if (step) *step = c->step;
    return KVS_OK;
}

// The layer's memory variables belong to the state: zero them whenever the
// state is replaced.
kvs_status clear_pml_memory(kvs_ctx* c) {
    if (c->pml_mem && c->pml_mem_count > 0) {
        API_HIP(c, hipMemsetAsync(c->pml_mem, 0, (size_t)c->pml_mem_count * tsize(c), c->stream));
        API_HIP(c, hipStreamSynchronize(c->stream));
    }
    return KVS_OK;
}

kvs_status kvs_set_pml(kvs_ctx* c, int32_t cells, double R, double alpha_max) {
    if (!c) return KVS_EINVAL;
    if (cells < 0) return fail(c, KVS_EINVAL, "pml: cells must be >= 0");
    if (cells > 0) {
        const kvs_grid& g = c->grid;
        if (std::min(g.nx, std::min(g.ny, g.nz)) < 2 * (int64_t)cells + 3)
            return fail(c, KVS_EINVAL, "pml: every extent must be at least 2 cells + 3");
        if (!(std::isfinite(R) && R > 0.0 && R <= 1.0)) return fail(c, KVS_EINVAL, "pml: R must be in (0, 1]");
        if (!std::isfinite(alpha_max)) return fail(c, KVS_EINVAL, "pml: alpha_max must be finite");
        if (c->sponge_cells > 0) return fail(c, KVS_EINVAL, "pml: the context has a sponge; use one or the other");
    }
    API_HIP(c, hipSetDevice(c->device));
    API_HIP(c, hipStreamSynchronize(c->stream));
    dfree(c->mem, c->pml_tab);
    dfree(c->mem, c->pml_mem);
    c->pml_mem_count = 0;
    c->pml_cells = 0;
    if (cells == 0) return KVS_OK;
    const kvs_grid& g = c->grid;
    int64_t count = 0;
    // per axis: two buffers of the 6 face memories (one read, the other
    // written each step) and the 3 divergence memories
    for (int a = 0; a < 3; ++a) count += 15 * kvs_pml_slab_cells(g, cells, a);
    API_HIP(c, c->mem.get(&c->pml_tab, tsize(c) * 4 * (size_t)(g.nx + g.ny + g.nz)));
    API_HIP(c, c->mem.get(&c->pml_mem, tsize(c) * (size_t)count));
    c->pml_mem_count = count;
    c->pml_cells = cells;
    c->pml_R = R;
    c->pml_alpha = alpha_max;
    c->pml_dirty = true;
    return clear_pml_memory(c);
}

kvs_status kvs_set_state(kvs_ctx* c, const double* u, const double* w, int64_t step) {
    if (!c) return KVS_EINVAL;
    if (!u || !w || step < 0) return fail(c, KVS_EINVAL, "bad state");
    const size_t bytes = sizeof(double) * 3 * c->N;
    double* tmp = nullptr;
    API_HIP(c, c->mem.get(&tmp, bytes));
    hipError_t e = hipSuccess;
    const double* src[2] = {u, w};
    void* dst[2] = {c->u[c->cur], c->w[c->cur]};
    for (int q = 0; q < 2 && e == hipSuccess; ++q) {
        e = hipMemcpyAsync(tmp, src[q], bytes, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = kvs_launch_cast(c, tmp, dst[q], 3 * c->N);
        if (e == hipSuccess) e = kvs_launch_zero_boundary(c, dst[q]);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    c->mem.put(tmp);
    if (e != hipSuccess) return fail(c, KVS_EDEVICE, std::string("set_state: ") + hipGetErrorString(e));
    c->step = step;
    return clear_pml_memory(c);
}

kvs_status kvs_set_state_curl(kvs_ctx* c, const double* A, int64_t step) {
    if (!c) return KVS_EINVAL;
    if (!A || step < 0) return fail(c, KVS_EINVAL, "curl state: A is NULL or step < 0");
    if (!c->have_dt) return fail(c, KVS_ESTATE, "curl state: no dt set");
    const size_t bytes = sizeof(double) * 3 * c->N;
    API_HIP(c, hipSetDevice(c->device));
    double* tmp = nullptr;
    API_HIP(c, c->mem.get(&tmp, bytes));
    hipError_t e = hipMemcpyAsync(tmp, A, bytes, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = kvs_launch_curl_state(c, tmp);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    c->mem.put(tmp);
    if (e != hipSuccess) return fail(c, KVS_EDEVICE, std::string("curl state: ") + hipGetErrorString(e));
    c->step = step;
    return clear_pml_memory(c);
}

kvs_status kvs_reset_state(kvs_ctx* c) {
    if (!c) return KVS_EINVAL;
    const size_t bytes = 3 * (size_t)c->N * tsize(c);
    for (int b = 0; b < 2; ++b) {
        API_HIP(c, hipMemsetAsync(c->u[b], 0, bytes, c->stream));
        API_HIP(c, hipMemsetAsync(c->w[b], 0, bytes, c->stream));
    }
    c->step = 0;
    c->trace_steps = 0;
    if (c->peak) API_HIP(c, hipMemsetAsync(c->peak, 0, (size_t)c->peak_cells * tsize(c), c->stream));
    return clear_pml_memory(c);
}

kvs_status kvs_set_peak_planes(kvs_ctx* c, const int32_t* axis, const int64_t* index, int32_t n) {
    if (!c) return KVS_EINVAL;
    if (n < 0 || n > KVS_MAX_PEAK_PLANES) return fail(c, KVS_EINVAL, "peak planes: n must be 0..KVS_MAX_PEAK_PLANES");
    if (n > 0 && (!axis || !index)) return fail(c, KVS_EINVAL, "peak planes: NULL axis or index");
    const kvs_grid& g = c->grid;
    const int64_t ext[3] = {g.nx, g.ny, g.nz};
    int64_t off[KVS_MAX_PEAK_PLANES] = {}, total = 0;
    for (int p = 0; p < n; ++p) {
        if (axis[p] < 0 || axis[p] > 2) return fail(c, KVS_EINVAL, "peak planes: axis must be 0..2");
        if (index[p] < 0 || index[p] >= ext[axis[p]])
            return fail(c, KVS_EINVAL, "peak plane " + std::to_string(p) + " outside the grid");
        for (int q = 0; q < p; ++q)
            if (axis[q] == axis[p] && index[q] == index[p])
                return fail(c, KVS_EINVAL, "peak planes: the same plane twice");
        off[p] = total;
        total += ext[axis[p] == 0 ? 1 : 0] * ext[axis[p] == 2 ? 1 : 2];
    }
    API_HIP(c, hipSetDevice(c->device));
    API_HIP(c, hipStreamSynchronize(c->stream));
    dfree(c->mem, c->peak);
    c->npeak = 0;
    c->peak_cells = 0;
    if (n == 0) return KVS_OK;
    API_HIP(c, c->mem.get(&c->peak, (size_t)total * tsize(c)));
    API_HIP(c, hipMemsetAsync(c->peak, 0, (size_t)total * tsize(c), c->stream));
    for (int p = 0; p < n; ++p) {
        c->peak_axis[p] = axis[p];
        c->peak_index[p] = index[p];
        c->peak_off[p] = off[p];
    }
    c->npeak = n;
    c->peak_cells = total;
    API_HIP(c, kvs_launch_peak_update(c, c->u[c->cur]));
    API_HIP(c, hipStreamSynchronize(c->stream));
    return KVS_OK;
}

kvs_status kvs_peak_map(const kvs_ctx* cc, int32_t axis, int64_t index, double* out) {
    kvs_ctx* c = const_cast<kvs_ctx*>(cc);
    if (!c) return KVS_EINVAL;
    if (!out) return fail(c, KVS_EINVAL, "peak map: out is NULL");
    int p = 0;
    while (p < c->npeak && !(c->peak_axis[p] == axis && c->peak_index[p] == index)) ++p;
    if (p == c->npeak) return fail(c, KVS_EINVAL, "peak map: plane not registered");
    const int64_t cells = (p + 1 < c->npeak ? c->peak_off[p + 1] : c->peak_cells) - c->peak_off[p];
    API_HIP(c, hipSetDevice(c->device));
    if (c->prec == KVS_FP64) {
        API_HIP(c, hipMemcpyAsync(out, static_cast<double*>(c->peak) + c->peak_off[p], sizeof(double) * cells,
                                  hipMemcpyDeviceToHost, c->stream));
        API_HIP(c, hipStreamSynchronize(c->stream));
    } else {
        std::vector<float> tmp((size_t)cells);
        API_HIP(c, hipMemcpyAsync(tmp.data(), static_cast<float*>(c->peak) + c->peak_off[p], sizeof(float) * cells,
                                  hipMemcpyDeviceToHost, c->stream));
        API_HIP(c, hipStreamSynchronize(c->stream));
        for (int64_t q = 0; q < cells; ++q) out[q] = (double)tmp[(size_t)q];
    }
    return KVS_OK;
}

// ---- acoustic radiation force ----------------------------------------------

kvs_status kvs_arf_begin(kvs_ctx* c, int32_t mode) {
    if (!c) return KVS_EINVAL;
    if (mode != KVS_ARF_PLANE && mode != KVS_ARF_POYNTING)
        return fail(c, KVS_EINVAL, "arf: mode must be KVS_ARF_PLANE or KVS_ARF_POYNTING");
    const int64_t need = (mode == KVS_ARF_PLANE ? 1 : 3) * c->N;
    API_HIP(c, hipSetDevice(c->device));
    if (c->arf_sum_cap < need) {
        API_HIP(c, hipStreamSynchronize(c->stream));
        dfree(c->mem, c->arf_sum);
        c->arf_sum_cap = 0;
        c->arf_mode = 0;
        API_HIP(c, c->mem.get(&c->arf_sum, sizeof(double) * (size_t)need));
        c->arf_sum_cap = need;
    }
    API_HIP(c, hipMemsetAsync(c->arf_sum, 0, sizeof(double) * (size_t)need, c->stream));
    c->arf_mode = mode;
    c->arf_samples = 0;
    return KVS_OK;
}

kvs_status kvs_arf_accumulate_device(kvs_ctx* c, const void* p, const void* v, int64_t nsamp, int32_t dtype) {
    if (!c) return KVS_EINVAL;
    if (c->arf_mode == 0) return fail(c, KVS_ESTATE, "arf: no kvs_arf_begin");
    if (nsamp < 1) return fail(c, KVS_EINVAL, "arf: nsamp must be >= 1");
    if (dtype != 0 && dtype != 1) return fail(c, KVS_EINVAL, "arf: dtype must be 0 (double) or 1 (float)");
    if (!p) return fail(c, KVS_EINVAL, "arf: p is NULL");
    if (c->arf_mode == KVS_ARF_POYNTING && !v) return fail(c, KVS_EINVAL, "arf: v is NULL in the Poynting form");
    if (c->arf_mode == KVS_ARF_PLANE && v) return fail(c, KVS_EINVAL, "arf: v must be NULL in the plane-wave form");
    API_HIP(c, hipSetDevice(c->device));
    API_HIP(c, kvs_launch_arf_accumulate(c, p, v, nsamp, dtype));
    c->arf_samples += nsamp;
    return KVS_OK;
}

kvs_status kvs_arf_accumulate(kvs_ctx* c, const double* p, const double* v, int64_t nsamp) {
    if (!c) return KVS_EINVAL;
    if (c->arf_mode == 0) return fail(c, KVS_ESTATE, "arf: no kvs_arf_begin");
    if (nsamp < 1) return fail(c, KVS_EINVAL, "arf: nsamp must be >= 1");
    if (!p) return fail(c, KVS_EINVAL, "arf: p is NULL");
    if (c->arf_mode == KVS_ARF_POYNTING && !v) return fail(c, KVS_EINVAL, "arf: v is NULL in the Poynting form");
    if (c->arf_mode == KVS_ARF_PLANE && v) return fail(c, KVS_EINVAL, "arf: v must be NULL in the plane-wave form");
    API_HIP(c, hipSetDevice(c->device));
    // stage one sample at a time (p, then v) through one device buffer
    const int64_t per = (v ? 4 : 1) * c->N;
    double* stage = nullptr;
    API_HIP(c, c->mem.get(&stage, sizeof(double) * (size_t)per));
    hipError_t e = hipSuccess;
    for (int64_t s = 0; s < nsamp && e == hipSuccess; ++s) {
        e = hipMemcpyAsync(stage, p + s * c->N, sizeof(double) * (size_t)c->N, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess && v)
            e = hipMemcpyAsync(stage + c->N, v + s * 3 * c->N, sizeof(double) * 3 * (size_t)c->N,
                               hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = kvs_launch_arf_accumulate(c, stage, v ? stage + c->N : nullptr, 1, 0);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    c->mem.put(stage);
    if (e != hipSuccess) return fail(c, KVS_EDEVICE, std::string("arf accumulate: ") + hipGetErrorString(e));
    c->arf_samples += nsamp;
    return KVS_OK;
}

kvs_status kvs_arf_get_sums(const kvs_ctx* cc, double* out, int64_t* nsamp) {
    kvs_ctx* c = const_cast<kvs_ctx*>(cc);
    if (!c) return KVS_EINVAL;
    if (c->arf_mode == 0) return fail(c, KVS_ESTATE, "arf: no kvs_arf_begin");
    if (nsamp) *nsamp = c->arf_samples;
    if (!out) return KVS_OK;
    const int64_t n = (c->arf_mode == KVS_ARF_PLANE ? 1 : 3) * c->N;
    API_HIP(c, hipSetDevice(c->device));
    API_HIP(c, hipMemcpyAsync(out, c->arf_sum, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost, c->stream));
    API_HIP(c, hipStreamSynchronize(c->stream));
    return KVS_OK;
}

kvs_status kvs_arf_set_force(kvs_ctx* c, const double* alpha, int64_t n_alpha, const double* cs, int64_t n_c,
                             const double* rho, int64_t n_rho, const uint8_t* mask, double n_pulse,
                             const double* beam_dir) {
    if (!c) return KVS_EINVAL;
    if (c->arf_mode == 0) return fail(c, KVS_ESTATE, "arf: no kvs_arf_begin");
    if (c->arf_samples == 0) return fail(c, KVS_ESTATE, "arf: no samples accumulated");
    const bool plane = c->arf_mode == KVS_ARF_PLANE;
    auto bad_count = [&](int64_t n) { return n != 1 && n != c->N; };
    if (!alpha || bad_count(n_alpha)) return fail(c, KVS_EINVAL, "arf: alpha needs 1 or N values");
    if (!cs || bad_count(n_c)) return fail(c, KVS_EINVAL, "arf: c needs 1 or N values");
    if (plane && (!rho || bad_count(n_rho))) return fail(c, KVS_EINVAL, "arf: rho needs 1 or N values");
    if (!(std::isfinite(n_pulse) && n_pulse > 0.0)) return fail(c, KVS_EINVAL, "arf: n_pulse must be > 0");
    for (int64_t q = 0; q < n_alpha; ++q)
        if (!(std::isfinite(alpha[q]) && alpha[q] >= 0.0)) return fail(c, KVS_EINVAL, "arf: alpha must be finite, >= 0");
    for (int64_t q = 0; q < n_c; ++q)
        if (!finite_pos(cs[q])) return fail(c, KVS_EINVAL, "arf: c must be finite, > 0");
    if (plane)
        for (int64_t q = 0; q < n_rho; ++q)
            if (!finite_pos(rho[q])) return fail(c, KVS_EINVAL, "arf: rho must be finite, > 0");
    double d[3] = {0.0, 0.0, 0.0};
    if (plane) {
        if (!beam_dir) return fail(c, KVS_EINVAL, "arf: beam_dir is NULL in the plane-wave form");
        const double n2 = beam_dir[0] * beam_dir[0] + beam_dir[1] * beam_dir[1] + beam_dir[2] * beam_dir[2];
        if (!(std::isfinite(n2) && n2 > 0.0)) return fail(c, KVS_EINVAL, "arf: beam_dir must be non-zero");
        const double nn = std::sqrt(n2);
        for (int q = 0; q < 3; ++q) d[q] = beam_dir[q] / nn;
    }
    API_HIP(c, hipSetDevice(c->device));
    // coefficient maps and mask staged in one temporary device buffer
    const int64_t nr = plane ? n_rho : 0;
    const size_t doubles = (size_t)(n_alpha + n_c + nr);
    const size_t bytes = sizeof(double) * doubles + (mask ? (size_t)c->N : 0);
    char* tmp = nullptr;
    API_HIP(c, c->mem.get(&tmp, bytes));
    double* dA = reinterpret_cast<double*>(tmp);
    double* dC = dA + n_alpha;
    double* dR = plane ? dC + n_c : nullptr;
    unsigned char* dM = mask ? reinterpret_cast<unsigned char*>(tmp + sizeof(double) * doubles) : nullptr;
    hipError_t e = hipMemcpyAsync(dA, alpha, sizeof(double) * n_alpha, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dC, cs, sizeof(double) * n_c, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && plane) e = hipMemcpyAsync(dR, rho, sizeof(double) * n_rho, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && mask) e = hipMemcpyAsync(dM, mask, (size_t)c->N, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = kvs_launch_arf_force(c, dA, n_alpha == 1 ? 0 : 1, dC, n_c == 1 ? 0 : 1, dR, n_rho == 1 ? 0 : 1, dM,
                                 n_pulse, d);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    c->mem.put(tmp);
    if (e != hipSuccess) return fail(c, KVS_EDEVICE, std::string("arf force: ") + hipGetErrorString(e));
    c->have_force = true;
    c->fs_current = false;
    return KVS_OK;
}

kvs_status kvs_strain_begin(kvs_ctx* c, const double* K, int64_t n_K) {
    if (!c) return KVS_EINVAL;
    if (!K || (n_K != 1 && n_K != c->N)) return fail(c, KVS_EINVAL, "strain: K needs 1 or N values");
    for (int64_t q = 0; q < n_K; ++q)
        if (!finite_pos(K[q])) return fail(c, KVS_EINVAL, "strain: K must be finite, > 0");
    API_HIP(c, hipSetDevice(c->device));
    API_HIP(c, hipStreamSynchronize(c->stream));
    if (!c->strain_peak) API_HIP(c, c->mem.get(&c->strain_peak, sizeof(double) * 2 * (size_t)c->N));
    if (c->strain_K_cap < n_K) {
        dfree(c->mem, c->strain_K);
        c->strain_K_cap = 0;
        API_HIP(c, c->mem.get(&c->strain_K, sizeof(double) * (size_t)n_K));
        c->strain_K_cap = n_K;
    }
    API_HIP(c, hipMemcpyAsync(c->strain_K, K, sizeof(double) * (size_t)n_K, hipMemcpyHostToDevice, c->stream));
    API_HIP(c, hipMemsetAsync(c->strain_peak, 0, sizeof(double) * 2 * (size_t)c->N, c->stream));
    API_HIP(c, hipStreamSynchronize(c->stream));
    c->strain_sK = n_K == 1 ? 0 : 1;
    c->strain_samples = 0;
    c->strain_on = true;
    return KVS_OK;
}

kvs_status kvs_strain_accumulate_device(kvs_ctx* c, const void* p, int64_t nsamp, int32_t dtype) {
    if (!c) return KVS_EINVAL;
    if (!c->strain_on) return fail(c, KVS_ESTATE, "strain: no kvs_strain_begin");
    if (nsamp < 1) return fail(c, KVS_EINVAL, "strain: nsamp must be >= 1");
    if (dtype != 0 && dtype != 1) return fail(c, KVS_EINVAL, "strain: dtype must be 0 (double) or 1 (float)");
    if (!p) return fail(c, KVS_EINVAL, "strain: p is NULL");
    API_HIP(c, hipSetDevice(c->device));
    API_HIP(c, kvs_launch_strain(c, p, nsamp, dtype));
    c->strain_samples += nsamp;
    return KVS_OK;
}

kvs_status kvs_strain_get(const kvs_ctx* cc, double* peak_strain, double* peak_gradient, int64_t* nsamp) {
    kvs_ctx* c = const_cast<kvs_ctx*>(cc);
    if (!c) return KVS_EINVAL;
    if (!c->strain_on) return fail(c, KVS_ESTATE, "strain: no kvs_strain_begin");
    if (nsamp) *nsamp = c->strain_samples;
    API_HIP(c, hipSetDevice(c->device));
    if (peak_strain)
        API_HIP(c, hipMemcpyAsync(peak_strain, c->strain_peak, sizeof(double) * (size_t)c->N, hipMemcpyDeviceToHost,
                                  c->stream));
    if (peak_gradient) {
        double* roots = nullptr;
        API_HIP(c, c->mem.get(&roots, sizeof(double) * (size_t)c->N));
        hipError_t e = kvs_launch_strain_roots(c, roots);
        if (e == hipSuccess)
            e = hipMemcpyAsync(peak_gradient, roots, sizeof(double) * (size_t)c->N, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        c->mem.put(roots);
        if (e != hipSuccess) return fail(c, KVS_EDEVICE, std::string("strain: ") + hipGetErrorString(e));
    }
    API_HIP(c, hipStreamSynchronize(c->stream));
    return KVS_OK;
}

kvs_status kvs_enable_kernel_timing(kvs_ctx* c, int32_t on) {
    if (!c) return KVS_EINVAL;
    if (on && !c->timing) {
        c->timed_ms = 0.0;
        c->timed_launches = 0;
        for (int q = 0; q < 2; ++q) {
            c->timed_ms_kind[q] = 0.0;
            c->timed_n_kind[q] = 0;
        }
        c->ev_used = 0;
    }
    if (!on && c->timing) {
        kvs_status s = flush_timing(c);
        if (s != KVS_OK) return s;
    }
    c->timing = on != 0;
    return KVS_OK;
}

kvs_status kvs_kernel_time(kvs_ctx* c, double* ms_total, int64_t* launches) {
    if (!c) return KVS_EINVAL;
    kvs_status s = flush_timing(c);
    if (s != KVS_OK) return s;
    if (ms_total) *ms_total = c->timed_ms;
    if (launches) *launches = c->timed_launches;
    return KVS_OK;
}

kvs_status kvs_kernel_time_split(kvs_ctx* c, double* ms, int64_t* launches) {
    if (!c) return KVS_EINVAL;
    kvs_status s = flush_timing(c);
    if (s != KVS_OK) return s;
    for (int q = 0; q < 2; ++q) {
        if (ms) ms[q] = c->timed_ms_kind[q];
        if (launches) launches[q] = c->timed_n_kind[q];
    }
    return KVS_OK;
}

int32_t kvs_num_step_variants(void) { return kvs_step_variant_count(); }

kvs_status kvs_set_step_variant(kvs_ctx* c, int32_t v) {
    if (!c) return KVS_EINVAL;
    if (v < 0 || v >= kvs_step_variant_count()) return fail(c, KVS_EINVAL, "no such step variant");
    c->step_variant = v;
    return KVS_OK;
}

kvs_status kvs_set_step_tuning(kvs_ctx* c, int32_t v, int32_t zchunk, int32_t remap) {
    if (!c) return KVS_EINVAL;
    if (v < 0 || v >= kvs_step_variant_count()) return fail(c, KVS_EINVAL, "no such step variant");
    if (zchunk < 0) return fail(c, KVS_EINVAL, "zchunk < 0");
    c->step_variant = v;
    c->step_zchunk = zchunk;
    c->step_remap = remap != 0;
    return KVS_OK;
}

kvs_status kvs_set_step_blocking(kvs_ctx* c, int32_t steps) {
    if (!c) return KVS_EINVAL;
    if (steps != 1 && steps != 2) return fail(c, KVS_EINVAL, "steps per launch must be 1 or 2");
    c->step_block = steps;
    return KVS_OK;
}

kvs_status kvs_set_direction_precision(kvs_ctx* c, int32_t prec) {
    if (!c) return KVS_EINVAL;
    if (prec != KVS_FP64 && prec != KVS_FP32) return fail(c, KVS_EINVAL, "direction precision must be FP64 or FP32");
    if (prec != c->dir_prec) c->p_dirty = true;
    c->dir_prec = prec;
    return KVS_OK;
}

kvs_status kvs_set_residual_precision(kvs_ctx* c, int32_t prec) {
    if (!c) return KVS_EINVAL;
    if (prec != KVS_FP64 && prec != KVS_FP32) return fail(c, KVS_EINVAL, "residual precision must be FP64 or FP32");
    c->res_prec = prec;
    return KVS_OK;
}

int32_t kvs_step_blocking_applies(const kvs_ctx* c) { return c && c->have_material && kvs_step2_supported(c) ? 1 : 0; }

kvs_status kvs_autotune_step(kvs_ctx* c, int32_t trial_steps, int32_t* chosen, double* ms_per_launch,
                             int32_t cap) {
    kvs_status s = need_material(c);
    if (s != KVS_OK) return s;
    if (!c->have_dt) return fail(c, KVS_ESTATE, "no time step set");
    if (trial_steps < 1) return fail(c, KVS_EINVAL, "trial_steps < 1");
    API_HIP(c, hipSetDevice(c->device));
    hipEvent_t e0, e1;
    API_HIP(c, hipEventCreate(&e0));
    API_HIP(c, hipEventCreate(&e1));
    const int nv = kvs_step_variant_count();
    const int zchunks[4] = {0, 16, 32, 64};  // auto split, and fixed segment lengths
    int best = 0, best_z = 0;
    double best_ms = 1e300;
    const int saved_z = c->step_zchunk;
    for (int v = 0; v < nv; ++v) {
        double v_best = 1e300;
        for (int zi = 0; zi < 4; ++zi) {
            c->step_zchunk = zchunks[zi];
            // warm-up launch, then timed launches; cur is not flipped, so every
            // launch recomputes the same next state from the same current state
            hipError_t e = kvs_launch_step_variant(c, 0.0, v);
            if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
            for (int q = 0; q < trial_steps && e == hipSuccess; ++q) e = kvs_launch_step_variant(c, 0.0, v);
            if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                c->step_zchunk = saved_z;
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                return fail(c, KVS_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
            }
            const double per = ms / trial_steps;
            v_best = std::min(v_best, per);
            if (per < best_ms) {
                best_ms = per;
                best = v;
                best_z = zchunks[zi];
            }
        }
        if (ms_per_launch && v < cap) ms_per_launch[v] = v_best;
    }
    c->step_zchunk = best_z;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->step_variant = best;
    if (chosen) *chosen = best;
    return KVS_OK;
}

// ---- batches -------------------------------------------------------------------

static kvs_status bfail(kvs_batch* b, kvs_status s, const std::string& msg) {
    if (b)
        b->err = msg;
    else
        g_create_err = msg;
    return s;
}

#define BATCH_HIP(b, call)                                                                                \
    do {                                                                                                  \
        hipError_t e_ = (call);                                                                           \
        if (e_ != hipSuccess) return bfail(b, KVS_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

static void batch_release(kvs_batch* b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (kvs_ctx* c : b->inst) kvs_destroy(c);
    b->inst.clear();
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
    dfree(b->mem, b->dev_params);
    dfree(b->mem, b->dev_work);
    dfree(b->mem, b->dev_params2);
    dfree(b->mem, b->dev_work2);
    dfree(b->mem, b->dev_ptabs2);
    dfree(b->mem, b->dev_probes);
    dfree(b->mem, b->traces);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    b->stream = nullptr;
}

kvs_status kvs_batch_create(const kvs_grid* grids, int32_t n, const kvs_opts* opts, kvs_batch** out) {
    if (!out) return bfail(nullptr, KVS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!grids || n < 1) return bfail(nullptr, KVS_EINVAL, "need at least one grid");
    kvs_opts o{};
    o.precision = KVS_FP32;
    o.sponge_sigma_max = -1.0;
    if (opts) o = *opts;
    if (o.device < 0) return bfail(nullptr, KVS_EINVAL, "device ordinal out of range");
    if (hipSetDevice(o.device) != hipSuccess) return bfail(nullptr, KVS_EDEVICE, "hipSetDevice failed");
    kvs_batch* b = new (std::nothrow) kvs_batch();
    if (!b) return bfail(nullptr, KVS_ENOMEM, "host allocation failed");
    if ((o.alloc == nullptr) != (o.free == nullptr)) {
        delete b;
        return bfail(nullptr, KVS_EINVAL, "alloc and free must be given together");
    }
    b->device = o.device;
    b->prec = o.precision;
    if (o.stream) {
        b->stream = (hipStream_t)o.stream;
    } else {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
            delete b;
            return bfail(nullptr, KVS_EDEVICE, "hipStreamCreate failed");
        }
        b->own_stream = true;
    }
    o.stream = b->stream;
    b->mem.alloc = o.alloc;
    b->mem.release = o.free;
    b->mem.user = o.alloc_user;
    b->mem.stream = b->stream;
    for (int32_t i = 0; i < n; ++i) {
        kvs_ctx* c = nullptr;
        kvs_status st = kvs_create(&grids[i], &o, &c);
        if (st != KVS_OK) {
            const std::string msg = "instance " + std::to_string(i) + ": " + kvs_last_error(nullptr);
            batch_release(b);
            delete b;
            return bfail(nullptr, st, msg);
        }
        b->inst.push_back(c);
    }
    b->probe_first.assign((size_t)n + 1, 0);
    *out = b;
    return KVS_OK;
}

void kvs_batch_destroy(kvs_batch* b) {
    if (!b) return;
    batch_release(b);
    delete b;
}

const char* kvs_batch_last_error(const kvs_batch* b) { return b ? b->err.c_str() : g_create_err.c_str(); }

kvs_ctx* kvs_batch_instance(kvs_batch* b, int32_t i) {
    if (!b || i < 0 || i >= (int32_t)b->inst.size()) return nullptr;
    return b->inst[(size_t)i];
}

kvs_status kvs_batch_share_projection(kvs_batch* b, int32_t src, int32_t dst) {
    if (!b) return KVS_EINVAL;
    kvs_ctx* s = kvs_batch_instance(b, src);
    kvs_ctx* d = kvs_batch_instance(b, dst);
    if (!s || !d) return bfail(b, KVS_EINVAL, "instance out of range");
    const kvs_grid &gs = s->grid, &gd = d->grid;
    if (gs.nx != gd.nx || gs.ny != gd.ny || gs.nz != gd.nz || gs.hx != gd.hx || gs.hy != gd.hy || gs.hz != gd.hz)
        return bfail(b, KVS_EINVAL, "share_projection needs identical grids");
    if (!s->fs_current) return bfail(b, KVS_ESTATE, "source instance has no current projection");
    if (src == dst) return KVS_OK;
    BATCH_HIP(b, hipMemcpyAsync(d->FS, s->FS, 3 * (size_t)s->N * tsize(s), hipMemcpyDeviceToDevice, b->stream));
    BATCH_HIP(b, hipStreamSynchronize(b->stream));
    d->fs_current = true;
    return KVS_OK;
}

// Probe tables of the two-step launches, for every instance with probes: one
// entry per 64-cell segment of each grid row (the row's offset into the probe
// table where that segment holds a probe, else -1), and per probed row nx
// instance-local probe indices.  Probe cells must be distinct and off the
// planes k = 0, nz - 1 (else two-step launches are not used).
static kvs_status batch_upload_probes2(kvs_batch* b) {
    const size_t ni = b->inst.size();
    dfree(b->mem, b->dev_ptabs2);
    b->rowtab2_off.assign(ni, -1);
    b->ptab2_off.assign(ni, -1);
    b->probes2_ok = true;
    std::vector<int> all;
    for (size_t i = 0; i < ni && b->probes2_ok; ++i) {
        const int64_t p0 = b->probe_first.empty() ? 0 : b->probe_first[i];
        const int64_t p1 = b->probe_first.empty() ? 0 : b->probe_first[i + 1];
        if (p1 == p0) continue;
        const kvs_grid& g = b->inst[i]->grid;
        const int64_t nseg = (g.nx + 63) / 64;
        std::vector<int> row((size_t)(g.ny * g.nz), -1), ptab;
        for (int64_t p = p0; p < p1 && b->probes2_ok; ++p) {
            const int64_t cell = b->probe_cell[(size_t)p];
            const int64_t x = cell % g.nx, y = (cell / g.nx) % g.ny, z = cell / (g.nx * g.ny);
            if (z == 0 || z == g.nz - 1) {
                b->probes2_ok = false;
                break;
            }
            int& off = row[(size_t)(y + g.ny * z)];
            if (off < 0) {
                if (ptab.size() + (size_t)g.nx > (size_t)INT_MAX) {
                    b->probes2_ok = false;  // offsets are 32-bit on the device
                    break;
                }
                off = (int)ptab.size();
                ptab.resize(ptab.size() + (size_t)g.nx, -1);
            }
            int& slot = ptab[(size_t)off + (size_t)x];
            if (slot >= 0) b->probes2_ok = false;  // the same cell twice
            slot = (int)(p - p0);
        }
        if (!b->probes2_ok) break;
        std::vector<int> seg((size_t)(g.ny * g.nz * nseg), -1);
        for (int64_t r = 0; r < g.ny * g.nz; ++r) {
            const int off = row[(size_t)r];
            if (off < 0) continue;
            for (int64_t x = 0; x < g.nx; ++x)
                if (ptab[(size_t)off + (size_t)x] >= 0) seg[(size_t)(r * nseg + x / 64)] = off;
        }
        b->rowtab2_off[i] = (int64_t)all.size();
        all.insert(all.end(), seg.begin(), seg.end());
        b->ptab2_off[i] = (int64_t)all.size();
        all.insert(all.end(), ptab.begin(), ptab.end());
    }
    if (!b->probes2_ok || all.empty()) {
        b->rowtab2_off.assign(ni, -1);
        b->ptab2_off.assign(ni, -1);
        return KVS_OK;
    }
    BATCH_HIP(b, b->mem.get(&b->dev_ptabs2, sizeof(int) * all.size()));
    BATCH_HIP(b, hipMemcpyAsync(b->dev_ptabs2, all.data(), sizeof(int) * all.size(), hipMemcpyHostToDevice,
                                b->stream));
    BATCH_HIP(b, hipStreamSynchronize(b->stream));
    return KVS_OK;
}

static kvs_status batch_upload_probes(kvs_batch* b) {
    const size_t np = b->probe_inst.size();
    dfree(b->mem, b->dev_probes);
    dfree(b->mem, b->traces);
    b->trace_cap = 0;
    b->trace_steps = 0;
    b->graph_valid = false;
    b->host_traces_valid = false;
    kvs_status s2 = batch_upload_probes2(b);
    if (s2 != KVS_OK) return s2;
    if (np == 0) return KVS_OK;
    // (instance, cell) pairs, then the first probe of every instance (n + 1
    // entries: the persistent path finds its instance's probes there)
    std::vector<int64_t> flat(2 * np + b->probe_first.size());
    for (size_t p = 0; p < np; ++p) {
        flat[2 * p] = b->probe_inst[p];
        flat[2 * p + 1] = b->probe_cell[p];
    }
    std::copy(b->probe_first.begin(), b->probe_first.end(), flat.begin() + 2 * np);
    BATCH_HIP(b, b->mem.get(&b->dev_probes, sizeof(int64_t) * flat.size()));
    BATCH_HIP(b, hipMemcpyAsync(b->dev_probes, flat.data(), sizeof(int64_t) * flat.size(), hipMemcpyHostToDevice,
                                b->stream));
    BATCH_HIP(b, hipStreamSynchronize(b->stream));
    return KVS_OK;
}

kvs_status kvs_batch_set_probes(kvs_batch* b, int32_t i, const int64_t* ijk, int64_t n) {
    if (!b) return KVS_EINVAL;
    kvs_ctx* c = kvs_batch_instance(b, i);
    if (!c) return bfail(b, KVS_EINVAL, "instance out of range");
    if (n < 0 || (n > 0 && !ijk)) return bfail(b, KVS_EINVAL, "bad probe list");
    const kvs_grid& g = c->grid;
    std::vector<int64_t> cells((size_t)n);
    for (int64_t p = 0; p < n; ++p) {
        const int64_t x = ijk[3 * p], y = ijk[3 * p + 1], z = ijk[3 * p + 2];
        if (x < 0 || x >= g.nx || y < 0 || y >= g.ny || z < 0 || z >= g.nz)
            return bfail(b, KVS_EINVAL, "probe " + std::to_string(p) + " outside instance " + std::to_string(i));
        cells[(size_t)p] = x + g.nx * (y + g.ny * z);
    }
    // rebuild the flat list with instance i's probes replaced
    std::vector<int64_t> pi, pc;
    const int ni = (int)b->inst.size();
    std::vector<int64_t> first((size_t)ni + 1, 0);
    for (int k = 0; k < ni; ++k) {
        first[(size_t)k] = (int64_t)pi.size();
        if (k == i) {
            for (int64_t p = 0; p < n; ++p) {
                pi.push_back(k);
                pc.push_back(cells[(size_t)p]);
            }
        } else {
            for (int64_t p = b->probe_first[(size_t)k]; p < b->probe_first[(size_t)k + 1]; ++p) {
                pi.push_back(k);
                pc.push_back(b->probe_cell[(size_t)p]);
            }
        }
    }
    first[(size_t)ni] = (int64_t)pi.size();
    b->probe_inst.swap(pi);
    b->probe_cell.swap(pc);
    b->probe_first.swap(first);
    return batch_upload_probes(b);
}

kvs_status kvs_batch_set_component(kvs_batch* b, int32_t comp) {
    if (!b) return KVS_EINVAL;
    if (comp < 0 || comp > 2) return bfail(b, KVS_EINVAL, "component must be 0..2");
    b->comp = comp;
    b->trace_steps = 0;
    b->graph_valid = false;
    b->host_traces_valid = false;
    return KVS_OK;
}

kvs_status kvs_batch_step(kvs_batch* b, int64_t nsteps) {
    if (!b) return KVS_EINVAL;
    if (nsteps < 0) return bfail(b, KVS_EINVAL, "nsteps < 0");
    if (nsteps == 0) return KVS_OK;
    for (size_t i = 0; i < b->inst.size(); ++i) {
        kvs_ctx* c = b->inst[i];
        const std::string who = "instance " + std::to_string(i) + ": ";
        if (!c->have_material || c->hetero) return bfail(b, KVS_ESTATE, who + "needs a uniform material");
        if (c->pml_cells > 0) return bfail(b, KVS_ESTATE, who + "absorbing layers are not batched");
        if (!c->have_dt) return bfail(b, KVS_ESTATE, who + "no time step set");
        if (c->step != b->step) return bfail(b, KVS_ESTATE, who + "stepped outside the batch");
        const int64_t n_env = (int64_t)c->env.size();
        for (int64_t n = b->step; n < std::min(b->step + nsteps, n_env); ++n)
            if (c->env[(size_t)n] != 0.0 && !c->fs_current)
                return bfail(b, KVS_ESTATE, who + "envelope on but no current projection");
    }
    BATCH_HIP(b, hipSetDevice(b->device));
    const int64_t np = (int64_t)b->probe_inst.size();
    if (np > 0 && b->trace_steps + nsteps > b->trace_cap) {
        const int64_t cap = std::max<int64_t>(b->trace_steps + nsteps, 2 * b->trace_cap);
        double* nb = nullptr;
        BATCH_HIP(b, b->mem.get(&nb, sizeof(double) * np * cap));
        if (b->traces && b->trace_steps > 0)
            BATCH_HIP(b, hipMemcpyAsync(nb, b->traces, sizeof(double) * np * b->trace_steps, hipMemcpyDeviceToDevice,
                                        b->stream));
        BATCH_HIP(b, hipStreamSynchronize(b->stream));
        dfree(b->mem, b->traces);
        b->traces = nb;
        b->trace_cap = cap;
        b->graph_valid = false;
    }
    BATCH_HIP(b, kvs_batch_prepare(b));
    int64_t flips = 0;
    BATCH_HIP(b, kvs_batch_run(b, nsteps, &flips));
    for (kvs_ctx* c : b->inst) {
        if (flips & 1) c->cur = 1 - c->cur;
        c->step += nsteps;
    }
    b->step += nsteps;
    if (np > 0) b->trace_steps += nsteps;
    b->host_traces_valid = false;
    return KVS_OK;
}

kvs_status kvs_batch_set_step_blocking(kvs_batch* b, int32_t steps) {
    if (!b) return KVS_EINVAL;
    if (steps != 1 && steps != 2) return bfail(b, KVS_EINVAL, "steps per launch must be 1 or 2");
    b->step_block = steps;
    b->graph_valid = false;
    return KVS_OK;
}

int32_t kvs_batch_step_blocking_applies(const kvs_batch* b) { return b && kvs_batch_two_step_supported(b) ? 1 : 0; }

kvs_status kvs_batch_set_persistent(kvs_batch* b, int32_t on) {
    if (!b) return KVS_EINVAL;
    b->small_ok = on != 0;
    b->graph_valid = false;
    return KVS_OK;
}

kvs_status kvs_batch_uses_persistent(const kvs_batch* b, int32_t* on) {
    if (!b || !on) return KVS_EINVAL;
    *on = kvs_batch_small_path(b) ? 1 : 0;
    return KVS_OK;
}

static void batch_retile(kvs_batch* b) {
    dfree(b->mem, b->dev_work);  // rebuilt for the new tile shape by the next prepare
    b->nwork = 0;
    b->graph_valid = false;
}

kvs_status kvs_batch_set_tuning(kvs_batch* b, int32_t variant, int32_t zchunk) {
    if (!b) return KVS_EINVAL;
    if ((variant < 0 || variant >= kvs_step_variant_count()) && variant != KVS_BATCH_FIT_ROWS)
        return bfail(b, KVS_EINVAL, "no such variant");
    if (zchunk < 1) return bfail(b, KVS_EINVAL, "zchunk < 1");
    b->variant = variant;
    b->zchunk = zchunk;
    batch_retile(b);
    return KVS_OK;
}

kvs_status kvs_batch_autotune(kvs_batch* b, int32_t trial_steps, int32_t* variant, int32_t* zchunk,
                              double* ms_per_launch, int32_t cap) {
    if (!b) return KVS_EINVAL;
    if (trial_steps < 1) return bfail(b, KVS_EINVAL, "trial_steps < 1");
    for (size_t i = 0; i < b->inst.size(); ++i) {
        kvs_ctx* c = b->inst[i];
        if (!c->have_material || c->hetero || !c->have_dt)
            return bfail(b, KVS_ESTATE, "instance " + std::to_string(i) + ": needs uniform material and dt");
    }
    BATCH_HIP(b, hipSetDevice(b->device));
    hipEvent_t e0, e1;
    BATCH_HIP(b, hipEventCreate(&e0));
    BATCH_HIP(b, hipEventCreate(&e1));
    const int nv = kvs_step_variant_count();
    const int zs[3] = {16, 32, 64};
    int best_v = b->variant, best_z = b->zchunk;
    double best = 1e300;
    hipError_t e = hipSuccess;
    // candidates: every variant for all instances, then the row-fitted tiling
    for (int vi = 0; vi <= nv && e == hipSuccess; ++vi) {
        const int v = vi < nv ? vi : KVS_BATCH_FIT_ROWS;
        double vbest = 1e300;
        for (int zi = 0; zi < 3 && e == hipSuccess; ++zi) {
            b->variant = v;
            b->zchunk = zs[zi];
            batch_retile(b);
            e = kvs_batch_prepare(b);
            if (e == hipSuccess) e = kvs_batch_trial_launch(b);
            if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
            for (int q = 0; q < trial_steps && e == hipSuccess; ++q) e = kvs_batch_trial_launch(b);
            if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            const double per = ms / trial_steps;
            vbest = std::min(vbest, per);
            if (e == hipSuccess && per < best) {
                best = per;
                best_v = v;
                best_z = zs[zi];
            }
        }
        if (ms_per_launch && vi < cap) ms_per_launch[vi] = vbest;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->variant = best_v;
    b->zchunk = best_z;
    batch_retile(b);
    if (e != hipSuccess) return bfail(b, KVS_EDEVICE, std::string("batch autotune: ") + hipGetErrorString(e));
    if (variant) *variant = best_v;
    if (zchunk) *zchunk = best_z;
    return KVS_OK;
}

kvs_status kvs_batch_reset(kvs_batch* b) {
    if (!b) return KVS_EINVAL;
    for (kvs_ctx* c : b->inst) {
        kvs_status s = kvs_reset_state(c);
        if (s != KVS_OK) return bfail(b, s, c->err);
    }
    b->step = 0;
    b->trace_steps = 0;
    b->host_traces_valid = false;
    return KVS_OK;
}

kvs_status kvs_batch_trace_count(const kvs_batch* b, int64_t* n) {
    if (!b || !n) return KVS_EINVAL;
    *n = b->trace_steps;
    return KVS_OK;
}

kvs_status kvs_batch_read_traces(kvs_batch* b, int32_t i, double* out, int64_t cap, int64_t* n_written) {
    if (!b) return KVS_EINVAL;
    if (!kvs_batch_instance(b, i)) return bfail(b, KVS_EINVAL, "instance out of range");
    if (cap < 0 || (cap > 0 && !out)) return bfail(b, KVS_EINVAL, "bad output buffer");
    const int64_t np = (int64_t)b->probe_inst.size();
    const int64_t p0 = b->probe_first[(size_t)i], p1 = b->probe_first[(size_t)i + 1];
    const int64_t per = p1 - p0;
    const int64_t rows = per > 0 ? std::min<int64_t>(b->trace_steps, cap / per) : 0;
    if (!b->host_traces_valid) {
        // one contiguous copy of every instance's traces; later calls slice it
        b->host_traces.resize((size_t)(np * b->trace_steps));
        if (!b->host_traces.empty())
            BATCH_HIP(b, hipMemcpyAsync(b->host_traces.data(), b->traces, sizeof(double) * b->host_traces.size(),
                                        hipMemcpyDeviceToHost, b->stream));
        BATCH_HIP(b, hipStreamSynchronize(b->stream));
        b->host_traces_valid = true;
    }
    for (int64_t r = 0; r < rows; ++r)
        std::copy_n(b->host_traces.data() + r * np + p0, per, out + r * per);
    const int64_t w = rows * per;
    if (n_written) *n_written = w;
    return KVS_OK;
}

}  // extern "C"
