// FDTD step kernel of one context (tile code in kvs_step_tile.hpp), its
// launch shapes, and the small per-cell helper kernels (material casts,
// dt^2/rho, stable dt, probe gather).
#include <hip/hip_ext.h>

#include "kvs_step_tile.hpp"

namespace {

// One context: tile from the block index (XCD-contiguous order when remap).
template <typename T, bool HET, bool VISC, bool FORCE, int BY, int VEC, int WX, int WPE>
__global__ __launch_bounds__(64 * WX * BY) __attribute__((amdgpu_waves_per_eu(WPE))) void step_kernel(
    const StepArgs<T> a) {
    if ((int)blockIdx.x < a.pblocks) {
        const long long p = (long long)blockIdx.x * (64 * WX * BY) + threadIdx.y * (64 * WX) + threadIdx.x;
        if (p < a.np) {
            const long long q = a.pcells[p];
            if (a.pcomp == 3) {
                a.pout[3 * p] = (double)a.u[q];
                a.pout[3 * p + 1] = (double)a.u[a.N + q];
                a.pout[3 * p + 2] = (double)a.u[2 * a.N + q];
            } else {
                a.pout[p] = (double)a.u[a.pcomp * a.N + q];
            }
        }
        return;
    }
    const int B = a.gx * a.gy * a.gz;
    const int b = (int)blockIdx.x - a.pblocks;
    const int t = a.remap ? tile_of(b, B) : b;
    step_tile<T, HET, VISC, FORCE, BY, VEC, WX>(a, t % a.gx, (t / a.gx) % a.gy, t / (a.gx * a.gy));
}

template <typename T, bool HET, bool VISC, bool FORCE, int BY, int VEC, int WX, int WPE = 1>
hipError_t launch_shape(kvs_ctx* c, StepArgs<T> a) {
    auto kern = step_kernel<T, HET, VISC, FORCE, BY, VEC, WX, WPE>;
    static const int cap = resident_blocks(kern, 64 * WX * BY);  // one value per instantiation
    a.gx = (a.nx + 64 * WX * VEC - 1) / (64 * WX * VEC);
    a.gy = (a.ny + BY - 1) / BY;
    a.kchunk = c->step_zchunk > 0 ? std::min(c->step_zchunk, a.nz - 2) : choose_kchunk(a.gx * a.gy, a.nz - 2, cap);
    a.gz = (a.nz - 2 + a.kchunk - 1) / a.kchunk;
    a.pblocks = a.pout ? (int)((a.np + 64 * WX * BY - 1) / (64 * WX * BY)) : 0;
    const int blocks = a.gx * a.gy * a.gz + a.pblocks;
    if (c->launch_ev[0])
        hipExtLaunchKernelGGL(kern, dim3(blocks), dim3(64 * WX, BY), 0, c->stream, c->launch_ev[0],
                              c->launch_ev[1], 0, a);
    else
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * WX, BY), 0, c->stream, a);
    return hipGetLastError();
}

template <typename T, bool HET, bool VISC, bool FORCE>
hipError_t launch_typed(kvs_ctx* c, const StepArgs<T>& a, int variant) {
    const int v = effective_variant(variant, sizeof(T) == 8, (a.nx % 2) != 0);
    if constexpr (sizeof(T) == 8) {
        switch (v) {
            case 1: return launch_shape<T, HET, VISC, FORCE, 8, 1, 1>(c, a);
            case 5: return launch_shape<T, HET, VISC, FORCE, 4, 1, 2>(c, a);
            default: return launch_shape<T, HET, VISC, FORCE, 4, 1, 1>(c, a);
        }
    } else {
        switch (v) {
            case 1: return launch_shape<T, HET, VISC, FORCE, 8, 1, 1>(c, a);
            case 2: return launch_shape<T, HET, VISC, FORCE, 4, 2, 1>(c, a);
            case 3: return launch_shape<T, HET, VISC, FORCE, 8, 2, 1>(c, a);
            case 4: return launch_shape<T, HET, VISC, FORCE, 16, 1, 1>(c, a);
            case 5: return launch_shape<T, HET, VISC, FORCE, 4, 1, 2>(c, a);
            case 6: return launch_shape<T, HET, VISC, FORCE, 8, 1, 2>(c, a);
            case 7: return launch_shape<T, HET, VISC, FORCE, 4, 1, 4>(c, a);
            default: return launch_shape<T, HET, VISC, FORCE, 4, 1, 1>(c, a);
        }
    }
}

template <typename T>
hipError_t launch_step_t(kvs_ctx* c, double gn, int variant) {
    const kvs_grid& g = c->grid;
    StepArgs<T> a{};
    const int nb = 1 - c->cur;
    a.u = static_cast<const T*>(c->u[c->cur]);
    a.w = static_cast<const T*>(c->w[c->cur]);
    a.un = static_cast<T*>(c->u[nb]);
    a.wn = static_cast<T*>(c->w[nb]);
    a.G = static_cast<const T*>(c->G);
    a.eta = static_cast<const T*>(c->eta);
    a.crho = static_cast<const T*>(c->crho);
    a.FS = static_cast<const T*>(c->FS);
    a.N = c->N;
    a.nx = (int)g.nx;
    a.ny = (int)g.ny;
    a.nz = (int)g.nz;
    a.L = c->sponge_cells;
    a.invL = a.L > 0 ? T(1.0 / a.L) : T(0);
    a.ihx2 = T(1.0 / (g.hx * g.hx));
    a.ihy2 = T(1.0 / (g.hy * g.hy));
    a.ihz2 = T(1.0 / (g.hz * g.hz));
    a.G0 = T(c->G0);
    a.eta_dt0 = T(c->eta0 / c->dt);
    a.crho0 = T(c->dt * c->dt / c->rho0);
    a.inv_dt = T(1.0 / c->dt);
    a.gn = T(gn);
    a.half_dt_smax = T(0.5 * c->sigma_max * c->dt);
    a.remap = c->step_remap;
    if (c->probe_fused_out) {
        a.pcells = reinterpret_cast<const long long*>(c->probe_cells);
        a.pout = c->probe_fused_out;
        a.np = c->nprobes;
        a.pcomp = c->probe_comp;
    }
    const bool F = gn != 0.0;
    if (c->hetero) {
        if (c->viscous)
            return F ? launch_typed<T, true, true, true>(c, a, variant) : launch_typed<T, true, true, false>(c, a, variant);
        return F ? launch_typed<T, true, false, true>(c, a, variant) : launch_typed<T, true, false, false>(c, a, variant);
    }
    if (c->viscous)
        return F ? launch_typed<T, false, true, true>(c, a, variant) : launch_typed<T, false, true, false>(c, a, variant);
    return F ? launch_typed<T, false, false, true>(c, a, variant) : launch_typed<T, false, false, false>(c, a, variant);
}

// ---- helpers ---------------------------------------------------------------

template <typename T>
__global__ void probe_kernel(const T* u, long long N, const int64_t* cells, int64_t np, int comp, double* out) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const long long cidx = cells[p];
    if (comp == 3) {
        out[3 * p + 0] = (double)u[cidx];
        out[3 * p + 1] = (double)u[N + cidx];
        out[3 * p + 2] = (double)u[2 * N + cidx];
    } else {
        out[p] = (double)u[comp * N + cidx];
    }
}

template <typename T>
__global__ void cast_kernel(const double* src, T* dst, int64_t n) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        dst[q] = (T)src[q];
}

template <typename T>
__global__ void widen_kernel(const T* src, double* dst, int64_t n) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        dst[q] = (double)src[q];
}

// material: G, eta, rho cast to T
template <typename T>
__global__ void material_kernel(const double* G, const double* rho, const double* eta, T* Gt, T* etat, T* rhot,
                                int64_t n) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        Gt[q] = (T)G[q];
        etat[q] = (T)eta[q];
        rhot[q] = (T)rho[q];
    }
}

// crho = dt^2 / rho, formed in double (dt * dt / rho) and rounded once to T
template <typename T>
__global__ void crho_kernel(const T* rho, T* crho, double dt, int64_t n) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        crho[q] = (T)(dt * dt / (double)rho[q]);
}

template <typename T>
__global__ void zero_boundary_kernel(T* f, int nx, int ny, int nz, long long N) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    const int i = (int)(q % nx), j = (int)((q / nx) % ny), k = (int)(q / ((long long)nx * ny));
    if (i == 0 || i == nx - 1 || j == 0 || j == ny - 1 || k == 0 || k == nz - 1) {
        f[q] = T(0);
        f[N + q] = T(0);
        f[2 * N + q] = T(0);
    }
}

__device__ __forceinline__ double hm64(double a, double b) { return 2.0 * a * b / (a + b); }

// Per interior cell: positive root of (Gmax/rho) S dt^2 + 2 (eta/rho) S dt = 1
// (A + 2B = 4); block minima of that bound and block maxima of sqrt(G/rho).
__global__ void stable_dt_kernel(const double* G, const double* rho, const double* eta, int nx, int ny, int nz,
                                 double S, double* part_dt, double* part_c) {
    __shared__ double sd[256], sc[256];
    const long long N = (long long)nx * ny * nz;
    double best = INFINITY, cmax = 0.0;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < N; q += (long long)gridDim.x * blockDim.x) {
        cmax = fmax(cmax, sqrt(G[q] / rho[q]));
        const int i = (int)(q % nx), j = (int)((q / nx) % ny), k = (int)(q / ((long long)nx * ny));
        if (i < 1 || i > nx - 2 || j < 1 || j > ny - 2 || k < 1 || k > nz - 2) continue;
        const long long st[3] = {1, nx, (long long)nx * ny};
        double gmax = 0.0;
        for (int ax = 0; ax < 3; ++ax) {
            gmax = fmax(gmax, hm64(G[q], G[q + st[ax]]));
            gmax = fmax(gmax, hm64(G[q], G[q - st[ax]]));
        }
        const double qa = gmax / rho[q] * S;
        const double qb = 2.0 * eta[q] / rho[q] * S;
        best = fmin(best, (-qb + sqrt(qb * qb + 4.0 * qa)) / (2.0 * qa));
    }
    sd[threadIdx.x] = best;
    sc[threadIdx.x] = cmax;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sd[threadIdx.x] = fmin(sd[threadIdx.x], sd[threadIdx.x + o]);
            sc[threadIdx.x] = fmax(sc[threadIdx.x], sc[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part_dt[blockIdx.x] = sd[0];
        part_c[blockIdx.x] = sc[0];
    }
}

__global__ void minmax_finalize_kernel(const double* part_dt, const double* part_c, int n, double* out) {
    __shared__ double sd[256], sc[256];
    double best = INFINITY, cmax = 0.0;
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
        best = fmin(best, part_dt[q]);
        cmax = fmax(cmax, part_c[q]);
    }
    sd[threadIdx.x] = best;
    sc[threadIdx.x] = cmax;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sd[threadIdx.x] = fmin(sd[threadIdx.x], sd[threadIdx.x + o]);
            sc[threadIdx.x] = fmax(sc[threadIdx.x], sc[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sd[0];
        out[1] = sc[0];
    }
}

int grid_blocks(int64_t n) { return (int)std::min<int64_t>((n + 255) / 256, 8192); }

}  // namespace

hipError_t kvs_launch_step(kvs_ctx* c, double gn) {
    return kvs_launch_step_variant(c, gn, c->step_variant);
}

hipError_t kvs_launch_step_variant(kvs_ctx* c, double gn, int variant) {
    if (variant < 0 || variant >= kNumVariants) variant = 0;
    return c->prec == KVS_FP32 ? launch_step_t<float>(c, gn, variant) : launch_step_t<double>(c, gn, variant);
}

int kvs_step_variant_count() { return kNumVariants; }

void kvs_step_variant_shape(int variant, int* by, int* vec, int* wx) {
    if (variant < 0 || variant >= kNumVariants) variant = 0;
    *by = kVariants[variant].by;
    *vec = kVariants[variant].vec;
    *wx = kVariants[variant].wx;
}

hipError_t kvs_launch_probe_gather(kvs_ctx* c, const void* u_new, int64_t slot) {
    if (c->nprobes == 0) return hipSuccess;
    const int nc = ncomp_of(c->probe_comp);
    double* out = c->traces + slot * c->nprobes * nc;
    const int blocks = (int)((c->nprobes + 255) / 256);
    if (c->prec == KVS_FP32)
        hipLaunchKernelGGL(probe_kernel<float>, dim3(blocks), dim3(256), 0, c->stream, static_cast<const float*>(u_new),
                           (long long)c->N, c->probe_cells, c->nprobes, c->probe_comp, out);
    else
        hipLaunchKernelGGL(probe_kernel<double>, dim3(blocks), dim3(256), 0, c->stream,
                           static_cast<const double*>(u_new), (long long)c->N, c->probe_cells, c->nprobes,
                           c->probe_comp, out);
    return hipGetLastError();
}

hipError_t kvs_launch_cast_material(kvs_ctx* c, const double* dG, const double* drho, const double* deta) {
    const int b = grid_blocks(c->N);
    if (c->prec == KVS_FP32)
        hipLaunchKernelGGL(material_kernel<float>, dim3(b), dim3(256), 0, c->stream, dG, drho, deta,
                           static_cast<float*>(c->G), static_cast<float*>(c->eta), static_cast<float*>(c->rho_t), c->N);
    else
        hipLaunchKernelGGL(material_kernel<double>, dim3(b), dim3(256), 0, c->stream, dG, drho, deta,
                           static_cast<double*>(c->G), static_cast<double*>(c->eta), static_cast<double*>(c->rho_t),
                           c->N);
    return hipGetLastError();
}

hipError_t kvs_launch_crho(kvs_ctx* c) {
    if (!c->hetero) return hipSuccess;
    const int b = grid_blocks(c->N);
    if (c->prec == KVS_FP32)
        hipLaunchKernelGGL(crho_kernel<float>, dim3(b), dim3(256), 0, c->stream, static_cast<const float*>(c->rho_t),
                           static_cast<float*>(c->crho), c->dt, c->N);
    else
        hipLaunchKernelGGL(crho_kernel<double>, dim3(b), dim3(256), 0, c->stream, static_cast<const double*>(c->rho_t),
                           static_cast<double*>(c->crho), c->dt, c->N);
    return hipGetLastError();
}

hipError_t kvs_launch_cast(kvs_ctx* c, const double* src, void* dst, int64_t n) {
    const int b = grid_blocks(n);
    if (c->prec == KVS_FP32)
        hipLaunchKernelGGL(cast_kernel<float>, dim3(b), dim3(256), 0, c->stream, src, static_cast<float*>(dst), n);
    else
        hipLaunchKernelGGL(cast_kernel<double>, dim3(b), dim3(256), 0, c->stream, src, static_cast<double*>(dst), n);
    return hipGetLastError();
}

hipError_t kvs_launch_widen(kvs_ctx* c, const void* src, double* dst, int64_t n) {
    const int b = grid_blocks(n);
    if (c->prec == KVS_FP32)
        hipLaunchKernelGGL(widen_kernel<float>, dim3(b), dim3(256), 0, c->stream, static_cast<const float*>(src), dst, n);
    else
        hipLaunchKernelGGL(widen_kernel<double>, dim3(b), dim3(256), 0, c->stream, static_cast<const double*>(src), dst,
                           n);
    return hipGetLastError();
}

hipError_t kvs_launch_f32_to_f64(kvs_ctx* c, const float* src, double* dst, int64_t n) {
    const int b = grid_blocks(n);
    hipLaunchKernelGGL(widen_kernel<float>, dim3(b), dim3(256), 0, c->stream, src, dst, n);
    return hipGetLastError();
}

hipError_t kvs_launch_zero_boundary(kvs_ctx* c, void* field3) {
    const int b = (int)((c->N + 255) / 256);
    const kvs_grid& g = c->grid;
    if (c->prec == KVS_FP32)
        hipLaunchKernelGGL(zero_boundary_kernel<float>, dim3(b), dim3(256), 0, c->stream, static_cast<float*>(field3),
                           (int)g.nx, (int)g.ny, (int)g.nz, (long long)c->N);
    else
        hipLaunchKernelGGL(zero_boundary_kernel<double>, dim3(b), dim3(256), 0, c->stream,
                           static_cast<double*>(field3), (int)g.nx, (int)g.ny, (int)g.nz, (long long)c->N);
    return hipGetLastError();
}

hipError_t kvs_launch_stable_dt(kvs_ctx* c, const double* dG, const double* drho, const double* deta, double* partial,
                                int64_t npartial, double* out) {
    const kvs_grid& g = c->grid;
    const double S = 1.0 / (g.hx * g.hx) + 1.0 / (g.hy * g.hy) + 1.0 / (g.hz * g.hz);
    const int nb = (int)std::min<int64_t>(npartial / 2, 1024);
    hipLaunchKernelGGL(stable_dt_kernel, dim3(nb), dim3(256), 0, c->stream, dG, drho, deta, (int)g.nx, (int)g.ny,
                       (int)g.nz, S, partial, partial + nb);
    hipLaunchKernelGGL(minmax_finalize_kernel, dim3(1), dim3(256), 0, c->stream, partial, partial + nb, nb, out);
    return hipGetLastError();
}
