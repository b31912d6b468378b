// FDTD step of the reduced Kelvin-Voigt shear equation on gfx950, plus the
// small per-cell helper kernels (material casts, dt^2/rho, stable dt,
// probe gather).
//
// Update (Sec. 3.1 leapfrog in summed form, Sec. 3.3 separable source,
// Sec. 3.5 Dirichlet layer), per interior cell and component c:
//   acc = div(G grad u_c) + (eta/dt) lap(w_c) + g_n f_S,c
//   w'  = a1 w_c + a2 acc,  a1 = (1-s)/(1+s), a2 = (dt^2/rho)/(1+s)
//   u'  = u_c + w'
// with s = sigma dt / 2 from the linear sponge ramp and harmonic face moduli.
//
// Kernel layout ("2.5-D" blocking).  A block of 64 x BY threads owns a 64 x BY
// column tile in the xy plane and marches over a chunk of z planes.  One
// 64-lane wavefront covers one 64-cell x row, so every global access is one
// fully coalesced 256 B (fp32) row segment.  Per plane the block stages the
// fields that are needed at xy neighbours (u, plus w when eta != 0, plus G
// when heterogeneous) in LDS with a one-cell halo; z neighbours live in a
// per-thread register queue (k-1, k, k+1, with k+2 prefetched).  Each cell's
// state is therefore read from HBM once per step; halo rows of adjacent tiles
// are served by L2 because tiles are issued XCD-contiguously (see tile_of).
#include "kvs_internal.hpp"

namespace {

template <typename T>
struct StepArgs {
    const T* u;     // [3][N] current u^n
    const T* w;     // [3][N] current w^n
    T* un;          // [3][N] u^{n+1}
    T* wn;          // [3][N] w^{n+1}
    const T* G;     // [N] (heterogeneous)
    const T* eta;   // [N] (heterogeneous)
    const T* crho;  // [N] dt^2/rho (heterogeneous)
    const T* FS;    // [3][N] projected force (when gn != 0)
    long long N;
    int nx, ny, nz;
    int gx, gy, gz;  // tiles per axis
    int kchunk;
    int L;           // sponge cells
    T invL;
    T ihx2, ihy2, ihz2;
    T G0, eta_dt0, crho0;  // homogeneous medium
    T inv_dt;
    T gn;
    T half_dt_smax;  // sigma_max * dt / 2
};

template <typename T>
__device__ __forceinline__ T harm(T a, T b);
template <>
__device__ __forceinline__ float harm<float>(float a, float b) {
    return 2.0f * a * b * __builtin_amdgcn_rcpf(a + b);
}
template <>
__device__ __forceinline__ double harm<double>(double a, double b) {
    return 2.0 * a * b / (a + b);
}

template <typename T>
__device__ __forceinline__ T recip(T x);
template <>
__device__ __forceinline__ float recip<float>(float x) {
    return 1.0f / x;
}
template <>
__device__ __forceinline__ double recip<double>(double x) {
    return 1.0 / x;
}

template <typename T>
__device__ __forceinline__ T ramp(int idx, int n, int L, T invL) {
    const int d = min(idx, n - 1 - idx);
    return d < L ? T(L - d) * invL : T(0);
}

// Tiles are numbered bx fastest, then by, then bz.  Hardware hands block b to
// XCD b % 8; remapping so that each XCD receives a contiguous range of tile
// numbers keeps y-adjacent tiles (which share halo rows) in the same L2.
__device__ __forceinline__ int tile_of(int b, int B) {
    const int xcd = b & 7, pos = b >> 3;
    const int per = B >> 3, rem = B & 7;
    return xcd * per + min(xcd, rem) + pos;
}

template <typename T, bool HET, bool VISC, bool FORCE, int BY>
__global__ __launch_bounds__(64 * BY) void step_kernel(const StepArgs<T> a) {
    static_assert(BY >= 2, "tile needs at least two rows");
    constexpr int NQ = 3 + (VISC ? 3 : 0) + (HET ? 1 : 0);
    constexpr int QG = VISC ? 6 : 3;
    __shared__ T lds[NQ][BY + 2][66];

    const int tx = threadIdx.x, ty = threadIdx.y;
    const int B = a.gx * a.gy * a.gz;
    const int t = tile_of(blockIdx.x, B);
    const int bx = t % a.gx;
    const int by = (t / a.gx) % a.gy;
    const int bz = t / (a.gx * a.gy);

    const int i = bx * 64 + tx;
    const int j = by * BY + ty;
    const int kb = 1 + bz * a.kchunk;
    const int ke = min(a.nz - 1, kb + a.kchunk);  // planes kb .. ke-1
    const bool in_x = i < a.nx, in_y = j < a.ny;
    const bool inb = in_x && in_y;
    const bool act = i >= 1 && i <= a.nx - 2 && j >= 1 && j <= a.ny - 2;
    const int sxy = a.nx * a.ny;
    const int col = inb ? i + a.nx * j : 0;

    const T* fp[NQ];
    fp[0] = a.u;
    fp[1] = a.u + a.N;
    fp[2] = a.u + 2 * a.N;
    if constexpr (VISC) {
        fp[3] = a.w;
        fp[4] = a.w + a.N;
        fp[5] = a.w + 2 * a.N;
    }
    if constexpr (HET) fp[QG] = a.G;

    // halo roles: first/last tile row loads the row below/above, first/last
    // lane loads the column left/right
    const bool hyl = in_x && ((ty == 0 && j >= 1) || (ty == BY - 1 && j + 1 < a.ny));
    const int hy_off = ty == 0 ? col - a.nx : col + a.nx;
    const int hy_row = ty == 0 ? 0 : BY + 1;
    const bool hxl = in_y && ((tx == 0 && i >= 1) || (tx == 63 && i + 1 < a.nx));
    const int hx_off = tx == 0 ? col - 1 : col + 1;
    const int hx_col = tx == 0 ? 0 : 65;

    T zm[NQ], zc[NQ], zp[NQ], zn[NQ], hyc[NQ], hyn[NQ], hxc[NQ], hxn[NQ];
#pragma unroll
    for (int f = 0; f < NQ; ++f) {
        zm[f] = inb ? fp[f][(kb - 1) * sxy + col] : T(0);
        zc[f] = inb ? fp[f][kb * sxy + col] : T(0);
        zp[f] = inb ? fp[f][(kb + 1) * sxy + col] : T(0);
        zn[f] = T(0);
        hyc[f] = hyl ? fp[f][kb * sxy + hy_off] : T(0);
        hxc[f] = hxl ? fp[f][kb * sxy + hx_off] : T(0);
        hyn[f] = T(0);
        hxn[f] = T(0);
    }

    T rxy = T(0);
    if (a.L > 0 && act) rxy = max(ramp<T>(i, a.nx, a.L, a.invL), ramp<T>(j, a.ny, a.L, a.invL));

    for (int k = kb; k < ke; ++k) {
        // prefetch centre values of plane k+2 and halos of plane k+1
        if (k + 2 <= ke && inb) {
#pragma unroll
            for (int f = 0; f < NQ; ++f) zn[f] = fp[f][(k + 2) * sxy + col];
        }
        if (k + 1 < ke) {
            if (hyl) {
#pragma unroll
                for (int f = 0; f < NQ; ++f) hyn[f] = fp[f][(k + 1) * sxy + hy_off];
            }
            if (hxl) {
#pragma unroll
                for (int f = 0; f < NQ; ++f) hxn[f] = fp[f][(k + 1) * sxy + hx_off];
            }
        }
        const int idx = k * sxy + col;
        // per-cell values used only here
        T wc_own[3] = {T(0), T(0), T(0)};
        T fsv[3] = {T(0), T(0), T(0)};
        T crho_c = a.crho0, eta_dt = a.eta_dt0;
        if (act) {
            if constexpr (!VISC) {
#pragma unroll
                for (int c = 0; c < 3; ++c) wc_own[c] = a.w[c * a.N + idx];
            }
            if constexpr (FORCE) {
#pragma unroll
                for (int c = 0; c < 3; ++c) fsv[c] = __builtin_nontemporal_load(a.FS + c * a.N + idx);
            }
            if constexpr (HET) {
                crho_c = __builtin_nontemporal_load(a.crho + idx);
                if constexpr (VISC) eta_dt = __builtin_nontemporal_load(a.eta + idx) * a.inv_dt;
            }
        }

        __syncthreads();  // previous plane fully consumed
#pragma unroll
        for (int f = 0; f < NQ; ++f) {
            lds[f][ty + 1][tx + 1] = zc[f];
            if (hyl) lds[f][hy_row][tx + 1] = hyc[f];
            if (hxl) lds[f][ty + 1][hx_col] = hxc[f];
        }
        __syncthreads();

        if (act) {
            T a1 = T(1), a2 = crho_c;
            if (a.L > 0) {
                const T s = a.half_dt_smax * max(rxy, ramp<T>(k, a.nz, a.L, a.invL));
                if (s > T(0)) {
                    const T inv = recip<T>(T(1) + s);
                    a1 = (T(1) - s) * inv;
                    a2 = crho_c * inv;
                }
            }
            T gxm, gxp, gym, gyp, gzm, gzp;
            if constexpr (HET) {
                const T Gc = zc[QG];
                gxm = harm<T>(Gc, lds[QG][ty + 1][tx]) * a.ihx2;
                gxp = harm<T>(Gc, lds[QG][ty + 1][tx + 2]) * a.ihx2;
                gym = harm<T>(Gc, lds[QG][ty][tx + 1]) * a.ihy2;
                gyp = harm<T>(Gc, lds[QG][ty + 2][tx + 1]) * a.ihy2;
                gzm = harm<T>(Gc, zm[QG]) * a.ihz2;
                gzp = harm<T>(Gc, zp[QG]) * a.ihz2;
            } else {
                gxm = gxp = a.G0 * a.ihx2;
                gym = gyp = a.G0 * a.ihy2;
                gzm = gzp = a.G0 * a.ihz2;
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T uc = zc[c];
                T acc = gxp * (lds[c][ty + 1][tx + 2] - uc) - gxm * (uc - lds[c][ty + 1][tx])
                      + gyp * (lds[c][ty + 2][tx + 1] - uc) - gym * (uc - lds[c][ty][tx + 1])
                      + gzp * (zp[c] - uc) - gzm * (uc - zm[c]);
                T wc;
                if constexpr (VISC) {
                    wc = zc[3 + c];
                    const T lw = (lds[3 + c][ty + 1][tx + 2] + lds[3 + c][ty + 1][tx] - T(2) * wc) * a.ihx2
                               + (lds[3 + c][ty + 2][tx + 1] + lds[3 + c][ty][tx + 1] - T(2) * wc) * a.ihy2
                               + (zp[3 + c] + zm[3 + c] - T(2) * wc) * a.ihz2;
                    acc += eta_dt * lw;
                } else {
                    wc = wc_own[c];
                }
                if constexpr (FORCE) acc += a.gn * fsv[c];
                const T wnew = a1 * wc + a2 * acc;
                __builtin_nontemporal_store(wnew, a.wn + c * a.N + idx);
                __builtin_nontemporal_store(uc + wnew, a.un + c * a.N + idx);
            }
        }
#pragma unroll
        for (int f = 0; f < NQ; ++f) {
            zm[f] = zc[f];
            zc[f] = zp[f];
            zp[f] = zn[f];
            hyc[f] = hyn[f];
            hxc[f] = hxn[f];
        }
    }
}

constexpr int kBY = 4;

template <typename T, bool HET, bool VISC, bool FORCE>
hipError_t launch_typed(kvs_ctx* c, const StepArgs<T>& a, int blocks) {
    hipLaunchKernelGGL((step_kernel<T, HET, VISC, FORCE, kBY>), dim3(blocks), dim3(64, kBY), 0, c->stream, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_step_t(kvs_ctx* c, double gn) {
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
    a.kchunk = (int)std::min<int64_t>(g.nz - 2, 32);
    a.gx = (a.nx + 63) / 64;
    a.gy = (a.ny + kBY - 1) / kBY;
    a.gz = (a.nz - 2 + a.kchunk - 1) / a.kchunk;
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
    const int blocks = a.gx * a.gy * a.gz;
    const bool F = gn != 0.0;
    if (c->hetero) {
        if (c->viscous) return F ? launch_typed<T, true, true, true>(c, a, blocks) : launch_typed<T, true, true, false>(c, a, blocks);
        return F ? launch_typed<T, true, false, true>(c, a, blocks) : launch_typed<T, true, false, false>(c, a, blocks);
    }
    if (c->viscous) return F ? launch_typed<T, false, true, true>(c, a, blocks) : launch_typed<T, false, true, false>(c, a, blocks);
    return F ? launch_typed<T, false, false, true>(c, a, blocks) : launch_typed<T, false, false, false>(c, a, blocks);
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
    return c->prec == KVS_FP32 ? launch_step_t<float>(c, gn) : launch_step_t<double>(c, gn);
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
