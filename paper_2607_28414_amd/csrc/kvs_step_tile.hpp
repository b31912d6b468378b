// The FDTD step's per-tile code, shared by the single-context step kernel
// and the batched step kernel, and the table of tile shapes.
//
// Update (Sec. 3.1 leapfrog in summed form, Sec. 3.3 separable source,
// Sec. 3.5 Dirichlet layer), per interior cell and component c:
//   acc = div(G grad u_c) + (eta/dt) lap(w_c) + g_n f_S,c
//   w'  = a1 w_c + a2 acc,  a1 = (1-s)/(1+s), a2 = (dt^2/rho)/(1+s)
//   u'  = u_c + w'
// with s = sigma dt / 2 from the linear sponge ramp and harmonic face moduli.
//
// Kernel layout ("2.5-D" blocking).  A block of 64 WX x BY threads owns a
// TX x BY column tile in the xy plane (TX = 64 WX VEC) and marches over a
// chunk of z planes.  One 64-lane wavefront covers 64 VEC consecutive cells of
// an x row, so every global access is a fully coalesced row segment; WX > 1
// puts several wavefronts side by side on a row, which spreads the two x-halo
// columns over a wider tile without more registers per lane.  Per plane the block stages the
// fields that are needed at xy neighbours (u, plus w when eta != 0, plus G
// when heterogeneous) in LDS with a one-cell halo; z neighbours live in a
// per-thread register queue (k-1, k, k+1, with k+2 prefetched).  Each cell's
// state is therefore read from HBM once per step; halo rows of adjacent tiles
// are served by L2 because tiles are issued XCD-contiguously (see tile_of).
#pragma once

#include "kvs_internal.hpp"
#include "kvs_tiling.hpp"

namespace {

using kvs_tiling::choose_kchunk;
using kvs_tiling::lds_barrier;
using kvs_tiling::resident_blocks;
using kvs_tiling::tile_of;

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
    int remap;       // 1: XCD-contiguous tile order
    // probe blocks: the first pblocks blocks of a launch copy the input state
    // (the previous step's result) at the probe cells into pout (probe p of
    // component pcomp at pout[p], or all components at pout[3 p + c]); the
    // remaining blocks are the tiles
    const long long* pcells;
    double* pout;
    long long np;
    int pcomp, pblocks;
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
__device__ __forceinline__ T ramp(int idx, int n, int L, T invL) {
    const int d = min(idx, n - 1 - idx);
    return d < L ? T(L - d) * invL : T(0);
}

template <typename T>
__device__ __forceinline__ T rcp_fast(T x);
template <>
__device__ __forceinline__ float rcp_fast<float>(float x) {
    return __builtin_amdgcn_rcpf(x);
}
template <>
__device__ __forceinline__ double rcp_fast<double>(double x) {
    return 1.0 / x;
}

// Vector of VEC consecutive x cells held by one lane.
template <typename T, int V>
struct VecT {
    typedef T type __attribute__((ext_vector_type(V)));
};
template <typename T>
struct VecT<T, 1> {
    typedef T type;
};

template <typename T, int V>
__device__ __forceinline__ void vload(const T* p, T (&o)[V]) {
    if constexpr (V == 1) {
        o[0] = *p;
    } else {
        const typename VecT<T, V>::type x = *reinterpret_cast<const typename VecT<T, V>::type*>(p);
#pragma unroll
        for (int v = 0; v < V; ++v) o[v] = x[v];
    }
}

template <typename T, int V>
__device__ __forceinline__ void vload_nt(const T* p, T (&o)[V]) {
    if constexpr (V == 1) {
        o[0] = __builtin_nontemporal_load(p);
    } else {
        const typename VecT<T, V>::type x =
            __builtin_nontemporal_load(reinterpret_cast<const typename VecT<T, V>::type*>(p));
#pragma unroll
        for (int v = 0; v < V; ++v) o[v] = x[v];
    }
}

template <typename T, int V>
__device__ __forceinline__ void vstore_nt(T* p, const T (&a)[V]) {
    if constexpr (V == 1) {
        __builtin_nontemporal_store(a[0], p);
    } else {
        typename VecT<T, V>::type x;
#pragma unroll
        for (int v = 0; v < V; ++v) x[v] = a[v];
        __builtin_nontemporal_store(x, reinterpret_cast<typename VecT<T, V>::type*>(p));
    }
}

template <typename T, int V>
__device__ __forceinline__ void vlds_write(T* p, const T (&a)[V]) {
    if constexpr (V == 1) {
        *p = a[0];
    } else {
        typename VecT<T, V>::type x;
#pragma unroll
        for (int v = 0; v < V; ++v) x[v] = a[v];
        *reinterpret_cast<typename VecT<T, V>::type*>(p) = x;
    }
}

// The loop body is straight-line on purpose: every lane issues every load
// (addresses clamped in bounds), writes LDS unconditionally (lanes without
// halo work into a dummy row) and stores unconditionally (values of cells
// that are not interior are 0, written into boundary cells that hold 0).
// Branch-free memory code lets the compiler count outstanding loads exactly,
// so the plane-ahead prefetch stays in flight across the barrier instead of
// being drained every plane.
//
// A lane owns VEC consecutive x cells (one dword or dwordx2 access per
// field); WX wavefronts cover TX = 64 WX VEC cells of one x row, a block BY
// rows.
// LDS row layout: [pad][left halo][TX cells][right halo][pad], so that every
// lane's VEC-wide write is naturally aligned, including the halo writes.
template <typename T, bool HET, bool VISC, bool FORCE, int BY, int VEC, int WX>
__device__ __forceinline__ void step_tile(const StepArgs<T>& a, int bx, int by, int bz) {
    static_assert(BY >= 3 && 2 * BY <= 64, "halo lane assignment needs 3 <= BY <= 32");
    static_assert(64 * WX * BY <= 1024, "at most 1024 threads per block");
    constexpr int NQ = 3 + (VISC ? 3 : 0) + (HET ? 1 : 0);
    constexpr int QG = VISC ? 6 : 3;
    constexpr int TX = 64 * WX * VEC;
    constexpr int W = TX + 4;
    constexpr int DUMMY = BY + 2;
    __shared__ T lds[2][NQ][BY + 3][W];

    const int tx = threadIdx.x, ty = threadIdx.y;
    const int nx = a.nx, ny = a.ny;
    const int i0 = bx * TX + VEC * tx;  // first of this lane's cells
    const int j = by * BY + ty;
    const int kb = 1 + bz * a.kchunk;
    const int ke = min(a.nz - 1, kb + a.kchunk);  // planes kb .. ke-1
    const bool inb = i0 < nx && j < ny;          // VEC > 1 needs nx % VEC == 0
    bool act[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) act[v] = i0 + v >= 1 && i0 + v <= nx - 2 && j >= 1 && j <= ny - 2;
    const int sxy = nx * ny;
    const int col = inb ? i0 + nx * j : 0;
    // store column: the lane's own cells; lanes outside the grid store zeros
    // into boundary row ny-1
    const int scol = inb ? col : min(i0, nx - VEC) + nx * (ny - 1);
    const int lcol = 2 + VEC * tx;  // LDS column of the lane's first cell

    // one halo slot per lane: wave 0 loads the row below the tile, wave BY-1
    // the row above, lanes 0..2BY-1 of wave 1 the VEC-wide pieces whose
    // last / first element is the left / right halo column of each row
    int h_off = col, h_row = DUMMY, h_col = lcol;
    bool h_real = true;
    if (ty == 0) {
        if (j >= 1 && i0 < nx) {
            h_off = col - nx;
            h_row = 0;
        }
    } else if (ty == BY - 1) {
        if (j + 1 < ny && i0 < nx) {
            h_off = col + nx;
            h_row = BY + 1;
        }
    } else if (ty == 1 && tx < 2 * BY) {
        h_real = false;
        const int row = tx % BY;
        const bool right = tx >= BY;
        const int ii = bx * TX + (right ? TX : -VEC);
        const int jj = by * BY + row;
        if (ii >= 0 && ii < nx && jj < ny) {
            h_off = ii + nx * jj;
            h_row = row + 1;
            h_col = right ? TX + 2 : 2 - VEC;
            h_real = true;
        }
    } else {
        h_real = false;
    }
    if (h_row == DUMMY) h_real = false;
    // a lane without halo work re-reads its own prefetch address (plane k+2)
    const int h_dz = h_real ? 1 : 2;

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

    // z register queue (k-1, k, k+1, prefetched k+2), halo of plane k (and
    // k+1 prefetched), per-cell values of plane k (and k+1 prefetched)
    T zm[NQ][VEC], zc[NQ][VEC], zp[NQ][VEC], zn[NQ][VEC], hc[NQ][VEC], hn[NQ][VEC];
    T wo_c[3][VEC], wo_n[3][VEC], fs_c[3][VEC], fs_n[3][VEC];
    T crho_c[VEC], crho_n[VEC], eta_c[VEC], eta_n[VEC];
#pragma unroll
    for (int f = 0; f < NQ; ++f) {
        vload<T, VEC>(fp[f] + (kb - 1) * sxy + col, zm[f]);
        vload<T, VEC>(fp[f] + kb * sxy + col, zc[f]);
        vload<T, VEC>(fp[f] + (kb + 1) * sxy + col, zp[f]);
        vload<T, VEC>(fp[f] + kb * sxy + h_off, hc[f]);
    }
    {
        const int q = kb * sxy + col;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                wo_c[c][v] = wo_n[c][v] = T(0);
                fs_c[c][v] = fs_n[c][v] = T(0);
            }
            if constexpr (!VISC) vload<T, VEC>(a.w + c * a.N + q, wo_c[c]);
            if constexpr (FORCE) vload<T, VEC>(a.FS + c * a.N + q, fs_c[c]);
        }
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            crho_c[v] = crho_n[v] = a.crho0;
            eta_c[v] = eta_n[v] = T(0);
        }
        if constexpr (HET) {
            vload<T, VEC>(a.crho + q, crho_c);
            if constexpr (VISC) vload<T, VEC>(a.eta + q, eta_c);
        }
    }

    T rxy[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v)
        rxy[v] = a.L > 0 ? max(ramp<T>(i0 + v, nx, a.L, a.invL), ramp<T>(j, ny, a.L, a.invL)) : T(0);
    const T ihx2 = a.ihx2, ihy2 = a.ihy2, ihz2 = a.ihz2;

    for (int k = kb; k < ke; ++k) {
        const int buf = k & 1;
#pragma unroll
        for (int f = 0; f < NQ; ++f) {
            vlds_write<T, VEC>(&lds[buf][f][ty + 1][lcol], zc[f]);
            vlds_write<T, VEC>(&lds[buf][f][h_row][h_col], hc[f]);
        }
        // prefetch: centre of plane k+2, halo and per-cell values of k+1
        // (clamped to planes that exist; the clamped values go unused)
        const int k2 = min(k + 2, ke);
        const int k1 = min(k + 1, ke - 1);
#pragma unroll
        for (int f = 0; f < NQ; ++f) {
            vload<T, VEC>(fp[f] + k2 * sxy + col, zn[f]);
            vload<T, VEC>(fp[f] + min(k + h_dz, ke) * sxy + h_off, hn[f]);
        }
        {
            const int q = k1 * sxy + col;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if constexpr (!VISC) vload<T, VEC>(a.w + c * a.N + q, wo_n[c]);
                if constexpr (FORCE) vload_nt<T, VEC>(a.FS + c * a.N + q, fs_n[c]);
            }
            if constexpr (HET) {
                vload_nt<T, VEC>(a.crho + q, crho_n);
                if constexpr (VISC) vload_nt<T, VEC>(a.eta + q, eta_n);
            }
        }
        lds_barrier();

        const T rz = a.L > 0 ? ramp<T>(k, a.nz, a.L, a.invL) : T(0);
        T uo[3][VEC], wo[3][VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const int lc = lcol + v;
            const T s = a.half_dt_smax * max(rxy[v], rz);
            const T inv1ps = rcp_fast<T>(T(1) + s);
            const T a1 = (T(1) - s) * inv1ps;
            const T a2 = crho_c[v] * inv1ps;
            const T eta_dt = HET ? eta_c[v] * a.inv_dt : a.eta_dt0;
            T gxm, gxp, gym, gyp, gzm, gzp;
            if constexpr (HET) {
                const T Gc = zc[QG][v];
                gxm = harm<T>(Gc, lds[buf][QG][ty + 1][lc - 1]) * ihx2;
                gxp = harm<T>(Gc, lds[buf][QG][ty + 1][lc + 1]) * ihx2;
                gym = harm<T>(Gc, lds[buf][QG][ty][lc]) * ihy2;
                gyp = harm<T>(Gc, lds[buf][QG][ty + 2][lc]) * ihy2;
                gzm = harm<T>(Gc, zm[QG][v]) * ihz2;
                gzp = harm<T>(Gc, zp[QG][v]) * ihz2;
            } else {
                gxm = gxp = a.G0 * ihx2;
                gym = gyp = a.G0 * ihy2;
                gzm = gzp = a.G0 * ihz2;
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T uc = zc[c][v];
                T acc = gxp * (lds[buf][c][ty + 1][lc + 1] - uc) - gxm * (uc - lds[buf][c][ty + 1][lc - 1])
                      + gyp * (lds[buf][c][ty + 2][lc] - uc) - gym * (uc - lds[buf][c][ty][lc])
                      + gzp * (zp[c][v] - uc) - gzm * (uc - zm[c][v]);
                T wc;
                if constexpr (VISC) {
                    wc = zc[3 + c][v];
                    const T lw = (lds[buf][3 + c][ty + 1][lc + 1] + lds[buf][3 + c][ty + 1][lc - 1] - T(2) * wc) * ihx2
                               + (lds[buf][3 + c][ty + 2][lc] + lds[buf][3 + c][ty][lc] - T(2) * wc) * ihy2
                               + (zp[3 + c][v] + zm[3 + c][v] - T(2) * wc) * ihz2;
                    acc += eta_dt * lw;
                } else {
                    wc = wo_c[c][v];
                }
                if constexpr (FORCE) acc += a.gn * fs_c[c][v];
                const T wnew = a1 * wc + a2 * acc;
                wo[c][v] = act[v] ? wnew : T(0);
                uo[c][v] = act[v] ? uc + wnew : T(0);
            }
        }
        const int sidx = k * sxy + scol;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            vstore_nt<T, VEC>(a.wn + c * a.N + sidx, wo[c]);
            vstore_nt<T, VEC>(a.un + c * a.N + sidx, uo[c]);
        }
#pragma unroll
        for (int f = 0; f < NQ; ++f)
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                zm[f][v] = zc[f][v];
                zc[f][v] = zp[f][v];
                zp[f][v] = zn[f][v];
                hc[f][v] = hn[f][v];
            }
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                wo_c[c][v] = wo_n[c][v];
                fs_c[c][v] = fs_n[c][v];
            }
            crho_c[v] = crho_n[v];
            eta_c[v] = eta_n[v];
        }
    }
}

// Step-kernel variants (tile rows BY, cells per lane VEC, wavefronts per row
// WX) chosen by kvs_autotune_step; variant 0 is the default.
struct StepVariant {
    int by, vec, wx, wpe;
};
// wpe: minimum waves per SIMD asked of the register allocator (1 = free)
constexpr StepVariant kVariants[] = {{4, 1, 1, 1}, {8, 1, 1, 1}, {4, 2, 1, 1}, {8, 2, 1, 1},
                                     {16, 1, 1, 1}, {4, 1, 2, 1}, {8, 1, 2, 1}, {4, 1, 4, 1}};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

// The shape a launch actually uses.  VEC = 2 needs an even nx so that every
// lane's pair is aligned and whole.  FP64 (the parity mode) uses one cell per
// lane and tiles of at most 8 rows and 128 columns: larger FP64 tiles spill
// registers or exceed the 160 KB of LDS (two buffered planes of 7 fields).
int effective_variant(int v, bool fp64, bool odd_nx) {
    if (v < 0 || v >= kNumVariants) v = 0;
    if (kVariants[v].vec == 2 && (fp64 || odd_nx)) v = kVariants[v].by == 8 ? 1 : 0;
    if (fp64) {
        if (v == 4) v = 1;
        if (v == 6 || v == 7) v = 5;
    }
    return v;
}

}  // namespace
