// Helmholtz projection of the body force (Sec. 3.2) on gfx950, all in FP64:
//   b = centred divergence of F on interior nodes,
//   CG on A phi = -b, A = -lap_h (interior mask after every update, phi_0 = 0
//   or a warm start, stop at sqrt(r.r / b.b) < tol, guards on p.Ap <= 0 and
//   non-finite inner products: Sec. 3.2.3),
//   f_S,a = (F_a(-a) + 2 F_a + F_a(+a))/4 - (phi(+a) - phi(-a))/(2 h_a).
//
// One CG iteration is two fused HBM sweeps plus two one-block finalize
// kernels, with every scalar (alpha, beta, r.r, the stop flag) kept on the
// device, so the host only polls a flag once per chunk of iterations:
//   sweep 1: p' = z + beta p (z = r, or r / diag(A) for Jacobi), A p' from
//            the 7-point stencil, block partials of p'.Ap'
//            (reads r, p; writes p': 24 B per cell)
//   finalize: alpha = r.z / p.Ap with the breakdown guard
//   sweep 2: A p' recomputed from p', phi += alpha p', r -= alpha Ap',
//            partials of r.r and r.z (reads phi, p', r; writes phi, r: 40 B)
//   finalize: beta, the stop test, the iteration count
// Recomputing A p' costs a few flops and saves storing and re-reading it.
// Flexible PCG (learned preconditioner): the update writes the new residual
// into a second buffer, and the network's output kernel, as it writes z, also
// sums z.r, z.r_old and r.r_old per block, from which the Polak-Ribiere beta
// z.(r - r_old) / (z_old . r_old) follows without another sweep.
// p is ping-ponged because sweep 1 reads p at neighbours while writing p'.
// Both sweeps are LDS-staged z-marches like the FDTD step (64 x 8 tiles,
// straight-line memory code, plane-ahead prefetch).
// Reductions are deterministic: fixed-shape wavefront shuffles inside a
// block, one partial per block, and a one-block fixed-order final sum.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <mutex>
#include <string>

#include "kvs_internal.hpp"
#include "kvs_tiling.hpp"

namespace {

using kvs_tiling::lds_barrier;

constexpr int CBY = 4;    // rows per block
constexpr int CKZ = 16;   // z planes per block

struct CgGeom {
    int nx, ny, nz, gx, gy, gz, kchunk;
    long long N;
    double ihx2, ihy2, ihz2;
    double i2hx, i2hy, i2hz;  // 1/(2h)
    double dinv;              // 1/diag(A)
};

enum { FIN_INIT = 0, FIN_ALPHA = 1, FIN_BETA = 2, FIN_TRUE = 3, FIN_FZ0 = 4, FIN_FBETA = 5, FIN_RESTART = 6, FIN_REPLACE = 7 };

using kvs_tiling::tile_of;

struct Tile {
    int i, j, kb, ke;
    bool act;
    int col;
};

__device__ __forceinline__ Tile tile_coords(const CgGeom& g) {
    const int B = g.gx * g.gy * g.gz;
    const int t = tile_of(blockIdx.x, B);
    const int bx = t % g.gx, by = (t / g.gx) % g.gy, bz = t / (g.gx * g.gy);
    Tile T;
    T.i = bx * 64 + threadIdx.x;
    T.j = by * CBY + threadIdx.y;
    T.kb = 1 + bz * g.kchunk;
    T.ke = min(g.nz - 1, T.kb + g.kchunk);
    T.act = T.i >= 1 && T.i <= g.nx - 2 && T.j >= 1 && T.j <= g.ny - 2;
    T.col = T.act ? T.i + g.nx * T.j : 0;
    return T;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum up to three values over the block; thread 0 writes them to partials
// [which * npart + block].
template <int NS>
__device__ __forceinline__ void block_partials(double v0, double v1, double v2, double* partials, int npart) {
    __shared__ double sh[3][CBY];
    const int lane = threadIdx.x, wid = threadIdx.y;
    v0 = wave_sum(v0);
    if (NS > 1) v1 = wave_sum(v1);
    if (NS > 2) v2 = wave_sum(v2);
    if (lane == 0) {
        sh[0][wid] = v0;
        if (NS > 1) sh[1][wid] = v1;
        if (NS > 2) sh[2][wid] = v2;
    }
    __syncthreads();
    if (lane == 0 && wid == 0) {
        double a = 0, b = 0, c = 0;
        for (int w = 0; w < CBY; ++w) {
            a += sh[0][w];
            if (NS > 1) b += sh[1][w];
            if (NS > 2) c += sh[2][w];
        }
        partials[blockIdx.x] = a;
        if (NS > 1) partials[npart + blockIdx.x] = b;
        if (NS > 2) partials[2 * npart + blockIdx.x] = c;
    }
}

__device__ __forceinline__ double div_at(const CgGeom& g, const double* F, int idx) {
    const int sy = g.nx, sz = g.nx * g.ny;
    const double* Fx = F;
    const double* Fy = F + g.N;
    const double* Fz = F + 2 * g.N;
    return (Fx[idx + 1] - Fx[idx - 1]) * g.i2hx + (Fy[idx + sy] - Fy[idx - sy]) * g.i2hy
         + (Fz[idx + sz] - Fz[idx - sz]) * g.i2hz;
}

__device__ __forceinline__ double negative_lap_at(const CgGeom& g, const double* q, int idx) {
    const int sy = g.nx, sz = g.nx * g.ny;
    const double c2 = 2.0 * q[idx];
    return -((q[idx + 1] + q[idx - 1] - c2) * g.ihx2 + (q[idx + sy] + q[idx - sy] - c2) * g.ihy2
             + (q[idx + sz] + q[idx - sz] - c2) * g.ihz2);
}

// r0 = -b - A phi0 (warm) or -b; partials of r.r, r.z, b.b
// r = -b (- A phi when warm) in FP64, stored as RT (float: the FP32
// residual of the plain CG, whose sums are of the stored values)
template <typename RT>
__global__ __launch_bounds__(64 * CBY) void cg_init_kernel(const CgGeom g, const double* F, const double* phi,
                                                           RT* r, int warm, double* partials, int npart) {
    const Tile t = tile_coords(g);
    const int sxy = g.nx * g.ny;
    double s1 = 0, s2 = 0, s3 = 0;
    if (t.act) {
        for (int k = t.kb; k < t.ke; ++k) {
            const int idx = k * sxy + t.col;
            const double b = div_at(g, F, idx);
            double rv = -b;
            if (warm) rv -= negative_lap_at(g, phi, idx);
            rv = (double)(RT)rv;
            r[idx] = (RT)rv;
            s1 += rv * rv;
            s2 += rv * (rv * g.dinv);
            s3 += b * b;
        }
    }
    block_partials<3>(s1, s2, s3, partials, npart);
}

// Geometry of the two CG sweeps: TX x BY tiles (TX = 64 WX: WX wavefronts
// side by side on a row), z segments of `kchunk`.  Wide rows spread the two
// x-halo columns over more cells: the widest of 256 x 4, 128 x 8 and 64 x 8
// whose padding of the row stays within 1/8 of it.
struct SweepGeom {
    int gx, gy, gz, kchunk;
};

struct SweepShape {
    int wx, by;
};

inline SweepShape sweep_shape(int nx) {
    auto waste_ok = [nx](int tx) { return 8 * (((nx + tx - 1) / tx) * tx - nx) <= nx; };
    if (waste_ok(256)) return {4, 4};
    if (waste_ok(128)) return {2, 8};
    return {1, 8};
}

// Per-lane tile coordinates and halo slot of a z-marching sweep (same
// scheme as the FDTD step: wave 0 loads the row below the tile, wave SBY-1
// the row above, lanes 0..2 SBY-1 of wave 1 the left/right columns; other
// lanes re-read their own plane-(k+2) address and write a dummy LDS row).
struct Lane {
    int i, j, kb, ke, col, scol, h_off, h_row, h_col, h_dz;
    bool act;
};

template <int WX, int SBY>
__device__ __forceinline__ Lane sweep_lane(const CgGeom& g, const SweepGeom& s) {
    constexpr int TX = 64 * WX;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int B = s.gx * s.gy * s.gz;
    const int t = tile_of(blockIdx.x, B);
    const int bx = t % s.gx, by = (t / s.gx) % s.gy, bz = t / (s.gx * s.gy);
    Lane L;
    L.i = bx * TX + tx;
    L.j = by * SBY + ty;
    L.kb = 1 + bz * s.kchunk;
    L.ke = min(g.nz - 1, L.kb + s.kchunk);
    const bool inb = L.i < g.nx && L.j < g.ny;
    L.act = L.i >= 1 && L.i <= g.nx - 2 && L.j >= 1 && L.j <= g.ny - 2;
    L.col = inb ? L.i + g.nx * L.j : 0;
    L.scol = min(L.i, g.nx - 1) + g.nx * min(L.j, g.ny - 1);
    L.h_off = L.col;
    L.h_row = SBY + 2;  // dummy row
    L.h_col = tx + 1;
    bool real = false;
    if (ty == 0) {
        if (L.j >= 1 && L.i < g.nx) {
            L.h_off = L.col - g.nx;
            L.h_row = 0;
            real = true;
        }
    } else if (ty == SBY - 1) {
        if (L.j + 1 < g.ny && L.i < g.nx) {
            L.h_off = L.col + g.nx;
            L.h_row = SBY + 1;
            real = true;
        }
    } else if (ty == 1 && tx < 2 * SBY) {
        const int row = tx % SBY;
        const bool right = tx >= SBY;
        const int ii = bx * TX + (right ? TX : -1);
        const int jj = by * SBY + row;
        if (ii >= 0 && ii < g.nx && jj < g.ny) {
            L.h_off = ii + g.nx * jj;
            L.h_row = row + 1;
            L.h_col = right ? TX + 1 : 0;
            real = true;
        }
    }
    L.h_dz = real ? 1 : 2;
    return L;
}

// Sum over the block (WX SBY waves) of up to two values; lane (0,0) writes
// them to partials[block] and partials[npart + block], in wave order.
template <int NS, int WX, int SBY>
__device__ __forceinline__ void sweep_partials(double v0, double v1, double* partials, int npart) {
    constexpr int NW = WX * SBY;
    __shared__ double sh[2][NW];
    v0 = wave_sum(v0);
    if (NS > 1) v1 = wave_sum(v1);
    const int wv = threadIdx.y * WX + threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        sh[0][wv] = v0;
        if (NS > 1) sh[1][wv] = v1;
    }
    __syncthreads();
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        double a = 0, b = 0;
        for (int w = 0; w < NW; ++w) {
            a += sh[0][w];
            if (NS > 1) b += sh[1][w];
        }
        partials[blockIdx.x] = a;
        if (NS > 1) partials[npart + blockIdx.x] = b;
    }
}

// sweep 1: p' = z + beta p, A p' = -lap p', partial p'.Ap'.  z = zs * src
// with src = r (CG: zs = 1, Jacobi: zs = 1/diag) or, in flexible PCG, the
// network output zf (zs = 1) unless this iteration fell back to Jacobi.
template <int WX, int SBY, typename PT, typename RT>
__global__ __launch_bounds__(64 * WX * SBY) void cg_dir_kernel(const CgGeom g, const SweepGeom sg, const RT* r_in,
                                                               const RT* zf, const PT* p_old, PT* p_new,
                                                               const CgState* st, double* partials, int npart) {
    if (st->done) return;
    __shared__ double lds[2][SBY + 3][64 * WX + 4];
    const Lane L = sweep_lane<WX, SBY>(g, sg);
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int sxy = g.nx * g.ny;
    const double beta = st->beta;
    const bool net_z = st->flexible && !st->zjacobi;
    // the network's z is stored like r: z itself in FP64, or (RT = float) the
    // FP32 sum before the output scale st->net_out it was formed with
    const RT* r = net_z ? zf : r_in;
    const double zs = net_z ? (sizeof(RT) == 4 ? st->net_out : 1.0)
                            : ((st->jacobi || (st->flexible && st->zjacobi)) ? g.dinv : 1.0);
    const bool first = beta == 0.0;
    // the new direction as stored (PT = float: rounded once); the stencil,
    // p.Ap and the update sweep all use this stored value
    auto pv = [&](double rv, double po) { return (double)(PT)(first ? rv * zs : rv * zs + beta * po); };
    const int kb = L.kb, ke = L.ke;
    double pm = pv(r[(kb - 1) * sxy + L.col], p_old[(kb - 1) * sxy + L.col]);
    double pc = pv(r[kb * sxy + L.col], p_old[kb * sxy + L.col]);
    double pp = pv(r[(kb + 1) * sxy + L.col], p_old[(kb + 1) * sxy + L.col]);
    double hc = pv(r[kb * sxy + L.h_off], p_old[kb * sxy + L.h_off]);
    double s1 = 0.0;
    for (int k = kb; k < ke; ++k) {
        const int buf = k & 1;
        lds[buf][ty + 1][tx + 1] = pc;
        lds[buf][L.h_row][L.h_col] = hc;
        const int q2 = min(k + 2, ke) * sxy + L.col;
        const int qh = min(k + L.h_dz, ke) * sxy + L.h_off;
        // streamed accesses (non-temporal): the old direction, read once per
        // iteration, and the new one, read by the next sweep from HBM anyway;
        // r stays cached for the update sweep
        const double rn = r[q2], on = __builtin_nontemporal_load(p_old + q2), hrn = r[qh], hon = p_old[qh];
        lds_barrier();
        const double c2 = 2.0 * pc;
        const double ap = -((lds[buf][ty + 1][tx + 2] + lds[buf][ty + 1][tx] - c2) * g.ihx2
                            + (lds[buf][ty + 2][tx + 1] + lds[buf][ty][tx + 1] - c2) * g.ihy2
                            + (pp + pm - c2) * g.ihz2);
        s1 += L.act ? pc * ap : 0.0;
        __builtin_nontemporal_store(L.act ? (PT)pc : (PT)0, p_new + k * sxy + L.scol);
        pm = pc;
        pc = pp;
        pp = pv(rn, on);
        hc = pv(hrn, hon);
    }
    sweep_partials<1, WX, SBY>(s1, 0.0, partials, npart);
}

// sweep 2: A p recomputed, phi += alpha p, r_out = r - alpha A p (r_out may
// be r itself), partials r.r, r.z
template <int WX, int SBY, typename PT, typename RT>
__global__ __launch_bounds__(64 * WX * SBY) void cg_upd_kernel(const CgGeom g, const SweepGeom sg, double* phi,
                                                               const RT* r, RT* r_out, const PT* p,
                                                               const CgState* st, double* partials, int npart) {
    if (st->done) return;
    __shared__ double lds[2][SBY + 3][64 * WX + 4];
    const Lane L = sweep_lane<WX, SBY>(g, sg);
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int sxy = g.nx * g.ny;
    const double alpha = st->alpha;
    const int kb = L.kb, ke = L.ke;
    double pm = p[(kb - 1) * sxy + L.col];
    double pc = p[kb * sxy + L.col];
    double pp = p[(kb + 1) * sxy + L.col];
    double hc = p[kb * sxy + L.h_off];
    double phc = phi[kb * sxy + L.col], rc = r[kb * sxy + L.col];
    double s1 = 0.0, s2 = 0.0;
    for (int k = kb; k < ke; ++k) {
        const int buf = k & 1;
        lds[buf][ty + 1][tx + 1] = pc;
        lds[buf][L.h_row][L.h_col] = hc;
        const double pn = p[min(k + 2, ke) * sxy + L.col];
        const double hn = p[min(k + L.h_dz, ke) * sxy + L.h_off];
        const int q1 = min(k + 1, ke - 1) * sxy + L.col;
        // streamed accesses (non-temporal): phi (read and written once per
        // iteration) and the stores; r and p stay cached for the next sweep
        const double phn = __builtin_nontemporal_load(phi + q1), rn = r[q1];
        lds_barrier();
        const double c2 = 2.0 * pc;
        const double ap = -((lds[buf][ty + 1][tx + 2] + lds[buf][ty + 1][tx] - c2) * g.ihx2
                            + (lds[buf][ty + 2][tx + 1] + lds[buf][ty][tx + 1] - c2) * g.ihy2
                            + (pp + pm - c2) * g.ihz2);
        const double phv = phc + alpha * pc;
        const double rv = (double)(RT)(rc - alpha * ap);  // as stored
        const int q = k * sxy + L.scol;
        __builtin_nontemporal_store(L.act ? phv : 0.0, phi + q);
        __builtin_nontemporal_store(L.act ? (RT)rv : (RT)0, r_out + q);
        s1 += L.act ? rv * rv : 0.0;
        s2 += L.act ? rv * (rv * g.dinv) : 0.0;
        pm = pc;
        pc = pp;
        pp = pn;
        hc = hn;
        phc = phn;
        rc = rn;
    }
    sweep_partials<2, WX, SBY>(s1, s2, partials, npart);
}


// partials of (-b - A phi)^2 and b^2
__global__ __launch_bounds__(64 * CBY) void cg_true_residual_kernel(const CgGeom g, const double* F, const double* phi,
                                                                    double* partials, int npart) {
    const Tile t = tile_coords(g);
    const int sxy = g.nx * g.ny;
    double s1 = 0, s3 = 0;
    if (t.act) {
        for (int k = t.kb; k < t.ke; ++k) {
            const int idx = k * sxy + t.col;
            const double b = div_at(g, F, idx);
            const double d = -b - negative_lap_at(g, phi, idx);
            s1 += d * d;
            s3 += b * b;
        }
    }
    block_partials<3>(s1, 0.0, s3, partials, npart);
}

template <typename T>
__global__ __launch_bounds__(64 * CBY) void grad_subtract_kernel(const CgGeom g, const double* F, const double* phi,
                                                                 T* FS) {
    const Tile t = tile_coords(g);
    if (!t.act) return;
    const int sxy = g.nx * g.ny;
    const int st[3] = {1, g.nx, sxy};
    const double i2h[3] = {g.i2hx, g.i2hy, g.i2hz};
    for (int k = t.kb; k < t.ke; ++k) {
        const int idx = k * sxy + t.col;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double* Fa = F + a * g.N;
            const double v = 0.25 * (Fa[idx - st[a]] + 2.0 * Fa[idx] + Fa[idx + st[a]])
                           - (phi[idx + st[a]] - phi[idx - st[a]]) * i2h[a];
            FS[a * g.N + idx] = (T)v;
        }
    }
}

// One block: fixed-order sums of the partials, then the scalar logic.
// partials[s * stride + q], q < count, s < nsum
__global__ __launch_bounds__(256) void cg_finalize_kernel(const double* partials, int count, int stride, int nsum,
                                                          int mode, CgState* st) {
    if (mode != FIN_INIT && mode != FIN_TRUE && mode != FIN_RESTART && st->done) return;
    // network scales of the flexible PCG from the current residual
    auto set_net_scales = [&](double rr) {
        const double rms = sqrt(rr / st->n_interior);
        st->net_in = rms > 0.0 ? 1.0 / rms : 0.0;
        st->net_out = rms * st->h2;
    };
    __shared__ double sh[3][256];
    for (int s = 0; s < nsum; ++s) {
        double acc = 0.0;
        for (int q = threadIdx.x; q < count; q += 256) acc += partials[s * stride + q];
        sh[s][threadIdx.x] = acc;
    }
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int s = 0; s < nsum; ++s) sh[s][threadIdx.x] += sh[s][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double s1 = sh[0][0];
    const double s2 = nsum > 1 ? sh[1][0] : 0.0;
    const double s3 = nsum > 2 ? sh[2][0] : 0.0;
    st->s1 = s1;
    st->s2 = s2;
    st->s3 = s3;
    if (mode == FIN_INIT) {
        st->rr0 = s1;
        st->rr = s1;
        st->rz = st->jacobi ? s2 : s1;
        st->bb = s3;
        st->iters = 0;
        st->beta = 0.0;
        st->alpha = 0.0;
        st->status = KVS_OK;
        st->done = 0;
        if (!isfinite(s1) || !isfinite(s3) || !isfinite(st->rz)) {
            st->status = KVS_EBREAKDOWN;
            st->done = 1;
        } else if (s1 == 0.0 || s3 == 0.0) {
            st->done = 1;  // nothing to solve, or b = 0 (phi is set to 0 by the host)
        } else if (st->fixed_iters <= 0 && !(1.0 >= sqrt(st->tol2))) {
            st->done = 1;  // tol > 1: the initial residual already satisfies the test
        }
        set_net_scales(s1);
    } else if (mode == FIN_FZ0) {
        // flexible PCG, first z: z.r, else fall back to Jacobi for this z
        if (s1 > 0.0 && isfinite(s1)) {
            st->rz = s1;
            st->zjacobi = 0;
        } else {
            st->rz = st->rr * st->dinv;
            st->zjacobi = 1;
            st->fallbacks += 1;
        }
    } else if (mode == FIN_FBETA) {
        // Polak-Ribiere: beta = z.(r - r_old) / (z_old . r_old); Jacobi z for
        // this iteration when z.r <= 0 or a product is not finite
        const double zr = s1, zro = s2, rro = s3;
        const double rz_old = st->rz;
        if (zr > 0.0 && isfinite(zr) && isfinite(zro)) {
            st->beta = (zr - zro) / rz_old;
            st->rz = zr;
            st->zjacobi = 0;
        } else {
            st->fallbacks += 1;
            st->zjacobi = 1;
            st->beta = st->dinv * (st->rr - rro) / rz_old;
            st->rz = st->rr * st->dinv;
        }
    } else if (mode == FIN_ALPHA) {
        st->pAp = s1;
        if (!(s1 > 0.0) || !isfinite(s1)) {
            st->status = KVS_EBREAKDOWN;
            st->done = 1;
        } else {
            st->alpha = st->rz / s1;
        }
    } else if (mode == FIN_BETA) {
        st->iters += 1;
        if (!isfinite(s1) || s1 < 0.0 || !isfinite(s2)) {
            st->status = KVS_EBREAKDOWN;
            st->done = 1;
            return;
        }
        if (st->flexible) {
            // residual, stop test and network scales only; beta comes later
            st->rr = s1;
            set_net_scales(s1);
            if (st->fixed_iters > 0) {
                if (st->iters >= st->fixed_iters) st->done = 1;
            } else if (sqrt(st->rr / st->bb) < sqrt(st->tol2)) {
                st->done = 1;
            } else if (st->iters >= st->max_iter) {
                st->status = KVS_ENOTCONV;
                st->done = 1;
            }
            return;
        }
        const double rz_new = st->jacobi ? s2 : s1;
        st->beta = rz_new / st->rz;
        st->rz = rz_new;
        st->rr = s1;
        if (st->fixed_iters > 0) {
            if (st->iters >= st->fixed_iters) st->done = 1;
        } else if (sqrt(st->rr / st->bb) < sqrt(st->tol2)) {
            st->done = 1;
        } else if (st->iters >= st->max_iter) {
            st->status = KVS_ENOTCONV;
            st->done = 1;
        }
    } else if (mode == FIN_RESTART) {
        // restart from the true residual r = -b - A phi: the iteration count
        // and b.b are kept, the direction is rebuilt from z alone (beta = 0)
        st->rr = s1;
        st->rz = st->jacobi ? s2 : s1;
        st->beta = 0.0;
        st->alpha = 0.0;
        st->done = 0;
        if (!isfinite(s1) || !isfinite(st->rz)) {
            st->status = KVS_EBREAKDOWN;
            st->done = 1;
        } else if (s1 == 0.0) {
            st->done = 1;
        }
        set_net_scales(s1);
    } else if (mode == FIN_REPLACE) {
        // reliable update of the FP32 residual: the recursive r was replaced
        // by the true residual -b - A phi; the direction is kept.  Flexible
        // PCG: z, its scalars and the network scales stay those of the
        // recursive r (a perturbation at the size of the drift, which the
        // flexible beta absorbs like any change of the preconditioner); only
        // r.r and the stop test are refreshed.
        if (st->flexible) {
            if (!isfinite(s1)) {
                st->status = KVS_EBREAKDOWN;
                st->done = 1;
                return;
            }
            st->rr = s1;
            if (st->fixed_iters <= 0 && sqrt(st->rr / st->bb) < sqrt(st->tol2)) st->done = 1;
            return;
        }
        // plain CG: beta, formed from the recursive z.r, is rescaled to the new one
        const double rz_new = st->jacobi ? s2 : s1;
        if (!isfinite(s1) || !isfinite(rz_new) || !(st->rz > 0.0)) {
            st->status = KVS_EBREAKDOWN;
            st->done = 1;
            return;
        }
        st->beta *= rz_new / st->rz;
        st->rz = rz_new;
        st->rr = s1;
        if (st->fixed_iters <= 0 && sqrt(st->rr / st->bb) < sqrt(st->tol2)) st->done = 1;
    } else {  // FIN_TRUE
        st->relres_true2 = s3 > 0.0 ? s1 / s3 : 0.0;
    }
}

CgGeom make_geom(const kvs_grid& gr) {
    CgGeom g{};
    g.nx = (int)gr.nx;
    g.ny = (int)gr.ny;
    g.nz = (int)gr.nz;
    g.kchunk = std::min<int>(CKZ, g.nz - 2);
    g.gx = (g.nx + 63) / 64;
    g.gy = (g.ny + CBY - 1) / CBY;
    g.gz = (g.nz - 2 + g.kchunk - 1) / g.kchunk;
    g.N = (long long)gr.nx * gr.ny * gr.nz;
    g.ihx2 = 1.0 / (gr.hx * gr.hx);
    g.ihy2 = 1.0 / (gr.hy * gr.hy);
    g.ihz2 = 1.0 / (gr.hz * gr.hz);
    g.i2hx = 1.0 / (2.0 * gr.hx);
    g.i2hy = 1.0 / (2.0 * gr.hy);
    g.i2hz = 1.0 / (2.0 * gr.hz);
    g.dinv = 1.0 / (2.0 * g.ihx2 + 2.0 * g.ihy2 + 2.0 * g.ihz2);
    return g;
}

int nblocks(const CgGeom& g) { return g.gx * g.gy * g.gz; }

// Error text of the projection driver: a fixed message or a HIP error
// (the text of a HIP error is a static string); no allocation.
struct CgErr {
    const char* what = nullptr;
    const char* hip = nullptr;
};

kvs_status cg_fail(CgErr& e, kvs_status s, const char* what, const char* hip = nullptr) {
    e.what = what;
    e.hip = hip;
    return s;
}

}  // namespace

int64_t kvs_cg_partials_needed(const kvs_grid& gr) {
    CgGeom g = make_geom(gr);
    const SweepShape sh = sweep_shape(g.nx);
    const int sweep_xy = ((g.nx + 64 * sh.wx - 1) / (64 * sh.wx)) * ((g.ny + sh.by - 1) / sh.by);
    return std::max<int64_t>(std::max<int64_t>(nblocks(g), kvs_tiling::max_tiled_blocks(sweep_xy, g.nz - 2)),
                             kvs_unet_out_blocks(gr));
}

#define CG_HIP(call)                                                      \
    do {                                                                  \
        hipError_t e_ = (call);                                           \
        if (e_ != hipSuccess) return cg_fail(err, KVS_EDEVICE, #call, hipGetErrorString(e_)); \
    } while (0)

namespace {

// One projection on explicit buffers: b = div F, the CG / Jacobi-PCG /
// flexible-PCG solve of A phi = -b, f_S = F - grad phi into FS (FP32 or FP64),
// the FP64 true residual.  Every buffer belongs to the caller; nothing is
// allocated here.  phi is the initial guess when B.warm (its outer layer must
// be 0), else it is cleared.  The outer layer of FS is not written.
struct CgBuffers {
    kvs_grid grid;
    hipStream_t stream;
    const double* F;
    double* phi;
    double* r;
    double* r2;  // flexible PCG only: the previous residual
    double* p[2];
    double* Ap;  // flexible PCG: the preconditioned residual z
    double* partials;
    int npart;
    CgState* cgs;       // device control block
    CgState* cgs_host;  // host mirror (pinned or not)
    void* FS;
    int fs_fp32;
    kvs_unet* net;
    bool warm;
    bool use_events;  // time with HIP events (else with the host clock)
    bool dir_fp32;    // p[] hold FP32 directions (the first half of each buffer)
    bool res_fp32;    // r (and r2, and the network's z) hold FP32 values
};

__global__ void fill_zero_kernel(double* a, long long n) {
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
        a[q] = 0.0;
}

hipError_t fill_zero(double* a, long long n, hipStream_t s) {
    const long long b = std::min<long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)std::max<long long>(b, 1)), dim3(256), 0, s, a, n);
    return hipGetLastError();
}

kvs_status cg_project(const CgBuffers& B, const kvs_solve_opts* o, kvs_solve_report* rep, CgErr& err) {
    const CgGeom g = make_geom(B.grid);
    const int nb = nblocks(g);
    const dim3 blk(64, CBY);
    double* part = B.partials;
    const int npart = B.npart;
    hipStream_t stream = B.stream;

    hipEvent_t e0 = nullptr, e1 = nullptr;
    const auto t0 = std::chrono::steady_clock::now();
    if (B.use_events) {
        CG_HIP(hipEventCreate(&e0));
        CG_HIP(hipEventCreate(&e1));
        CG_HIP(hipEventRecord(e0, stream));
    }

    const bool flexible = o->precond == KVS_PC_UNET;
    if (flexible && (!B.net || !B.r2)) return cg_fail(err, KVS_ESTATE, "flexible PCG needs a network and a second residual buffer");
    CgState init{};
    init.tol2 = o->tol * o->tol;
    init.max_iter = o->max_iter;
    init.fixed_iters = o->fixed_iters;
    init.jacobi = o->precond == KVS_PC_JACOBI ? 1 : 0;
    init.flexible = flexible ? 1 : 0;
    init.dinv = g.dinv;
    init.h2 = B.grid.hx * B.grid.hx;
    init.n_interior = (double)(g.nx - 2) * (double)(g.ny - 2) * (double)(g.nz - 2);
    *B.cgs_host = init;
    CG_HIP(hipMemcpyAsync(B.cgs, B.cgs_host, sizeof(CgState), hipMemcpyHostToDevice, stream));
    const bool warm = B.warm;
    if (!warm) CG_HIP(fill_zero(B.phi, g.N, stream));

    // the residual buffers (and, in flexible PCG, z) hold FP32 values with
    // B.res_fp32
    const bool res32 = B.res_fp32;
    // z = U(r) from the network, stored as r is (FP32: the sum before the
    // output scale), with the partial sums for the flexible PCG's scalars
    auto precondition = [&](const double* r_buf, const UnetDots* dots, int* nbo) {
        if (res32)
            return kvs_unet_precondition32(B.net, reinterpret_cast<const float*>(r_buf), reinterpret_cast<float*>(B.Ap),
                                           B.grid, &B.cgs->net_in, &B.cgs->net_out, &B.cgs->done, stream, dots, nbo);
        return kvs_unet_precondition(B.net, r_buf, B.Ap, B.grid, &B.cgs->net_in, &B.cgs->net_out, &B.cgs->done, stream,
                                     dots, nbo);
    };
    auto launch_init = [&](double* rbuf, int warm_flag) {
        if (res32)
            hipLaunchKernelGGL(cg_init_kernel<float>, dim3(nb), blk, 0, stream, g, B.F, B.phi,
                               reinterpret_cast<float*>(rbuf), warm_flag, part, npart);
        else
            hipLaunchKernelGGL(cg_init_kernel<double>, dim3(nb), blk, 0, stream, g, B.F, B.phi, rbuf, warm_flag, part,
                               npart);
    };
    launch_init(B.r, warm ? 1 : 0);
    hipLaunchKernelGGL(cg_finalize_kernel, dim3(1), dim3(256), 0, stream, part, nb, npart, 3, (int)FIN_INIT, B.cgs);
    CG_HIP(hipGetLastError());

    const SweepShape shp = sweep_shape(g.nx);
    SweepGeom sg{};
    sg.gx = (g.nx + 64 * shp.wx - 1) / (64 * shp.wx);
    sg.gy = (g.ny + shp.by - 1) / shp.by;
    {
        static const int cap1 = kvs_tiling::resident_blocks(cg_dir_kernel<1, 8, double, double>, 512);
        static const int cap2 = kvs_tiling::resident_blocks(cg_dir_kernel<2, 8, double, double>, 1024);
        static const int cap4 = kvs_tiling::resident_blocks(cg_dir_kernel<4, 4, double, double>, 1024);
        const int cap = shp.wx == 4 ? cap4 : (shp.wx == 2 ? cap2 : cap1);
        sg.kchunk = kvs_tiling::choose_kchunk(sg.gx * sg.gy, g.nz - 2, cap);
        sg.gz = (g.nz - 2 + sg.kchunk - 1) / sg.kchunk;
    }
    const int nbs = sg.gx * sg.gy * sg.gz;
    const dim3 sblk(64 * shp.wx, shp.by);
    // the direction buffers hold PT values (B.dir_fp32: float), the residual
    // buffers RT values (res32: float)
    auto launch_dir_t = [&](auto ptag, auto rtag, const double* r_buf, const double* zf_buf, const double* p_old_buf,
                            double* p_new_buf) {
        using PT = decltype(ptag);
        using RT = decltype(rtag);
        const RT* r_in = reinterpret_cast<const RT*>(r_buf);
        const RT* zf = reinterpret_cast<const RT*>(zf_buf);
        const PT* p_old = reinterpret_cast<const PT*>(p_old_buf);
        PT* p_new = reinterpret_cast<PT*>(p_new_buf);
        if (shp.wx == 4)
            hipLaunchKernelGGL((cg_dir_kernel<4, 4, PT, RT>), dim3(nbs), sblk, 0, stream, g, sg, r_in, zf, p_old,
                               p_new, B.cgs, part, npart);
        else if (shp.wx == 2)
            hipLaunchKernelGGL((cg_dir_kernel<2, 8, PT, RT>), dim3(nbs), sblk, 0, stream, g, sg, r_in, zf, p_old,
                               p_new, B.cgs, part, npart);
        else
            hipLaunchKernelGGL((cg_dir_kernel<1, 8, PT, RT>), dim3(nbs), sblk, 0, stream, g, sg, r_in, zf, p_old,
                               p_new, B.cgs, part, npart);
    };
    auto launch_upd_t = [&](auto ptag, auto rtag, const double* r_buf, double* r_out_buf, const double* p_buf) {
        using PT = decltype(ptag);
        using RT = decltype(rtag);
        const RT* r_in = reinterpret_cast<const RT*>(r_buf);
        RT* r_out = reinterpret_cast<RT*>(r_out_buf);
        const PT* pv = reinterpret_cast<const PT*>(p_buf);
        if (shp.wx == 4)
            hipLaunchKernelGGL((cg_upd_kernel<4, 4, PT, RT>), dim3(nbs), sblk, 0, stream, g, sg, B.phi, r_in, r_out,
                               pv, B.cgs, part, npart);
        else if (shp.wx == 2)
            hipLaunchKernelGGL((cg_upd_kernel<2, 8, PT, RT>), dim3(nbs), sblk, 0, stream, g, sg, B.phi, r_in, r_out,
                               pv, B.cgs, part, npart);
        else
            hipLaunchKernelGGL((cg_upd_kernel<1, 8, PT, RT>), dim3(nbs), sblk, 0, stream, g, sg, B.phi, r_in, r_out,
                               pv, B.cgs, part, npart);
    };
    auto launch_dir = [&](const double* r_in, const double* zf, const double* p_old, double* p_new) {
        if (B.dir_fp32 && res32)
            launch_dir_t(float{}, float{}, r_in, zf, p_old, p_new);
        else if (B.dir_fp32)
            launch_dir_t(float{}, double{}, r_in, zf, p_old, p_new);
        else if (res32)
            launch_dir_t(double{}, float{}, r_in, zf, p_old, p_new);
        else
            launch_dir_t(double{}, double{}, r_in, zf, p_old, p_new);
    };
    auto launch_upd = [&](const double* r_in, double* r_out, const double* pv) {
        if (B.dir_fp32 && res32)
            launch_upd_t(float{}, float{}, r_in, r_out, pv);
        else if (B.dir_fp32)
            launch_upd_t(float{}, double{}, r_in, r_out, pv);
        else if (res32)
            launch_upd_t(double{}, float{}, r_in, r_out, pv);
        else
            launch_upd_t(double{}, double{}, r_in, r_out, pv);
    };
    int pi = 0;  // p[pi] holds the current search direction
    const long long cap = (o->fixed_iters > 0 ? o->fixed_iters : o->max_iter) + 1;
    double* z = B.Ap;  // flexible PCG: the preconditioned residual
    const int* stop = &B.cgs->done;
    // flexible PCG keeps the previous residual for beta: the update writes
    // the new residual into the other buffer (rb[ri] is the current one)
    double* rb[2] = {B.r, flexible ? B.r2 : B.r};
    int ri = 0;
    if (flexible) {
        // z = U(r) and the partial sums of z.r from the network's output kernel
        const UnetDots dots{nullptr, part, npart};
        int nbo = 0;
        CG_HIP(precondition(rb[0], &dots, &nbo));
        hipLaunchKernelGGL(cg_finalize_kernel, dim3(1), dim3(256), 0, stream, part, nbo, npart, 3, (int)FIN_FZ0,
                           B.cgs);
        CG_HIP(hipGetLastError());
    }
    // Iterate until the device sets the stop flag (tolerance on the recursive
    // residual, max_iter, fixed_iters or a breakdown).
    // Reliable updates of an FP32 residual: its rounding at every update
    // makes the recursive r drift from -b - A phi by about 6e-8 of the
    // largest |r| since it was last exact, so whenever r.r has fallen by
    // kReplace since then (checked where the host reads the state), r is
    // recomputed from phi in FP64 and beta rescaled to it (FIN_REPLACE).
    constexpr double kReplace = 1e-4;  // r.r ratio: |r| down by 100
    auto iterate = [&]() -> kvs_status {
        int chunk = flexible ? 2 : 4;
        long long launched = 0;
        double rr_ref = -1.0;  // r.r when r was last exact (first read of this call)
        while (true) {
            for (int m = 0; m < chunk; ++m) {
                launch_dir(rb[ri], z, B.p[pi], B.p[1 - pi]);
                hipLaunchKernelGGL(cg_finalize_kernel, dim3(1), dim3(256), 0, stream, part, nbs, npart, 1,
                                   (int)FIN_ALPHA, B.cgs);
                launch_upd(rb[ri], rb[1 - ri], B.p[1 - pi]);
                hipLaunchKernelGGL(cg_finalize_kernel, dim3(1), dim3(256), 0, stream, part, nbs, npart, 2,
                                   (int)FIN_BETA, B.cgs);
                if (flexible) {
                    // z = U(r_new) with the partial sums of z.r_new, z.r_old, r_new.r_old
                    const UnetDots dots{rb[ri], part, npart};
                    int nbo = 0;
                    CG_HIP(precondition(rb[1 - ri], &dots, &nbo));
                    hipLaunchKernelGGL(cg_finalize_kernel, dim3(1), dim3(256), 0, stream, part, nbo, npart, 3,
                                       (int)FIN_FBETA, B.cgs);
                    ri = 1 - ri;
                }
                pi = 1 - pi;
            }
            CG_HIP(hipGetLastError());
            launched += chunk;
            CG_HIP(hipMemcpyAsync(B.cgs_host, B.cgs, sizeof(CgState), hipMemcpyDeviceToHost, stream));
            CG_HIP(hipStreamSynchronize(stream));
            if (B.cgs_host->done) break;
            if (launched > cap) return cg_fail(err, KVS_EDEVICE, "CG: iteration cap passed without a stop flag");
            if (res32) {
                if (rr_ref < 0.0) {
                    rr_ref = B.cgs_host->rr;
                } else if (B.cgs_host->rr < kReplace * rr_ref) {
                    launch_init(rb[ri], 1);
                    hipLaunchKernelGGL(cg_finalize_kernel, dim3(1), dim3(256), 0, stream, part, nb, npart, 3,
                                       (int)FIN_REPLACE, B.cgs);
                    CG_HIP(hipGetLastError());
                    rr_ref = B.cgs_host->rr;
                }
            }
            chunk = std::min(chunk * 2, flexible ? 8 : 64);
        }
        return KVS_OK;
    };
    {
        const kvs_status ist = iterate();
        if (ist != KVS_OK) return ist;
    }
    // b = 0 gives phi = 0, also when a warm start began from an earlier phi
    if (warm && B.cgs_host->bb == 0.0) CG_HIP(fill_zero(B.phi, g.N, stream));
    // Launches after the stop flag return at once; the host-side flip of pi
    // may then be off by those, which is harmless: the next solve (or restart)
    // starts with beta = 0, which rebuilds the direction from z alone.

    // Confirmation on the true residual (always for the flexible PCG, whose
    // recursive residual can drift from the true one when the preconditioner
    // changes between iterations; on request for CG / Jacobi-PCG): when the
    // recursive residual met tol but ||-b - A phi|| / ||b|| did not, restart
    // from the true residual and continue, counting iterations on.
    const bool confirm = (flexible || res32 || o->confirm_true) && o->fixed_iters <= 0;
    for (int restarts = 0;; ++restarts) {
        hipLaunchKernelGGL(cg_true_residual_kernel, dim3(nb), blk, 0, stream, g, B.F, B.phi, part, npart);
        hipLaunchKernelGGL(cg_finalize_kernel, dim3(1), dim3(256), 0, stream, part, nb, npart, 3, (int)FIN_TRUE,
                           B.cgs);
        CG_HIP(hipGetLastError());
        if (!confirm) break;
        CG_HIP(hipMemcpyAsync(B.cgs_host, B.cgs, sizeof(CgState), hipMemcpyDeviceToHost, stream));
        CG_HIP(hipStreamSynchronize(stream));
        const CgState& h = *B.cgs_host;
        if (h.status != KVS_OK || h.bb == 0.0 || !(h.relres_true2 >= h.tol2) || h.iters >= h.max_iter ||
            restarts >= 8)
            break;
        launch_init(rb[ri], 1);
        hipLaunchKernelGGL(cg_finalize_kernel, dim3(1), dim3(256), 0, stream, part, nb, npart, 3, (int)FIN_RESTART,
                           B.cgs);
        if (flexible) {
            const UnetDots dots{nullptr, part, npart};
            int nbo = 0;
            CG_HIP(precondition(rb[ri], &dots, &nbo));
            hipLaunchKernelGGL(cg_finalize_kernel, dim3(1), dim3(256), 0, stream, part, nbo, npart, 3, (int)FIN_FZ0,
                               B.cgs);
        }
        CG_HIP(hipGetLastError());
        const kvs_status ist = iterate();
        if (ist != KVS_OK) return ist;
    }
    const int status = B.cgs_host->status;
    if (status != KVS_EBREAKDOWN) {
        if (B.fs_fp32)
            hipLaunchKernelGGL(grad_subtract_kernel<float>, dim3(nb), blk, 0, stream, g, B.F, B.phi,
                               static_cast<float*>(B.FS));
        else
            hipLaunchKernelGGL(grad_subtract_kernel<double>, dim3(nb), blk, 0, stream, g, B.F, B.phi,
                               static_cast<double*>(B.FS));
    }
    CG_HIP(hipGetLastError());
    if (B.use_events) CG_HIP(hipEventRecord(e1, stream));
    CG_HIP(hipMemcpyAsync(B.cgs_host, B.cgs, sizeof(CgState), hipMemcpyDeviceToHost, stream));
    CG_HIP(hipStreamSynchronize(stream));
    float ms = 0.f;
    if (B.use_events) {
        CG_HIP(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    } else {
        ms = (float)std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    const CgState& s = *B.cgs_host;
    if (rep) {
        rep->iters = s.iters;
        rep->relres_recursive = s.bb > 0 ? std::sqrt(s.rr / s.bb) : 0.0;
        rep->relres_true = std::sqrt(s.relres_true2);
        rep->ms = ms;
        rep->status = s.status;
    }
    if (s.status == KVS_ENOTCONV) return cg_fail(err, KVS_ENOTCONV, "projection: CG reached max_iter above tolerance");
    if (s.status == KVS_EBREAKDOWN)
        return cg_fail(err, KVS_EBREAKDOWN, "projection: CG breakdown (p.Ap <= 0 or non-finite inner product)");
    return (kvs_status)s.status;
}

std::string cg_message(const CgErr& e) {
    std::string m = e.what ? e.what : "";
    if (e.hip) m += std::string(": ") + e.hip;
    return m;
}

}  // namespace

kvs_status kvs_run_projection(kvs_ctx* c, const kvs_solve_opts* o, kvs_solve_report* rep) {
    if (o->precond == KVS_PC_UNET && !c->r2) {
        const hipError_t e = c->mem.get(&c->r2, sizeof(double) * c->N);
        if (e != hipSuccess) {
            c->err = std::string("device allocation (second residual): ") + hipGetErrorString(e);
            return KVS_ENOMEM;
        }
        // its outer layer is read as zeros (by the sweeps and the network)
        // and never written: clear what the allocator handed over
        const hipError_t ez = fill_zero(c->r2, (long long)c->N, c->stream);
        if (ez != hipSuccess) {
            c->err = std::string("fill_zero_kernel: ") + hipGetErrorString(ez);
            return KVS_EDEVICE;
        }
    }
    CgBuffers B{};
    B.grid = c->grid;
    B.stream = c->stream;
    B.F = c->F;
    B.phi = c->phi;
    B.r = c->r;
    B.r2 = c->r2;
    B.p[0] = c->p[0];
    B.p[1] = c->p[1];
    B.Ap = c->Ap;
    B.partials = c->partials;
    B.npart = (int)c->npart;
    B.cgs = c->cgs;
    B.cgs_host = c->cgs_host;
    B.FS = c->FS;
    B.fs_fp32 = c->prec == KVS_FP32;
    B.net = c->net;
    B.warm = o->warm_start && c->have_phi;
    B.use_events = true;
    B.dir_fp32 = c->dir_prec == KVS_FP32;
    B.res_fp32 = c->res_prec == KVS_FP32;
    // the residual buffers' outer layer is read as zeros by the sweeps: clear
    // them when this solve views them at the other width than the last one
    if (B.res_fp32 != c->r_view32) {
        for (double* v : {c->r, c->r2}) {
            if (!v) continue;
            const hipError_t e = fill_zero(v, (long long)c->N, c->stream);
            if (e != hipSuccess) {
                c->err = std::string("fill_zero_kernel: ") + hipGetErrorString(e);
                return KVS_EDEVICE;
            }
        }
        c->r_view32 = B.res_fp32;
    }
    if (c->p_dirty) {
        for (double* v : {c->p[0], c->p[1]}) {
            const hipError_t e = fill_zero(v, (long long)c->N, c->stream);
            if (e != hipSuccess) {
                c->err = std::string("fill_zero_kernel: ") + hipGetErrorString(e);
                return KVS_EDEVICE;
            }
        }
        c->p_dirty = false;
    }
    CgErr err;
    const kvs_status st = cg_project(B, o, rep, err);
    if (st == KVS_EDEVICE && err.hip) {  // a HIP failure: the solve did not finish
        c->err = cg_message(err);
        return st;
    }
    if (st != KVS_OK && st != KVS_ENOTCONV && st != KVS_EBREAKDOWN) {
        c->err = cg_message(err);
        return st;
    }
    const CgState& s = *c->cgs_host;
    c->have_phi = true;
    if (s.status != KVS_EBREAKDOWN) c->fs_current = true;
    c->last_fallbacks = s.fallbacks;
    if (st != KVS_OK) c->err = cg_message(err);
    return st;
}

// ---- projection without allocation ------------------------------------------
//
// The CG work vectors, block partials and control block of
// kvs_project_noalloc live in one file-scope device array, `scratch`, of
// KVS_NOALLOC_SCRATCH_BYTES.  Each device holds its own copy; its address is
// taken once per device with hipGetSymbolAddress (the array's name is a host
// stand-in, never a device pointer) and every later use goes through that
// address.  Calls on one device share the array: calls that overlap on one
// device race.  Layout: CgState | partials (3 npart) | r | p0 | p1 | Ap.

namespace {

constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[KVS_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

thread_local char g_noalloc_err[256] = "";

kvs_status noalloc_fail(kvs_status s, const char* what, const char* detail = nullptr) {
    std::snprintf(g_noalloc_err, sizeof(g_noalloc_err), "%s%s%s", what, detail ? ": " : "", detail ? detail : "");
    return s;
}

// The device address of this device's scratch array (looked up once per
// device with the device current).
kvs_status scratch_address(int device, unsigned char** out) {
    if (device < 0 || device >= kMaxDevices) return noalloc_fail(KVS_EINVAL, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return noalloc_fail(KVS_EDEVICE, "hipGetSymbolAddress(scratch)", hipGetErrorString(e));
        g_scratch_ptr[device] = ptr;
    }
    *out = static_cast<unsigned char*>(g_scratch_ptr[device]);
    return KVS_OK;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Bytes of scratch a projection of `g` needs.
size_t noalloc_bytes(const kvs_grid& g, int64_t npart) {
    const size_t N = (size_t)g.nx * (size_t)g.ny * (size_t)g.nz;
    return align256(sizeof(CgState)) + align256(3 * (size_t)npart * sizeof(double)) + 4 * align256(N * sizeof(double));
}

// Zero the outer layer of `ncomp` consecutive scalar fields of double.
__global__ void zero_outer_kernel(double* f, int nx, int ny, int nz, int ncomp) {
    const long long N = (long long)nx * ny * nz;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < N * ncomp;
         q += (long long)gridDim.x * blockDim.x) {
        const long long c = q % N;
        const int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / ((long long)nx * ny));
        if (i == 0 || i == nx - 1 || j == 0 || j == ny - 1 || k == 0 || k == nz - 1) f[q] = 0.0;
    }
}

}  // namespace

kvs_status kvs_project_noalloc(const kvs_grid* grid, const double* F, double* phi, double* FS,
                               const kvs_solve_opts* opts, int32_t device, void* stream, kvs_solve_report* rep) {
    g_noalloc_err[0] = 0;
    if (!grid || !F || !phi || !FS) return noalloc_fail(KVS_EINVAL, "grid, F, phi and FS must be non-NULL");
    const kvs_grid& g = *grid;
    if (g.nx < 3 || g.ny < 3 || g.nz < 3 || !(g.hx > 0) || !(g.hy > 0) || !(g.hz > 0) || !std::isfinite(g.hx) ||
        !std::isfinite(g.hy) || !std::isfinite(g.hz))
        return noalloc_fail(KVS_EINVAL, "grid needs n >= 3 per axis and finite spacings > 0");
    kvs_solve_opts o{};
    o.tol = 1e-8;
    o.max_iter = 10000;
    o.precond = KVS_PC_JACOBI;
    if (opts) o = *opts;
    if (o.fixed_iters < 0) return noalloc_fail(KVS_EINVAL, "fixed_iters < 0");
    if (o.fixed_iters == 0 && !(o.tol > 0.0 && std::isfinite(o.tol))) return noalloc_fail(KVS_EINVAL, "tol must be > 0");
    if (o.max_iter <= 0) return noalloc_fail(KVS_EINVAL, "max_iter must be > 0");
    if (o.precond != KVS_PC_NONE && o.precond != KVS_PC_JACOBI)
        return noalloc_fail(KVS_EINVAL, "the allocation-free projection runs CG or Jacobi-PCG only");
    const int64_t npart = std::max<int64_t>(kvs_cg_partials_needed(g), 2048);
    const size_t need = noalloc_bytes(g, npart);
    if ((double)g.nx * (double)g.ny * (double)g.nz > 2.0e9 || need > (size_t)KVS_NOALLOC_SCRATCH_BYTES) {
        char detail[160];
        std::snprintf(detail, sizeof(detail), "grid %lldx%lldx%lld needs %zu bytes of scratch, the maximum is %zu",
                      (long long)g.nx, (long long)g.ny, (long long)g.nz, need, (size_t)KVS_NOALLOC_SCRATCH_BYTES);
        return noalloc_fail(KVS_EINVAL, "grid too large for the allocation-free projection", detail);
    }
    {
        const hipError_t e = hipSetDevice(device);
        if (e != hipSuccess) return noalloc_fail(KVS_EDEVICE, "hipSetDevice", hipGetErrorString(e));
    }
    unsigned char* base = nullptr;
    {
        const kvs_status st = scratch_address(device, &base);
        if (st != KVS_OK) return st;
    }
    const size_t N = (size_t)g.nx * (size_t)g.ny * (size_t)g.nz;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        unsigned char* q = base + off;
        off += align256(bytes);
        return q;
    };
    CgState host_state{};
    CgBuffers B{};
    B.grid = g;
    B.stream = static_cast<hipStream_t>(stream);
    B.F = F;
    B.phi = phi;
    B.cgs = reinterpret_cast<CgState*>(take(sizeof(CgState)));
    B.partials = reinterpret_cast<double*>(take(3 * (size_t)npart * sizeof(double)));
    B.npart = (int)npart;
    B.r = reinterpret_cast<double*>(take(N * sizeof(double)));
    B.p[0] = reinterpret_cast<double*>(take(N * sizeof(double)));
    B.p[1] = reinterpret_cast<double*>(take(N * sizeof(double)));
    B.Ap = reinterpret_cast<double*>(take(N * sizeof(double)));
    B.r2 = nullptr;
    B.cgs_host = &host_state;
    B.FS = FS;
    B.fs_fp32 = 0;
    B.net = nullptr;
    B.warm = o.warm_start != 0;
    B.use_events = false;
    // The sweeps read the outer layer of r and of both directions (never
    // written there, 0 in a context since its creation): the shared array
    // holds whatever the last call left, so clear them on every call.
    for (double* v : {B.r, B.p[0], B.p[1]}) {
        const hipError_t e = fill_zero(v, (long long)N, B.stream);
        if (e != hipSuccess) return noalloc_fail(KVS_EDEVICE, "fill_zero_kernel", hipGetErrorString(e));
    }
    // outer layers: phi (a warm start's guess) and FS are 0 there
    const unsigned nbz = (unsigned)std::min<size_t>((3 * N + 255) / 256, 4096);
    if (B.warm) hipLaunchKernelGGL(zero_outer_kernel, dim3(nbz), dim3(256), 0, B.stream, phi, (int)g.nx, (int)g.ny,
                                   (int)g.nz, 1);
    hipLaunchKernelGGL(zero_outer_kernel, dim3(nbz), dim3(256), 0, B.stream, FS, (int)g.nx, (int)g.ny, (int)g.nz, 3);
    {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return noalloc_fail(KVS_EDEVICE, "zero_outer_kernel", hipGetErrorString(e));
    }
    CgErr err;
    const kvs_status st = cg_project(B, &o, rep, err);
    if (st != KVS_OK) noalloc_fail(st, err.what ? err.what : "projection failed", err.hip);
    return st;
}

const char* kvs_noalloc_last_error(void) { return g_noalloc_err; }
