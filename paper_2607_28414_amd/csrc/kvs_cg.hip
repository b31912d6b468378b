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
#include <cmath>

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

enum { FIN_INIT = 0, FIN_ALPHA = 1, FIN_BETA = 2, FIN_TRUE = 3, FIN_FZ0 = 4, FIN_FBETA = 5, FIN_RESTART = 6 };

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
__global__ __launch_bounds__(64 * CBY) void cg_init_kernel(const CgGeom g, const double* F, const double* phi,
                                                           double* r, int warm, double* partials, int npart) {
    const Tile t = tile_coords(g);
    const int sxy = g.nx * g.ny;
    double s1 = 0, s2 = 0, s3 = 0;
    if (t.act) {
        for (int k = t.kb; k < t.ke; ++k) {
            const int idx = k * sxy + t.col;
            const double b = div_at(g, F, idx);
            double rv = -b;
            if (warm) rv -= negative_lap_at(g, phi, idx);
            r[idx] = rv;
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
template <int WX, int SBY>
__global__ __launch_bounds__(64 * WX * SBY) void cg_dir_kernel(const CgGeom g, const SweepGeom sg, const double* r_in,
                                                               const double* zf, const double* p_old, double* p_new,
                                                               const CgState* st, double* partials, int npart) {
    if (st->done) return;
    __shared__ double lds[2][SBY + 3][64 * WX + 4];
    const Lane L = sweep_lane<WX, SBY>(g, sg);
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int sxy = g.nx * g.ny;
    const double beta = st->beta;
    const bool net_z = st->flexible && !st->zjacobi;
    const double* r = net_z ? zf : r_in;
    const double zs = (st->jacobi || (st->flexible && st->zjacobi)) ? g.dinv : 1.0;
    const bool first = beta == 0.0;
    auto pv = [&](double rv, double po) { return first ? rv * zs : rv * zs + beta * po; };
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
        const double rn = r[q2], on = p_old[q2], hrn = r[qh], hon = p_old[qh];
        lds_barrier();
        const double c2 = 2.0 * pc;
        const double ap = -((lds[buf][ty + 1][tx + 2] + lds[buf][ty + 1][tx] - c2) * g.ihx2
                            + (lds[buf][ty + 2][tx + 1] + lds[buf][ty][tx + 1] - c2) * g.ihy2
                            + (pp + pm - c2) * g.ihz2);
        s1 += L.act ? pc * ap : 0.0;
        p_new[k * sxy + L.scol] = L.act ? pc : 0.0;
        pm = pc;
        pc = pp;
        pp = pv(rn, on);
        hc = pv(hrn, hon);
    }
    sweep_partials<1, WX, SBY>(s1, 0.0, partials, npart);
}

// sweep 2: A p recomputed, phi += alpha p, r_out = r - alpha A p (r_out may
// be r itself), partials r.r, r.z
template <int WX, int SBY>
__global__ __launch_bounds__(64 * WX * SBY) void cg_upd_kernel(const CgGeom g, const SweepGeom sg, double* phi,
                                                               const double* r, double* r_out, const double* p,
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
        const double phn = phi[q1], rn = r[q1];
        lds_barrier();
        const double c2 = 2.0 * pc;
        const double ap = -((lds[buf][ty + 1][tx + 2] + lds[buf][ty + 1][tx] - c2) * g.ihx2
                            + (lds[buf][ty + 2][tx + 1] + lds[buf][ty][tx + 1] - c2) * g.ihy2
                            + (pp + pm - c2) * g.ihz2);
        const double phv = phc + alpha * pc;
        const double rv = rc - alpha * ap;
        const int q = k * sxy + L.scol;
        phi[q] = L.act ? phv : 0.0;
        r_out[q] = L.act ? rv : 0.0;
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

kvs_status fail(kvs_ctx* c, kvs_status s, const std::string& msg) {
    c->err = msg;
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

#define CG_HIP(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return fail(c, KVS_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

kvs_status kvs_run_projection(kvs_ctx* c, const kvs_solve_opts* o, kvs_solve_report* rep) {
    const CgGeom g = make_geom(c->grid);
    const int nb = nblocks(g);
    const dim3 blk(64, CBY);
    double* part = c->partials;
    const int npart = (int)c->npart;

    hipEvent_t e0, e1;
    CG_HIP(hipEventCreate(&e0));
    CG_HIP(hipEventCreate(&e1));
    CG_HIP(hipEventRecord(e0, c->stream));

    const bool flexible = o->precond == KVS_PC_UNET;
    CgState init{};
    init.tol2 = o->tol * o->tol;
    init.max_iter = o->max_iter;
    init.fixed_iters = o->fixed_iters;
    init.jacobi = o->precond == KVS_PC_JACOBI ? 1 : 0;
    init.flexible = flexible ? 1 : 0;
    init.dinv = g.dinv;
    init.h2 = c->grid.hx * c->grid.hx;
    init.n_interior = (double)(g.nx - 2) * (double)(g.ny - 2) * (double)(g.nz - 2);
    *c->cgs_host = init;
    CG_HIP(hipMemcpyAsync(c->cgs, c->cgs_host, sizeof(CgState), hipMemcpyHostToDevice, c->stream));
    const bool warm = o->warm_start && c->have_phi;
    if (!warm) CG_HIP(hipMemsetAsync(c->phi, 0, sizeof(double) * c->N, c->stream));

    hipLaunchKernelGGL(cg_init_kernel, dim3(nb), blk, 0, c->stream, g, c->F, c->phi, c->r, warm ? 1 : 0, part, npart);
    hipLaunchKernelGGL(cg_finalize_kernel, dim3(1), dim3(256), 0, c->stream, part, nb, npart, 3, (int)FIN_INIT, c->cgs);
    CG_HIP(hipGetLastError());

    const SweepShape shp = sweep_shape(g.nx);
    SweepGeom sg{};
    sg.gx = (g.nx + 64 * shp.wx - 1) / (64 * shp.wx);
    sg.gy = (g.ny + shp.by - 1) / shp.by;
    {
        static const int cap1 = kvs_tiling::resident_blocks(cg_dir_kernel<1, 8>, 512);
        static const int cap2 = kvs_tiling::resident_blocks(cg_dir_kernel<2, 8>, 1024);
        static const int cap4 = kvs_tiling::resident_blocks(cg_dir_kernel<4, 4>, 1024);
        const int cap = shp.wx == 4 ? cap4 : (shp.wx == 2 ? cap2 : cap1);
        sg.kchunk = kvs_tiling::choose_kchunk(sg.gx * sg.gy, g.nz - 2, cap);
        sg.gz = (g.nz - 2 + sg.kchunk - 1) / sg.kchunk;
    }
    const int nbs = sg.gx * sg.gy * sg.gz;
    const dim3 sblk(64 * shp.wx, shp.by);
    auto launch_dir = [&](const double* r_in, const double* zf, const double* p_old, double* p_new) {
        if (shp.wx == 4)
            hipLaunchKernelGGL((cg_dir_kernel<4, 4>), dim3(nbs), sblk, 0, c->stream, g, sg, r_in, zf, p_old, p_new,
                               c->cgs, part, npart);
        else if (shp.wx == 2)
            hipLaunchKernelGGL((cg_dir_kernel<2, 8>), dim3(nbs), sblk, 0, c->stream, g, sg, r_in, zf, p_old, p_new,
                               c->cgs, part, npart);
        else
            hipLaunchKernelGGL((cg_dir_kernel<1, 8>), dim3(nbs), sblk, 0, c->stream, g, sg, r_in, zf, p_old, p_new,
                               c->cgs, part, npart);
    };
    auto launch_upd = [&](const double* r_in, double* r_out, const double* pv) {
        if (shp.wx == 4)
            hipLaunchKernelGGL((cg_upd_kernel<4, 4>), dim3(nbs), sblk, 0, c->stream, g, sg, c->phi, r_in, r_out, pv,
                               c->cgs, part, npart);
        else if (shp.wx == 2)
            hipLaunchKernelGGL((cg_upd_kernel<2, 8>), dim3(nbs), sblk, 0, c->stream, g, sg, c->phi, r_in, r_out, pv,
                               c->cgs, part, npart);
        else
            hipLaunchKernelGGL((cg_upd_kernel<1, 8>), dim3(nbs), sblk, 0, c->stream, g, sg, c->phi, r_in, r_out, pv,
                               c->cgs, part, npart);
    };
    int pi = 0;  // p[pi] holds the current search direction
    const long long cap = (o->fixed_iters > 0 ? o->fixed_iters : o->max_iter) + 1;
    double* z = c->Ap;  // flexible PCG: the preconditioned residual
    const int* stop = &c->cgs->done;
    // flexible PCG keeps the previous residual for beta: the update writes
    // the new residual into the other buffer (rb[ri] is the current one)
    if (flexible && !c->r2) CG_HIP(hipMalloc(&c->r2, sizeof(double) * c->N));
    double* rb[2] = {c->r, flexible ? c->r2 : c->r};
    int ri = 0;
    if (flexible) {
        // z = U(r) and the partial sums of z.r from the network's output kernel
        const UnetDots dots{nullptr, part, npart};
        int nbo = 0;
        CG_HIP(kvs_unet_precondition(c->net, rb[0], z, c->grid, &c->cgs->net_in, &c->cgs->net_out, stop, c->stream,
                                     &dots, &nbo));
        hipLaunchKernelGGL(cg_finalize_kernel, dim3(1), dim3(256), 0, c->stream, part, nbo, npart, 3, (int)FIN_FZ0,
                           c->cgs);
        CG_HIP(hipGetLastError());
    }
    // Iterate until the device sets the stop flag (tolerance on the recursive
    // residual, max_iter, fixed_iters or a breakdown).
    auto iterate = [&]() -> kvs_status {
    int chunk = flexible ? 2 : 4;
    long long launched = 0;
    while (true) {
        for (int m = 0; m < chunk; ++m) {
            launch_dir(rb[ri], z, c->p[pi], c->p[1 - pi]);
            hipLaunchKernelGGL(cg_finalize_kernel, dim3(1), dim3(256), 0, c->stream, part, nbs, npart, 1, (int)FIN_ALPHA,
                               c->cgs);
            launch_upd(rb[ri], rb[1 - ri], c->p[1 - pi]);
            hipLaunchKernelGGL(cg_finalize_kernel, dim3(1), dim3(256), 0, c->stream, part, nbs, npart, 2, (int)FIN_BETA,
                               c->cgs);
            if (flexible) {
                // z = U(r_new) with the partial sums of z.r_new, z.r_old, r_new.r_old
                const UnetDots dots{rb[ri], part, npart};
                int nbo = 0;
                CG_HIP(kvs_unet_precondition(c->net, rb[1 - ri], z, c->grid, &c->cgs->net_in, &c->cgs->net_out, stop,
                                             c->stream, &dots, &nbo));
                hipLaunchKernelGGL(cg_finalize_kernel, dim3(1), dim3(256), 0, c->stream, part, nbo, npart, 3,
                                   (int)FIN_FBETA, c->cgs);
                ri = 1 - ri;
            }
            pi = 1 - pi;
        }
        CG_HIP(hipGetLastError());
        launched += chunk;
        CG_HIP(hipMemcpyAsync(c->cgs_host, c->cgs, sizeof(CgState), hipMemcpyDeviceToHost, c->stream));
        CG_HIP(hipStreamSynchronize(c->stream));
        if (c->cgs_host->done) break;
        if (launched > cap) return fail(c, KVS_EDEVICE, "CG: iteration cap passed without a stop flag");
        chunk = std::min(chunk * 2, flexible ? 8 : 64);
    }
    return KVS_OK;
    };
    {
        const kvs_status ist = iterate();
        if (ist != KVS_OK) return ist;
    }
    // b = 0 gives phi = 0, also when a warm start began from an earlier phi
    if (warm && c->cgs_host->bb == 0.0) CG_HIP(hipMemsetAsync(c->phi, 0, sizeof(double) * c->N, c->stream));
    // Launches after the stop flag return at once; the host-side flip of pi
    // may then be off by those, which is harmless: the next solve (or restart)
    // starts with beta = 0, which rebuilds the direction from z alone.

    // Confirmation on the true residual (always for the flexible PCG, whose
    // recursive residual can drift from the true one when the preconditioner
    // changes between iterations; on request for CG / Jacobi-PCG): when the
    // recursive residual met tol but ||-b - A phi|| / ||b|| did not, restart
    // from the true residual and continue, counting iterations on.
    const bool confirm = (flexible || o->confirm_true) && o->fixed_iters <= 0;
    for (int restarts = 0;; ++restarts) {
        hipLaunchKernelGGL(cg_true_residual_kernel, dim3(nb), blk, 0, c->stream, g, c->F, c->phi, part, npart);
        hipLaunchKernelGGL(cg_finalize_kernel, dim3(1), dim3(256), 0, c->stream, part, nb, npart, 3, (int)FIN_TRUE,
                           c->cgs);
        CG_HIP(hipGetLastError());
        if (!confirm) break;
        CG_HIP(hipMemcpyAsync(c->cgs_host, c->cgs, sizeof(CgState), hipMemcpyDeviceToHost, c->stream));
        CG_HIP(hipStreamSynchronize(c->stream));
        const CgState& h = *c->cgs_host;
        if (h.status != KVS_OK || h.bb == 0.0 || !(h.relres_true2 >= h.tol2) || h.iters >= h.max_iter ||
            restarts >= 8)
            break;
        hipLaunchKernelGGL(cg_init_kernel, dim3(nb), blk, 0, c->stream, g, c->F, c->phi, rb[ri], 1, part, npart);
        hipLaunchKernelGGL(cg_finalize_kernel, dim3(1), dim3(256), 0, c->stream, part, nb, npart, 3,
                           (int)FIN_RESTART, c->cgs);
        if (flexible) {
            const UnetDots dots{nullptr, part, npart};
            int nbo = 0;
            CG_HIP(kvs_unet_precondition(c->net, rb[ri], z, c->grid, &c->cgs->net_in, &c->cgs->net_out, stop,
                                         c->stream, &dots, &nbo));
            hipLaunchKernelGGL(cg_finalize_kernel, dim3(1), dim3(256), 0, c->stream, part, nbo, npart, 3,
                               (int)FIN_FZ0, c->cgs);
        }
        CG_HIP(hipGetLastError());
        const kvs_status ist = iterate();
        if (ist != KVS_OK) return ist;
    }
    const int status = c->cgs_host->status;
    if (status != KVS_EBREAKDOWN) {
        if (c->prec == KVS_FP32)
            hipLaunchKernelGGL(grad_subtract_kernel<float>, dim3(nb), blk, 0, c->stream, g, c->F, c->phi,
                               static_cast<float*>(c->FS));
        else
            hipLaunchKernelGGL(grad_subtract_kernel<double>, dim3(nb), blk, 0, c->stream, g, c->F, c->phi,
                               static_cast<double*>(c->FS));
    }
    CG_HIP(hipGetLastError());
    CG_HIP(hipEventRecord(e1, c->stream));
    CG_HIP(hipMemcpyAsync(c->cgs_host, c->cgs, sizeof(CgState), hipMemcpyDeviceToHost, c->stream));
    CG_HIP(hipStreamSynchronize(c->stream));
    float ms = 0.f;
    CG_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);

    const CgState& s = *c->cgs_host;
    c->have_phi = true;
    if (s.status != KVS_EBREAKDOWN) c->fs_current = true;
    c->last_fallbacks = s.fallbacks;
    if (rep) {
        rep->iters = s.iters;
        rep->relres_recursive = s.bb > 0 ? std::sqrt(s.rr / s.bb) : 0.0;
        rep->relres_true = std::sqrt(s.relres_true2);
        rep->ms = ms;
        rep->status = s.status;
    }
    if (s.status != KVS_OK)
        c->err = s.status == KVS_ENOTCONV ? "projection: CG reached max_iter above tolerance"
                                          : "projection: CG breakdown (p.Ap <= 0 or non-finite inner product)";
    return (kvs_status)s.status;
}
