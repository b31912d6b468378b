// Two FDTD steps per pass over the state (temporal blocking) for FP32 viscous
// media, heterogeneous or homogeneous, whose x rows fit one tile
// (nx <= 64 WX): the Sec. 3.1 update of kvs_step_tile.hpp applied twice, with
// the same FP32 operations in the same order, so the result is bitwise that
// of two one-step launches.  The per-tile code, shared by the single-context
// kernel (kvs_step2.hip) and the batched one (kvs_batch.hip).
//
// A block of 64 WX x R threads owns R - 2 output rows y0 .. y0 + R - 3 of
// every plane of a z segment.  Thread row r (0 .. R - 1) computes the
// intermediate state (step n + 1) on row y0 - 1 + r, i.e. the output rows and
// one row on each side, from the input state staged in LDS on rows
// y0 - 2 .. y0 + R - 1 (its z neighbours in a per-thread register queue);
// thread rows 1 .. R - 2 then advance their rows to step n + 2 from the
// intermediate state staged in LDS (z neighbours again in registers).  The march computes the intermediate
// state one plane ahead of the second step: at iteration k it forms plane k
// of step n + 1 and plane k - 1 of step n + 2, so one barrier per plane
// orders both.  Per two cell-updates the input is read and the output written
// once (60 B); the intermediate rows on each side and the intermediate planes
// at the segment ends are computed twice (R / (R - 2) / 2 + 1/2 updates of
// arithmetic per output cell-update: 1.5 for R = 4).  The kernel is bound by
// vector-ALU issue, not HBM.
//
// Face moduli: harm(G, G') / h^2 = 2 G G' / (G + G') / h^2 is formed as
// (G G') rcp(G + G') (2 / h^2).  Scaling by 2 is exact, so this is the same
// rounded value as the one-step kernel's ((2 G) G') rcp(G + G') / h^2, and it
// does not depend on the operand order (products and sums commute exactly):
// the z- face of plane k is the z+ face of plane k - 1, carried over, and the
// second step reuses the faces of the first.
//
// Probe values of the intermediate state: written by the thread that owns its
// cell (output rows, planes of its own segment), found through a table with
// one entry per 64-cell row segment that is fetched a plane ahead with the
// other prefetches (a lookup per plane would drain the prefetch queue).
#pragma once

#include "kvs_step_tile.hpp"

namespace {

constexpr int S2_ROWS = 4;  // thread rows of the single-context tiles (two output rows)

struct Step2Args {
    StepArgs<float> a;
    const int* rowtab;  // [nz][ny][ceil(nx / 64)]: offset of row (j, k) in ptab where
                        // its 64-cell segment holds a probe, else -1
    const int* ptab;    // per probed row, nx entries: probe index or -1
    double* pmid;       // trace slot of the intermediate state
};

// Global-memory views of the argument pointers: a pointer read from a table
// in memory (the batched launch) is otherwise generic, and flat accesses also
// count against the LDS wait counter, so the wait before each barrier would
// drain the plane-ahead prefetch.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> glob(T* p) {
    return (gptr<T>)p;
}

// One tile of R thread rows: output rows (R - 2) by .. (R - 2) by + R - 3 of
// the planes of z segment bz (thread rows 1 .. R - 2; rows 0 and R - 1 form
// the intermediate state of the rows next to them).
template <bool HET, int WX, int R>
__device__ __forceinline__ void step2_tile(const Step2Args& A2, int by, int bz) {
    static_assert(R >= 3 && 64 * WX * R <= 1024, "3 .. 1024 / (64 WX) thread rows");
    const StepArgs<float>& a = A2.a;
    constexpr int TX = 64 * WX, W = TX + 2;  // LDS row: cell i at column i + 1
    constexpr int NQ = HET ? 7 : 6;          // u (3), w (3), G (heterogeneous)
    __shared__ float sn[2][NQ][R + 2][W];  // input planes, rows y0 - 2 .. y0 + R - 1
    __shared__ float s1[2][6][R][W];       // intermediate planes, rows y0 - 1 .. y0 + R - 2

    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int y0 = (R - 2) * by;
    const int kb = 1 + bz * a.kchunk;
    const int ke = min(nz - 1, kb + a.kchunk);  // output planes kb .. ke - 1
    // a wavefront is 64 threads of one thread row (blockDim.x = 64 WX), so the
    // row index is uniform across it: kept in a scalar register, the row tests
    // below are scalar branches
    const int tx = threadIdx.x, ty = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int i = tx, j = y0 - 1 + ty;  // this thread's cell column and row
    const int lc = i + 1;
    const bool inrow = i < nx && j >= 0 && j < ny;
    const bool act = i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2;  // interior in x and y
    const bool own = ty >= 1 && ty <= R - 2;                           // output rows
    // the output rows carry both steps: issued first, they reach the second
    // step while the halo rows still form the first, instead of running it
    // alone at the end of each plane (2 % per step at 256^3)
    if (own) __builtin_amdgcn_s_setprio(1);
    const int sxy = nx * ny;
    const int col = inrow ? i + nx * j : 0;
    // halo rows of the input plane: thread row 0 loads row y0 - 2 (LDS row 0),
    // thread row R - 1 row y0 + R - 1 (LDS row R + 1); rows outside the grid
    // stage zeros
    const bool hload = ty == 0 || ty == R - 1;
    const int hj = ty == 0 ? y0 - 2 : y0 + R - 1;
    const bool hin = hload && i < nx && hj >= 0 && hj < ny;
    const int hcol = hin ? i + nx * hj : 0;
    const int hrow = ty == 0 ? 0 : R + 1;

    gptr<const float> fp[NQ];
    fp[0] = glob(a.u);
    fp[1] = glob(a.u + a.N);
    fp[2] = glob(a.u + 2 * a.N);
    fp[3] = glob(a.w);
    fp[4] = glob(a.w + a.N);
    fp[5] = glob(a.w + 2 * a.N);
    if constexpr (HET) fp[NQ - 1] = glob(a.G);
    const gptr<const float> crho_g = glob(a.crho), eta_g = glob(a.eta);
    auto clampz = [&](int k) { return min(max(k, 0), nz - 1); };
    const float rx = a.L > 0 ? ramp<float>(i, nx, a.L, a.invL) : 0.f;
    const float rxy = a.L > 0 ? max(rx, ramp<float>(j, ny, a.L, a.invL)) : 0.f;
    const float ihx2 = a.ihx2, ihy2 = a.ihy2, ihz2 = a.ihz2;
    const float h2x = 2.f * ihx2, h2y = 2.f * ihy2, h2z = 2.f * ihz2;
    auto face = [](float g, float gn, float h2) { return g * gn * __builtin_amdgcn_rcpf(g + gn) * h2; };
    // probes: this wavefront's row-segment entry of the table (tx >> 6 is the
    // wavefront's index in its row)
    const bool probes = A2.pmid != nullptr && own && j < ny;  // uniform across a wavefront
    const int nseg = (nx + 63) >> 6;
    const gptr<const int> rowtab_j = glob(probes ? A2.rowtab + j * nseg + (tx >> 6) : nullptr);
    auto rowoff = [&](int k) { return k >= kb && k < ke ? rowtab_j[ny * nseg * k] : -1; };

    // input queue (planes k - 1, k, k + 1, prefetched k + 2) of this cell,
    // halo row value (plane k, prefetched k + 1), per-cell material (k, k + 1)
    float zm[NQ], zc[NQ], zp[NQ], zn[NQ], hc[NQ], hn[NQ];
    const int k0 = kb - 1;  // first intermediate plane
#pragma unroll
    for (int f = 0; f < NQ; ++f) {
        zm[f] = fp[f][clampz(k0 - 1) * sxy + col];
        zc[f] = fp[f][clampz(k0) * sxy + col];
        zp[f] = fp[f][clampz(k0 + 1) * sxy + col];
        hc[f] = hn[f] = 0.f;
    }
    if (hload) {
#pragma unroll
        for (int f = 0; f < NQ; ++f) hc[f] = fp[f][clampz(k0) * sxy + hcol];
    }
    // heterogeneous: z- face of the current plane; homogeneous: the six faces
    // G / h^2 of the one-step kernel, constant
    float fz = 0.f, gx0 = 0.f, gy0 = 0.f, gz0 = 0.f;
    float crho_c = a.crho0, eta_c = 0.f;
    if constexpr (HET) {
        fz = face(zc[NQ - 1], zm[NQ - 1], h2z);
        crho_c = crho_g[clampz(k0) * sxy + col];
        eta_c = eta_g[clampz(k0) * sxy + col];
    } else {
        gx0 = a.G0 * ihx2;
        gy0 = a.G0 * ihy2;
        gz0 = a.G0 * ihz2;
    }
    float crho_n = 0.f, eta_n = 0.f;
    // intermediate state of this cell at planes k - 2, k - 1 (q: plane k, just
    // formed), the face moduli and material of plane k - 1, for the second step
    float qm[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, qc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float fprev[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float crho_p = crho_c, eta_p = eta_c;  // homogeneous: the constants throughout
    int poff = probes ? rowoff(k0) : -1, poff_n = -1;
    for (int k = k0; k <= ke; ++k) {
        const int buf = k & 1;
#pragma unroll
        for (int f = 0; f < NQ; ++f) sn[buf][f][ty + 1][lc] = inrow ? zc[f] : 0.f;
        if (hload) {
#pragma unroll
            for (int f = 0; f < NQ; ++f) sn[buf][f][hrow][lc] = hin ? hc[f] : 0.f;
        }
        // prefetch plane k + 2 of the queue, the halo and material of k + 1 and
        // the probe entry of k + 1
#pragma unroll
        for (int f = 0; f < NQ; ++f) zn[f] = fp[f][clampz(k + 2) * sxy + col];
        if (hload) {
#pragma unroll
            for (int f = 0; f < NQ; ++f) hn[f] = fp[f][clampz(k + 1) * sxy + hcol];
        }
        if constexpr (HET) {
            crho_n = __builtin_nontemporal_load(crho_g + clampz(k + 1) * sxy + col);
            eta_n = __builtin_nontemporal_load(eta_g + clampz(k + 1) * sxy + col);
        }
        if (probes) poff_n = rowoff(k + 1);
        lds_barrier();

        // ---- step n + 1 at (i, j, k) ----
        const bool a1c = act && k >= 1 && k <= nz - 2;
        float fcur[6];
        float q[6];
        {
            if constexpr (HET) {
                const float Gc = zc[NQ - 1];
                fcur[0] = face(Gc, sn[buf][NQ - 1][ty + 1][lc - 1], h2x);
                fcur[1] = face(Gc, sn[buf][NQ - 1][ty + 1][lc + 1], h2x);
                fcur[2] = face(Gc, sn[buf][NQ - 1][ty][lc], h2y);
                fcur[3] = face(Gc, sn[buf][NQ - 1][ty + 2][lc], h2y);
                fcur[4] = fz;
                fcur[5] = face(Gc, zp[NQ - 1], h2z);
            } else {
                fcur[0] = fcur[1] = gx0;
                fcur[2] = fcur[3] = gy0;
                fcur[4] = fcur[5] = gz0;
            }
            const float rz = a.L > 0 ? ramp<float>(k, nz, a.L, a.invL) : 0.f;
            const float s = a.half_dt_smax * max(rxy, rz);
            const float inv1ps = rcp_fast<float>(1.f + s);
            const float c1 = (1.f - s) * inv1ps;
            const float c2 = crho_c * inv1ps;
            const float eta_dt = HET ? eta_c * a.inv_dt : a.eta_dt0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float uc = zc[c];
                float acc = fcur[1] * (sn[buf][c][ty + 1][lc + 1] - uc) - fcur[0] * (uc - sn[buf][c][ty + 1][lc - 1])
                          + fcur[3] * (sn[buf][c][ty + 2][lc] - uc) - fcur[2] * (uc - sn[buf][c][ty][lc])
                          + fcur[5] * (zp[c] - uc) - fcur[4] * (uc - zm[c]);
                const float wc = zc[3 + c];
                const float lw = (sn[buf][3 + c][ty + 1][lc + 1] + sn[buf][3 + c][ty + 1][lc - 1] - 2.f * wc) * ihx2
                               + (sn[buf][3 + c][ty + 2][lc] + sn[buf][3 + c][ty][lc] - 2.f * wc) * ihy2
                               + (zp[3 + c] + zm[3 + c] - 2.f * wc) * ihz2;
                acc += eta_dt * lw;
                const float wnew = c1 * wc + c2 * acc;
                q[3 + c] = a1c ? wnew : 0.f;
                q[c] = a1c ? uc + wnew : 0.f;
            }
        }
#pragma unroll
        for (int f = 0; f < 6; ++f) s1[buf][f][ty][lc] = q[f];
        if (poff >= 0 && inrow) {
            const int p = glob(A2.ptab)[poff + i];
            if (p >= 0) {
                if (a.pcomp == 3) {
                    glob(A2.pmid)[3 * p] = (double)q[0];
                    glob(A2.pmid)[3 * p + 1] = (double)q[1];
                    glob(A2.pmid)[3 * p + 2] = (double)q[2];
                } else {
                    glob(A2.pmid)[p] = (double)q[a.pcomp];
                }
            }
        }

        // ---- step n + 2 at (i, j, k - 1), output rows ----
        const int k2 = k - 1;
        if (own && k2 >= kb && k2 < ke) {
            const int bb = k2 & 1;
            const float rz = a.L > 0 ? ramp<float>(k2, nz, a.L, a.invL) : 0.f;
            const float s = a.half_dt_smax * max(rxy, rz);
            const float inv1ps = rcp_fast<float>(1.f + s);
            const float c1 = (1.f - s) * inv1ps;
            const float c2 = crho_p * inv1ps;
            const float eta_dt = HET ? eta_p * a.inv_dt : a.eta_dt0;
            float uo[3], wo[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float uc = qc[c];
                float acc = fprev[1] * (s1[bb][c][ty][lc + 1] - uc) - fprev[0] * (uc - s1[bb][c][ty][lc - 1])
                          + fprev[3] * (s1[bb][c][ty + 1][lc] - uc) - fprev[2] * (uc - s1[bb][c][ty - 1][lc])
                          + fprev[5] * (q[c] - uc) - fprev[4] * (uc - qm[c]);
                const float wc = qc[3 + c];
                const float lw = (s1[bb][3 + c][ty][lc + 1] + s1[bb][3 + c][ty][lc - 1] - 2.f * wc) * ihx2
                               + (s1[bb][3 + c][ty + 1][lc] + s1[bb][3 + c][ty - 1][lc] - 2.f * wc) * ihy2
                               + (q[3 + c] + qm[3 + c] - 2.f * wc) * ihz2;
                acc += eta_dt * lw;
                const float wnew = c1 * wc + c2 * acc;
                wo[c] = act ? wnew : 0.f;
                uo[c] = act ? uc + wnew : 0.f;
            }
            if (inrow) {
                const int sidx = k2 * sxy + col;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    __builtin_nontemporal_store(wo[c], glob(a.wn) + c * a.N + sidx);
                    __builtin_nontemporal_store(uo[c], glob(a.un) + c * a.N + sidx);
                }
            }
        }
        // ---- advance the queues ----
#pragma unroll
        for (int f = 0; f < NQ; ++f) {
            zm[f] = zc[f];
            zc[f] = zp[f];
            zp[f] = zn[f];
            hc[f] = hn[f];
        }
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            qm[f] = qc[f];
            qc[f] = q[f];
            fprev[f] = fcur[f];
        }
        poff = poff_n;
        if constexpr (HET) fz = fcur[5];
        if constexpr (HET) {
            crho_p = crho_c;
            eta_p = eta_c;
            crho_c = crho_n;
            eta_c = eta_n;
        }
    }
}

}  // namespace
