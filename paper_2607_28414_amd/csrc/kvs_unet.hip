// Learned preconditioner: a small linear 3-level U-Net on gfx950 (BF16
// activations and weights, FP32 accumulation on MFMA), its backward pass and
// an Adam optimiser, used inside a flexible PCG for the projection's
// Poisson solve.
//
// Network (channels C0, C1, C2; no biases, no nonlinearity, so the
// preconditioner is a fixed linear operator):
//   e0 = conv(r; 1 -> C0)                                   level 0 (full grid)
//   e1 = conv(pool(e0); C0 -> C1)                           level 1 (1/2 per axis)
//   b  = conv(pool(e1); C1 -> C2), then conv(C2 -> C2, dilation 2, 4, ...),
//        then conv(C2 -> C1)                                level 2 (1/4 per axis)
//   g1 = conv(e1 + up(b); C1 -> C0)                         level 1
//   g0 = conv(e0 + up(g1); C0 -> C0)                        level 0
//   z  = conv(g0; C0 -> 1)                                  level 0
// conv = 3x3x3 (dilated) cross-correlation with zero padding, pool = mean of
// the (up to 8) children, up = nearest-neighbour copy.  The additive skip
// inputs are formed while the next conv reads its operand, so no upsampled
// tensor is stored.
//
// Layout: activations channels-last [z][y][x][C] in BF16; conv weights
// W[co][k] with k = tap * CI + ci (tap = 9 dz + 3 dy + dx over {0,1,2}^3),
// K padded with zeros to a multiple of 32.  MFMA: each wavefront computes
// 16 consecutive voxels x CO channels as D[co][voxel] = W[co][k] X[k][voxel]
// with v_mfma_f32_16x16x32_bf16 (A operand = weights, B operand = the
// activation patch; 8 consecutive k of one tap are 8 consecutive channels,
// one 16-byte load).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "kvs_internal.hpp"
#include "kvs_tiling.hpp"

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short short4v __attribute__((ext_vector_type(4)));

namespace {

struct Dims {
    int nx, ny, nz;
    __host__ __device__ long long n() const { return (long long)nx * ny * nz; }
};

// The network input x = bf16(fp32(in_scale r)): the scaled FP64 residual is
// rounded to FP32, then to BF16 (nearest even at each step).  The FP32 value
// goes through an empty asm statement; without it the compiler merges the two
// conversions into one direct conversion from FP64, which rounds once (and
// takes a nine-instruction round-to-odd sequence more per value).
__device__ __forceinline__ bf16 bf16_via_f32(double x) {
    float f = (float)x;
    asm volatile("" : "+v"(f));
    return (bf16)f;
}

// 16 bytes of zeros: the source of taps outside the grid in the gathering conv
__device__ __attribute__((aligned(16))) bf16 kZeroRow[8];

// Bricks of 16 x NV x 4 voxels covering a grid (counts along x, y, z);
// bx = 0 selects blocks of consecutive voxels instead.
struct Bricks {
    int bx, by, bz;
};

__host__ __device__ inline Dims coarse(Dims d) { return Dims{(d.nx + 1) / 2, (d.ny + 1) / 2, (d.nz + 1) / 2}; }

__device__ __forceinline__ int tap_dx(int tap) { return tap % 3 - 1; }
__device__ __forceinline__ int tap_dy(int tap) { return (tap / 3) % 3 - 1; }
__device__ __forceinline__ int tap_dz(int tap) { return tap / 9 - 1; }

// ---- forward kernels (MFMA) --------------------------------------------------

__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// 16x16x16 BF16 MFMA (K = 16: four k per lane)
__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(short4v, a), __builtin_bit_cast(short4v, b), c,
                                                     0, 0, 0);
}

// Convolution at the coarse levels:
// out[v][co] = sum_{tap, ci} W[co][tap * CI + ci] * in(v + dil * tap)[ci],
// in(p) = A[p][ci], zero outside the grid.
// Each wavefront computes NV groups of 16 consecutive voxels for all CO
// channels.  The weights are staged in LDS in slabs of WS K-chunks (double
// buffered through registers) and shared by the block's 4 wavefronts, so a
// block reads them from L2 once; the activation taps are gathered per group
// (constant offsets for wavefronts away from the boundary).  Outputs are
// rounded once (BF16) or stored as FP32.  Every wavefront runs the slab loop
// (its barriers) even when its voxels lie beyond the grid.
// The register budget is capped for two wavefronts per SIMD: uncapped, the
// 64-channel instances took 260 registers and ran one wavefront per SIMD,
// which leaves the gather loads' latency exposed.
constexpr int WS = 6;  // K chunks per weight slab

template <int CI, int CO, int NV, typename OUT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void conv3_mfma(const bf16* __restrict__ A, Dims d,
                                                  int dil, Bricks bk, const bf16* __restrict__ W,
                                                  OUT* __restrict__ out, const int* stop) {
    static_assert(CI % 8 == 0 && CO % 16 == 0, "channel counts");
    constexpr int K = 27 * CI;
    constexpr int KP = (K + 31) / 32 * 32;
    constexpr int NC = KP / 32;
    constexpr int NSL = (NC + WS - 1) / WS;
    constexpr int MT = CO / 16;
    constexpr int WROW = 32 * WS + 8;                 // bf16 per output row of a slab (padded)
    constexpr int ITEMS = CO * 4 * WS;                // 16-byte items per slab
    constexpr int IPT = (ITEMS + 255) / 256;
    __shared__ __attribute__((aligned(16))) bf16 wsl[2][CO * WROW];
    if (stop && *stop) return;
    const int t = threadIdx.x, lane = t & 63;
    // Voxels of the block: with bricks (dilation 1), brick (kx, ky, kz) of
    // 16 x NV x 4 voxels, wavefront w taking layer z = w, group g row y = g,
    // lane vl column x = vl (a compact 3-D footprint per XCD); otherwise 4 x
    // 16 NV consecutive voxels in memory order.
    const int blk = kvs_tiling::tile_of((int)blockIdx.x, (int)gridDim.x);
    const int vl = lane & 15, kg = lane >> 4;
    int gx[NV], gy[NV], gz[NV];
    bool valid[NV];
    int vox[NV];  // voxel counts stay below 2^31
    if (bk.bx > 0) {
        const int kx = blk % bk.bx, ky = (blk / bk.bx) % bk.by, kz = blk / (bk.bx * bk.by);
#pragma unroll
        for (int g = 0; g < NV; ++g) {
            gx[g] = 16 * kx + vl;
            gy[g] = NV * ky + g;
            gz[g] = 4 * kz + (t >> 6);
            valid[g] = gx[g] < d.nx && gy[g] < d.ny && gz[g] < d.nz;
            vox[g] = valid[g] ? gx[g] + d.nx * (gy[g] + d.ny * gz[g]) : 0;
        }
    } else {
        const long long v0 = ((long long)blk * 4 + (t >> 6)) * (16 * NV);
#pragma unroll
        for (int g = 0; g < NV; ++g) {
            const long long v = v0 + 16 * g + vl;
            valid[g] = v < d.n();
            const unsigned vc = valid[g] ? (unsigned)v : 0u, row = vc / (unsigned)d.nx;
            gx[g] = (int)(vc - row * (unsigned)d.nx);
            gy[g] = (int)(row % (unsigned)d.ny);
            gz[g] = (int)(row / (unsigned)d.ny);
            vox[g] = (int)vc;
        }
    }
    bool deep = true;
#pragma unroll
    for (int g = 0; g < NV; ++g)
        deep = deep && valid[g] && gx[g] >= dil && gx[g] < d.nx - dil && gy[g] >= dil && gy[g] < d.ny - dil &&
               gz[g] >= dil && gz[g] < d.nz - dil;
    const bool fast = __all(deep);
    const bf16* base[NV];
#pragma unroll
    for (int g = 0; g < NV; ++g) base[g] = A + (size_t)vox[g] * CI;
    // taps whose source voxel lies inside the grid: bit tap of tm[g]
    unsigned tm[NV];
#pragma unroll
    for (int g = 0; g < NV; ++g) {
        const unsigned mx = (gx[g] >= dil ? 1u : 0u) | 2u | (gx[g] + dil < d.nx ? 4u : 0u);
        const unsigned my = (gy[g] >= dil ? 1u : 0u) | 2u | (gy[g] + dil < d.ny ? 4u : 0u);
        const unsigned mz = (gz[g] >= dil ? 1u : 0u) | 2u | (gz[g] + dil < d.nz ? 4u : 0u);
        unsigned m = 0u;
#pragma unroll
        for (int tap = 0; tap < 27; ++tap)
            m |= ((mx >> (tap % 3)) & (my >> ((tap / 3) % 3)) & (mz >> (tap / 9)) & 1u) << tap;
        tm[g] = valid[g] ? m : 0u;
    }
    // per chunk and lane group: source offset (elements) and tap index; taps
    // >= 27 (K padding) have zero weights and take tap 26's offset
    static_assert(NC * 4 <= 256, "one tap-table entry per thread");
    __shared__ int2 ktab[NC * 4];
    if (t < NC * 4) {
        const int k0 = (t / 4) * 32 + 8 * (t % 4), tap = k0 / CI, tc = min(tap, 26);
        ktab[t] = int2{dil * (tap_dx(tc) + d.nx * tap_dy(tc) + d.nx * d.ny * tap_dz(tc)) * CI + k0 % CI, tap};
    }

    // weight slab staging: item -> (output row, 16-byte piece of the slab)
    bf16x8 wreg[IPT];
    auto wload = [&](int sl) {
#pragma unroll
        for (int h = 0; h < IPT; ++h) {
            const int it = min(t + 256 * h, ITEMS - 1);
            const int co = it / (4 * WS), q = it % (4 * WS);
            const int kcol = min(32 * WS * sl + 8 * q, KP - 8);  // past the last chunk: any valid address
            wreg[h] = *reinterpret_cast<const bf16x8*>(W + (size_t)co * KP + kcol);
        }
    };
    auto wstore = [&](int buf) {
#pragma unroll
        for (int h = 0; h < IPT; ++h) {
            const int it = t + 256 * h;
            if (it >= ITEMS) break;
            const int co = it / (4 * WS), q = it % (4 * WS);
            *reinterpret_cast<bf16x8*>(&wsl[buf][co * WROW + 8 * q]) = wreg[h];
        }
    };

    f32x4 acc[NV][MT];
#pragma unroll
    for (int g = 0; g < NV; ++g)
#pragma unroll
        for (int m = 0; m < MT; ++m) acc[g][m] = f32x4{0.f, 0.f, 0.f, 0.f};

    // Activation patch of chunk kc for every group.  Loads are unconditional
    // (clamped addresses; chunks past the end re-read the last one) and masked
    // when the patch is used, so the gather of chunk kc + 1 stays in flight
    // while chunk kc runs, across the LDS-only barriers.  Two patch buffers
    // alternate by chunk parity (no register copies that would wait on a
    // load), and the interior case (constant offsets, no masks) is its own
    // loop.
    auto run = [&](auto fast_tag) {
        constexpr bool FAST = decltype(fast_tag)::value;
        // out-of-grid taps read a row of zeros instead of being masked
        auto gather = [&](int kc, bf16x8 (&a8)[NV]) {
            const int2 e = ktab[min(kc, NC - 1) * 4 + kg];
#pragma unroll
            for (int g = 0; g < NV; ++g) {
                const bf16* src = base[g] + e.x;
                if constexpr (!FAST) src = ((tm[g] >> e.y) & 1u) ? src : kZeroRow;
                a8[g] = *reinterpret_cast<const bf16x8*>(src);
            }
        };
        auto compute = [&](int kc, const bf16x8 (&a8)[NV]) {
            const int sl = kc / WS, kk = kc % WS;
            if (kk == 0) {
                if (sl > 0) {
                    kvs_tiling::lds_barrier();  // every wavefront is done with the old slab of this buffer
                    wstore(sl & 1);
                    kvs_tiling::lds_barrier();
                }
                if (sl + 1 < NSL) wload(sl + 1);
            }
            bf16x8 wf[MT];
#pragma unroll
            for (int m = 0; m < MT; ++m)
                wf[m] = *reinterpret_cast<const bf16x8*>(&wsl[sl & 1][(16 * m + vl) * WROW + 32 * kk + 8 * kg]);
#pragma unroll
            for (int g = 0; g < NV; ++g)
#pragma unroll
                for (int m = 0; m < MT; ++m) acc[g][m] = mfma32(wf[m], a8[g], acc[g][m]);
        };
        // the scheduling barriers keep each gather ahead of the chunk that
        // runs while it is in flight (left alone, the scheduler moves loads
        // next to their use)
        bf16x8 pa[NV], pb[NV];
        gather(0, pa);
        for (int kc = 0; kc < NC; kc += 2) {
            gather(kc + 1, pb);
            __builtin_amdgcn_sched_barrier(0);
            compute(kc, pa);
            __builtin_amdgcn_sched_barrier(0);
            if (kc + 1 < NC) {
                gather(kc + 2, pa);
                __builtin_amdgcn_sched_barrier(0);
                compute(kc + 1, pb);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    };

    wload(0);
    wstore(0);
    kvs_tiling::lds_barrier();
    if (fast)
        run(std::true_type{});
    else
        run(std::false_type{});
#pragma unroll
    for (int g = 0; g < NV; ++g) {
        if (!valid[g]) continue;
        const size_t v = (size_t)vox[g];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            if constexpr (sizeof(OUT) == 2) {
                bf16x4 o;
#pragma unroll
                for (int i = 0; i < 4; ++i) o[i] = (bf16)acc[g][m][i];
                *reinterpret_cast<bf16x4*>(out + v * CO + 16 * m + 4 * kg) = o;
            } else {
                *reinterpret_cast<f32x4*>(out + v * CO + 16 * m + 4 * kg) = acc[g][m];
            }
        }
    }
}

// Convolution on sub-lattice bricks (any dilation; 32 or 64 input channels,
// the 1/4-resolution bottleneck): a convolution with dilation d is d^3
// independent undilated convolutions on the sub-lattices x = a + d i,
// y = b + d j, z = c + d k.  A block owns an 8 x 8 x 4 LZ brick of one
// sub-lattice (all CO channels) and stages the brick's input with its
// one-voxel halo (10 x 10 x (4 LZ + 2) voxels, zeros outside the grid) in
// LDS, 32 input channels per pass; wavefront w computes z layers LZ w ..
// LZ w + LZ - 1 of the brick, 4 LZ groups of 16 voxels (two 8-voxel rows
// each) x CO channels, with
// both MFMA operands read from LDS: every staged activation serves the 27
// taps of up to 27 outputs from LDS instead of 27 gathers through the L1.
// The weights of three taps at a time are staged in LDS, the next three
// loaded into registers while the current ones are used.  Same sum as
// conv3_mfma in another order (taps of the first 32 channels, then of the
// next 32), FP32 accumulation, one rounding of the output.
constexpr int SB_X = 8, SB_Y = 8;         // output brick (sub-lattice voxels): 8 x 8 x 4 LZ
constexpr int SH_X = SB_X + 2, SH_Y = SB_Y + 2;  // staged brick with halo: 10 x 10 x (4 LZ + 2)
// z layers of the brick per wavefront: 2 for up to 32 output channels (the
// weight slabs are small enough for a 10 x 10 x 10 staged brick at two blocks
// per CU, and each weight fragment then serves 8 voxel groups), else 1
constexpr int sub_lz(int co) { return co <= 32 ? 2 : 1; }
constexpr int SVS = 32;            // LDS voxel stride (bf16; padding to 40 or 48 measured no faster)
constexpr int STAPS = 3;           // taps per weight slab
constexpr int SWROW = 32 * STAPS + 8;  // bf16 per output-channel row of a slab (padded)

struct SubBricks {
    int bx, by, bz;  // bricks per sub-lattice axis
};

template <int CI, int CO, typename OUT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void conv3_sub(
    const bf16* __restrict__ A, Dims d, int dil, SubBricks sb, const bf16* __restrict__ W, OUT* __restrict__ out,
    const int* stop) {
    static_assert(CI % 32 == 0 && CO % 16 == 0 && CO <= 64, "channel counts");
    constexpr int LZ = sub_lz(CO), NG = 4 * LZ;  // z layers per wavefront, voxel groups per wavefront
    constexpr int SB_Z = 4 * LZ, SH_Z = SB_Z + 2, SH_V = SH_X * SH_Y * SH_Z;
    constexpr int NH = CI / 32;      // passes of 32 input channels
    constexpr int MT = CO / 16;      // output-channel tiles
    constexpr int KP = 27 * CI;      // weight row length (a multiple of 32)
    constexpr int NSL = 27 / STAPS;  // weight slabs per pass
    constexpr int WITEMS = CO * STAPS * 4;  // 16-byte pieces per slab
    constexpr int WIPT = (WITEMS + 255) / 256;
    constexpr int XITEMS = SH_V * 4;        // 16-byte pieces of a staged pass
    constexpr int XIPT = (XITEMS + 255) / 256;
    __shared__ __attribute__((aligned(16))) bf16 xs[SH_V * SVS];
    __shared__ __attribute__((aligned(16))) bf16 ws[2][CO * SWROW];
    if (stop && *stop) return;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int vl = lane & 15, kg = lane >> 4;
    int q = kvs_tiling::tile_of((int)blockIdx.x, (int)gridDim.x);
    const int bi = q % sb.bx;
    q /= sb.bx;
    const int bj = q % sb.by;
    q /= sb.by;
    const int bk = q % sb.bz;
    q /= sb.bz;
    const int sa = q % dil, sbb = (q / dil) % dil, sc = q / (dil * dil);  // sub-lattice
    const int i0 = bi * SB_X, j0 = bj * SB_Y, k0 = bk * SB_Z;

    // staged pieces of this thread: source offset (elements, channel 0) or -1
    int xsrc[XIPT];
#pragma unroll
    for (int h = 0; h < XIPT; ++h) {
        const int p = t + 256 * h;
        xsrc[h] = -1;
        if (p < XITEMS) {
            const int v = p >> 2, hx = v % SH_X, hy = (v / SH_X) % SH_Y, hz = v / (SH_X * SH_Y);
            const int gx = sa + dil * (i0 + hx - 1), gy = sbb + dil * (j0 + hy - 1), gz = sc + dil * (k0 + hz - 1);
            if (gx >= 0 && gx < d.nx && gy >= 0 && gy < d.ny && gz >= 0 && gz < d.nz)
                xsrc[h] = (gx + d.nx * (gy + d.ny * gz)) * CI + 8 * (p & 3);
        }
    }
    // the pieces of one pass, loaded into registers (the next pass's while
    // the current one runs), then written to LDS
    bf16x8 xn[XIPT];
    auto xload = [&](int pass) {
        const bf16* Ap = A + 32 * pass;  // uniform base, per-lane 32-bit offsets
#pragma unroll
        for (int h = 0; h < XIPT; ++h) {
            bf16x8 v = {};
            if (xsrc[h] >= 0) v = *reinterpret_cast<const bf16x8*>(Ap + xsrc[h]);
            xn[h] = v;
        }
    };
    auto xstore = [&]() {
#pragma unroll
        for (int h = 0; h < XIPT; ++h) {
            const int p = t + 256 * h;
            if (p >= XITEMS) break;
            *reinterpret_cast<bf16x8*>(&xs[(p >> 2) * SVS + 8 * (p & 3)]) = xn[h];
        }
    };
    // weight slab (pass, slab): rows co, taps 3 slab .. 3 slab + 2, channels 32 pass .. + 31
    bf16x8 wreg[WIPT];
    int woff[WIPT];  // this thread's pieces of a slab: offset from the slab's first weight
#pragma unroll
    for (int h = 0; h < WIPT; ++h) {
        const int it = min(t + 256 * h, WITEMS - 1);
        const int co = it / (4 * STAPS), r = it % (4 * STAPS);
        woff[h] = co * KP + (r >> 2) * CI + 8 * (r & 3);
    }
    auto wload = [&](int pass, int sl) {
        const bf16* Wp = W + STAPS * sl * CI + 32 * pass;  // uniform base
#pragma unroll
        for (int h = 0; h < WIPT; ++h) wreg[h] = *reinterpret_cast<const bf16x8*>(Wp + woff[h]);
    };
    auto wstore = [&](int buf) {
#pragma unroll
        for (int h = 0; h < WIPT; ++h) {
            const int it = t + 256 * h;
            if (it >= WITEMS) break;
            const int co = it / (4 * STAPS), r = it % (4 * STAPS);
            *reinterpret_cast<bf16x8*>(&ws[buf][co * SWROW + 8 * r]) = wreg[h];
        }
    };

    f32x4 acc[NG][MT];
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int m = 0; m < MT; ++m) acc[g][m] = f32x4{0.f, 0.f, 0.f, 0.f};
    // staged voxel of group g at tap offset (0, 0, 0): x = vl % 8,
    // y = 2 (g % 4) + vl / 8, z = LZ wv + g / 4
    int xv[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) xv[g] = (vl & 7) + SH_X * (2 * (g & 3) + (vl >> 3) + SH_Y * (LZ * wv + (g >> 2)));

#pragma unroll 1
    for (int pass = 0; pass < NH; ++pass) {
        // (the barrier that ends the previous pass's last slab: every
        // wavefront is done with xs and both weight buffers)
        if (pass == 0) xload(0);
        xstore();
        if (pass + 1 < NH) xload(pass + 1);
        wload(pass, 0);
        wstore(0);
        kvs_tiling::lds_barrier();
        // (kept rolled: fully unrolled, with immediate tap offsets, it ran
        // 15-25 % slower)
#pragma unroll 1
        for (int sl = 0; sl < NSL; ++sl) {
            if (sl + 1 < NSL) wload(pass, sl + 1);
            const bf16* wb = ws[sl & 1];
#pragma unroll
            for (int tt = 0; tt < STAPS; ++tt) {
                const int tap = STAPS * sl + tt;
                const int off = tap % 3 + SH_X * ((tap / 3) % 3 + SH_Y * (tap / 9));
                bf16x8 xf[NG], wf[MT];
#pragma unroll
                for (int g = 0; g < NG; ++g) xf[g] = *reinterpret_cast<const bf16x8*>(&xs[(xv[g] + off) * SVS + 8 * kg]);
#pragma unroll
                for (int m = 0; m < MT; ++m)
                    wf[m] = *reinterpret_cast<const bf16x8*>(&wb[(16 * m + vl) * SWROW + 32 * tt + 8 * kg]);
#pragma unroll
                for (int g = 0; g < NG; ++g)
#pragma unroll
                    for (int m = 0; m < MT; ++m) acc[g][m] = mfma32(wf[m], xf[g], acc[g][m]);
            }
            if (sl + 1 < NSL) wstore((sl + 1) & 1);
            kvs_tiling::lds_barrier();
        }
    }
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        const int x = i0 + (vl & 7), y = j0 + 2 * (g & 3) + (vl >> 3), z = k0 + LZ * wv + (g >> 2);
        const int gx = sa + dil * x, gy = sbb + dil * y, gz = sc + dil * z;
        if (gx >= d.nx || gy >= d.ny || gz >= d.nz) continue;
        const size_t v = (size_t)gx + (size_t)d.nx * (gy + (size_t)d.ny * gz);
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            if constexpr (sizeof(OUT) == 2) {
                bf16x4 o;
#pragma unroll
                for (int i = 0; i < 4; ++i) o[i] = (bf16)acc[g][m][i];
                *reinterpret_cast<bf16x4*>(out + v * CO + 16 * m + 4 * kg) = o;
            } else {
                *reinterpret_cast<f32x4*>(out + v * CO + 16 * m + 4 * kg) = acc[g][m];
            }
        }
    }
}

// Convolution with dilation 1 as an LDS-staged z-march (same result as
// conv3_mfma).  A block owns a 32 x TY column of output voxels and marches up
// a z segment; the haloed input planes z - 1, z, z + 1 (34 x (TY + 2) voxels,
// channel stride CI + 8 against bank conflicts) live in an LDS ring, the
// plane after next is prefetched into registers.  Each wavefront owns
// TY / 2 groups of 16 voxels along x and keeps its weight fragments of all
// chunks in registers.  With PROJ (CO = 16) the epilogue also forms the
// pointwise projection gz = sum_c wp[c] bf16(out[c]) (FP32), and `out` may
// be null (only gz is needed at inference).
template <int CI, int TY>
struct ZmGeom {
    static constexpr int TX = 32, HX = TX + 2, HY = TY + 2, HV = HX * HY;
    static constexpr int VS = CI + 8;                    // LDS voxel stride (bf16)
    static constexpr int PL = HV * VS;                   // plane (bf16)
    static constexpr int ITEMS = HV * (CI / 8);          // 16-byte items per plane
    static constexpr int IPT = (ITEMS + 255) / 256;      // items per thread
};

// Two wavefronts per SIMD where the register file allows it without spills
// (the 32 -> 32 instance keeps its registers and runs one).
constexpr int zm_waves(int ci, int co) { return ci == 32 && co == 32 ? 1 : 2; }

template <int CI, int CO, int TY, bool PROJ, typename OUT, bool POOL = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(zm_waves(CI, CO)))) void conv3_zm(const bf16* __restrict__ A, Dims d, int ntx, int nty, int zchunk,
                                                const bf16* __restrict__ W, OUT* __restrict__ out,
                                                const float* __restrict__ wp, float* __restrict__ gz,
                                                const int* stop, bf16* __restrict__ pooled) {
    using G = ZmGeom<CI, TY>;
    constexpr int K = 27 * CI, KP = (K + 31) / 32 * 32, NC = KP / 32, MT = CO / 16, NG = TY / 2;
    static_assert(TY % 2 == 0 && CI % 8 == 0 && CO % 16 == 0 && (!PROJ || CO == 16), "tile");
    // POOL: the BF16 outputs are also pooled into `pooled` (mean of the
    // existing 2 x 2 x 2 children): a wavefront's groups g and g + 2 are the
    // rows 2w and 2w + 1, x pairs are neighbouring lanes, z pairs consecutive
    // planes of the segment (segments start on even planes)
    static_assert(!POOL || (NG == 4 && sizeof(OUT) == 2 && !PROJ), "pooling layout");
    float ps[2][MT][4];
#pragma unroll
    for (int xh = 0; xh < 2; ++xh)
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int i = 0; i < 4; ++i) ps[xh][m][i] = 0.f;
    __shared__ __attribute__((aligned(16))) bf16 lds[3 * G::PL];
    if (stop && *stop) return;
    const int blk = kvs_tiling::tile_of((int)blockIdx.x, (int)gridDim.x);
    const int tx = blk % ntx, t2 = blk / ntx;
    const int ty = t2 % nty, tz = t2 / nty;
    const int x0 = tx * G::TX, y0 = ty * TY;
    const int zs = tz * zchunk, ze = min(d.nz, zs + zchunk);
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, vl = lane & 15, kg = lane >> 4;
    const int pbase = zs - 1;  // ring slot of plane p: (p - pbase) % 3
    // staging: item -> (haloed voxel, 8 channels)
    bf16x8 pa[G::IPT];
    bool pm[G::IPT];
    auto sload = [&](int p) {
#pragma unroll
        for (int h = 0; h < G::IPT; ++h) {
            const int it = min(t + 256 * h, G::ITEMS - 1);
            const int hv = it / (CI / 8), c8 = it % (CI / 8);
            const int gx = x0 - 1 + hv % G::HX, gy = y0 - 1 + hv / G::HX;
            pm[h] = t + 256 * h < G::ITEMS && p >= 0 && p < d.nz && gx >= 0 && gx < d.nx && gy >= 0 && gy < d.ny;
            const int cx = min(max(gx, 0), d.nx - 1), cy = min(max(gy, 0), d.ny - 1), cz = min(max(p, 0), d.nz - 1);
            pa[h] = *reinterpret_cast<const bf16x8*>(A + ((size_t)cx + (size_t)d.nx * (size_t)(cy + d.ny * cz)) * CI + 8 * c8);
        }
    };
    auto sstore = [&](int p) {
        bf16* slot = lds + ((p - pbase) % 3) * G::PL;
#pragma unroll
        for (int h = 0; h < G::IPT; ++h) {
            const int it = t + 256 * h;
            if (it >= G::ITEMS) break;
            const int hv = it / (CI / 8), c8 = it % (CI / 8);
            bf16x8 v;
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = pm[h] ? pa[h][j] : (bf16)0.f;
            *reinterpret_cast<bf16x8*>(slot + hv * G::VS + 8 * c8) = v;
        }
    };
    // this lane's weight fragments of every chunk, held for the whole segment
    bf16x8 wreg[NC][MT];
#pragma unroll
    for (int kc = 0; kc < NC; ++kc)
#pragma unroll
        for (int m = 0; m < MT; ++m)
            wreg[kc][m] = *reinterpret_cast<const bf16x8*>(W + (size_t)(16 * m + vl) * KP + kc * 32 + 8 * kg);
    // group g of wavefront w: plane row (w NG + g) / 2, x half (w NG + g) % 2
    const int lane_base = (w * NG / 2) * G::HX * G::VS + vl * G::VS;
    sload(zs - 1);
    sstore(zs - 1);
    sload(zs);
    sstore(zs);
    sload(zs + 1);
    sstore(zs + 1);
    sload(zs + 2);
    kvs_tiling::lds_barrier();
    for (int z = zs; z < ze; ++z) {
        const int s0 = ((z - 1 - pbase) % 3) * G::PL, s1 = ((z - pbase) % 3) * G::PL, s2 = ((z + 1 - pbase) % 3) * G::PL;
        f32x4 acc[NG][MT];
#pragma unroll
        for (int g = 0; g < NG; ++g)
#pragma unroll
            for (int m = 0; m < MT; ++m) acc[g][m] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < NC; ++kc) {
            // chunk kc covers k = 32 kc + 8 kg .. + 7: one tap, 8 channels;
            // k >= 27 CI has zero weights and reads a valid tap instead
            const int k0 = kc * 32 + 8 * kg;
            const int tap = min(k0 / CI, 26), ci0 = k0 % CI;
            const int tdz = tap_dz(tap);
            const int toff = (tdz < 0 ? s0 : (tdz == 0 ? s1 : s2)) +
                             ((1 + tap_dy(tap)) * G::HX + 1 + tap_dx(tap)) * G::VS + ci0 + lane_base;
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const int gdelta = ((g >> 1) * G::HX + 16 * (g & 1)) * G::VS;
                const bf16x8 xb = *reinterpret_cast<const bf16x8*>(lds + toff + gdelta);
#pragma unroll
                for (int m = 0; m < MT; ++m) acc[g][m] = mfma32(wreg[kc][m], xb, acc[g][m]);
            }
        }
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            const int gl = w * NG + g;
            const int gx = x0 + 16 * (gl & 1) + vl, gy = y0 + (gl >> 1);
            const bool inside = gx < d.nx && gy < d.ny;
            const size_t v = (size_t)min(gx, d.nx - 1) + (size_t)d.nx * (size_t)(min(gy, d.ny - 1) + d.ny * z);
            if constexpr (PROJ) {
                // lane holds channels 4 kg .. 4 kg + 3 of voxel vl; sum over the 4 lane groups
                float pz = 0.f;
#pragma unroll
                for (int i = 0; i < 4; ++i) pz = fmaf(wp[4 * kg + i], (float)(bf16)acc[g][0][i], pz);
                pz += __shfl_xor(pz, 16);
                pz += __shfl_xor(pz, 32);
                if (inside && kg == 0) gz[v] = pz;
            }
            if (!inside || !out) continue;
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                if constexpr (sizeof(OUT) == 2) {
                    bf16x4 o;
#pragma unroll
                    for (int i = 0; i < 4; ++i) o[i] = (bf16)acc[g][m][i];
                    *reinterpret_cast<bf16x4*>(out + v * CO + 16 * m + 4 * kg) = o;
                } else {
                    *reinterpret_cast<f32x4*>(out + v * CO + 16 * m + 4 * kg) = acc[g][m];
                }
            }
        }
        if constexpr (POOL) {
#pragma unroll
            for (int xh = 0; xh < 2; ++xh)
#pragma unroll
                for (int gg = 0; gg < 2; ++gg) {
                    const int gl = w * NG + xh + 2 * gg;
                    const bool in = x0 + 16 * (gl & 1) + vl < d.nx && y0 + (gl >> 1) < d.ny;
#pragma unroll
                    for (int m = 0; m < MT; ++m)
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            ps[xh][m][i] += in ? (float)(bf16)acc[xh + 2 * gg][m][i] : 0.f;
                }
            if ((z & 1) || z == d.nz - 1) {
                const Dims c = coarse(d);
                const int Z = z >> 1, Y = (y0 >> 1) + w;
#pragma unroll
                for (int xh = 0; xh < 2; ++xh) {
                    const int X = (x0 + 16 * xh + vl) >> 1;
                    const int cnt = (min(2 * X + 2, d.nx) - 2 * X) * (min(2 * Y + 2, d.ny) - 2 * Y) *
                                    (min(2 * Z + 2, d.nz) - 2 * Z);
#pragma unroll
                    for (int m = 0; m < MT; ++m) {
                        bf16x4 o;
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const float v = ps[xh][m][i] + __shfl_xor(ps[xh][m][i], 1);
                            o[i] = (bf16)(v / (float)cnt);
                            ps[xh][m][i] = 0.f;
                        }
                        if ((vl & 1) == 0 && X < c.nx && Y < c.ny)
                            *reinterpret_cast<bf16x4*>(pooled + ((size_t)(Z * c.ny + Y) * c.nx + X) * CO + 16 * m +
                                                       4 * kg) = o;
                    }
                }
            }
        }
        if (z + 1 < ze) {
            kvs_tiling::lds_barrier();  // plane z - 1 no longer read
            sstore(z + 2);
            if (z + 3 <= ze) sload(z + 3);
            kvs_tiling::lds_barrier();
        }
    }
}

// voxel groups per wavefront: fewer for wide inputs or outputs (register budget)
constexpr int conv_nv(int ci, int co) { return (co >= 64 || ci >= 32) ? 4 : 8; }

// Scales of the network input and output: device values (the flexible PCG
// computes them from the residual norm without a host round trip) or host
// values; `stop` (device flag) makes every kernel return at once.
struct NetCtl {
    const double* in_dev;
    const double* out_dev;
    const int* stop;
    double in_v, out_v;
};

// Level 0 of the encoder: p0 = bf16(pool(conv(x; W0))) with x = bf16(in_scale
// r) and e0 = conv(x; W0) unrounded.  For a coarse voxel whose 8 children all
// exist, the mean of the children's 3x3x3 convs is one 4x4x4 stride-2 conv of
// x with the composed weights Wp[c][s] = 1/8 sum_o W0[c][s - o] (s = 0..3 per
// axis from the fine voxel 2V - 1, o the child offset): K = 64, two MFMA
// chunks per 16 coarse voxels.  Wp is carried as a BF16 pair (hi + lo, two
// MFMAs per chunk), so the result is FP32-accurate before its one BF16
// rounding.  Coarse voxels with a missing child (odd fine extents) are
// recomputed exactly by pool0_edge_kernel afterwards.
// A block owns FP_CX x FP_CY coarse voxels of each coarse plane (wavefront w:
// coarse row Y0 + w, FP_CX / 16 groups of 16 along x) and marches up a
// segment of coarse planes; the fine planes of x it needs (two new ones per
// coarse plane, halo 1 at the low side and 2 at the high side) are staged as
// BF16 in a 6-plane LDS ring, loaded one coarse plane ahead (one barrier per
// coarse plane).  Lane (v, kg) of a chunk reads 2 rows x 4 consecutive fine x.
constexpr int FP_CX = 64, FP_CY = 4;
constexpr int FP_RX = 2 * FP_CX + 2, FP_RY = 2 * FP_CY + 2, FP_RS = FP_RX + 2, FP_RN = FP_RY * FP_RS, FP_SLOTS = 6;
constexpr int FP_ITEMS = FP_RX * FP_RY;            // staged values per fine plane
constexpr int FP_IPT = (FP_ITEMS + 255) / 256;     // per thread

template <typename RT>  // the residual as stored: FP64, or FP32 (the flexible PCG's FP32 storage)
__global__ __launch_bounds__(256) void first_pool_kernel(const RT* __restrict__ r, NetCtl ctl, Dims d, int ntx,
                                                         int nty, int zchunk, const bf16* __restrict__ Wp,
                                                         bf16* __restrict__ p0) {
    __shared__ __attribute__((aligned(16))) bf16 xs[FP_SLOTS * FP_RN];
    if (ctl.stop && *ctl.stop) return;
    const double in_scale = ctl.in_dev ? *ctl.in_dev : ctl.in_v;
    const Dims c = coarse(d);
    const int blk = kvs_tiling::tile_of((int)blockIdx.x, (int)gridDim.x);
    const int tx = blk % ntx, t2 = blk / ntx;
    const int ty = t2 % nty, tz = t2 / nty;
    const int X0 = tx * FP_CX, Y0 = ty * FP_CY;
    const int Zs = tz * zchunk, Ze = min(c.nz, Zs + zchunk);
    const int fx0 = 2 * X0 - 1, fy0 = 2 * Y0 - 1;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, vl = lane & 15, kg = lane >> 4;
    const int sxy = d.nx * d.ny;
    const int pbase = 2 * Zs - 1;  // ring slot of fine plane p: (p - pbase) % FP_SLOTS
    // composed weights, chunk ch, hi and lo: A[row = channel vl][k = 8 kg + j]
    bf16x8 wa[2][2];
#pragma unroll
    for (int ch = 0; ch < 2; ++ch)
#pragma unroll
        for (int hl = 0; hl < 2; ++hl)
            wa[ch][hl] = *reinterpret_cast<const bf16x8*>(Wp + (size_t)hl * 16 * 64 + vl * 64 + 32 * ch + 8 * kg);
    // Loads are unconditional from clamped (in-bounds) addresses and masked
    // when stored to LDS, so that a prefetch stays in flight until then.
    auto fload = [&](int p, double (&v)[FP_IPT], bool (&m)[FP_IPT]) {
#pragma unroll
        for (int h = 0; h < FP_IPT; ++h) {
            const int i = min(t + 256 * h, FP_ITEMS - 1);
            const int gx = fx0 + i % FP_RX, gy = fy0 + i / FP_RX;
            m[h] = t + 256 * h < FP_ITEMS && p >= 0 && p < d.nz && gx >= 0 && gx < d.nx && gy >= 0 && gy < d.ny;
            const int pc = min(max(p, 0), d.nz - 1), yc = min(max(gy, 0), d.ny - 1), xc = min(max(gx, 0), d.nx - 1);
            v[h] = r[(size_t)pc * sxy + (size_t)(yc * d.nx + xc)];
        }
    };
    auto fstore = [&](int p, const double (&v)[FP_IPT], const bool (&m)[FP_IPT]) {
        bf16* sl = xs + ((p - pbase) % FP_SLOTS) * FP_RN;
#pragma unroll
        for (int h = 0; h < FP_IPT; ++h) {
            const int i = t + 256 * h;
            if (h + 1 < FP_IPT || i < FP_ITEMS)
                sl[(i / FP_RX) * FP_RS + i % FP_RX] = m[h] ? bf16_via_f32(in_scale * v[h]) : (bf16)0.f;
        }
    };
    double va[FP_IPT], vb[FP_IPT];
    bool ma[FP_IPT], mb[FP_IPT];
    fload(pbase, va, ma);
    fload(pbase + 1, vb, mb);
    fstore(pbase, va, ma);
    fstore(pbase + 1, vb, mb);
    fload(2 * Zs + 1, va, ma);
    fload(2 * Zs + 2, vb, mb);
    const int Y = Y0 + w;
    for (int Z = Zs; Z < Ze; ++Z) {
        fstore(2 * Z + 1, va, ma);
        fstore(2 * Z + 2, vb, mb);
        if (Z + 1 < Ze) {
            fload(2 * Z + 3, va, ma);
            fload(2 * Z + 4, vb, mb);
        }
        kvs_tiling::lds_barrier();
        // rows of this lane's chunk: fine plane 2Z - 1 + 2 ch + (kg >> 1),
        // tile rows 2w + 2 (kg & 1) and the next
        int rb[2];
#pragma unroll
        for (int ch = 0; ch < 2; ++ch)
            rb[ch] = ((2 * Z - 1 + 2 * ch + (kg >> 1) - pbase) % FP_SLOTS) * FP_RN + (2 * w + 2 * (kg & 1)) * FP_RS;
#pragma unroll
        for (int g = 0; g < FP_CX / 16; ++g) {
            const int col = 2 * (16 * g + vl);  // even: 4-byte aligned pairs
            f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ch = 0; ch < 2; ++ch) {
                const bf16* q = xs + rb[ch] + col;
                typedef unsigned int u32;
                const u32 a0 = *reinterpret_cast<const u32*>(q), a1 = *reinterpret_cast<const u32*>(q + 2);
                const u32 b0 = *reinterpret_cast<const u32*>(q + FP_RS), b1 = *reinterpret_cast<const u32*>(q + FP_RS + 2);
                typedef u32 u32x4 __attribute__((ext_vector_type(4)));
                const bf16x8 xb = __builtin_bit_cast(bf16x8, u32x4{a0, a1, b0, b1});
                acc = mfma32(wa[ch][0], xb, acc);
                acc = mfma32(wa[ch][1], xb, acc);
            }
            const int X = X0 + 16 * g + vl;
            if (X < c.nx && Y < c.ny) {
                bf16x4 o;
#pragma unroll
                for (int i = 0; i < 4; ++i) o[i] = (bf16)acc[i];
                *reinterpret_cast<bf16x4*>(p0 + ((size_t)(Z * c.ny + Y) * c.nx + X) * 16 + 4 * kg) = o;
            }
        }
    }
}

// p0 of the coarse voxels with a missing child (the last coarse index along
// an axis whose fine extent is odd): the exact mean over the existing
// children of e0 = conv(x; W0) (unrounded, FP32), rounded once.  One thread
// per such voxel and channel; the faces are enumerated x, then y, then z
// (voxels on two faces are written twice with the same value).
template <typename RT>
__global__ void pool0_edge_kernel(const RT* __restrict__ r, NetCtl ctl, Dims d, const bf16* __restrict__ W0,
                                  bf16* __restrict__ p0) {
    if (ctl.stop && *ctl.stop) return;
    const Dims c = coarse(d);
    const long long fx = (d.nx & 1) ? (long long)c.ny * c.nz : 0, fy = (d.ny & 1) ? (long long)c.nx * c.nz : 0;
    const long long fz = (d.nz & 1) ? (long long)c.nx * c.ny : 0;
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long v = q / 16;
    const int ch = (int)(q % 16);
    if (v >= fx + fy + fz) return;
    int X, Y, Z;
    if (v < fx) {
        X = c.nx - 1, Y = (int)(v % c.ny), Z = (int)(v / c.ny);
    } else if (v < fx + fy) {
        const long long u = v - fx;
        Y = c.ny - 1, X = (int)(u % c.nx), Z = (int)(u / c.nx);
    } else {
        const long long u = v - fx - fy;
        Z = c.nz - 1, X = (int)(u % c.nx), Y = (int)(u / c.nx);
    }
    const double in_scale = ctl.in_dev ? *ctl.in_dev : ctl.in_v;
    float sum = 0.f;
    int cnt = 0;
    for (int oz = 0; oz < 2; ++oz)
        for (int oy = 0; oy < 2; ++oy)
            for (int ox = 0; ox < 2; ++ox) {
                const int x = 2 * X + ox, y = 2 * Y + oy, z = 2 * Z + oz;
                if (x >= d.nx || y >= d.ny || z >= d.nz) continue;
                ++cnt;
                for (int tap = 0; tap < 27; ++tap) {
                    const int gx = x + tap_dx(tap), gy = y + tap_dy(tap), gzz = z + tap_dz(tap);
                    if (gx < 0 || gx >= d.nx || gy < 0 || gy >= d.ny || gzz < 0 || gzz >= d.nz) continue;
                    const float xv = (float)bf16_via_f32(in_scale * r[((size_t)gzz * d.ny + gy) * d.nx + gx]);
                    sum = fmaf((float)W0[ch * 32 + tap], xv, sum);
                }
            }
    p0[((size_t)(Z * c.ny + Y) * c.nx + X) * 16 + ch] = (bf16)(sum / (float)cnt);
}

// Cell-centred trilinear interpolation (factor 2), per axis: parent I and
// the neighbour J on the fine cell's side (clamped), weights 3/4 and 1/4.
__device__ __forceinline__ void up_axis(int i, int nc, int& I, int& J) {
    I = i >> 1;
    J = (i & 1) ? min(I + 1, nc - 1) : max(I - 1, 0);
}

// Output of the network at the fine level as one 5x5x5 stencil:
//   z(v) = out_scale * (sum_t Wc[t] x(v + t) + up(gz)(v)) on the interior,
//   0 on the outer layer, x = bf16(in_scale r) (0 outside the grid),
//   Wc = W_out composed with W0 (summed over the C0 channels).
// An interior output reads e0 = conv(x; W0) only at voxels inside the grid,
// so conv(e0; W_out) there equals the composed stencil of x exactly; e0 is
// taken unrounded on this path.  125 FP32 FMAs per voxel replace the C0
// channels of e0 and the 27-tap gather.
// A block owns ZO_TX x ZO_TY outputs per plane (a lane: one x column, two
// adjacent rows) and marches up a z segment.  Each x plane (halo 2) is staged
// once in a double-buffered LDS plane, read as a 6 x 5 window per lane, and
// added with the five dz slices of Wc into rolling sums for the outputs two
// planes below to two above; the lowest is then complete.  The coarse
// correction is interpolated in z while it is staged (one LDS tile per
// output plane) and bilinearly in the plane.  One barrier per plane; x and
// gz are loaded one plane ahead.
constexpr int ZO_TX = 64, ZO_TY = 8;
constexpr int ZO_RX = ZO_TX + 4, ZO_RY = ZO_TY + 4, ZO_RS = 72, ZO_PLANE = ZO_RY * ZO_RS;
constexpr int ZO_NX = ZO_RX * ZO_RY;  // staged x values per plane (816)
constexpr int ZO_GX = ZO_TX / 2 + 2, ZO_GY = ZO_TY / 2 + 2, ZO_GN = ZO_GX * ZO_GY;  // coarse tile 34 x 6

// RT: the residual as stored (r and r_old); ZF32: z is stored as the FP32
// sum before the output scale (the flexible PCG's FP32 storage, which applies
// the scale where it reads z), else as out_scale times it in FP64.
template <typename RT, bool ZF32>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void zout_kernel(const RT* __restrict__ r, NetCtl ctl, Dims d, int ntx,
                                                   int nty, int zchunk, const float* __restrict__ Wc,
                                                   const float* __restrict__ gz,
                                                   std::conditional_t<ZF32, float, double>* __restrict__ z,
                                                   const RT* __restrict__ r_old, double* __restrict__ part,
                                                   int npart) {
    __shared__ float xs[2][ZO_PLANE];
    __shared__ float gs[2][ZO_GN];
    // FP64 residual of the block's own outputs, kept from the staging of
    // plane q (iteration q) until output plane q is finished (iteration q + 2)
    __shared__ double rring[4][ZO_TY][ZO_TX];
    // weights, one dz slice per 28 floats (16-byte aligned slices, read as
    // float4 broadcasts; as scalar operands all 125 would not fit the SGPRs)
    __shared__ __attribute__((aligned(16))) float wsh[5 * 28];
    if (ctl.stop && *ctl.stop) return;
    if (threadIdx.x < 125) wsh[(threadIdx.x / 25) * 28 + threadIdx.x % 25] = Wc[threadIdx.x];
    const double in_scale = ctl.in_dev ? *ctl.in_dev : ctl.in_v;
    const double out_scale = ctl.out_dev ? *ctl.out_dev : ctl.out_v;
    const int blk = kvs_tiling::tile_of((int)blockIdx.x, (int)gridDim.x);
    const int tx = blk % ntx, t2 = blk / ntx;
    const int ty = t2 % nty, tz = t2 / nty;
    const int x0 = tx * ZO_TX, y0 = ty * ZO_TY;
    const int zs = tz * zchunk, ze = min(d.nz, zs + zchunk);
    const int t = threadIdx.x, lx = t & 63, ya = 2 * (t >> 6);
    const int sxy = d.nx * d.ny;
    const Dims c = coarse(d);

    // x plane: value i of the haloed tile (row i / ZO_RX, column i % ZO_RX);
    // loads are unconditional from clamped addresses, masked when stored
    auto xload = [&](int p, int h, double& v, bool& m) {
        const int i = t + 256 * h;
        const int ic = min(i, ZO_NX - 1);
        const int gx = x0 - 2 + ic % ZO_RX, gy = y0 - 2 + ic / ZO_RX;
        m = i < ZO_NX && p >= 0 && p < d.nz && gx >= 0 && gx < d.nx && gy >= 0 && gy < d.ny;
        const int pc = min(max(p, 0), d.nz - 1), yc = min(max(gy, 0), d.ny - 1), xc = min(max(gx, 0), d.nx - 1);
        v = r[(size_t)pc * sxy + (size_t)(yc * d.nx + xc)];
    };
    // coarse tile entry t: column X0 - 1 + t % ZO_GX, row Y0 - 1 + t / ZO_GX
    // (clamped; outputs only reference entries inside the coarse grid)
    const int gcol = min(t, ZO_GN - 1) % ZO_GX, grow = min(t, ZO_GN - 1) / ZO_GX;
    const int gX = min(max(x0 / 2 - 1 + gcol, 0), c.nx - 1), gY = min(max(y0 / 2 - 1 + grow, 0), c.ny - 1);
    auto gload = [&](int o, float& a, float& b) {
        int Iz, Jz;
        up_axis(min(max(o, 0), d.nz - 1), c.nz, Iz, Jz);
        const size_t col = (size_t)gY * c.nx + gX;
        a = gz[(size_t)Iz * c.ny * c.nx + col];
        b = gz[(size_t)Jz * c.ny * c.nx + col];
    };
    // this lane's outputs: column x, rows y and y + 1 (clamped for the gz
    // indices; outputs outside the grid are not stored)
    const int xo = x0 + lx, yo = y0 + ya;
    int Ix, Jx, Iy0, Jy0, Iy1, Jy1;
    up_axis(min(xo, d.nx - 1), c.nx, Ix, Jx);
    up_axis(min(yo, d.ny - 1), c.ny, Iy0, Jy0);
    up_axis(min(yo + 1, d.ny - 1), c.ny, Iy1, Jy1);
    const int cx0 = x0 / 2 - 1, cy0 = y0 / 2 - 1;
    const int gIx = Ix - cx0, gJx = Jx - cx0;
    const int gI0 = (Iy0 - cy0) * ZO_GX, gJ0 = (Jy0 - cy0) * ZO_GX;
    const int gI1 = (Iy1 - cy0) * ZO_GX, gJ1 = (Jy1 - cy0) * ZO_GX;
    const bool inx = xo >= 1 && xo <= d.nx - 2;
    const bool st0 = xo < d.nx && yo < d.ny, st1 = xo < d.nx && yo + 1 < d.ny;
    const bool in0 = inx && yo >= 1 && yo <= d.ny - 2, in1 = inx && yo + 1 >= 1 && yo + 1 <= d.ny - 2;
    const int lbase = ya * ZO_RS + lx;  // window origin: tile row ya, column lx

    double xv[4];
    bool xm[4];
    float ga = 0.f, gb = 0.f;
#pragma unroll
    for (int h = 0; h < 4; ++h) xload(zs - 2, h, xv[h], xm[h]);
    float a0[5] = {0.f, 0.f, 0.f, 0.f, 0.f}, a1[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    double dzr = 0.0, dzo = 0.0, dro = 0.0;  // partial inner products (part != null)
    for (int p = zs - 2; p <= ze + 1; ++p) {
        const int buf = (p - zs) & 1;
        float* xb = xs[buf];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int i = t + 256 * h;
            if (h < 3 || i < ZO_NX) {
                const int ic = min(i, ZO_NX - 1);
                xb[(ic / ZO_RX) * ZO_RS + ic % ZO_RX] = xm[h] ? (float)bf16_via_f32(in_scale * xv[h]) : 0.f;
                if (part) {
                    const int row = ic / ZO_RX - 2, col = ic % ZO_RX - 2;
                    if (row >= 0 && row < ZO_TY && col >= 0 && col < ZO_TX) rring[p & 3][row][col] = xm[h] ? xv[h] : 0.0;
                }
            }
        }
        // r_old at this iteration's outputs (plane p - 2), used after the stencil
        double ro0 = 0.0, ro1 = 0.0;
        if (r_old && p - 2 >= zs && p - 2 < ze) {
            const size_t zq = (size_t)(p - 2) * sxy + (size_t)yo * d.nx + xo;
            ro0 = r_old[st0 ? zq : 0];
            ro1 = r_old[st1 ? zq + d.nx : 0];
        }
        // output plane p - 2; the interpolations are written as explicit FMAs
        // (0.25 x is exact, so each weighted pair is rounded once) rather than
        // left to the compiler's contraction, which may pick either product
        if (t < ZO_GN) gs[buf][t] = fmaf(0.75f, ga, 0.25f * gb);
        if (p + 1 <= ze + 1) {
#pragma unroll
            for (int h = 0; h < 4; ++h) xload(p + 1, h, xv[h], xm[h]);
        }
        if (p - 1 >= zs && p - 1 < ze) gload(p - 1, ga, gb);
        kvs_tiling::lds_barrier();
        float v[6][5];
#pragma unroll
        for (int rr = 0; rr < 6; ++rr)
#pragma unroll
            for (int cc = 0; cc < 5; ++cc) v[rr][cc] = xb[lbase + rr * ZO_RS + cc];
        // plane p contributes to output p - 2 + k with the dz = 2 - k slice
        // the weight slice of the next k is read while this one is used; the
        // scheduling barriers keep two slices live at most
        // an opaque base offset keeps the weight reads in the loop (hoisted
        // out, all 125 would stay live in registers)
        int wo = 0;
        asm volatile("" : "+s"(wo));
        const float* wb = wsh + wo;
        float4 wc[7], wn[7];
#pragma unroll
        for (int q = 0; q < 7; ++q) wc[q] = *reinterpret_cast<const float4*>(wb + 4 * 28 + 4 * q);
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            if (k < 4) {
#pragma unroll
                for (int q = 0; q < 7; ++q) wn[q] = *reinterpret_cast<const float4*>(wb + (3 - k) * 28 + 4 * q);
            }
            __builtin_amdgcn_sched_barrier(0);
            const float* wk = reinterpret_cast<const float*>(wc);
#pragma unroll
            for (int dy = 0; dy < 5; ++dy)
#pragma unroll
                for (int dx = 0; dx < 5; ++dx) {
                    const float wt = wk[dy * 5 + dx];
                    a0[k] = fmaf(wt, v[dy][dx], a0[k]);
                    a1[k] = fmaf(wt, v[dy + 1][dx], a1[k]);
                }
            // the sums of this slice are final here (not sunk to the loop end,
            // where every slice's weights would be live at once)
            asm volatile("" : "+v"(a0[k]), "+v"(a1[k]));
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < 7; ++q) wc[q] = wn[q];
        }
        const int o = p - 2;
        if (o >= zs && o < ze) {
            const float* g = gs[buf];
            const float up0 = fmaf(0.75f, fmaf(0.75f, g[gI0 + gIx], 0.25f * g[gI0 + gJx]),
                                   0.25f * fmaf(0.75f, g[gJ0 + gIx], 0.25f * g[gJ0 + gJx]));
            const float up1 = fmaf(0.75f, fmaf(0.75f, g[gI1 + gIx], 0.25f * g[gI1 + gJx]),
                                   0.25f * fmaf(0.75f, g[gJ1 + gIx], 0.25f * g[gJ1 + gJx]));
            const bool inz = o >= 1 && o <= d.nz - 2;
            const size_t zo = (size_t)o * sxy + (size_t)yo * d.nx + xo;
            const float zu0 = in0 && inz ? a0[0] + up0 : 0.f, zu1 = in1 && inz ? a1[0] + up1 : 0.f;
            const double z0 = out_scale * (double)zu0;
            const double z1 = out_scale * (double)zu1;
            if constexpr (ZF32) {
                if (st0) z[zo] = zu0;
                if (st1) z[zo + d.nx] = zu1;
            } else {
                if (st0) z[zo] = z0;
                if (st1) z[zo + d.nx] = z1;
            }
            if (part) {
                // residuals at this lane's two outputs (outputs past the grid
                // have z = 0 and are left out of r.r_old)
                const double rn0 = rring[o & 3][ya][lx], rn1 = rring[o & 3][ya + 1][lx];
                dzr += z0 * rn0 + z1 * rn1;
                dzo += z0 * ro0 + z1 * ro1;
                dro += (in0 && inz ? rn0 * ro0 : 0.0) + (in1 && inz ? rn1 * ro1 : 0.0);
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            a0[k] = a0[k + 1];
            a1[k] = a1[k + 1];
        }
        a0[4] = 0.f;
        a1[4] = 0.f;
    }
    if (part) {
        // fixed-order block sums: wavefront butterflies, then wavefront 0
        __shared__ double dsum[3][4];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            dzr += __shfl_xor(dzr, o);
            dzo += __shfl_xor(dzo, o);
            dro += __shfl_xor(dro, o);
        }
        if ((t & 63) == 0) {
            dsum[0][t >> 6] = dzr;
            dsum[1][t >> 6] = dzo;
            dsum[2][t >> 6] = dro;
        }
        __syncthreads();
        if (t == 0) {
            part[blockIdx.x] = (dsum[0][0] + dsum[0][1]) + (dsum[0][2] + dsum[0][3]);
            part[npart + blockIdx.x] = (dsum[1][0] + dsum[1][1]) + (dsum[1][2] + dsum[1][3]);
            part[2 * npart + blockIdx.x] = (dsum[2][0] + dsum[2][1]) + (dsum[2][2] + dsum[2][3]);
        }
    }
}

// e0 = bf16(conv(x; W0)) at every voxel, for a training forward pass that
// keeps it (the backward pass of the output layer reads it).
__global__ void e0_keep_kernel(const double* __restrict__ r, NetCtl ctl, Dims d, const bf16* __restrict__ W0,
                               bf16* __restrict__ e0) {
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= d.n()) return;
    const double in_scale = ctl.in_dev ? *ctl.in_dev : ctl.in_v;
    const int x = (int)(v % d.nx), y = (int)((v / d.nx) % d.ny), zz = (int)(v / ((long long)d.nx * d.ny));
    float xt[27];
    for (int tap = 0; tap < 27; ++tap) {
        const int gx = x + tap_dx(tap), gy = y + tap_dy(tap), gzz = zz + tap_dz(tap);
        const bool in = gx >= 0 && gx < d.nx && gy >= 0 && gy < d.ny && gzz >= 0 && gzz < d.nz;
        xt[tap] = in ? (float)bf16_via_f32(in_scale * r[((size_t)gzz * d.ny + gy) * d.nx + gx]) : 0.f;
    }
    for (int c0 = 0; c0 < 16; c0 += 8) {
        bf16x8 o;
        for (int c = 0; c < 8; ++c) {
            float s = 0.f;
            for (int tap = 0; tap < 27; ++tap) s = fmaf((float)W0[(c0 + c) * 32 + tap], xt[tap], s);
            o[c] = (bf16)s;
        }
        *reinterpret_cast<bf16x8*>(e0 + v * 16 + c0) = o;
    }
}

// Skip input of a decoder level: out(v) = bf16(A(v) + up(B)(v)) with up the
// cell-centred trilinear interpolation from the coarser grid (8 channels per
// thread; the 8 coarse values summed in FP32).
template <int C>
__global__ __launch_bounds__(256) void skip_up_kernel(const bf16* __restrict__ A, const bf16* __restrict__ B, Dims d,
                                                      bf16* __restrict__ out, const int* stop) {
    if (stop && *stop) return;
    const Dims c = coarse(d);
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long v = t / (C / 8);
    const int c8 = (int)(t % (C / 8)) * 8;
    if (v >= d.n()) return;
    const unsigned vu = (unsigned)v, row = vu / (unsigned)d.nx;
    const int x = (int)(vu - row * (unsigned)d.nx), y = (int)(row % (unsigned)d.ny), z = (int)(row / (unsigned)d.ny);
    int Ix, Jx, Iy, Jy, Iz, Jz;
    up_axis(x, c.nx, Ix, Jx);
    up_axis(y, c.ny, Iy, Jy);
    up_axis(z, c.nz, Iz, Jz);
    const int zz[2] = {Iz, Jz}, yy[2] = {Iy, Jy}, xx[2] = {Ix, Jx};
    bf16x8 cv[8];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int e = 0; e < 2; ++e)
                cv[4 * a + 2 * b + e] =
                    *reinterpret_cast<const bf16x8*>(B + (((size_t)zz[a] * c.ny + yy[b]) * c.nx + xx[e]) * C + c8);
    const bf16x8 a8 = *reinterpret_cast<const bf16x8*>(A + (size_t)v * C + c8);
    bf16x8 o;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        float u = 0.f;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            u = fmaf(((q >> 2) ? 0.25f : 0.75f) * (((q >> 1) & 1) ? 0.25f : 0.75f) * ((q & 1) ? 0.25f : 0.75f),
                     (float)cv[q][j], u);
        o[j] = (bf16)((float)a8[j] + u);
    }
    *reinterpret_cast<bf16x8*>(out + (size_t)v * C + c8) = o;
}

hipError_t launch_skip_up(int ch, const bf16* A, const bf16* B, Dims d, bf16* out, hipStream_t s, const int* stop) {
    const long long threads = d.n() * (ch / 8);
    const int nb = (int)((threads + 255) / 256);
    switch (ch) {
        case 8: hipLaunchKernelGGL(skip_up_kernel<8>, dim3(nb), dim3(256), 0, s, A, B, d, out, stop); break;
        case 16: hipLaunchKernelGGL(skip_up_kernel<16>, dim3(nb), dim3(256), 0, s, A, B, d, out, stop); break;
        case 32: hipLaunchKernelGGL(skip_up_kernel<32>, dim3(nb), dim3(256), 0, s, A, B, d, out, stop); break;
        case 64: hipLaunchKernelGGL(skip_up_kernel<64>, dim3(nb), dim3(256), 0, s, A, B, d, out, stop); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// rows of a z-march tile: LDS of about 50-60 KB per block for any CI
constexpr int zm_rows(int ci) { return ci <= 16 ? 8 : (ci <= 32 ? 4 : 2); }

template <int CI, int CO, bool PROJ, typename OUT, bool POOL = false>
hipError_t launch_zm(const bf16* A, Dims d, const bf16* W, OUT* out, const float* wp, float* gz, hipStream_t s,
                     const int* stop, bf16* pooled = nullptr) {
    constexpr int TY = zm_rows(CI);
    auto kern = conv3_zm<CI, CO, TY, PROJ, OUT, POOL>;
    static const int cap = kvs_tiling::resident_blocks(kern, 256);
    const int ntx = (d.nx + 31) / 32, nty = (d.ny + TY - 1) / TY;
    int zchunk = kvs_tiling::choose_kchunk(ntx * nty, d.nz, cap);
    if (POOL) zchunk += zchunk & 1;  // segments start on even planes (z pairs of the pooling)
    const int nb = ntx * nty * ((d.nz + zchunk - 1) / zchunk);
    hipLaunchKernelGGL(kern, dim3(nb), dim3(256), 0, s, A, d, ntx, nty, zchunk, W, out, wp, gz, stop, pooled);
    return hipGetLastError();
}

// dispatch of the MFMA conv over the channel pairs this network uses:
// dilation 1 with up to 32 channels -> LDS z-march; dilated or 64-channel
// layers (the 1/4-resolution bottleneck, 32 or 64 input channels) ->
// sub-lattice bricks; the gathering kernel for the rest (fewer than 32 input
// channels with dilation or 64 output channels)
template <typename OUT>
hipError_t launch_conv(int ci, int co, const bf16* A, Dims d, int dil, const bf16* W, OUT* out, hipStream_t s,
                       const int* stop = nullptr) {
#define KVS_CONV_CASE(CI_, CO_)                                                                                \
    if (ci == CI_ && co == CO_) {                                                                              \
        if constexpr (CI_ <= 32 && CO_ <= 32) {                                                                \
            if (dil == 1) return launch_zm<CI_, CO_, false, OUT>(A, d, W, out, nullptr, nullptr, s, stop);     \
        }                                                                                                      \
        if constexpr (CI_ % 32 == 0) {                                                                         \
            if (d.n() * CI_ < (1LL << 31)) {                                                                   \
                const int ex = (d.nx + dil - 1) / dil, ey = (d.ny + dil - 1) / dil, ez = (d.nz + dil - 1) / dil; \
                constexpr int SBZ = 4 * sub_lz(CO_);                                                           \
                const SubBricks sb{(ex + SB_X - 1) / SB_X, (ey + SB_Y - 1) / SB_Y, (ez + SBZ - 1) / SBZ};        \
                const long long nsb = (long long)dil * dil * dil * sb.bx * sb.by * sb.bz;                     \
                if (nsb >= (1LL << 31)) return hipErrorInvalidValue;                                           \
                hipLaunchKernelGGL((conv3_sub<CI_, CO_, OUT>), dim3((unsigned)nsb), dim3(256), 0, s, A, d, dil, sb, \
                                   W, out, stop);                                                              \
                return hipGetLastError();                                                                      \
            }                                                                                                  \
        }                                                                                                      \
        constexpr int NV = conv_nv(CI_, CO_);                                                                  \
        /* bricks for dilation 1 (measured faster there; with dilation the       \
           linear order was as fast and wastes no lanes on partial bricks) */    \
        const Bricks bk = dil == 1 ? Bricks{(d.nx + 15) / 16, (d.ny + NV - 1) / NV, (d.nz + 3) / 4}                \
                                   : Bricks{0, 0, 0};                                                          \
        const long long nb = dil == 1 ? (long long)bk.bx * bk.by * bk.bz : (d.n() + 64 * NV - 1) / (64 * NV);  \
        if (nb >= (1LL << 31)) return hipErrorInvalidValue;                                                    \
        hipLaunchKernelGGL((conv3_mfma<CI_, CO_, NV, OUT>), dim3((unsigned)nb), dim3(256), 0, s, A, d, dil, bk, W, \
                           out, stop);                                                                         \
        return hipGetLastError();                                                                              \
    }
    KVS_CONV_CASE(16, 32)
    KVS_CONV_CASE(32, 64)
    KVS_CONV_CASE(64, 64)
    KVS_CONV_CASE(64, 32)
    KVS_CONV_CASE(32, 16)
    KVS_CONV_CASE(16, 16)
    KVS_CONV_CASE(8, 16)
    KVS_CONV_CASE(32, 32)
#undef KVS_CONV_CASE
    return hipErrorInvalidValue;
}

struct OutLaunch {
    int ntx, nty, zchunk, nblocks;
};

OutLaunch first_pool_launch(Dims d) {
    const Dims c = coarse(d);
    OutLaunch L;
    L.ntx = (c.nx + FP_CX - 1) / FP_CX;
    L.nty = (c.ny + FP_CY - 1) / FP_CY;
    static const int cap = kvs_tiling::resident_blocks(first_pool_kernel<double>, 256);
    L.zchunk = kvs_tiling::choose_kchunk(L.ntx * L.nty, c.nz, cap);
    L.nblocks = L.ntx * L.nty * ((c.nz + L.zchunk - 1) / L.zchunk);
    return L;
}

OutLaunch out_launch(Dims d) {
    OutLaunch L;
    L.ntx = (d.nx + ZO_TX - 1) / ZO_TX;
    L.nty = (d.ny + ZO_TY - 1) / ZO_TY;
    static const int cap = kvs_tiling::resident_blocks(zout_kernel<double, false>, 256);
    L.zchunk = kvs_tiling::choose_kchunk(L.ntx * L.nty, d.nz, cap);
    L.nblocks = L.ntx * L.nty * ((d.nz + L.zchunk - 1) / L.zchunk);
    return L;
}

}  // namespace

// ---- training kernels ------------------------------------------------------------

namespace {

__global__ void f32_to_bf16(const float* __restrict__ a, bf16* __restrict__ b, long long n) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) b[q] = (bf16)a[q];
}

// Weight gradient of one conv: part[tap][blk][co * CI + ci] =
//   sum over the block's voxels v of x(v + dil tap)[ci] * dy[v][co],
// x(p) = A[p] as the forward read it (or, FIRST, the scaled FP64 input
// rounded to BF16); dy in FP32.  64 voxels are staged in
// LDS at a time; each thread owns a fixed set of (co, ci) pairs.
template <int CI, int CO, bool FIRST>
__global__ __launch_bounds__(256) void dw_partial(const bf16* __restrict__ A, const double* __restrict__ r,
                                                  double in_scale, Dims d, int dil,
                                                  const float* __restrict__ dy, float* __restrict__ part) {
    constexpr int NP = CI * CO;
    constexpr int PER = (NP + 255) / 256;
    __shared__ float xs[64][CI];
    __shared__ float ys[64][CO];
    const int tap = blockIdx.y;
    const int ox = dil * tap_dx(tap), oy = dil * tap_dy(tap), oz = dil * tap_dz(tap);
    const long long N = d.n();
    float acc[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) acc[q] = 0.f;
    for (long long base = (long long)blockIdx.x * 64; base < N; base += (long long)gridDim.x * 64) {
        for (int idx = threadIdx.x; idx < 64 * CI; idx += 256) {
            const int vox = idx / CI, c = idx % CI;
            const long long v = base + vox;
            float val = 0.f;
            if (v < N) {
                const int x = (int)(v % d.nx) + ox, y = (int)((v / d.nx) % d.ny) + oy,
                          z = (int)(v / ((long long)d.nx * d.ny)) + oz;
                if (x >= 0 && x < d.nx && y >= 0 && y < d.ny && z >= 0 && z < d.nz) {
                    const long long p = x + (long long)d.nx * (y + (long long)d.ny * z);
                    if constexpr (FIRST) {
                        val = (float)bf16_via_f32(in_scale * r[p]);
                    } else {
                        val = (float)A[p * CI + c];
                    }
                }
            }
            xs[vox][c] = val;
        }
        for (int idx = threadIdx.x; idx < 64 * CO; idx += 256) {
            const int vox = idx / CO, c = idx % CO;
            const long long v = base + vox;
            ys[vox][c] = v < N ? dy[v * CO + c] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int pidx = threadIdx.x + 256 * q;
            if (pidx < NP) {
                const int co = pidx / CI, ci = pidx % CI;
                float a = acc[q];
                for (int vox = 0; vox < 64; ++vox) a += xs[vox][ci] * ys[vox][co];
                acc[q] = a;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int pidx = threadIdx.x + 256 * q;
        if (pidx < NP) part[((long long)tap * gridDim.x + blockIdx.x) * NP + pidx] = acc[q];
    }
}

// grad[co][tap * CI + ci] (+)= sum over blocks, fixed order
__global__ void dw_reduce(const float* __restrict__ part, int nblk, int CI, int CO, float* __restrict__ grad,
                          int accumulate) {
    const int NP = CI * CO;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 27LL * NP) return;
    const int tap = (int)(t / NP), pidx = (int)(t % NP);
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += part[((long long)tap * nblk + b) * NP + pidx];
    const int co = pidx / CI, ci = pidx % CI;
    float* g = grad + (long long)co * 27 * CI + tap * CI + ci;
    *g = accumulate ? *g + s : s;
}

// dg[v][ci] = sum_tap W[tap][ci] * dz[v - tap]   (output layer, one channel)
template <int CI>
__global__ void out_backward(const float* __restrict__ dz, Dims d, const float* __restrict__ W, float* __restrict__ dg) {
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= d.n()) return;
    const int x = (int)(v % d.nx), y = (int)((v / d.nx) % d.ny), z = (int)(v / ((long long)d.nx * d.ny));
    float acc[CI];
#pragma unroll
    for (int c = 0; c < CI; ++c) acc[c] = 0.f;
    for (int tap = 0; tap < 27; ++tap) {
        const int px = x - tap_dx(tap), py = y - tap_dy(tap), pz = z - tap_dz(tap);
        if (px < 0 || px >= d.nx || py < 0 || py >= d.ny || pz < 0 || pz >= d.nz) continue;
        const float g = dz[px + (long long)d.nx * (py + (long long)d.ny * pz)];
#pragma unroll
        for (int c = 0; c < CI; ++c) acc[c] += W[tap * CI + c] * g;
    }
#pragma unroll
    for (int c = 0; c < CI; ++c) dg[v * CI + c] = acc[c];
}

// weight of fine cell i in the interpolation of coarse cell V (one axis)
__device__ __forceinline__ float up_weight(int i, int V, int nc) {
    int I, J;
    up_axis(i, nc, I, J);
    return (I == V ? 0.75f : 0.f) + (J == V ? 0.25f : 0.f);
}

// adjoint of the trilinear interpolation: dc[V][c] = sum over the fine cells
// 2V-1 .. 2V+2 (per axis) of their interpolation weight on V times df
__global__ void up_adjoint(const float* __restrict__ df, Dims d, int C, float* __restrict__ dc) {
    const Dims cd = coarse(d);
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cd.n() * C) return;
    const long long V = t / C;
    const int c = (int)(t % C);
    const int X = (int)(V % cd.nx), Y = (int)((V / cd.nx) % cd.ny), Z = (int)(V / ((long long)cd.nx * cd.ny));
    float s = 0.f;
    for (int z = 2 * Z - 1; z <= 2 * Z + 2; ++z) {
        if (z < 0 || z >= d.nz) continue;
        const float wz = up_weight(z, Z, cd.nz);
        if (wz == 0.f) continue;
        for (int y = 2 * Y - 1; y <= 2 * Y + 2; ++y) {
            if (y < 0 || y >= d.ny) continue;
            const float wy = up_weight(y, Y, cd.ny);
            if (wy == 0.f) continue;
            for (int x = 2 * X - 1; x <= 2 * X + 2; ++x) {
                if (x < 0 || x >= d.nx) continue;
                const float wx = up_weight(x, X, cd.nx);
                if (wx == 0.f) continue;
                s = fmaf(wz * wy * wx, df[(x + (long long)d.nx * (y + (long long)d.ny * z)) * C + c], s);
            }
        }
    }
    dc[t] = s;
}

// pointwise projection gz = g . wp (C channels): block partials of
// sum_V g[V][c] dgz[V] for the weight gradient ...
template <int C>
__global__ __launch_bounds__(256) void proj_grad_partial(const bf16* __restrict__ g, const float* __restrict__ dgz,
                                                         long long n, float* __restrict__ part) {
    __shared__ float sh[256];
    float acc = 0.f;
    const int c = threadIdx.x % C;
    for (long long v = (long long)blockIdx.x * (256 / C) + threadIdx.x / C; v < n; v += (long long)gridDim.x * (256 / C))
        acc = fmaf((float)g[v * C + c], dgz[v], acc);
    sh[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < C) {
        float s = 0.f;
        for (int q = threadIdx.x; q < 256; q += C) s += sh[q];
        part[(long long)blockIdx.x * C + threadIdx.x] = s;
    }
}

__global__ void proj_grad_reduce(const float* __restrict__ part, int nblk, int C, float* __restrict__ grad,
                                 int accumulate) {
    const int c = threadIdx.x;
    if (c >= C) return;
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += part[(long long)b * C + c];
    grad[c] = accumulate ? grad[c] + s : s;
}

// ... and its adjoint dg[V][c] = wp[c] dgz[V]
__global__ void proj_adjoint(const float* __restrict__ dgz, const float* __restrict__ wp, long long n, int C,
                             float* __restrict__ dg) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n * C) dg[t] = wp[t % C] * dgz[t / C];
}

// adjoint of mean pooling, added: df[v][c] += dc[v/2][c] / (children of v/2)
__global__ void pool_adjoint_add(const float* __restrict__ dc, Dims d, int C, float* __restrict__ df) {
    const Dims cd = coarse(d);
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= d.n() * C) return;
    const long long v = t / C;
    const int c = (int)(t % C);
    const int x = (int)(v % d.nx), y = (int)((v / d.nx) % d.ny), z = (int)(v / ((long long)d.nx * d.ny));
    const int X = x >> 1, Y = y >> 1, Z = z >> 1;
    const int cnt = (std::min(2 * X + 2, d.nx) - 2 * X) * (std::min(2 * Y + 2, d.ny) - 2 * Y) * (std::min(2 * Z + 2, d.nz) - 2 * Z);
    df[t] += dc[(X + (long long)cd.nx * (Y + (long long)cd.ny * Z)) * C + c] / (float)cnt;
}

// A-norm loss of the unit-spacing Poisson operator A = -lap (interior):
// e = z - xs; dz_raw = A e (0 outside the interior); block partials of
// e.Ae and xs.A xs.
__global__ void anorm_loss(const double* __restrict__ z, const double* __restrict__ xs, Dims d,
                           double* __restrict__ dz_raw, double* __restrict__ part) {
    __shared__ double sh[2][256];
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double s1 = 0.0, s2 = 0.0;
    if (v < d.n()) {
        const int x = (int)(v % d.nx), y = (int)((v / d.nx) % d.ny), zz = (int)(v / ((long long)d.nx * d.ny));
        double ae = 0.0;
        if (x >= 1 && x <= d.nx - 2 && y >= 1 && y <= d.ny - 2 && zz >= 1 && zz <= d.nz - 2) {
            const long long sy = d.nx, sz = (long long)d.nx * d.ny;
            auto e = [&](long long q) { return z[q] - xs[q]; };
            ae = 6.0 * e(v) - e(v - 1) - e(v + 1) - e(v - sy) - e(v + sy) - e(v - sz) - e(v + sz);
            const double ax = 6.0 * xs[v] - xs[v - 1] - xs[v + 1] - xs[v - sy] - xs[v + sy] - xs[v - sz] - xs[v + sz];
            s1 = e(v) * ae;
            s2 = xs[v] * ax;
        }
        dz_raw[v] = ae;
    }
    sh[0][threadIdx.x] = s1;
    sh[1][threadIdx.x] = s2;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + o];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sh[0][0];
        part[2 * blockIdx.x + 1] = sh[1][0];
    }
}

__global__ void scale_to_f32(const double* __restrict__ a, double s, float* __restrict__ b, long long n) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) b[q] = (float)(s * a[q]);
}

__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, long long n, float lr, float b1, float b2, float eps, float c1,
                            float c2, float gscale) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const float gq = g[q] * gscale;
    const float mq = b1 * m[q] + (1.f - b1) * gq;
    const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    w[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

// x = xs - xk, then both scaled later
__global__ void sub_kernel(const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ out,
                           long long n) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) out[q] = a[q] - b[q];
}

__global__ void scale_kernel(double* __restrict__ a, double s, long long n) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) a[q] *= s;
}

// y = A x = -lap_h x on the interior (0 elsewhere); block partials of y.y
__global__ void apply_A_kernel(const double* __restrict__ x, Dims d, double ihx2, double ihy2, double ihz2,
                               double* __restrict__ y, double* __restrict__ part) {
    __shared__ double sh[256];
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    if (v < d.n()) {
        const int i = (int)(v % d.nx), j = (int)((v / d.nx) % d.ny), k = (int)(v / ((long long)d.nx * d.ny));
        double a = 0.0;
        if (i >= 1 && i <= d.nx - 2 && j >= 1 && j <= d.ny - 2 && k >= 1 && k <= d.nz - 2) {
            const long long sy = d.nx, sz = (long long)d.nx * d.ny;
            const double c2 = 2.0 * x[v];
            a = -((x[v + 1] + x[v - 1] - c2) * ihx2 + (x[v + sy] + x[v - sy] - c2) * ihy2 +
                  (x[v + sz] + x[v - sz] - c2) * ihz2);
            s = a * a;
        }
        y[v] = a;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

int nblocks256(long long n) { return (int)((n + 255) / 256); }

}  // namespace

// ---- network object ------------------------------------------------------------

struct UnetLayerDesc {
    int ci, co, dil, level;  // dil 0: pointwise (one tap); level of the output
    int taps() const { return dil > 0 ? 27 : 1; }
};

struct kvs_unet {
    int c0 = 16, c1 = 32, c2 = 64, nbott = 4;
    std::vector<UnetLayerDesc> layers;  // 0 first, 1 enc1, 2.. bottleneck, dec1, projection, out
    std::vector<int64_t> w_off, wt_off;  // offsets of each layer's bf16 weights (forward, transposed)
    std::vector<int64_t> kp, kpt;        // padded K per layer (forward, transposed)
    std::vector<int64_t> m_off;          // offset of each layer in the flat master layout
    int64_t n_w = 0, n_wt = 0, n_master = 0;
    bf16* w = nullptr;       // device bf16 forward weights
    bf16* wt = nullptr;      // device bf16 transposed weights (for the backward pass)
    float* w_proj = nullptr; // device fp32 (bf16-rounded) projection weights [C0]
    float* w_out = nullptr;  // device fp32 (bf16-rounded) output weights [27][C0] (backward pass)
    float* w_comp = nullptr; // device fp32 composed output stencil [5][5][5] (dz, dy, dx): W_out after W0
    bf16* w_pool = nullptr;  // device bf16 pair (hi, lo) of the composed pooled first conv [2][16][64]
    float* master = nullptr; // device fp32 master weights (flat)
    float* grad = nullptr;   // device fp32 gradient (flat, same layout)
    float* adam_m = nullptr;
    float* adam_v = nullptr;
    int64_t adam_t = 0;
    std::vector<float> host_master;
    // activations of the last grid: p0, e1, p1, bottleneck outputs, i1 (kept
    // for the backward pass), gz; g1 (1/2 resolution) and e0 (full
    // resolution) only when a forward pass is asked to keep them (training)
    Dims dims{0, 0, 0};
    bf16 *p0 = nullptr, *e1 = nullptr, *p1 = nullptr, *i1 = nullptr, *g1 = nullptr;
    float* gz = nullptr;
    std::vector<bf16*> bott;
    bf16* e0k = nullptr;
    Dims e0_dims{0, 0, 0};
    bool kept = false;  // the last forward pass stored g1 and e0 for this grid
    // training buffers (allocated on first use)
    Dims tdims{0, 0, 0};
    float *de0 = nullptr, *dp0 = nullptr, *dg1 = nullptr, *de1 = nullptr, *dp1 = nullptr, *dgz = nullptr;
    std::vector<float*> dbott;  // gradient of each bottleneck output, and of its input p1 (last)
    bf16* gb = nullptr;         // bf16 staging of a gradient (conv^T input)
    float* dzf = nullptr;
    double* dz_raw = nullptr;
    double* part = nullptr;
    float* wpart = nullptr;
    int64_t wpart_n = 0;
    std::string err;
};

namespace {

template <typename P>
void ufree(P*& p) {
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

void unet_free_acts(kvs_unet* u) {
    for (bf16** p : {&u->p0, &u->e1, &u->p1, &u->i1, &u->g1, &u->e0k}) ufree(*p);
    ufree(u->gz);
    for (bf16*& p : u->bott) ufree(p);
    u->bott.clear();
    u->dims = Dims{0, 0, 0};
    u->e0_dims = Dims{0, 0, 0};
    u->kept = false;
}

void unet_free_train(kvs_unet* u) {
    for (float** p : {&u->de0, &u->dp0, &u->dg1, &u->de1, &u->dp1, &u->dgz, &u->dzf}) ufree(*p);
    for (float*& p : u->dbott) ufree(p);
    u->dbott.clear();
    ufree(u->gb);
    ufree(u->dz_raw);
    ufree(u->part);
    ufree(u->wpart);
    u->wpart_n = 0;
    u->tdims = Dims{0, 0, 0};
}

hipError_t unet_ensure_acts(kvs_unet* u, Dims d) {
    if (u->p0 && u->dims.nx == d.nx && u->dims.ny == d.ny && u->dims.nz == d.nz) return hipSuccess;
    unet_free_acts(u);
    const Dims d1 = coarse(d), d2 = coarse(d1);
    const long long n1 = d1.n(), n2 = d2.n();
    hipError_t e = hipMalloc(&u->p0, sizeof(bf16) * n1 * u->c0);
    if (e == hipSuccess) e = hipMalloc(&u->e1, sizeof(bf16) * n1 * u->c1);
    if (e == hipSuccess) e = hipMalloc(&u->i1, sizeof(bf16) * n1 * u->c1);
    if (e == hipSuccess) e = hipMalloc(&u->g1, sizeof(bf16) * n1 * u->c0);
    if (e == hipSuccess) e = hipMalloc(&u->gz, sizeof(float) * n1);
    if (e == hipSuccess) e = hipMalloc(&u->p1, sizeof(bf16) * n2 * u->c1);
    for (int q = 0; q < u->nbott && e == hipSuccess; ++q) {
        bf16* b = nullptr;
        e = hipMalloc(&b, sizeof(bf16) * n2 * u->c2);
        u->bott.push_back(b);
    }
    if (e != hipSuccess) {
        unet_free_acts(u);
        return e;
    }
    u->dims = d;
    return hipSuccess;
}

// e0 at full resolution, for a forward pass that keeps it
hipError_t unet_ensure_e0(kvs_unet* u, Dims d) {
    if (u->e0k && u->e0_dims.nx == d.nx && u->e0_dims.ny == d.ny && u->e0_dims.nz == d.nz) return hipSuccess;
    ufree(u->e0k);
    u->e0_dims = Dims{0, 0, 0};
    hipError_t e = hipMalloc(&u->e0k, sizeof(bf16) * d.n() * u->c0);
    if (e == hipSuccess) u->e0_dims = d;
    return e;
}

hipError_t unet_ensure_train(kvs_unet* u, Dims d) {
    if (u->de0 && u->tdims.nx == d.nx && u->tdims.ny == d.ny && u->tdims.nz == d.nz) return hipSuccess;
    unet_free_train(u);
    const Dims d1 = coarse(d), d2 = coarse(d1);
    const long long n0 = d.n(), n1 = d1.n(), n2 = d2.n();
    hipError_t e = hipMalloc(&u->de0, sizeof(float) * n0 * u->c0);
    if (e == hipSuccess) e = hipMalloc(&u->dp0, sizeof(float) * n1 * u->c0);
    if (e == hipSuccess) e = hipMalloc(&u->dg1, sizeof(float) * n1 * u->c0);
    if (e == hipSuccess) e = hipMalloc(&u->dgz, sizeof(float) * n1);
    if (e == hipSuccess) e = hipMalloc(&u->de1, sizeof(float) * n1 * u->c1);
    if (e == hipSuccess) e = hipMalloc(&u->dp1, sizeof(float) * n2 * u->c1);
    for (int q = 0; q < u->nbott && e == hipSuccess; ++q) {
        float* b = nullptr;
        e = hipMalloc(&b, sizeof(float) * n2 * u->c2);
        u->dbott.push_back(b);
    }
    if (e == hipSuccess) e = hipMalloc(&u->gb, sizeof(bf16) * std::max(n1 * u->c1, n2 * u->c2));
    if (e == hipSuccess) e = hipMalloc(&u->dzf, sizeof(float) * n0);
    if (e == hipSuccess) e = hipMalloc(&u->dz_raw, sizeof(double) * n0);
    if (e == hipSuccess) e = hipMalloc(&u->part, sizeof(double) * 2 * nblocks256(n0));
    if (e != hipSuccess) {
        unet_free_train(u);
        return e;
    }
    u->tdims = d;
    return hipSuccess;
}


void build_layers(kvs_unet* u) {
    u->layers.clear();
    u->layers.push_back({1, u->c0, 1, 0});      // e0
    u->layers.push_back({u->c0, u->c1, 1, 1});  // e1 = conv(pool e0)
    u->layers.push_back({u->c1, u->c2, 1, 2});  // bottleneck in
    int dil = 2;
    for (int q = 0; q < u->nbott - 2; ++q, dil *= 2) u->layers.push_back({u->c2, u->c2, dil, 2});
    u->layers.push_back({u->c2, u->c1, 1, 2});  // bottleneck out
    u->layers.push_back({u->c1, u->c0, 1, 1});  // g1 = conv(e1 + up b)
    u->layers.push_back({u->c0, 1, 0, 1});      // gz = g1 . wp
    u->layers.push_back({u->c0, 1, 1, 0});      // z = conv(e0) + up(gz)
    u->w_off.clear();
    u->wt_off.clear();
    u->kp.clear();
    u->kpt.clear();
    u->m_off.clear();
    int64_t off = 0, offt = 0, offm = 0;
    const size_t nconv = u->layers.size() - 2;  // 27-tap layers with MFMA weight layouts
    for (size_t l = 0; l < u->layers.size(); ++l) {
        const UnetLayerDesc& L = u->layers[l];
        u->m_off.push_back(offm);
        offm += (int64_t)L.taps() * L.ci * L.co;
        if (l >= nconv) continue;
        const int64_t kp = L.ci == 1 ? 32 : (27 * L.ci + 31) / 32 * 32;
        const int64_t kpt = (27 * L.co + 31) / 32 * 32;
        u->w_off.push_back(off);
        u->kp.push_back(kp);
        off += kp * L.co;
        u->wt_off.push_back(offt);
        u->kpt.push_back(kpt);
        offt += L.ci == 1 ? 0 : kpt * L.ci;
    }
    u->n_w = off;
    u->n_wt = offt;
    u->n_master = offm;
}

}  // namespace

// Network application: z = out_scale * U(in_scale * r) (scales from ctl);
// keep: also store g1 (1/2 resolution) and e0 (full resolution) for a
// backward pass.
// RT, ZF32: the storage of r and z (zout_kernel); keep needs FP64 r.
template <typename RT = double, bool ZF32 = false>
hipError_t kvs_unet_apply(kvs_unet* u, const RT* r, const NetCtl& ctl, std::conditional_t<ZF32, float, double>* z, Dims d,
                          hipStream_t s, bool keep = false, const UnetDots* dots = nullptr, int* nblocks = nullptr) {
    if (d.n() >= (1LL << 31)) return hipErrorInvalidValue;  // 32-bit voxel indices in the kernels
    hipError_t e = unet_ensure_acts(u, d);
    if (e == hipSuccess && keep) e = unet_ensure_e0(u, d);
    if (e != hipSuccess) return e;
    u->kept = false;
    const Dims d1 = coarse(d), d2 = coarse(d1);
    const std::vector<UnetLayerDesc>& L = u->layers;
    const int nl = (int)L.size();
    const int ld1 = nl - 3;
    const int* stop = ctl.stop;
    const OutLaunch fl = first_pool_launch(d);
    hipLaunchKernelGGL(first_pool_kernel<RT>, dim3(fl.nblocks), dim3(256), 0, s, r, ctl, d, fl.ntx, fl.nty, fl.zchunk,
                       u->w_pool, u->p0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((d.nx | d.ny | d.nz) & 1) {
        const Dims c = coarse(d);
        const long long faces = ((d.nx & 1) ? (long long)c.ny * c.nz : 0) + ((d.ny & 1) ? (long long)c.nx * c.nz : 0) +
                                ((d.nz & 1) ? (long long)c.nx * c.ny : 0);
        hipLaunchKernelGGL(pool0_edge_kernel<RT>, dim3(nblocks256(faces * 16)), dim3(256), 0, s, r, ctl, d,
                           u->w + u->w_off[0], u->p0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // e1 = conv(p0) and its pooling p1 in one z-march
    if ((e = launch_zm<16, 32, false, bf16, true>(u->p0, d1, u->w + u->w_off[1], u->e1, nullptr, nullptr, s, stop,
                                                  u->p1)) != hipSuccess)
        return e;
    const bf16* in = u->p1;
    for (int l = 2; l < ld1; ++l) {
        bf16* out = u->bott[(size_t)(l - 2)];
        if ((e = launch_conv(L[l].ci, L[l].co, in, d2, L[l].dil, u->w + u->w_off[l], out, s, stop)) != hipSuccess)
            return e;
        in = out;
    }
    if ((e = launch_skip_up(u->c1, u->e1, in, d1, u->i1, s, stop)) != hipSuccess) return e;
    if ((e = launch_zm<32, 16, true, bf16>(u->i1, d1, u->w + u->w_off[ld1], keep ? u->g1 : nullptr, u->w_proj, u->gz,
                                          s, stop)) != hipSuccess)
        return e;
    const OutLaunch ol = out_launch(d);
    if (dots && ol.nblocks > dots->npart) return hipErrorInvalidValue;  // partials sized at context creation
    hipLaunchKernelGGL((zout_kernel<RT, ZF32>), dim3(ol.nblocks), dim3(256), 0, s, r, ctl, d, ol.ntx, ol.nty, ol.zchunk,
                       u->w_comp, u->gz, z, dots ? static_cast<const RT*>(dots->r_old) : nullptr,
                       dots ? dots->part : nullptr, dots ? dots->npart : 0);
    if (nblocks) *nblocks = ol.nblocks;
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if constexpr (std::is_same_v<RT, double>) {
        if (keep) {
            hipLaunchKernelGGL(e0_keep_kernel, dim3(nblocks256(d.n())), dim3(256), 0, s, r, ctl, d,
                               u->w + u->w_off[0], u->e0k);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    } else if (keep) {
        return hipErrorInvalidValue;
    }
    u->kept = keep;
    return hipSuccess;
}

hipError_t kvs_unet_precondition(kvs_unet* u, const double* r, double* z, const kvs_grid& g, const double* in_scale,
                                 const double* out_scale, const int* stop, hipStream_t s, const UnetDots* dots,
                                 int* nblocks) {
    NetCtl ctl{in_scale, out_scale, stop, 1.0, 1.0};
    return kvs_unet_apply(u, r, ctl, z, Dims{(int)g.nx, (int)g.ny, (int)g.nz}, s, false, dots, nblocks);
}

hipError_t kvs_unet_precondition32(kvs_unet* u, const float* r, float* z_sum, const kvs_grid& g,
                                   const double* in_scale, const double* out_scale, const int* stop, hipStream_t s,
                                   const UnetDots* dots, int* nblocks) {
    NetCtl ctl{in_scale, out_scale, stop, 1.0, 1.0};
    return kvs_unet_apply<float, true>(u, r, ctl, z_sum, Dims{(int)g.nx, (int)g.ny, (int)g.nz}, s, false, dots,
                                       nblocks);
}

int64_t kvs_unet_out_blocks(const kvs_grid& g) {
    return out_launch(Dims{(int)g.nx, (int)g.ny, (int)g.nz}).nblocks;
}

namespace {

// dispatch of the weight-gradient reduction
hipError_t launch_dw(kvs_unet* u, int ci, int co, bool first, const bf16* A, const double* r,
                     double in_scale, Dims d, int dil, const float* dy, int64_t m_off, int accumulate, hipStream_t s) {
    const int nblk = (int)std::min<long long>(256, (d.n() + 63) / 64);
    const int64_t need = 27LL * nblk * ci * co;
    if (need > u->wpart_n) {
        ufree(u->wpart);
        hipError_t e = hipMalloc(&u->wpart, sizeof(float) * need);
        if (e != hipSuccess) return e;
        u->wpart_n = need;
    }
    const dim3 grid(nblk, 27);
#define KVS_DW_CASE(CI_, CO_, F_)                                                                                  \
    if (ci == CI_ && co == CO_ && first == F_) {                                                                   \
        hipLaunchKernelGGL((dw_partial<CI_, CO_, F_>), grid, dim3(256), 0, s, A, r, in_scale, d, dil, dy, u->wpart); \
    } else
    KVS_DW_CASE(1, 16, true)
    KVS_DW_CASE(16, 32, false)
    KVS_DW_CASE(32, 64, false)
    KVS_DW_CASE(64, 64, false)
    KVS_DW_CASE(64, 32, false)
    KVS_DW_CASE(32, 16, false)
    KVS_DW_CASE(16, 16, false)
    KVS_DW_CASE(16, 1, false) { return hipErrorInvalidValue; }
#undef KVS_DW_CASE
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(dw_reduce, dim3(nblocks256(27LL * ci * co)), dim3(256), 0, s, u->wpart, nblk, ci, co,
                       u->grad + m_off, accumulate);
    return hipGetLastError();
}

hipError_t to_bf16(const float* a, bf16* b, long long n, hipStream_t s) {
    hipLaunchKernelGGL(f32_to_bf16, dim3(nblocks256(n)), dim3(256), 0, s, a, b, n);
    return hipGetLastError();
}

// Backward pass of the last forward (input r, in_scale), given the FP32
// gradient dzf of the raw network output (before out_scale) on the interior.
// Accumulates (or writes) the flat FP32 weight gradient.
hipError_t unet_backward(kvs_unet* u, const double* r, double in_scale, Dims d, int accumulate, hipStream_t s) {
    hipError_t e = unet_ensure_train(u, d);
    if (e != hipSuccess) return e;
    const Dims d1 = coarse(d), d2 = coarse(d1);
    const std::vector<UnetLayerDesc>& L = u->layers;
    const int nl = (int)L.size();
    const int lo = nl - 1, lp = nl - 2, ld1 = nl - 3;
    const int c0 = u->c0, c1 = u->c1;
    // output: z = conv(e0; W_out) + up(gz)
    if ((e = launch_dw(u, c0, 1, false, u->e0k, nullptr, 0.0, d, 1, u->dzf, u->m_off[lo], accumulate, s)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(out_backward<16>, dim3(nblocks256(d.n())), dim3(256), 0, s, u->dzf, d, u->w_out, u->de0);
    hipLaunchKernelGGL(up_adjoint, dim3(nblocks256(d1.n())), dim3(256), 0, s, u->dzf, d, 1, u->dgz);
    // projection gz = g1 . wp
    {
        const int nblk = (int)std::min<long long>(256, (d1.n() + 15) / 16);
        if ((long long)nblk * c0 > u->wpart_n) {
            ufree(u->wpart);
            if ((e = hipMalloc(&u->wpart, sizeof(float) * nblk * c0)) != hipSuccess) return e;
            u->wpart_n = (int64_t)nblk * c0;
        }
        hipLaunchKernelGGL(proj_grad_partial<16>, dim3(nblk), dim3(256), 0, s, u->g1, u->dgz, d1.n(), u->wpart);
        hipLaunchKernelGGL(proj_grad_reduce, dim3(1), dim3(64), 0, s, u->wpart, nblk, c0, u->grad + u->m_off[lp],
                           accumulate);
        hipLaunchKernelGGL(proj_adjoint, dim3(nblocks256(d1.n() * c0)), dim3(256), 0, s, u->dgz, u->w_proj, d1.n(), c0,
                           u->dg1);
    }
    // dec1: g1 = conv(i1), i1 = e1 + up(b_last)
    if ((e = launch_dw(u, c1, c0, false, u->i1, nullptr, 0.0, d1, 1, u->dg1, u->m_off[ld1], accumulate, s)) !=
        hipSuccess)
        return e;
    if ((e = to_bf16(u->dg1, u->gb, d1.n() * c0, s)) != hipSuccess) return e;
    if ((e = launch_conv(c0, c1, u->gb, d1, 1, u->wt + u->wt_off[ld1], u->de1, s)) != hipSuccess) return e;
    float* dcur = u->dbott[(size_t)(u->nbott - 1)];  // gradient of the last bottleneck output (C1 channels)
    hipLaunchKernelGGL(up_adjoint, dim3(nblocks256(d2.n() * c1)), dim3(256), 0, s, u->de1, d1, c1, dcur);
    // bottleneck, last to first
    for (int l = ld1 - 1; l >= 2; --l) {
        const int q = l - 2;
        const bf16* xin = q == 0 ? u->p1 : u->bott[(size_t)(q - 1)];
        float* dxin = q == 0 ? u->dp1 : u->dbott[(size_t)(q - 1)];
        if ((e = launch_dw(u, L[l].ci, L[l].co, false, xin, nullptr, 0.0, d2, L[l].dil, dcur, u->m_off[l], accumulate,
                           s)) != hipSuccess)
            return e;
        if ((e = to_bf16(dcur, u->gb, d2.n() * L[l].co, s)) != hipSuccess) return e;
        if ((e = launch_conv(L[l].co, L[l].ci, u->gb, d2, L[l].dil, u->wt + u->wt_off[l], dxin, s)) != hipSuccess)
            return e;
        dcur = dxin;
    }
    // pool(e1) -> bottleneck input
    hipLaunchKernelGGL(pool_adjoint_add, dim3(nblocks256(d1.n() * c1)), dim3(256), 0, s, u->dp1, d1, c1, u->de1);
    // e1 = conv(pool e0)
    if ((e = launch_dw(u, c0, c1, false, u->p0, nullptr, 0.0, d1, 1, u->de1, u->m_off[1], accumulate, s)) != hipSuccess)
        return e;
    if ((e = to_bf16(u->de1, u->gb, d1.n() * c1, s)) != hipSuccess) return e;
    if ((e = launch_conv(c1, c0, u->gb, d1, 1, u->wt + u->wt_off[1], u->dp0, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(pool_adjoint_add, dim3(nblocks256(d.n() * c0)), dim3(256), 0, s, u->dp0, d, c0, u->de0);
    // e0 = conv(in_scale r)
    return launch_dw(u, 1, c0, true, nullptr, r, in_scale, d, 1, u->de0, u->m_off[0], accumulate, s);
}

}  // namespace


// ---- C ABI ---------------------------------------------------------------------

namespace {
thread_local std::string g_unet_err;
kvs_status ufail(kvs_unet* u, kvs_status s, const std::string& m) {
    if (u)
        u->err = m;
    else
        g_unet_err = m;
    return s;
}

// host master -> device master, bf16 forward / transposed layouts, fp32 out
kvs_status upload_weights(kvs_unet* u) {
    std::vector<bf16> wb((size_t)u->n_w, (bf16)0.f), wtb((size_t)std::max<int64_t>(u->n_wt, 1), (bf16)0.f);
    const int nl = (int)u->layers.size();
    for (int l = 0; l < nl - 2; ++l) {
        const UnetLayerDesc& L = u->layers[(size_t)l];
        const float* m = u->host_master.data() + u->m_off[(size_t)l];
        const int64_t K = 27LL * L.ci, kp = u->kp[(size_t)l], kpt = u->kpt[(size_t)l];
        for (int co = 0; co < L.co; ++co)
            for (int64_t k = 0; k < K; ++k) wb[(size_t)(u->w_off[(size_t)l] + co * kp + k)] = (bf16)m[co * K + k];
        if (L.ci == 1) continue;
        // transposed: Wt[ci][tap' * co + c] = W[c][(26 - tap') * ci + ci]
        for (int ci = 0; ci < L.ci; ++ci)
            for (int tp = 0; tp < 27; ++tp)
                for (int c = 0; c < L.co; ++c)
                    wtb[(size_t)(u->wt_off[(size_t)l] + ci * kpt + tp * L.co + c)] =
                        (bf16)m[(int64_t)c * K + (26 - tp) * L.ci + ci];
    }
    std::vector<float> wpj((size_t)u->c0);
    const float* mp = u->host_master.data() + u->m_off[(size_t)(nl - 2)];
    for (size_t q = 0; q < wpj.size(); ++q) wpj[q] = (float)(bf16)mp[q];
    std::vector<float> wo((size_t)27 * u->c0);
    const float* mo = u->host_master.data() + u->m_off[(size_t)(nl - 1)];
    for (size_t q = 0; q < wo.size(); ++q) wo[q] = (float)(bf16)mo[q];
    // composed output stencil: Wc[t1 + t2] += sum_c W_out[t1][c] W0[c][t2]
    // (bf16-rounded factors, FP64 sums, one rounding to FP32)
    std::vector<double> wc(125, 0.0);
    const float* m0 = u->host_master.data() + u->m_off[0];  // W0[c][tap], ci = 1
    for (int t1 = 0; t1 < 27; ++t1)
        for (int t2 = 0; t2 < 27; ++t2) {
            const int dz = t1 / 9 + t2 / 9, dy = (t1 / 3) % 3 + (t2 / 3) % 3, dx = t1 % 3 + t2 % 3;
            double acc = 0.0;
            for (int c = 0; c < u->c0; ++c) acc += (double)wo[(size_t)(t1 * u->c0 + c)] * (double)(float)(bf16)m0[c * 27 + t2];
            wc[(size_t)(25 * dz + 5 * dy + dx)] += acc;
        }
    std::vector<float> wcf(wc.begin(), wc.end());
    // pooled first conv: Wp[c][s] = 1/8 sum_o W0[c][s - o], s = (sz, sy, sx) in
    // 0..3 (k = 16 sz + 4 sy + sx), o in {0, 1}^3; as a BF16 pair hi + lo
    std::vector<bf16> wpl((size_t)2 * 16 * 64);
    for (int ch = 0; ch < 16; ++ch)
        for (int k = 0; k < 64; ++k) {
            const int sz = k / 16, sy = (k / 4) % 4, sx = k % 4;
            double acc = 0.0;
            for (int o = 0; o < 8; ++o) {
                const int tz = sz - (o >> 2), ty = sy - ((o >> 1) & 1), tx = sx - (o & 1);
                if (tz < 0 || tz > 2 || ty < 0 || ty > 2 || tx < 0 || tx > 2) continue;
                acc += (double)(float)(bf16)m0[ch * 27 + 9 * tz + 3 * ty + tx];
            }
            acc *= 0.125;
            const bf16 hi = (bf16)(float)acc;
            wpl[(size_t)ch * 64 + k] = hi;
            wpl[(size_t)16 * 64 + ch * 64 + k] = (bf16)(float)(acc - (double)(float)hi);
        }
    if (hipMemcpy(u->w, wb.data(), sizeof(bf16) * wb.size(), hipMemcpyHostToDevice) != hipSuccess ||
        (u->n_wt > 0 && hipMemcpy(u->wt, wtb.data(), sizeof(bf16) * u->n_wt, hipMemcpyHostToDevice) != hipSuccess) ||
        hipMemcpy(u->w_proj, wpj.data(), sizeof(float) * wpj.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(u->w_out, wo.data(), sizeof(float) * wo.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(u->w_comp, wcf.data(), sizeof(float) * wcf.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(u->w_pool, wpl.data(), sizeof(bf16) * wpl.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(u->master, u->host_master.data(), sizeof(float) * u->n_master, hipMemcpyHostToDevice) != hipSuccess)
        return ufail(u, KVS_EDEVICE, "weight upload failed");
    return KVS_OK;
}

Dims dims_of(int64_t nx, int64_t ny, int64_t nz) { return Dims{(int)nx, (int)ny, (int)nz}; }
}  // namespace

extern "C" {

kvs_status kvs_unet_create(const int32_t* channels, int32_t n_bottleneck, kvs_unet** out) {
    if (!out) return ufail(nullptr, KVS_EINVAL, "out is NULL");
    *out = nullptr;
    const int c0 = channels ? channels[0] : 16, c1 = channels ? channels[1] : 32, c2 = channels ? channels[2] : 64;
    if (c0 != 16 || c1 != 32 || c2 != 64) return ufail(nullptr, KVS_EINVAL, "supported channel counts: 16, 32, 64");
    if (n_bottleneck < 2 || n_bottleneck > 8) return ufail(nullptr, KVS_EINVAL, "n_bottleneck must be 2..8");
    kvs_unet* u = new (std::nothrow) kvs_unet();
    if (!u) return ufail(nullptr, KVS_ENOMEM, "host allocation failed");
    u->c0 = c0;
    u->c1 = c1;
    u->c2 = c2;
    u->nbott = n_bottleneck;
    build_layers(u);
    u->host_master.assign((size_t)u->n_master, 0.f);
    bool ok = hipMalloc(&u->w, sizeof(bf16) * u->n_w) == hipSuccess;
    ok = ok && hipMalloc(&u->wt, sizeof(bf16) * std::max<int64_t>(u->n_wt, 1)) == hipSuccess;
    ok = ok && hipMalloc(&u->w_proj, sizeof(float) * c0) == hipSuccess;
    ok = ok && hipMalloc(&u->w_out, sizeof(float) * 27 * c0) == hipSuccess;
    ok = ok && hipMalloc(&u->w_comp, sizeof(float) * 125) == hipSuccess;
    ok = ok && hipMalloc(&u->w_pool, sizeof(bf16) * 2 * 16 * 64) == hipSuccess;
    for (float** p : {&u->master, &u->grad, &u->adam_m, &u->adam_v})
        ok = ok && hipMalloc(p, sizeof(float) * u->n_master) == hipSuccess;
    ok = ok && hipMemset(u->grad, 0, sizeof(float) * u->n_master) == hipSuccess;
    ok = ok && hipMemset(u->adam_m, 0, sizeof(float) * u->n_master) == hipSuccess;
    ok = ok && hipMemset(u->adam_v, 0, sizeof(float) * u->n_master) == hipSuccess;
    if (!ok) {
        kvs_unet_destroy(u);
        return ufail(nullptr, KVS_ENOMEM, "device allocation failed");
    }
    kvs_status s = upload_weights(u);
    if (s != KVS_OK) {
        kvs_unet_destroy(u);
        return s;
    }
    *out = u;
    return KVS_OK;
}

void kvs_unet_destroy(kvs_unet* u) {
    if (!u) return;
    (void)hipDeviceSynchronize();
    unet_free_acts(u);
    unet_free_train(u);
    ufree(u->w);
    ufree(u->wt);
    ufree(u->w_proj);
    ufree(u->w_out);
    ufree(u->w_comp);
    ufree(u->w_pool);
    ufree(u->master);
    ufree(u->grad);
    ufree(u->adam_m);
    ufree(u->adam_v);
    delete u;
}

const char* kvs_unet_last_error(const kvs_unet* u) { return u ? u->err.c_str() : g_unet_err.c_str(); }

int64_t kvs_unet_num_weights(const kvs_unet* u) { return u ? u->n_master : 0; }

int32_t kvs_unet_num_layers(const kvs_unet* u) { return u ? (int32_t)u->layers.size() : 0; }

kvs_status kvs_unet_layer(const kvs_unet* u, int32_t l, int32_t* ci, int32_t* co, int32_t* dil, int32_t* taps) {
    if (!u || l < 0 || l >= (int32_t)u->layers.size()) return KVS_EINVAL;
    const UnetLayerDesc& L = u->layers[(size_t)l];
    if (ci) *ci = L.ci;
    if (co) *co = L.co;
    if (dil) *dil = L.dil;
    if (taps) *taps = L.taps();
    return KVS_OK;
}

kvs_status kvs_unet_set_weights(kvs_unet* u, const float* w, int64_t n) {
    if (!u || !w) return KVS_EINVAL;
    if (n != u->n_master) return ufail(u, KVS_EINVAL, "wrong weight count");
    std::memcpy(u->host_master.data(), w, sizeof(float) * n);
    u->adam_t = 0;
    if (hipMemset(u->adam_m, 0, sizeof(float) * n) != hipSuccess || hipMemset(u->adam_v, 0, sizeof(float) * n) != hipSuccess)
        return ufail(u, KVS_EDEVICE, "reset of the optimiser state failed");
    return upload_weights(u);
}

kvs_status kvs_unet_get_weights(const kvs_unet* u, float* w, int64_t n) {
    if (!u || !w) return KVS_EINVAL;
    if (n != u->n_master) return KVS_EINVAL;
    std::memcpy(w, u->host_master.data(), sizeof(float) * n);
    return KVS_OK;
}

kvs_status kvs_unet_forward(kvs_unet* u, const double* r, double in_scale, double out_scale, double* z, int64_t nx,
                            int64_t ny, int64_t nz, void* stream) {
    if (!u || !r || !z) return KVS_EINVAL;
    if (nx < 3 || ny < 3 || nz < 3) return ufail(u, KVS_EINVAL, "grid needs >= 3 nodes per axis");
    NetCtl ctl{nullptr, nullptr, nullptr, in_scale, out_scale};
    hipError_t e = kvs_unet_apply(u, r, ctl, z, dims_of(nx, ny, nz), (hipStream_t)stream, true);
    if (e != hipSuccess) return ufail(u, KVS_EDEVICE, std::string("unet forward: ") + hipGetErrorString(e));
    return KVS_OK;
}

kvs_status kvs_unet_backward(kvs_unet* u, const double* r, double in_scale, const double* dz, double dz_scale,
                             int64_t nx, int64_t ny, int64_t nz, int32_t accumulate, void* stream) {
    if (!u || !r || !dz) return KVS_EINVAL;
    const Dims d = dims_of(nx, ny, nz);
    if (!u->kept || u->dims.nx != d.nx || u->dims.ny != d.ny || u->dims.nz != d.nz)
        return ufail(u, KVS_ESTATE, "backward needs a forward pass on the same grid first");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = unet_ensure_train(u, d);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(scale_to_f32, dim3(nblocks256(d.n())), dim3(256), 0, s, dz, dz_scale, u->dzf, d.n());
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = unet_backward(u, r, in_scale, d, accumulate, s);
    if (e != hipSuccess) return ufail(u, KVS_EDEVICE, std::string("unet backward: ") + hipGetErrorString(e));
    return KVS_OK;
}

kvs_status kvs_unet_get_grad(const kvs_unet* u, float* g, int64_t n) {
    if (!u || !g || n != u->n_master) return KVS_EINVAL;
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(g, u->grad, sizeof(float) * n, hipMemcpyDeviceToHost) != hipSuccess)
        return KVS_EDEVICE;
    return KVS_OK;
}

kvs_status kvs_unet_train_sample(kvs_unet* u, const double* b, const double* xs, int64_t nx, int64_t ny, int64_t nz,
                                 int32_t accumulate, double* loss, void* stream) {
    if (!u || !b || !xs) return KVS_EINVAL;
    const Dims d = dims_of(nx, ny, nz);
    hipStream_t s = (hipStream_t)stream;
    NetCtl ctl{nullptr, nullptr, nullptr, 1.0, 1.0};
    hipError_t e = unet_ensure_train(u, d);
    double* z = nullptr;
    if (e == hipSuccess) e = hipMalloc(&z, sizeof(double) * d.n());
    if (e == hipSuccess) e = kvs_unet_apply(u, b, ctl, z, d, s, true);
    const int nb = nblocks256(d.n());
    std::vector<double> part((size_t)2 * nb);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(anorm_loss, dim3(nb), dim3(256), 0, s, z, xs, d, u->dz_raw, u->part);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(part.data(), u->part, sizeof(double) * part.size(), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    double eAe = 0.0, xAx = 0.0;
    for (int q = 0; q < nb; ++q) {
        eAe += part[(size_t)2 * q];
        xAx += part[(size_t)2 * q + 1];
    }
    if (e == hipSuccess && !(xAx > 0.0)) {
        (void)hipFree(z);
        return ufail(u, KVS_EINVAL, "training target has zero A-norm");
    }
    // L = e.Ae / xAx, dL/dz = 2 A e / xAx
    if (e == hipSuccess) {
        hipLaunchKernelGGL(scale_to_f32, dim3(nb), dim3(256), 0, s, u->dz_raw, 2.0 / xAx, u->dzf, d.n());
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = unet_backward(u, b, 1.0, d, accumulate, s);
    if (z) (void)hipFree(z);
    if (e != hipSuccess) return ufail(u, KVS_EDEVICE, std::string("unet train: ") + hipGetErrorString(e));
    if (loss) *loss = eAe / xAx;
    return KVS_OK;
}

kvs_status kvs_unet_adam_step(kvs_unet* u, double lr, int32_t n_samples, void* stream) {
    if (!u || n_samples < 1 || !(lr > 0.0)) return KVS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    u->adam_t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)u->adam_t), c2 = 1.f - std::pow(b2, (float)u->adam_t);
    hipLaunchKernelGGL(adam_kernel, dim3(nblocks256(u->n_master)), dim3(256), 0, s, u->master, u->grad, u->adam_m,
                       u->adam_v, (long long)u->n_master, (float)lr, b1, b2, 1e-8f, c1, c2, 1.f / (float)n_samples);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(u->host_master.data(), u->master, sizeof(float) * u->n_master, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return ufail(u, KVS_EDEVICE, std::string("adam: ") + hipGetErrorString(e));
    return upload_weights(u);
}

kvs_status kvs_unet_sample_from_x(double* x, double* b, int64_t nx, int64_t ny, int64_t nz, double* b_rms,
                                  void* stream) {
    if (!x || !b || nx < 3 || ny < 3 || nz < 3) return ufail(nullptr, KVS_EINVAL, "bad arguments");
    const Dims d = dims_of(nx, ny, nz);
    if (d.n() >= (1LL << 31)) return ufail(nullptr, KVS_EINVAL, "grid too large");
    hipStream_t s = (hipStream_t)stream;
    const int nb = nblocks256(d.n());
    double* part = nullptr;
    hipError_t e = hipMalloc(&part, sizeof(double) * nb);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(apply_A_kernel, dim3(nb), dim3(256), 0, s, x, d, 1.0, 1.0, 1.0, b, part);
        e = hipGetLastError();
    }
    std::vector<double> hp((size_t)nb);
    if (e == hipSuccess) e = hipMemcpyAsync(hp.data(), part, sizeof(double) * nb, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (part) (void)hipFree(part);
    if (e != hipSuccess) return ufail(nullptr, KVS_EDEVICE, std::string("sample: ") + hipGetErrorString(e));
    double bb = 0.0;
    for (double v : hp) bb += v;
    const double rms = std::sqrt(bb / ((double)(nx - 2) * (double)(ny - 2) * (double)(nz - 2)));
    if (!(rms > 0.0)) return ufail(nullptr, KVS_EINVAL, "A x vanishes on the interior");
    hipLaunchKernelGGL(scale_kernel, dim3(nb), dim3(256), 0, s, b, 1.0 / rms, d.n());
    hipLaunchKernelGGL(scale_kernel, dim3(nb), dim3(256), 0, s, x, 1.0 / rms, d.n());
    if (hipStreamSynchronize(s) != hipSuccess) return ufail(nullptr, KVS_EDEVICE, "sample: scaling failed");
    if (b_rms) *b_rms = rms;
    return KVS_OK;
}

int64_t kvs_unet_conv_kpad(int32_t ci) { return ci == 1 ? 32 : (27 * (int64_t)ci + 31) / 32 * 32; }

kvs_status kvs_unet_conv_check(int32_t ci, int32_t co, int32_t dil, const uint16_t* A, const uint16_t* B, int64_t nx,
                               int64_t ny, int64_t nz, const uint16_t* W, uint16_t* out) {
    if (!A || !W || !out || nx < 1 || ny < 1 || nz < 1 || dil < 1) return ufail(nullptr, KVS_EINVAL, "bad arguments");
    const Dims d{(int)nx, (int)ny, (int)nz};
    const Dims c = coarse(d);
    const size_t na = (size_t)d.n() * ci, nbb = B ? (size_t)c.n() * ci : 0, nw = (size_t)co * kvs_unet_conv_kpad(ci),
                 no = (size_t)d.n() * co;
    bf16 *dA = nullptr, *dB = nullptr, *dI = nullptr, *dW = nullptr, *dO = nullptr;
    hipError_t e = hipMalloc(&dA, 2 * na);
    if (e == hipSuccess && B) e = hipMalloc(&dB, 2 * nbb);
    if (e == hipSuccess && B) e = hipMalloc(&dI, 2 * na);
    if (e == hipSuccess) e = hipMalloc(&dW, 2 * nw);
    if (e == hipSuccess) e = hipMalloc(&dO, 2 * no);
    if (e == hipSuccess) e = hipMemcpy(dA, A, 2 * na, hipMemcpyHostToDevice);
    if (e == hipSuccess && B) e = hipMemcpy(dB, B, 2 * nbb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dW, W, 2 * nw, hipMemcpyHostToDevice);
    // with a skip input: in = bf16(A + up(B)) first, then the convolution
    if (e == hipSuccess && B) e = launch_skip_up(ci, dA, dB, d, dI, nullptr, nullptr);
    if (e == hipSuccess) e = launch_conv(ci, co, B ? dI : dA, d, dil, dW, dO, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(out, dO, 2 * no, hipMemcpyDeviceToHost);
    for (bf16* p : {dA, dB, dI, dW, dO})
        if (p) (void)hipFree(p);
    if (e != hipSuccess) return ufail(nullptr, KVS_EDEVICE, std::string("conv check: ") + hipGetErrorString(e));
    return KVS_OK;
}

// Training pair from the solver's own projection on ctx (FP64 context):
// phi* = converged solution of the current force (Jacobi-PCG to 1e-11); with
// k_snapshot > 0 the pair is the CG error after k iterations,
// x = phi* - phi_k, else x = phi*; b = A x with the context's spacing; both
// scaled so that b has unit RMS.  b, x: device fields of N doubles.
kvs_status kvs_unet_make_sample(kvs_ctx* c, int64_t k_snapshot, int32_t precond, double* b, double* x,
                                double* b_rms) {
    if (!c || !b || !x || k_snapshot < 0 || (precond != KVS_PC_JACOBI && precond != KVS_PC_UNET)) return KVS_EINVAL;
    const Dims d{(int)c->grid.nx, (int)c->grid.ny, (int)c->grid.nz};
    kvs_solve_opts o{};
    o.tol = 1e-11;
    o.max_iter = 100000;
    o.precond = KVS_PC_JACOBI;
    kvs_status st = kvs_project(c, &o, nullptr);
    if (st != KVS_OK) return st;
    hipStream_t s = c->stream;
    const int nb = nblocks256(d.n());
    hipError_t e = hipMemcpyAsync(x, c->phi, sizeof(double) * d.n(), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && k_snapshot > 0) {
        o.fixed_iters = k_snapshot;
        o.precond = (kvs_precond)precond;
        if (hipStreamSynchronize(s) != hipSuccess) return KVS_EDEVICE;
        st = kvs_project(c, &o, nullptr);
        if (st != KVS_OK) return st;
        hipLaunchKernelGGL(sub_kernel, dim3(nb), dim3(256), 0, s, x, c->phi, x, d.n());
        e = hipGetLastError();
    }
    double* part = nullptr;
    if (e == hipSuccess) e = hipMalloc(&part, sizeof(double) * nb);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(apply_A_kernel, dim3(nb), dim3(256), 0, s, x, d, 1.0 / (c->grid.hx * c->grid.hx),
                           1.0 / (c->grid.hy * c->grid.hy), 1.0 / (c->grid.hz * c->grid.hz), b, part);
        e = hipGetLastError();
    }
    std::vector<double> hp((size_t)nb);
    if (e == hipSuccess) e = hipMemcpyAsync(hp.data(), part, sizeof(double) * nb, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (part) (void)hipFree(part);
    if (e != hipSuccess) return KVS_EDEVICE;
    double bb = 0.0;
    for (double v : hp) bb += v;
    const long long nint = (long long)(d.nx - 2) * (d.ny - 2) * (d.nz - 2);
    const double rms = std::sqrt(bb / (double)nint);
    if (!(rms > 0.0)) return KVS_EINVAL;
    hipLaunchKernelGGL(scale_kernel, dim3(nb), dim3(256), 0, s, b, 1.0 / rms, d.n());
    hipLaunchKernelGGL(scale_kernel, dim3(nb), dim3(256), 0, s, x, 1.0 / rms, d.n());
    if (hipStreamSynchronize(s) != hipSuccess) return KVS_EDEVICE;
    if (b_rms) *b_rms = rms;
    return KVS_OK;
}

}  // extern "C"
