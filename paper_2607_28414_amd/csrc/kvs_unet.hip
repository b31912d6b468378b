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
#include <vector>

#include "kvs_internal.hpp"

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

struct Dims {
    int nx, ny, nz;
    __host__ __device__ long long n() const { return (long long)nx * ny * nz; }
};

__host__ __device__ inline Dims coarse(Dims d) { return Dims{(d.nx + 1) / 2, (d.ny + 1) / 2, (d.nz + 1) / 2}; }

__device__ __forceinline__ int tap_dx(int tap) { return tap % 3 - 1; }
__device__ __forceinline__ int tap_dy(int tap) { return (tap / 3) % 3 - 1; }
__device__ __forceinline__ int tap_dz(int tap) { return tap / 9 - 1; }

// ---- forward conv (MFMA) -----------------------------------------------------
// out[v][co] = sum_{tap, ci} W[co][tap * CI + ci] * in(v + dil * tap)[ci],
// in(p) = A[p][ci] + (B ? B[p / 2][ci] : 0), zero outside the grid.
// out may be BF16 (store) — every output is rounded once, to nearest even.
template <int CI, int CO>
__global__ __launch_bounds__(256) void conv3_mfma(const bf16* __restrict__ A, const bf16* __restrict__ B, Dims d,
                                                  int dil, const bf16* __restrict__ W, bf16* __restrict__ out) {
    static_assert(CI % 8 == 0 && CO % 16 == 0, "channel counts");
    constexpr int K = 27 * CI;
    constexpr int KP = (K + 31) / 32 * 32;
    constexpr int MT = CO / 16;
    const int lane = threadIdx.x & 63;
    const long long wave = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int vl = lane & 15, kg = lane >> 4;
    const long long N = d.n();
    const long long v = wave * 16 + vl;
    const bool valid = v < N;
    const long long vc = valid ? v : 0;
    const int x = (int)(vc % d.nx), y = (int)((vc / d.nx) % d.ny), z = (int)(vc / ((long long)d.nx * d.ny));
    const Dims dB = coarse(d);
    f32x4 acc[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) acc[m] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < KP / 32; ++kc) {
        const int k0 = kc * 32 + 8 * kg;
        const int tap = k0 / CI, ci0 = k0 % CI;
        bf16x8 xb;
        float xf[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (tap < 27 && valid) {
            const int px = x + dil * tap_dx(tap), py = y + dil * tap_dy(tap), pz = z + dil * tap_dz(tap);
            if (px >= 0 && px < d.nx && py >= 0 && py < d.ny && pz >= 0 && pz < d.nz) {
                const long long p = px + (long long)d.nx * (py + (long long)d.ny * pz);
                const bf16x8 a8 = *reinterpret_cast<const bf16x8*>(A + p * CI + ci0);
#pragma unroll
                for (int j = 0; j < 8; ++j) xf[j] = (float)a8[j];
                if (B) {
                    const long long q = (px >> 1) + (long long)dB.nx * ((py >> 1) + (long long)dB.ny * (pz >> 1));
                    const bf16x8 b8 = *reinterpret_cast<const bf16x8*>(B + q * CI + ci0);
#pragma unroll
                    for (int j = 0; j < 8; ++j) xf[j] += (float)b8[j];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) xb[j] = (bf16)xf[j];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const bf16x8 w8 = *reinterpret_cast<const bf16x8*>(W + (long long)(16 * m + vl) * KP + k0);
            acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w8, xb, acc[m], 0, 0, 0);
        }
    }
    if (!valid) return;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        bf16x4 o;
#pragma unroll
        for (int i = 0; i < 4; ++i) o[i] = (bf16)acc[m][i];
        *reinterpret_cast<bf16x4*>(out + v * CO + 16 * m + 4 * kg) = o;
    }
}

// first layer: one input channel read from an FP64 field, scaled
template <int CO>
__global__ __launch_bounds__(256) void conv3_first(const double* __restrict__ r, double in_scale, Dims d,
                                                   const bf16* __restrict__ W, bf16* __restrict__ out) {
    constexpr int MT = CO / 16;
    const int lane = threadIdx.x & 63;
    const long long wave = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int vl = lane & 15, kg = lane >> 4;
    const long long N = d.n();
    const long long v = wave * 16 + vl;
    const bool valid = v < N;
    const long long vc = valid ? v : 0;
    const int x = (int)(vc % d.nx), y = (int)((vc / d.nx) % d.ny), z = (int)(vc / ((long long)d.nx * d.ny));
    bf16x8 xb;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int tap = 8 * kg + j;
        float val = 0.f;
        if (tap < 27 && valid) {
            const int px = x + tap_dx(tap), py = y + tap_dy(tap), pz = z + tap_dz(tap);
            if (px >= 0 && px < d.nx && py >= 0 && py < d.ny && pz >= 0 && pz < d.nz)
                val = (float)(in_scale * r[px + (long long)d.nx * (py + (long long)d.ny * pz)]);
        }
        xb[j] = (bf16)val;
    }
    f32x4 acc[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        const bf16x8 w8 = *reinterpret_cast<const bf16x8*>(W + (16 * m + vl) * 32 + 8 * kg);
        acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w8, xb, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
    }
    if (!valid) return;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        bf16x4 o;
#pragma unroll
        for (int i = 0; i < 4; ++i) o[i] = (bf16)acc[m][i];
        *reinterpret_cast<bf16x4*>(out + v * CO + 16 * m + 4 * kg) = o;
    }
}

// output layer: one channel, FP64 result scaled, 0 outside the interior
template <int CI>
__global__ __launch_bounds__(256) void conv3_out(const bf16* __restrict__ g, Dims d, const float* __restrict__ W,
                                                 double out_scale, double* __restrict__ z) {
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= d.n()) return;
    const int x = (int)(v % d.nx), y = (int)((v / d.nx) % d.ny), zz = (int)(v / ((long long)d.nx * d.ny));
    if (x < 1 || x > d.nx - 2 || y < 1 || y > d.ny - 2 || zz < 1 || zz > d.nz - 2) {
        z[v] = 0.0;
        return;
    }
    float acc = 0.f;
    for (int tap = 0; tap < 27; ++tap) {
        const long long p = (x + tap_dx(tap)) + (long long)d.nx * ((y + tap_dy(tap)) + (long long)d.ny * (zz + tap_dz(tap)));
#pragma unroll
        for (int c8 = 0; c8 < CI; c8 += 8) {
            const bf16x8 a8 = *reinterpret_cast<const bf16x8*>(g + p * CI + c8);
#pragma unroll
            for (int j = 0; j < 8; ++j) acc += W[tap * CI + c8 + j] * (float)a8[j];
        }
    }
    z[v] = out_scale * (double)acc;
}

// mean of the children of coarse voxel V (8 channels per thread)
template <int C>
__global__ void pool2(const bf16* __restrict__ fine, Dims d, bf16* __restrict__ out) {
    const Dims c = coarse(d);
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long V = t / (C / 8);
    const int c8 = (int)(t % (C / 8)) * 8;
    if (V >= c.n()) return;
    const int X = (int)(V % c.nx), Y = (int)((V / c.nx) % c.ny), Z = (int)(V / ((long long)c.nx * c.ny));
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int cnt = 0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const int x = 2 * X + dx, y = 2 * Y + dy, z = 2 * Z + dz;
                if (x >= d.nx || y >= d.ny || z >= d.nz) continue;
                const bf16x8 a8 = *reinterpret_cast<const bf16x8*>(fine + (x + (long long)d.nx * (y + (long long)d.ny * z)) * C + c8);
#pragma unroll
                for (int j = 0; j < 8; ++j) s[j] += (float)a8[j];
                ++cnt;
            }
    bf16x8 o;
#pragma unroll
    for (int j = 0; j < 8; ++j) o[j] = (bf16)(s[j] / (float)cnt);
    *reinterpret_cast<bf16x8*>(out + V * C + c8) = o;
}

int blocks_for_waves(long long voxels) { return (int)((voxels + 63) / 64); }

}  // namespace

// ---- network object ------------------------------------------------------------

struct UnetLayerDesc {
    int ci, co, dil, level;  // level of the output
    bool skip_in;            // input = skip tensor + up(previous)
};

struct kvs_unet {
    int c0 = 16, c1 = 32, c2 = 64, nbott = 4;
    std::vector<UnetLayerDesc> layers;  // 0 first, 1 enc1, 2.. bottleneck, dec1, dec0, out
    std::vector<int64_t> w_off;         // offset of each layer's bf16 weights (elements)
    std::vector<int64_t> kp;            // padded K per layer
    int64_t n_w = 0;                    // total bf16 weight elements
    bf16* w = nullptr;                  // device bf16 weights (inference layout)
    float* w_out = nullptr;             // device fp32 weights of the output layer [27][C0]
    std::vector<float> host_master;     // fp32 master weights, layer by layer, [co][27*ci] (out: [27][c0])
    // activation buffers for the last grid
    Dims dims{0, 0, 0};
    bf16 *e0 = nullptr, *p0 = nullptr, *e1 = nullptr, *p1 = nullptr, *ba = nullptr, *bb = nullptr, *g1 = nullptr,
         *g0 = nullptr;
    std::string err;
};

namespace {

void unet_free_acts(kvs_unet* u) {
    for (bf16** p : {&u->e0, &u->p0, &u->e1, &u->p1, &u->ba, &u->bb, &u->g1, &u->g0}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
}

hipError_t unet_ensure_acts(kvs_unet* u, Dims d) {
    if (u->e0 && u->dims.nx == d.nx && u->dims.ny == d.ny && u->dims.nz == d.nz) return hipSuccess;
    unet_free_acts(u);
    const Dims d1 = coarse(d), d2 = coarse(d1);
    const long long n0 = d.n(), n1 = d1.n(), n2 = d2.n();
    hipError_t e = hipMalloc(&u->e0, sizeof(bf16) * n0 * u->c0);
    if (e == hipSuccess) e = hipMalloc(&u->g0, sizeof(bf16) * n0 * u->c0);
    if (e == hipSuccess) e = hipMalloc(&u->p0, sizeof(bf16) * n1 * u->c0);
    if (e == hipSuccess) e = hipMalloc(&u->e1, sizeof(bf16) * n1 * u->c1);
    if (e == hipSuccess) e = hipMalloc(&u->g1, sizeof(bf16) * n1 * u->c0);
    if (e == hipSuccess) e = hipMalloc(&u->p1, sizeof(bf16) * n2 * u->c1);
    if (e == hipSuccess) e = hipMalloc(&u->ba, sizeof(bf16) * n2 * u->c2);
    if (e == hipSuccess) e = hipMalloc(&u->bb, sizeof(bf16) * n2 * u->c2);
    if (e != hipSuccess) {
        unet_free_acts(u);
        return e;
    }
    u->dims = d;
    return hipSuccess;
}

// dispatch of the MFMA conv over the channel pairs this network uses
hipError_t launch_conv(int ci, int co, const bf16* A, const bf16* B, Dims d, int dil, const bf16* W, bf16* out,
                       hipStream_t s) {
    const int nb = blocks_for_waves(d.n());
#define KVS_CONV_CASE(CI_, CO_)                                                                          \
    if (ci == CI_ && co == CO_) {                                                                        \
        hipLaunchKernelGGL((conv3_mfma<CI_, CO_>), dim3(nb), dim3(256), 0, s, A, B, d, dil, W, out);    \
        return hipGetLastError();                                                                        \
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

hipError_t launch_pool(int c, const bf16* fine, Dims d, bf16* out, hipStream_t s) {
    const long long threads = coarse(d).n() * (c / 8);
    const int nb = (int)((threads + 255) / 256);
    switch (c) {
        case 8: hipLaunchKernelGGL(pool2<8>, dim3(nb), dim3(256), 0, s, fine, d, out); break;
        case 16: hipLaunchKernelGGL(pool2<16>, dim3(nb), dim3(256), 0, s, fine, d, out); break;
        case 32: hipLaunchKernelGGL(pool2<32>, dim3(nb), dim3(256), 0, s, fine, d, out); break;
        case 64: hipLaunchKernelGGL(pool2<64>, dim3(nb), dim3(256), 0, s, fine, d, out); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

void build_layers(kvs_unet* u) {
    u->layers.clear();
    u->layers.push_back({1, u->c0, 1, 0, false});      // e0
    u->layers.push_back({u->c0, u->c1, 1, 1, false});  // e1 = conv(pool e0)
    u->layers.push_back({u->c1, u->c2, 1, 2, false});  // bottleneck in
    int dil = 2;
    for (int q = 0; q < u->nbott - 2; ++q, dil *= 2) u->layers.push_back({u->c2, u->c2, dil, 2, false});
    u->layers.push_back({u->c2, u->c1, 1, 2, false});  // bottleneck out
    u->layers.push_back({u->c1, u->c0, 1, 1, true});   // g1 = conv(e1 + up b)
    u->layers.push_back({u->c0, u->c0, 1, 0, true});   // g0 = conv(e0 + up g1)
    u->layers.push_back({u->c0, 1, 1, 0, false});      // z
    u->w_off.clear();
    u->kp.clear();
    int64_t off = 0;
    for (size_t l = 0; l + 1 < u->layers.size(); ++l) {
        const UnetLayerDesc& L = u->layers[l];
        const int64_t kp = L.ci == 1 ? 32 : (27 * L.ci + 31) / 32 * 32;
        u->w_off.push_back(off);
        u->kp.push_back(kp);
        off += kp * L.co;
    }
    u->n_w = off;
}

}  // namespace

hipError_t kvs_unet_apply(kvs_unet* u, const double* r, double in_scale, double out_scale, double* z, Dims d,
                          hipStream_t s);

hipError_t kvs_unet_apply(kvs_unet* u, const double* r, double in_scale, double out_scale, double* z, Dims d,
                          hipStream_t s) {
    hipError_t e = unet_ensure_acts(u, d);
    if (e != hipSuccess) return e;
    const Dims d1 = coarse(d), d2 = coarse(d1);
    const std::vector<UnetLayerDesc>& L = u->layers;
    const int nl = (int)L.size();
    // e0
    {
        const int nb = blocks_for_waves(d.n());
        const bf16* W = u->w + u->w_off[0];
        hipLaunchKernelGGL(conv3_first<16>, dim3(nb), dim3(256), 0, s, r, in_scale, d, W, u->e0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = launch_pool(u->c0, u->e0, d, u->p0, s)) != hipSuccess) return e;
    if ((e = launch_conv(u->c0, u->c1, u->p0, nullptr, d1, 1, u->w + u->w_off[1], u->e1, s)) != hipSuccess) return e;
    if ((e = launch_pool(u->c1, u->e1, d1, u->p1, s)) != hipSuccess) return e;
    // bottleneck: layers 2 .. nl-4
    const bf16* in = u->p1;
    bf16* outb = u->ba;
    for (int l = 2; l <= nl - 4; ++l) {
        if ((e = launch_conv(L[l].ci, L[l].co, in, nullptr, d2, L[l].dil, u->w + u->w_off[l], outb, s)) != hipSuccess)
            return e;
        in = outb;
        outb = outb == u->ba ? u->bb : u->ba;
    }
    const int ld1 = nl - 3, ld0 = nl - 2, lo = nl - 1;
    if ((e = launch_conv(u->c1, u->c0, u->e1, in, d1, 1, u->w + u->w_off[ld1], u->g1, s)) != hipSuccess) return e;
    if ((e = launch_conv(u->c0, u->c0, u->e0, u->g1, d, 1, u->w + u->w_off[ld0], u->g0, s)) != hipSuccess) return e;
    (void)lo;
    {
        const int nb = (int)((d.n() + 255) / 256);
        hipLaunchKernelGGL(conv3_out<16>, dim3(nb), dim3(256), 0, s, u->g0, d, u->w_out, out_scale, z);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

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

// fp32 master -> device bf16 (inference layout) and fp32 output weights
kvs_status upload_weights(kvs_unet* u) {
    std::vector<bf16> wb((size_t)u->n_w, (bf16)0.f);
    size_t m = 0;
    const int nl = (int)u->layers.size();
    for (int l = 0; l < nl - 1; ++l) {
        const UnetLayerDesc& L = u->layers[(size_t)l];
        const int64_t K = 27 * L.ci, kp = u->kp[(size_t)l];
        for (int co = 0; co < L.co; ++co)
            for (int64_t k = 0; k < K; ++k) wb[(size_t)(u->w_off[(size_t)l] + co * kp + k)] = (bf16)u->host_master[m++];
    }
    std::vector<float> wo((size_t)27 * u->c0);
    for (size_t q = 0; q < wo.size(); ++q) wo[q] = (float)(bf16)u->host_master[m++];
    if (hipMemcpy(u->w, wb.data(), sizeof(bf16) * wb.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(u->w_out, wo.data(), sizeof(float) * wo.size(), hipMemcpyHostToDevice) != hipSuccess)
        return ufail(u, KVS_EDEVICE, "weight upload failed");
    return KVS_OK;
}

int64_t master_count(const kvs_unet* u) {
    int64_t n = 0;
    for (const UnetLayerDesc& L : u->layers) n += (int64_t)27 * L.ci * L.co;
    return n;
}
}  // namespace

extern "C" {

kvs_status kvs_unet_create(const int32_t* channels, int32_t n_bottleneck, kvs_unet** out) {
    if (!out) return ufail(nullptr, KVS_EINVAL, "out is NULL");
    *out = nullptr;
    const int c0 = channels ? channels[0] : 16, c1 = channels ? channels[1] : 32, c2 = channels ? channels[2] : 64;
    if (c0 != 16 || c1 != 32 || c2 != 64)
        return ufail(nullptr, KVS_EINVAL, "supported channel counts: 16, 32, 64");
    if (n_bottleneck < 2 || n_bottleneck > 8) return ufail(nullptr, KVS_EINVAL, "n_bottleneck must be 2..8");
    kvs_unet* u = new (std::nothrow) kvs_unet();
    if (!u) return ufail(nullptr, KVS_ENOMEM, "host allocation failed");
    u->c0 = c0;
    u->c1 = c1;
    u->c2 = c2;
    u->nbott = n_bottleneck;
    build_layers(u);
    u->host_master.assign((size_t)master_count(u), 0.f);
    if (hipMalloc(&u->w, sizeof(bf16) * u->n_w) != hipSuccess ||
        hipMalloc(&u->w_out, sizeof(float) * 27 * c0) != hipSuccess) {
        if (u->w) (void)hipFree(u->w);
        delete u;
        return ufail(nullptr, KVS_ENOMEM, "device allocation failed");
    }
    kvs_status s = upload_weights(u);
    if (s != KVS_OK) return s;
    *out = u;
    return KVS_OK;
}

void kvs_unet_destroy(kvs_unet* u) {
    if (!u) return;
    unet_free_acts(u);
    if (u->w) (void)hipFree(u->w);
    if (u->w_out) (void)hipFree(u->w_out);
    delete u;
}

const char* kvs_unet_last_error(const kvs_unet* u) { return u ? u->err.c_str() : g_unet_err.c_str(); }

int64_t kvs_unet_num_weights(const kvs_unet* u) { return u ? (int64_t)u->host_master.size() : 0; }

kvs_status kvs_unet_set_weights(kvs_unet* u, const float* w, int64_t n) {
    if (!u || !w) return KVS_EINVAL;
    if (n != (int64_t)u->host_master.size()) return ufail(u, KVS_EINVAL, "wrong weight count");
    std::memcpy(u->host_master.data(), w, sizeof(float) * n);
    return upload_weights(u);
}

kvs_status kvs_unet_get_weights(const kvs_unet* u, float* w, int64_t n) {
    if (!u || !w) return KVS_EINVAL;
    if (n != (int64_t)u->host_master.size()) return KVS_EINVAL;
    std::memcpy(w, u->host_master.data(), sizeof(float) * n);
    return KVS_OK;
}

kvs_status kvs_unet_forward(kvs_unet* u, const double* r, double in_scale, double out_scale, double* z, int64_t nx,
                            int64_t ny, int64_t nz, void* stream) {
    if (!u || !r || !z) return KVS_EINVAL;
    if (nx < 3 || ny < 3 || nz < 3) return ufail(u, KVS_EINVAL, "grid needs >= 3 nodes per axis");
    const Dims d{(int)nx, (int)ny, (int)nz};
    hipError_t e = kvs_unet_apply(u, r, in_scale, out_scale, z, d, (hipStream_t)stream);
    if (e != hipSuccess) return ufail(u, KVS_EDEVICE, std::string("unet forward: ") + hipGetErrorString(e));
    return KVS_OK;
}

// One MFMA conv on host buffers (BF16 bit patterns), for verification:
// out[v][co] = sum W[co][tap*ci + c] * (A[p][c] + B[p/2][c]), W padded to
// kvs_unet_conv_kpad(ci) columns.
int64_t kvs_unet_conv_kpad(int32_t ci) { return ci == 1 ? 32 : (27 * (int64_t)ci + 31) / 32 * 32; }

kvs_status kvs_unet_conv_check(int32_t ci, int32_t co, int32_t dil, const uint16_t* A, const uint16_t* B, int64_t nx,
                               int64_t ny, int64_t nz, const uint16_t* W, uint16_t* out) {
    if (!A || !W || !out || nx < 1 || ny < 1 || nz < 1 || dil < 1) return ufail(nullptr, KVS_EINVAL, "bad arguments");
    const Dims d{(int)nx, (int)ny, (int)nz};
    const Dims c = coarse(d);
    const size_t na = (size_t)d.n() * ci, nbb = B ? (size_t)c.n() * ci : 0, nw = (size_t)co * kvs_unet_conv_kpad(ci),
                 no = (size_t)d.n() * co;
    bf16 *dA = nullptr, *dB = nullptr, *dW = nullptr, *dO = nullptr;
    hipError_t e = hipMalloc(&dA, 2 * na);
    if (e == hipSuccess && B) e = hipMalloc(&dB, 2 * nbb);
    if (e == hipSuccess) e = hipMalloc(&dW, 2 * nw);
    if (e == hipSuccess) e = hipMalloc(&dO, 2 * no);
    if (e == hipSuccess) e = hipMemcpy(dA, A, 2 * na, hipMemcpyHostToDevice);
    if (e == hipSuccess && B) e = hipMemcpy(dB, B, 2 * nbb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dW, W, 2 * nw, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_conv(ci, co, dA, dB, d, dil, dW, dO, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(out, dO, 2 * no, hipMemcpyDeviceToHost);
    for (bf16* p : {dA, dB, dW, dO})
        if (p) (void)hipFree(p);
    if (e != hipSuccess) return ufail(nullptr, KVS_EDEVICE, std::string("conv check: ") + hipGetErrorString(e));
    return KVS_OK;
}

}  // extern "C"
