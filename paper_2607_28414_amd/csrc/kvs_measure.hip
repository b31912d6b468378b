// Streaming references for the FDTD step kernels' rooflines: kernels with a
// step's memory pattern and no stencil.  The heterogeneous step reads 9 FP32
// values per cell (three components each of u and w, and the three per-cell
// material values) and writes 6 (the new u and w), 60 B; the homogeneous
// batched step reads 6 and writes 6, 48 B.  Each stream is contiguous, with
// 16-byte non-temporal loads and stores (the fastest of the simple forms
// measured: plain accesses, one or several vectors per thread, 4 to 32 blocks
// per CU), grid-stride over 16 blocks per CU.  The bandwidth is the practical
// ceiling for a kernel that moves a step's bytes once; a step kernel's
// fraction of it separates stencil and tiling losses from what HBM delivers
// to that read/write mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "kvs_internal.hpp"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

struct StreamPtrs {
    const f4* in[9];
    f4* out[6];
    long long n4;
};

// R reads and W writes per element (W <= R): every output mixes three inputs
// so that no load is dead.
template <int R, int W>
__global__ __launch_bounds__(256) void stream_kernel(const StreamPtrs s) {
    static_assert(W <= R && R <= 9 && W <= 6 && R <= W + 3, "every input feeds an output");
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < s.n4; q += stride) {
        f4 v[R];
#pragma unroll
        for (int a = 0; a < R; ++a) v[a] = __builtin_nontemporal_load(&s.in[a][q]);
#pragma unroll
        for (int b = 0; b < W; ++b)
            __builtin_nontemporal_store(v[b] + v[(b + 3) % R] * v[(R - 3 + b % 3) % R], &s.out[b][q]);
    }
}

}  // namespace

kvs_status kvs_measure_stream_rw(int32_t device, int64_t n, int32_t reads, int32_t writes, int32_t reps,
                                 double* gbs) {
    if (!gbs || n < 1024 || reps < 1) return KVS_EINVAL;
    if (!((reads == 9 && writes == 6) || (reads == 6 && writes == 6))) return KVS_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return KVS_EDEVICE;
    const long long n4 = (n + 3) / 4;
    const int nbuf = reads + writes;
    std::vector<void*> bufs((size_t)nbuf, nullptr);
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    kvs_status ret = KVS_OK;
    for (auto& b : bufs)
        if (hipMalloc(&b, sizeof(f4) * (size_t)n4) != hipSuccess) ret = KVS_ENOMEM;
    if (ret == KVS_OK && (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
                          hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        ret = KVS_EDEVICE;
    if (ret == KVS_OK) {
        for (auto& b : bufs)
            if (hipMemsetAsync(b, 0, sizeof(f4) * (size_t)n4, st) != hipSuccess) ret = KVS_EDEVICE;
    }
    if (ret == KVS_OK) {
        StreamPtrs s{};
        for (int a = 0; a < reads; ++a) s.in[a] = static_cast<const f4*>(bufs[(size_t)a]);
        for (int b = 0; b < writes; ++b) s.out[b] = static_cast<f4*>(bufs[(size_t)(reads + b)]);
        s.n4 = n4;
        hipDeviceProp_t prop;
        (void)hipGetDeviceProperties(&prop, device);
        const int blocks = std::max(1, prop.multiProcessorCount) * 16;
        std::vector<float> ms;
        for (int r = 0; r <= reps && ret == KVS_OK; ++r) {  // the first launch is not timed
            (void)hipEventRecord(e0, st);
            if (reads == 9)
                hipLaunchKernelGGL((stream_kernel<9, 6>), dim3(blocks), dim3(256), 0, st, s);
            else
                hipLaunchKernelGGL((stream_kernel<6, 6>), dim3(blocks), dim3(256), 0, st, s);
            (void)hipEventRecord(e1, st);
            if (hipEventSynchronize(e1) != hipSuccess) ret = KVS_EDEVICE;
            float t = 0.f;
            (void)hipEventElapsedTime(&t, e0, e1);
            if (r > 0) ms.push_back(t);
        }
        if (ret == KVS_OK) {
            std::sort(ms.begin(), ms.end());
            const double med = ms[ms.size() / 2];
            *gbs = (double)nbuf * 16.0 * (double)n4 / (med * 1e-3) / 1e9;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    for (auto b : bufs)
        if (b) (void)hipFree(b);
    return ret;
}

kvs_status kvs_measure_stream(int32_t device, int64_t n, int32_t reps, double* gbs) {
    return kvs_measure_stream_rw(device, n, 9, 6, reps, gbs);
}
