// Tiling helpers shared by the stencil kernels (FDTD step and CG sweeps).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

namespace kvs_tiling {

// Tiles are numbered x fastest, then y, then z.  The hardware hands block b
// to XCD b % 8; remapping so that each XCD receives a contiguous range of
// tile numbers keeps y-adjacent tiles (which share halo rows) in one L2.
__device__ __forceinline__ int tile_of(int b, int B) {
    const int xcd = b & 7, pos = b >> 3;
    const int per = B >> 3, rem = B & 7;
    return xcd * per + min(xcd, rem) + pos;
}

// Workgroup barrier that orders LDS only.  __syncthreads() also fences
// global memory, which makes every wave drain its outstanding global loads
// (the plane-ahead prefetch) at each barrier; the stencils only share LDS.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Blocks of one kernel instance that fit on the chip at once.
template <typename K>
int resident_blocks(K kernel, int threads) {
    int dev = 0, per_cu = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 1024;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu <= 0)
        per_cu = 1;
    return per_cu * prop.multiProcessorCount;
}

// Split z into segments so that (xy tiles) x (segments) fills whole rounds of
// resident blocks; fewer, longer segments re-read fewer halo planes.
inline int choose_kchunk(int xytiles, int planes, int cap) {
    int best_seg = 1;
    double best = -1.0;
    const int max_seg = std::max(1, planes / 8);
    for (int seg = 1; seg <= max_seg; ++seg) {
        const int chunk = (planes + seg - 1) / seg;
        const int nseg = (planes + chunk - 1) / chunk;
        const long long blocks = (long long)xytiles * nseg;
        const long long rounds = (blocks + cap - 1) / cap;
        const double fill = (double)blocks / (double)(rounds * cap);
        const double halo = 2.0 / (double)chunk;
        const double score = fill / (1.0 + halo);
        if (score > best + 1e-9) {
            best = score;
            best_seg = seg;
        }
    }
    return (planes + best_seg - 1) / best_seg;
}

// Upper bound on the blocks any tiled launch over `planes` z planes uses:
// at least 8 planes per segment.
inline long long max_tiled_blocks(int xytiles, int planes) {
    return (long long)xytiles * std::max(1, (planes + 7) / 8);
}

}  // namespace kvs_tiling
