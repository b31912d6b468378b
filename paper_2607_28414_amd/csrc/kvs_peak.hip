// Peak displacement maps: after every step, the running maximum of
// |u| = sqrt(ux^2 + uy^2 + uz^2) on registered grid planes (the |u| slices
// and peak displacement of the transcranial demonstration, Sec. 5.1).
//
// One y-row of blocks per plane and a grid-stride loop over the plane's
// cells, the plane's first in-plane axis fastest.  z and y planes read whole
// x rows (coalesced); an x plane reads one cell per row, which is inherent to
// that slice and costs a few microseconds per step on the largest grids.
#include "kvs_internal.hpp"

namespace {

// NaN wins over every number, so an unstable run shows in the map instead of
// hiding behind a plain max.
template <typename T>
__global__ void peak_kernel(const T* u, long long N, int nx, int ny, PeakPlanes P, T* maps) {
    const int p = blockIdx.y;
    const int axis = P.axis[p];
    const long long idx = P.index[p];
    const long long n1 = P.n1[p], cells = n1 * P.n2[p];
    T* m = maps + P.off[p];
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < cells;
         q += (long long)gridDim.x * blockDim.x) {
        const long long a = q % n1, b = q / n1;
        const long long i = axis == 0 ? idx : a;
        const long long j = axis == 0 ? a : (axis == 1 ? idx : b);
        const long long k = axis == 2 ? idx : b;
        const long long c = i + nx * (j + ny * k);
        const T x = u[c], y = u[N + c], z = u[2 * N + c];
        const T v = sqrt(x * x + y * y + z * z);
        const T old = m[q];
        m[q] = (v > old || __builtin_isnan(v)) ? v : old;
    }
}

}  // namespace

hipError_t kvs_launch_peak_update(kvs_ctx* c, const void* u_new) {
    if (c->npeak == 0) return hipSuccess;
    PeakPlanes P{};
    long long most = 0;
    for (int p = 0; p < c->npeak; ++p) {
        const int a = c->peak_axis[p];
        P.axis[p] = a;
        P.index[p] = c->peak_index[p];
        P.n1[p] = a == 0 ? c->grid.ny : c->grid.nx;
        P.n2[p] = a == 2 ? c->grid.ny : c->grid.nz;
        P.off[p] = c->peak_off[p];
        most = std::max(most, (long long)P.n1[p] * P.n2[p]);
    }
    const dim3 grid((unsigned)std::min<long long>((most + 255) / 256, 1024), (unsigned)c->npeak);
    if (c->prec == KVS_FP32)
        hipLaunchKernelGGL(peak_kernel<float>, grid, dim3(256), 0, c->stream, static_cast<const float*>(u_new),
                           (long long)c->N, (int)c->grid.nx, (int)c->grid.ny, P, static_cast<float*>(c->peak));
    else
        hipLaunchKernelGGL(peak_kernel<double>, grid, dim3(256), 0, c->stream, static_cast<const double*>(u_new),
                           (long long)c->N, (int)c->grid.nx, (int)c->grid.ny, P, static_cast<double*>(c->peak));
    return hipGetLastError();
}
