// Curl-based initial state (Sec. 3.5: a divergence-free initial velocity
// built as the curl of a vector potential, the source of the wavespeed
// validation of Sec. 4.1).  In the summed form the state is (u, w) with
// w = u^0 - u^{-1}; an initial velocity v0 at rest displacement gives u = 0,
// w = dt v0.  v0 = curl_h A with the grid's centred first differences on the
// interior nodes and 0 on the outer (Dirichlet) layer, in FP64, then stored
// in the state precision.  One pass over the cells; the six neighbour reads
// of A per component are served by the caches.
#include "kvs_internal.hpp"

namespace {

template <typename T>
__global__ __launch_bounds__(256) void curl_state_kernel(const double* __restrict__ A, long long N, int nx, int ny,
                                                         int nz, double two_hx, double two_hy, double two_hz,
                                                         double dt, T* __restrict__ u, T* __restrict__ w) {
#pragma clang fp contract(off)
    const long long sxy = (long long)nx * ny;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx);
        const int y = (int)((i / nx) % ny);
        const int z = (int)(i / sxy);
        double c0 = 0.0, c1 = 0.0, c2 = 0.0;
        if (x >= 1 && x <= nx - 2 && y >= 1 && y <= ny - 2 && z >= 1 && z <= nz - 2) {
            const double* Ax = A;
            const double* Ay = A + N;
            const double* Az = A + 2 * N;
            const double dyAz = (Az[i + nx] - Az[i - nx]) / two_hy;
            const double dzAy = (Ay[i + sxy] - Ay[i - sxy]) / two_hz;
            const double dzAx = (Ax[i + sxy] - Ax[i - sxy]) / two_hz;
            const double dxAz = (Az[i + 1] - Az[i - 1]) / two_hx;
            const double dxAy = (Ay[i + 1] - Ay[i - 1]) / two_hx;
            const double dyAx = (Ax[i + nx] - Ax[i - nx]) / two_hy;
            c0 = dt * (dyAz - dzAy);
            c1 = dt * (dzAx - dxAz);
            c2 = dt * (dxAy - dyAx);
        }
        w[i] = (T)c0;
        w[N + i] = (T)c1;
        w[2 * N + i] = (T)c2;
        u[i] = T(0);
        u[N + i] = T(0);
        u[2 * N + i] = T(0);
    }
}

}  // namespace

hipError_t kvs_launch_curl_state(kvs_ctx* c, const double* A) {
    const kvs_grid& g = c->grid;
    const long long N = (long long)c->N;
    const unsigned blocks = (unsigned)std::min<long long>((N + 255) / 256, 16384);
    if (c->prec == KVS_FP32)
        hipLaunchKernelGGL(curl_state_kernel<float>, dim3(blocks), dim3(256), 0, c->stream, A, N, (int)g.nx,
                           (int)g.ny, (int)g.nz, 2.0 * g.hx, 2.0 * g.hy, 2.0 * g.hz, c->dt,
                           static_cast<float*>(c->u[c->cur]), static_cast<float*>(c->w[c->cur]));
    else
        hipLaunchKernelGGL(curl_state_kernel<double>, dim3(blocks), dim3(256), 0, c->stream, A, N, (int)g.nx,
                           (int)g.ny, (int)g.nz, 2.0 * g.hx, 2.0 * g.hy, 2.0 * g.hz, c->dt,
                           static_cast<double*>(c->u[c->cur]), static_cast<double*>(c->w[c->cur]));
    return hipGetLastError();
}
