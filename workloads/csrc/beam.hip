// Synthetic acoustic samples on the device: the focused tone burst of
// workloads.acoustic_beam_samples (a Gaussian beam along +z focused at a
// point, waist w0, wavelength c / f0, attenuated by exp(-alpha (z - z_min)),
// `cycles` periods of `per` samples, silent afterwards; v = p n / (rho c) with
// n the normalised local direction of the phase front (x / R, y / R, 1)),
// evaluated per cell in FP64 in the order of the numpy generator and cast to
// the sample type.  Input drawing for benchmarks and tests (it stands in for
// an acoustic solver's output); the solver library does not use it.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace {

struct Beam {
    int nx, ny, nz;
    double hx, hy, hz;
    double fx, fy, fz;  // focus
    double f0, c, rho, alpha, p0, w0;
    int per, cycles;
    long long s0;
    int nsamp;
};

template <typename T>
__global__ void beam_kernel(const Beam b, T* p, T* v) {
#pragma clang fp contract(off)
    const long long N = (long long)b.nx * b.ny * b.nz;
    const double pi = 3.14159265358979323846;
    const double zmin = (double)(0 - b.nz / 2) * b.hz;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < N; q += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(q % b.nx), j = (int)((q / b.nx) % b.ny), k = (int)(q / ((long long)b.nx * b.ny));
        const double x = (double)(i - b.nx / 2) * b.hx - b.fx;
        const double y = (double)(j - b.ny / 2) * b.hy - b.fy;
        const double z = (double)(k - b.nz / 2) * b.hz;
        const double dz = z - b.fz;
        const double lam = b.c / b.f0;
        const double kw = 2 * pi / lam;
        const double zr = pi * (b.w0 * b.w0) / lam;
        const double w = b.w0 * sqrt(1 + (dz / zr) * (dz / zr));
        const double inv_r = dz / (dz * dz + zr * zr);
        const double rr = x * x + y * y;
        const double amp = b.p0 * (b.w0 / w) * exp(-rr / (w * w)) * exp(-b.alpha * (z - zmin));
        const double phase = kw * dz + kw * rr * inv_r / 2 - atan(dz / zr);
        const double nxv = x * inv_r, nyv = y * inv_r;
        const double norm = sqrt(nxv * nxv + nyv * nyv + 1.0);
        const double scale = 1.0 / (b.rho * b.c);
        for (int s = 0; s < b.nsamp; ++s) {
            const long long sg = b.s0 + s;
            const double pv = sg < (long long)b.per * b.cycles ? amp * cos(2 * pi * (double)sg / b.per - phase) : 0.0;
            p[s * N + q] = (T)pv;
            if (v) {
                v[(3LL * s + 0) * N + q] = (T)(pv * (scale * nxv / norm));
                v[(3LL * s + 1) * N + q] = (T)(pv * (scale * nyv / norm));
                v[(3LL * s + 2) * N + q] = (T)(pv * (scale / norm));
            }
        }
    }
}

}  // namespace

// p [nsamp][N], v [nsamp][3][N] (or NULL): device buffers of float (dtype 1)
// or double (dtype 0).  Returns 0 on success, else the HIP error code.
extern "C" int wl_beam_samples(int nx, int ny, int nz, double hx, double hy, double hz, double fx, double fy,
                               double fz, double f0, double c, double rho, double alpha, double p0, double w0, int per,
                               int cycles, long long s0, int nsamp, int dtype, void* p, void* v, void* stream) {
    Beam b{nx, ny, nz, hx, hy, hz, fx, fy, fz, f0, c, rho, alpha, p0, w0, per, cycles, s0, nsamp};
    const long long N = (long long)nx * ny * nz;
    const unsigned blocks = (unsigned)((N + 255) / 256 < 65536 ? (N + 255) / 256 : 65536);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dtype == 1)
        hipLaunchKernelGGL(beam_kernel<float>, dim3(blocks), dim3(256), 0, s, b, static_cast<float*>(p),
                           static_cast<float*>(v));
    else
        hipLaunchKernelGGL(beam_kernel<double>, dim3(blocks), dim3(256), 0, s, b, static_cast<double*>(p),
                           static_cast<double*>(v));
    return (int)hipGetLastError();
}
