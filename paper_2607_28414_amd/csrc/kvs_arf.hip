// Acoustic radiation body force from a time series of the acoustic field
// (Sec. 3.4: plane-wave form, Eq. isppa_norm; Poynting form, Eq. arf_poynting),
// and the peak acoustic strain maps of Sec. 5.2 from the pressure series.
//
// Three streaming kernels:
//   arf_acc_kernel   folds nsamp samples of p (and v) into per-cell FP64 sums,
//                    S += p^2 (plane-wave form) or S_i += p v_i (Poynting form),
//                    sample by sample in the order given;
//   arf_force_kernel turns the sums into the force pattern F (FP64, [3][N]);
//   strain_kernel    folds pressure samples into the peak |eps| and peak
//                    |grad eps| maps.
//
// The accumulation is HBM-bound (16 B of FP32 input per cell and sample in
// the Poynting form, plus one read and one write of the sums per launch):
// each lane owns VEC consecutive cells so that every access is a 16-byte
// vector load of a contiguous run, the samples of one launch are streamed
// with non-temporal loads (read once), and the sums stay in registers across
// the launch's samples.  Products and sums are FP64 and are not contracted
// into fused multiply-adds, so the result is the plain sequential sum.
#include "kvs_internal.hpp"

namespace {

template <typename T, int V>
struct Vec {
    typedef T type __attribute__((ext_vector_type(V)));
};

template <typename T, int V>
__device__ __forceinline__ void load_nt(const T* p, double (&o)[V]) {
    if constexpr (V == 1) {
        o[0] = (double)__builtin_nontemporal_load(p);
    } else {
        const typename Vec<T, V>::type x = __builtin_nontemporal_load(reinterpret_cast<const typename Vec<T, V>::type*>(p));
#pragma unroll
        for (int j = 0; j < V; ++j) o[j] = (double)x[j];
    }
}

// MODE 1: plane-wave form (one sum), MODE 2: Poynting form (three sums).
// Lane t owns cells [V t, V t + V); the host picks V > 1 only when N is a
// multiple of V and the inputs are 16-byte aligned, so no lane straddles the
// end of a sample.
template <typename T, int MODE, int V>
__global__ __launch_bounds__(256) void arf_acc_kernel(const T* __restrict__ p, const T* __restrict__ v, long long N,
                                                      int nsamp, double* __restrict__ S) {
#pragma clang fp contract(off)
    constexpr int NS = MODE == 1 ? 1 : 3;
    const long long c0 = ((long long)blockIdx.x * blockDim.x + threadIdx.x) * V;
    if (c0 >= N) return;
    double acc[NS][V];
#pragma unroll
    for (int i = 0; i < NS; ++i)
#pragma unroll
        for (int j = 0; j < V; ++j) acc[i][j] = S[i * N + c0 + j];
#pragma unroll 2
    for (int s = 0; s < nsamp; ++s) {
        double ps[V];
        load_nt<T, V>(p + (long long)s * N + c0, ps);
        if constexpr (MODE == 1) {
#pragma unroll
            for (int j = 0; j < V; ++j) acc[0][j] = acc[0][j] + ps[j] * ps[j];
        } else {
            const T* vs = v + (long long)s * 3 * N + c0;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                double vi[V];
                load_nt<T, V>(vs + i * N, vi);
#pragma unroll
                for (int j = 0; j < V; ++j) acc[i][j] = acc[i][j] + ps[j] * vi[j];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < NS; ++i)
#pragma unroll
        for (int j = 0; j < V; ++j) S[i * N + c0 + j] = acc[i][j];
}

// Coefficient maps are indexed with stride 0 (one uniform value) or 1 (a
// value per cell).  mask == nullptr keeps every cell.
struct ForceArgs {
    const double* S;
    long long N;
    int mode;
    const double* alpha;
    const double* c;
    const double* rho;
    int sa, sc, sr;
    const unsigned char* mask;
    double n_pulse;
    double d0, d1, d2;  // unit beam direction (plane-wave form)
    double* F;
};

__global__ __launch_bounds__(256) void arf_force_kernel(const ForceArgs a) {
#pragma clang fp contract(off)
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < a.N;
         i += (long long)gridDim.x * blockDim.x) {
        const bool keep = a.mask == nullptr || a.mask[i] != 0;
        const double al = a.alpha[i * a.sa], cc = a.c[i * a.sc];
        const double coef = 2.0 * al / cc;
        double f0, f1, f2;
        if (a.mode == 1) {
            const double intensity = a.S[i] / (a.rho[i * a.sr] * cc * a.n_pulse);
            const double b0 = coef * intensity;
            f0 = b0 * a.d0;
            f1 = b0 * a.d1;
            f2 = b0 * a.d2;
        } else {
            f0 = coef * (a.S[i] / a.n_pulse);
            f1 = coef * (a.S[a.N + i] / a.n_pulse);
            f2 = coef * (a.S[2 * a.N + i] / a.n_pulse);
        }
        a.F[i] = keep ? f0 : 0.0;
        a.F[a.N + i] = keep ? f1 : 0.0;
        a.F[2 * a.N + i] = keep ? f2 : 0.0;
    }
}

// Peak acoustic strain eps = -p / K and peak |grad eps| (Sec. 5.2), one lane
// per cell, the launch's samples in order.  The cell's own strain is the
// division -p / K (so the peak-strain map is the definition's value); the six
// neighbour strains in the gradient use the neighbours' 1/K, formed once per
// launch, and the differences are scaled by 1/(2 h): products instead of
// nine more FP64 divisions per cell and sample, which made the kernel bound
// by FP64 issue (each gradient term differs from the divided form by a few
// roundings).  The neighbours' p reads hit the caches: concurrent blocks
// cover adjacent rows and planes.  Running maxima in registers; a NaN, once
// seen, stays.  The gradient map holds the running maximum of |grad eps|^2:
// the square root is monotone and correctly rounded, so taking it once when
// the map is read gives the maximum of the roots exactly.
template <typename T>
__global__ __launch_bounds__(256) void strain_kernel(const T* __restrict__ p, long long N, int nsamp, int nx, int ny,
                                                     int nz, const double* __restrict__ K, int sK, double inv_2hx,
                                                     double inv_2hy, double inv_2hz, double* __restrict__ peak) {
#pragma clang fp contract(off)
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const long long sxy = (long long)nx * ny;
    const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / sxy);
    const bool inner = x >= 1 && x <= nx - 2 && y >= 1 && y <= ny - 2 && z >= 1 && z <= nz - 2;
    const double Kc = K[i * sK];
    const long long off[6] = {-1, 1, -(long long)nx, nx, -sxy, sxy};
    double rK[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) rK[q] = inner ? -1.0 / K[(i + off[q]) * sK] : 0.0;
    double pe = peak[i], pg = peak[N + i];
    for (int s = 0; s < nsamp; ++s) {
        const T* ps = p + (long long)s * N;
        const double e = -(double)ps[i] / Kc;
        const double ae = fabs(e);
        pe = (ae > pe || __builtin_isnan(ae)) ? ae : pe;
        if (inner) {
            double en[6];
#pragma unroll
            for (int q = 0; q < 6; ++q) en[q] = (double)ps[i + off[q]] * rK[q];
            const double gx = (en[1] - en[0]) * inv_2hx;
            const double gy = (en[3] - en[2]) * inv_2hy;
            const double gz = (en[5] - en[4]) * inv_2hz;
            const double g2 = gx * gx + gy * gy + gz * gz;
            pg = (g2 > pg || __builtin_isnan(g2)) ? g2 : pg;
        }
    }
    peak[i] = pe;
    peak[N + i] = pg;
}

template <typename T, int MODE, int V>
void launch_acc(hipStream_t s, const void* p, const void* v, long long N, int nsamp, double* S) {
    const long long lanes = (N + V - 1) / V;
    const unsigned blocks = (unsigned)((lanes + 255) / 256);
    hipLaunchKernelGGL((arf_acc_kernel<T, MODE, V>), dim3(blocks), dim3(256), 0, s, static_cast<const T*>(p),
                       static_cast<const T*>(v), N, nsamp, S);
}

template <typename T, int MODE>
void launch_acc_mode(hipStream_t s, const void* p, const void* v, long long N, int nsamp, double* S) {
    constexpr int V = sizeof(T) == 4 ? 4 : 2;  // 16-byte accesses
    const bool aligned = (reinterpret_cast<uintptr_t>(p) % 16 == 0) &&
                         (MODE == 1 || reinterpret_cast<uintptr_t>(v) % 16 == 0) && (N % V == 0);
    if (aligned)
        launch_acc<T, MODE, V>(s, p, v, N, nsamp, S);
    else
        launch_acc<T, MODE, 1>(s, p, v, N, nsamp, S);
}

}  // namespace

// Samples per launch: bounds the index arithmetic of one launch and keeps
// a launch short enough to interleave with other work on the stream.
static constexpr int64_t kMaxSamplesPerLaunch = 64;

hipError_t kvs_launch_arf_accumulate(kvs_ctx* c, const void* p, const void* v, int64_t nsamp, int dtype) {
    const long long N = (long long)c->N;
    const size_t es = dtype == 1 ? sizeof(float) : sizeof(double);
    for (int64_t s0 = 0; s0 < nsamp; s0 += kMaxSamplesPerLaunch) {
        const int ns = (int)std::min<int64_t>(kMaxSamplesPerLaunch, nsamp - s0);
        const char* ps = static_cast<const char*>(p) + (size_t)s0 * N * es;
        const char* vs = v ? static_cast<const char*>(v) + (size_t)s0 * 3 * N * es : nullptr;
        if (c->arf_mode == 1)
            dtype == 1 ? launch_acc_mode<float, 1>(c->stream, ps, vs, N, ns, c->arf_sum)
                       : launch_acc_mode<double, 1>(c->stream, ps, vs, N, ns, c->arf_sum);
        else
            dtype == 1 ? launch_acc_mode<float, 2>(c->stream, ps, vs, N, ns, c->arf_sum)
                       : launch_acc_mode<double, 2>(c->stream, ps, vs, N, ns, c->arf_sum);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t kvs_launch_strain(kvs_ctx* c, const void* p, int64_t nsamp, int dtype) {
    const kvs_grid& g = c->grid;
    const long long N = (long long)c->N;
    const size_t es = dtype == 1 ? sizeof(float) : sizeof(double);
    const unsigned blocks = (unsigned)((N + 255) / 256);
    for (int64_t s0 = 0; s0 < nsamp; s0 += kMaxSamplesPerLaunch) {
        const int ns = (int)std::min<int64_t>(kMaxSamplesPerLaunch, nsamp - s0);
        const void* ps = static_cast<const char*>(p) + (size_t)s0 * N * es;
        if (dtype == 1)
            hipLaunchKernelGGL(strain_kernel<float>, dim3(blocks), dim3(256), 0, c->stream, static_cast<const float*>(ps),
                               N, ns, (int)g.nx, (int)g.ny, (int)g.nz, c->strain_K, c->strain_sK, 0.5 / g.hx,
                               0.5 / g.hy, 0.5 / g.hz, c->strain_peak);
        else
            hipLaunchKernelGGL(strain_kernel<double>, dim3(blocks), dim3(256), 0, c->stream,
                               static_cast<const double*>(ps), N, ns, (int)g.nx, (int)g.ny, (int)g.nz, c->strain_K,
                               c->strain_sK, 0.5 / g.hx, 0.5 / g.hy, 0.5 / g.hz, c->strain_peak);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

namespace {
// The gradient map's square roots (the map holds squares while samples are
// folded in).
__global__ __launch_bounds__(256) void sqrt_kernel(const double* __restrict__ in, double* __restrict__ out,
                                                   long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        out[i] = sqrt(in[i]);
}
}  // namespace

hipError_t kvs_launch_strain_roots(kvs_ctx* c, double* out) {
    const long long N = (long long)c->N;
    const unsigned blocks = (unsigned)std::min<long long>((N + 255) / 256, 16384);
    hipLaunchKernelGGL(sqrt_kernel, dim3(blocks), dim3(256), 0, c->stream, c->strain_peak + N, out, N);
    return hipGetLastError();
}

hipError_t kvs_launch_arf_force(kvs_ctx* c, const double* alpha, int sa, const double* cs, int sc, const double* rho,
                                int sr, const unsigned char* mask, double n_pulse, const double d[3]) {
    ForceArgs a{};
    a.S = c->arf_sum;
    a.N = (long long)c->N;
    a.mode = c->arf_mode;
    a.alpha = alpha;
    a.c = cs;
    a.rho = rho ? rho : cs;  // unread in the Poynting form
    a.sa = sa;
    a.sc = sc;
    a.sr = rho ? sr : 0;
    a.mask = mask;
    a.n_pulse = n_pulse;
    a.d0 = d[0];
    a.d1 = d[1];
    a.d2 = d[2];
    a.F = c->F;
    const unsigned blocks = (unsigned)std::min<long long>((a.N + 255) / 256, 16384);
    hipLaunchKernelGGL(arf_force_kernel, dim3(blocks), dim3(256), 0, c->stream, a);
    return hipGetLastError();
}
