// Body-force patterns from their closed form, written on the device into the
// context's force buffer (the F that kvs_project divides, solves and
// subtracts from).  The focused push of the separable source (Sec. 3.3: b0, a
// Gaussian along a beam axis; the Gaussian excitation of Sec. 4.4) and the
// time-varying workload's pattern (a Gaussian whose focus moves, times a
// random-phase plane-wave modulation) share one form: on every node
//   F_axis = F0 exp(-lat^2 / (2 s_l^2) - ax^2 / (2 s_a^2)) M(x),
//   M(x)   = 1 + a sum_m cos(k_m . x + phi_m),
// the other two components 0, with x = ((i - nx/2) hx, (j - ny/2) hy,
// (k - nz/2) hz) the node coordinates, ax = x_axis - c_axis the axial offset
// from the focus c and lat^2 the sum of the squared lateral offsets (lateral
// axes in increasing order).  Optionally F = 0 outside a box around the focus
// (|lateral offset| <= box_l on each lateral axis, |ax| <= box_a).
// Arithmetic is FP64, evaluated in the order written, without contraction
// into fused multiply-adds, so that a plain evaluation of the same formula
// on the host agrees to the last bits of exp and cos.
#include "kvs_internal.hpp"

namespace {

struct ForceArgs {
    int nx, ny, nz, axis, nmodes;
    long long N;
    double hx, hy, hz;
    double F0, c[3];
    double den_l, den_a;  // 2 s^2
    double box_l, box_a;  // < 0: no box
    double amp;
    double k[KVS_MAX_FORCE_MODES][3];
    double phase[KVS_MAX_FORCE_MODES];
};

__global__ __launch_bounds__(256) void force_pattern_kernel(const ForceArgs a, double* F) {
#pragma clang fp contract(off)
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < a.N; q += stride) {
        const int i = (int)(q % a.nx);
        const int j = (int)((q / a.nx) % a.ny);
        const int k = (int)(q / ((long long)a.nx * a.ny));
        const double x[3] = {(double)(i - a.nx / 2) * a.hx, (double)(j - a.ny / 2) * a.hy,
                             (double)(k - a.nz / 2) * a.hz};
        double off[3];
        for (int d = 0; d < 3; ++d) off[d] = x[d] - a.c[d];
        bool inside = true;
        double lat2 = 0.0;
        bool first = true;
        for (int d = 0; d < 3; ++d) {
            if (d == a.axis) continue;
            if (a.box_l >= 0.0 && !(fabs(off[d]) <= a.box_l)) inside = false;
            const double s = off[d] * off[d];
            lat2 = first ? s : lat2 + s;
            first = false;
        }
        const double ax = off[a.axis];
        if (a.box_a >= 0.0 && !(fabs(ax) <= a.box_a)) inside = false;
        double v = 0.0;
        if (inside) {
            const double g = exp(-lat2 / a.den_l - (ax * ax) / a.den_a);
            double M = 1.0;
            for (int m = 0; m < a.nmodes; ++m) {
                const double arg = a.k[m][0] * x[0] + a.k[m][1] * x[1] + a.k[m][2] * x[2] + a.phase[m];
                M = M + a.amp * cos(arg);
            }
            v = a.F0 * g * M;
        }
        for (int d = 0; d < 3; ++d) F[d * a.N + q] = d == a.axis ? v : 0.0;
    }
}

}  // namespace

hipError_t kvs_launch_force_pattern(kvs_ctx* c, const kvs_force_pattern* p) {
    ForceArgs a{};
    const kvs_grid& g = c->grid;
    a.nx = (int)g.nx;
    a.ny = (int)g.ny;
    a.nz = (int)g.nz;
    a.N = c->N;
    a.hx = g.hx;
    a.hy = g.hy;
    a.hz = g.hz;
    a.axis = p->axis;
    a.F0 = p->F0;
    for (int d = 0; d < 3; ++d) a.c[d] = p->centre[d];
    a.den_l = 2.0 * (p->sigma_lateral * p->sigma_lateral);
    a.den_a = 2.0 * (p->sigma_axial * p->sigma_axial);
    a.box_l = p->box_lateral;
    a.box_a = p->box_axial;
    a.nmodes = p->n_modes;
    a.amp = p->mod_amp;
    for (int m = 0; m < p->n_modes; ++m) {
        for (int d = 0; d < 3; ++d) a.k[m][d] = p->k[m][d];
        a.phase[m] = p->phase[m];
    }
    const long long blocks = std::min<long long>((c->N + 255) / 256, 65536);
    hipLaunchKernelGGL(force_pattern_kernel, dim3((unsigned)blocks), dim3(256), 0, c->stream, a, c->F);
    return hipGetLastError();
}
