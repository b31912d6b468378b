// Two FDTD steps per launch for one context (the tile code is in
// kvs_step2_tile.hpp).  The first pblocks blocks copy the launch's input state
// (the previous step's result) at the probe cells, as in the one-step kernel;
// the remaining blocks are the tiles, numbered XCD by XCD.
#include <hip/hip_ext.h>

#include "kvs_step2_tile.hpp"

namespace {

template <bool HET, int WX>
__global__ __launch_bounds__(64 * WX * S2_ROWS) void step2_kernel(const Step2Args A2) {
    const StepArgs<float>& a = A2.a;
    if ((int)blockIdx.x < a.pblocks) {
        const long long p = (long long)blockIdx.x * (64 * WX * S2_ROWS) + threadIdx.y * (64 * WX) + threadIdx.x;
        if (p < a.np) {
            const long long q = a.pcells[p];
            if (a.pcomp == 3) {
                a.pout[3 * p] = (double)a.u[q];
                a.pout[3 * p + 1] = (double)a.u[a.N + q];
                a.pout[3 * p + 2] = (double)a.u[2 * a.N + q];
            } else {
                a.pout[p] = (double)a.u[a.pcomp * a.N + q];
            }
        }
        return;
    }
    const int B = a.gy * a.gz;
    const int b = (int)blockIdx.x - a.pblocks;
    const int t = a.remap ? tile_of(b, B) : b;
    step2_tile<HET, WX, S2_ROWS>(A2, t % a.gy, t / a.gy);
}

template <bool HET, int WX>
hipError_t launch_wx(kvs_ctx* c, const Step2Args& A0) {
    Step2Args A2 = A0;
    StepArgs<float>& a = A2.a;
    auto kern = step2_kernel<HET, WX>;
    static const int cap = resident_blocks(kern, 64 * WX * S2_ROWS);
    a.gx = 1;
    a.gy = (a.ny + 1) / 2;
    a.kchunk = c->step_zchunk > 0 ? std::min(c->step_zchunk, a.nz - 2) : choose_kchunk(a.gy, a.nz - 2, cap);
    a.gz = (a.nz - 2 + a.kchunk - 1) / a.kchunk;
    a.pblocks = a.pout ? (int)((a.np + 64 * WX * S2_ROWS - 1) / (64 * WX * S2_ROWS)) : 0;
    const int blocks = a.gy * a.gz + a.pblocks;
    if (c->launch_ev[0])
        hipExtLaunchKernelGGL(kern, dim3(blocks), dim3(64 * WX, S2_ROWS), 0, c->stream, c->launch_ev[0],
                              c->launch_ev[1], 0, A2);
    else
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * WX, S2_ROWS), 0, c->stream, A2);
    return hipGetLastError();
}

}  // namespace

bool kvs_step2_supported(const kvs_ctx* c) {
    // cell offsets within a field are 32-bit
    return c->prec == KVS_FP32 && c->viscous && c->npeak == 0 && c->pml_cells == 0 &&
           c->grid.nx <= 256 && c->N < ((int64_t)1 << 31) && (c->nprobes == 0 || c->probe_rows_ok);
}

hipError_t kvs_launch_step2(kvs_ctx* c) {
    const kvs_grid& g = c->grid;
    Step2Args A2{};
    StepArgs<float>& a = A2.a;
    const int nb = 1 - c->cur;
    a.u = static_cast<const float*>(c->u[c->cur]);
    a.w = static_cast<const float*>(c->w[c->cur]);
    a.un = static_cast<float*>(c->u[nb]);
    a.wn = static_cast<float*>(c->w[nb]);
    a.G = static_cast<const float*>(c->G);
    a.eta = static_cast<const float*>(c->eta);
    a.crho = static_cast<const float*>(c->crho);
    a.N = c->N;
    a.nx = (int)g.nx;
    a.ny = (int)g.ny;
    a.nz = (int)g.nz;
    a.L = c->sponge_cells;
    a.invL = a.L > 0 ? (float)(1.0 / a.L) : 0.f;
    a.ihx2 = (float)(1.0 / (g.hx * g.hx));
    a.ihy2 = (float)(1.0 / (g.hy * g.hy));
    a.ihz2 = (float)(1.0 / (g.hz * g.hz));
    a.G0 = (float)c->G0;
    a.eta_dt0 = (float)(c->eta0 / c->dt);
    a.crho0 = (float)(c->dt * c->dt / c->rho0);
    a.inv_dt = (float)(1.0 / c->dt);
    a.half_dt_smax = (float)(0.5 * c->sigma_max * c->dt);
    a.remap = c->step_remap;
    if (c->probe_fused_out) {
        a.pcells = reinterpret_cast<const long long*>(c->probe_cells);
        a.pout = c->probe_fused_out;
        a.np = c->nprobes;
        a.pcomp = c->probe_comp;
    }
    if (c->nprobes > 0) {
        A2.rowtab = c->probe_rowtab;
        A2.ptab = c->probe_ptab;
        A2.pmid = c->probe_mid_out;
        a.pcomp = c->probe_comp;
    }
    if (c->hetero) return g.nx <= 128 ? launch_wx<true, 2>(c, A2) : launch_wx<true, 4>(c, A2);
    return g.nx <= 128 ? launch_wx<false, 2>(c, A2) : launch_wx<false, 4>(c, A2);
}
