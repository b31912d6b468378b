// Absorbing layer (convolutional PML) for the reduced Kelvin-Voigt shear
// update.  The paper terminates the grid with a Dirichlet layer and names
// perfectly matched layers as the remedy for its reflections (Sec. 3.5,
// Sec. 7) without a formulation; the one implemented here stretches each
// axis, s_a = 1 + d_a / (alpha + i w), in both spatial derivatives of each
// term of the Sec. 3.1 update, in recursive-convolution form:
//
//   face fluxes      F_el = G_f (u(+a) - u) / h_a,   F_w = (w(+a) - w) / h_a,
//                    psi <- b_f psi + c_f F,  stretched flux F + psi;
//   cell divergence  D_a = (stretched F_el(+) - (-)) / h_a
//                          + (eta / dt) (stretched F_w(+) - (-)) / h_a,
//                    phi <- b_c phi + c_c D_a,  stretched D_a + phi;
//   update           w' = w + (dt^2 / rho) (sum_a stretched D_a + g_n f_S),
//                    u' = u + w'   (no sponge with the layer),
//
// with b = exp(-(d + alpha) dt), c = d / (d + alpha) (b - 1), d = d0 q^2 over
// the layer's depth q, alpha constant inside the layer (default
// pi c_max / (10 L h_min), the frequency of a wave ten layer widths long; a
// shift that vanished anywhere in the layer would leave the interior free to
// drift by a uniform static displacement).
//
// The layer is L cells next to every Dirichlet face.  The main step kernel
// updates every cell with the plain scheme; one layer pass per step then
// corrects the layer cells: for each axis whose layer holds the cell it
// advances the memories of the cell's two faces from the old state (read
// from one buffer; the cell writes the face towards the wall into the other
// buffer, so every face is written once, and the buffers swap every step),
// advances the cell's divergence memory phi and adds to the new state the
// difference the stretched derivatives make.  Memory variables live only in
// the slabs: along axis a, indices [0, T) and [n_a - 1 - T, n_a - 1) with
// T = L + 1, which hold the faces i + 1/2 and the cells i that the layer
// uses.
#include <algorithm>
#include <cmath>
#include <vector>

#include "kvs_internal.hpp"

namespace {

template <typename T>
__device__ __forceinline__ T harm2(T a, T b) {
    return T(2) * a * b / (a + b);
}

template <typename T>
struct PmlAxis {
    const T* tab;     // [4][n]: b at cells, c at cells, b at faces (i + 1/2), c at faces
    const T* psin;    // [6][M]: face memories psi_el (3 components), psi_w (3), this step's
    T* psout;         // [6][M]: the same, next step's
    T* phi;           // [3][M]: divergence memories (updated in place)
    long long M;      // slab cells of this axis
    int n;            // extent
    T ih;             // 1 / h
};

template <typename T>
struct PmlArgs {
    const T* u;
    const T* w;
    T* un;
    T* wn;
    const T* G;     // [N] or null (uniform G0)
    const T* eta;   // [N] or null (uniform eta_dt0)
    const T* crho;  // [N] or null (uniform crho0)
    T G0, eta_dt0, crho0, inv_dt;
    long long N;
    int nx, ny, nz, L, Ts;
    PmlAxis<T> ax[3];
    // band boxes for pass 2: [6] x (i0, i1, j0, j1, k0, k1) and prefix counts
    int box[6][6];
    long long start[7];
};

__device__ __forceinline__ int slab_of(int i, int n, int Ts) { return i < Ts ? i : Ts + (i - (n - 1 - Ts)); }

// slab-cell index of (position s along the axis, the other two coordinates)
__device__ __forceinline__ long long slab_index(int a, int s, int i, int j, int k, int nx, int ny, int Ts) {
    if (a == 0) return s + (long long)(2 * Ts) * (j + (long long)ny * k);
    if (a == 1) return i + (long long)nx * (s + (long long)(2 * Ts) * k);
    return i + (long long)nx * (j + (long long)ny * s);
}

// The layer pass: the layer cells, enumerated box by box (each cell once).
// With no sponge the plain update is linear in acc (w' = w + (dt^2/rho) acc),
// so the cell only adds the layer's part to what the step kernel wrote:
// acc_layer - acc_plain = sum over the axes whose layer holds the cell of
// (psi differences) / h + phi, where psi on the cell's two faces and phi
// advance with that axis's fluxes and full stretched divergence.  Axes whose
// layer does not hold the cell are left to the step kernel (there psi = phi
// = 0).  The face towards the wall is the cell's to write (in the low layer
// its face i - 1/2, in the high layer i + 1/2); the face at the layer's
// inner edge has c = 0 and keeps its zero.
template <typename T>
__global__ __launch_bounds__(256) void pml_cell_kernel(const PmlArgs<T> a) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.start[6]) return;
    int b = 0;
    while (t >= a.start[b + 1]) ++b;
    const int* bx = a.box[b];
    const int ex = bx[1] - bx[0] + 1, ey = bx[3] - bx[2] + 1;
    const long long lt = t - a.start[b];
    const int i = bx[0] + (int)(lt % ex);
    const int j = bx[2] + (int)((lt / ex) % ey);
    const int k = bx[4] + (int)(lt / ((long long)ex * ey));
    const int pos[3] = {i, j, k};
    const long long cell = i + (long long)a.nx * (j + (long long)a.ny * k);
    const long long strides[3] = {1, a.nx, (long long)a.nx * a.ny};
    const T Gc = a.G ? a.G[cell] : a.G0;
    const T eta_dt = a.eta ? a.eta[cell] * a.inv_dt : a.eta_dt0;
    const T cr = a.crho ? a.crho[cell] : a.crho0;
    T dacc[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int A = 0; A < 3; ++A) {
        const PmlAxis<T>& X = a.ax[A];
        const int ia = pos[A];
        if (!(ia <= a.L || ia >= X.n - 1 - a.L)) continue;
        const bool low = ia <= a.L;
        const long long st = strides[A];
        const T Gm = a.G ? harm2<T>(Gc, a.G[cell - st]) : a.G0;
        const T Gp = a.G ? harm2<T>(Gc, a.G[cell + st]) : a.G0;
        const long long mp = slab_index(A, slab_of(ia, X.n, a.Ts), i, j, k, a.nx, a.ny, a.Ts);      // face ia + 1/2, cell ia
        const long long mm = slab_index(A, slab_of(ia - 1, X.n, a.Ts), i, j, k, a.nx, a.ny, a.Ts);  // face ia - 1/2
        const long long mo = low ? mm : mp;                                                            // the face this cell writes
        const T bc = X.tab[ia], cc = X.tab[X.n + ia];
        const T bfm = X.tab[2 * X.n + ia - 1], cfm = X.tab[3 * X.n + ia - 1];
        const T bfp = X.tab[2 * X.n + ia], cfp = X.tab[3 * X.n + ia];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const long long o = c * a.N;
            const T uc = a.u[o + cell], wc = a.w[o + cell];
            const T Fp = Gp * ((a.u[o + cell + st] - uc) * X.ih), Fm = Gm * ((uc - a.u[o + cell - st]) * X.ih);
            const T Wp = (a.w[o + cell + st] - wc) * X.ih, Wm = (wc - a.w[o + cell - st]) * X.ih;
            const T pe_p = bfp * X.psin[c * X.M + mp] + cfp * Fp, pe_m = bfm * X.psin[c * X.M + mm] + cfm * Fm;
            const T pw_p = bfp * X.psin[(3 + c) * X.M + mp] + cfp * Wp;
            const T pw_m = bfm * X.psin[(3 + c) * X.M + mm] + cfm * Wm;
            X.psout[c * X.M + mo] = low ? pe_m : pe_p;
            X.psout[(3 + c) * X.M + mo] = low ? pw_m : pw_p;
            const T D = ((Fp + pe_p) - (Fm + pe_m)) * X.ih + eta_dt * (((Wp + pw_p) - (Wm + pw_m)) * X.ih);
            T* ph = X.phi + c * X.M + mp;
            const T phi = bc * *ph + cc * D;
            *ph = phi;
            dacc[c] += ((pe_p - pe_m) + eta_dt * (pw_p - pw_m)) * X.ih + phi;
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const long long o = c * a.N;
        const T d = cr * dacc[c];
        a.wn[o + cell] += d;
        a.un[o + cell] += d;
    }
}

// Profile coefficients (FP64) of one axis: cells i and faces i + 1/2.
void axis_table(int n, int L, double h, double cmax, double dt, double R, double alpha, std::vector<double>& tab) {
    const double d0 = 3.0 * cmax * std::log(1.0 / R) / (2.0 * L * h);
    tab.assign((size_t)4 * n, 0.0);
    auto coef = [&](double x, double* b, double* c) {
        const double q = std::max((L + 0.5 - x) / L, (x - (n - 1.5 - L)) / L);
        if (!(q > 0.0)) {
            *b = 1.0;
            *c = 0.0;
            return;
        }
        const double d = d0 * q * q;
        *b = std::exp(-(d + alpha) * dt);
        *c = d > 0.0 ? d / (d + alpha) * (*b - 1.0) : 0.0;
    };
    for (int i = 0; i < n; ++i) coef((double)i, &tab[(size_t)i], &tab[(size_t)n + i]);
    for (int i = 0; i + 1 < n; ++i) coef(i + 0.5, &tab[(size_t)2 * n + i], &tab[(size_t)3 * n + i]);
    tab[(size_t)3 * n - 1] = 1.0;  // no face past the last node
    tab[(size_t)4 * n - 1] = 0.0;
}

template <typename T>
hipError_t build_t(kvs_ctx* c) {
    const kvs_grid& g = c->grid;
    const int ext[3] = {(int)g.nx, (int)g.ny, (int)g.nz};
    const double hh[3] = {g.hx, g.hy, g.hz};
    const double alpha = c->pml_alpha >= 0.0 ? c->pml_alpha : kvs_pml_default_alpha(g, c->cmax, c->pml_cells);
    std::vector<T> all;
    for (int A = 0; A < 3; ++A) {
        std::vector<double> tab;
        axis_table(ext[A], c->pml_cells, hh[A], c->cmax, c->dt, c->pml_R, alpha, tab);
        for (double v : tab) all.push_back((T)v);
    }
    hipError_t e = hipMemcpyAsync(c->pml_tab, all.data(), sizeof(T) * all.size(), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return e;
}

template <typename T>
hipError_t launch_t(kvs_ctx* c) {
    const kvs_grid& g = c->grid;
    PmlArgs<T> a{};
    const int nb = 1 - c->cur;
    a.u = static_cast<const T*>(c->u[c->cur]);
    a.w = static_cast<const T*>(c->w[c->cur]);
    a.un = static_cast<T*>(c->u[nb]);
    a.wn = static_cast<T*>(c->w[nb]);
    a.G = c->hetero ? static_cast<const T*>(c->G) : nullptr;
    a.eta = c->hetero && c->viscous ? static_cast<const T*>(c->eta) : nullptr;
    a.crho = c->hetero ? static_cast<const T*>(c->crho) : nullptr;
    a.G0 = T(c->G0);
    a.eta_dt0 = c->hetero ? T(0) : T(c->eta0 / c->dt);
    a.crho0 = T(c->dt * c->dt / c->rho0);
    a.inv_dt = T(1.0 / c->dt);
    a.N = (long long)c->N;
    a.nx = (int)g.nx;
    a.ny = (int)g.ny;
    a.nz = (int)g.nz;
    a.L = c->pml_cells;
    a.Ts = c->pml_cells + 1;
    const int ext[3] = {a.nx, a.ny, a.nz};
    const double hh[3] = {g.hx, g.hy, g.hz};
    // memory per axis: face-memory buffers 0 and 1 (6 slabs each), then phi
    // (3 slabs); this step reads the buffer of the state's parity
    const T* tab = static_cast<const T*>(c->pml_tab);
    T* mem = static_cast<T*>(c->pml_mem);
    for (int A = 0; A < 3; ++A) {
        const long long M = kvs_pml_slab_cells(g, c->pml_cells, A);
        a.ax[A].tab = tab;
        a.ax[A].psin = mem + (c->cur ? 6 * M : 0);
        a.ax[A].psout = mem + (c->cur ? 0 : 6 * M);
        a.ax[A].phi = mem + 12 * M;
        a.ax[A].n = ext[A];
        a.ax[A].ih = T(1.0 / hh[A]);
        a.ax[A].M = M;
        tab += 4 * ext[A];
        mem += 15 * M;
    }
    const int L = a.L, nx = a.nx, ny = a.ny, nz = a.nz;
    const int boxes[6][6] = {
        {1, nx - 2, 1, ny - 2, 1, L},
        {1, nx - 2, 1, ny - 2, nz - 1 - L, nz - 2},
        {1, nx - 2, 1, L, L + 1, nz - 2 - L},
        {1, nx - 2, ny - 1 - L, ny - 2, L + 1, nz - 2 - L},
        {1, L, L + 1, ny - 2 - L, L + 1, nz - 2 - L},
        {nx - 1 - L, nx - 2, L + 1, ny - 2 - L, L + 1, nz - 2 - L},
    };
    a.start[0] = 0;
    for (int b = 0; b < 6; ++b) {
        for (int q = 0; q < 6; ++q) a.box[b][q] = boxes[b][q];
        const long long v = (long long)(boxes[b][1] - boxes[b][0] + 1) * (boxes[b][3] - boxes[b][2] + 1) *
                            (boxes[b][5] - boxes[b][4] + 1);
        a.start[b + 1] = a.start[b] + v;
    }
    hipLaunchKernelGGL(pml_cell_kernel<T>, dim3((unsigned)((a.start[6] + 255) / 256)), dim3(256), 0, c->stream, a);
    return hipGetLastError();
}

}  // namespace

double kvs_pml_default_alpha(const kvs_grid& g, double cmax, int L) {
    return 3.14159265358979323846 * cmax / (10.0 * L * std::min(g.hx, std::min(g.hy, g.hz)));
}

int64_t kvs_pml_slab_cells(const kvs_grid& g, int L, int axis) {
    const int64_t T2 = 2 * (int64_t)(L + 1);
    if (axis == 0) return T2 * g.ny * g.nz;
    if (axis == 1) return g.nx * T2 * g.nz;
    return g.nx * g.ny * T2;
}

hipError_t kvs_pml_build(kvs_ctx* c) { return c->prec == KVS_FP32 ? build_t<float>(c) : build_t<double>(c); }

hipError_t kvs_launch_pml(kvs_ctx* c, double gn) {
    (void)gn;  // the force term is the step kernel's; the layer changes the stencil terms only
    return c->prec == KVS_FP32 ? launch_t<float>(c) : launch_t<double>(c);
}
