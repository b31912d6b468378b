// Internal declarations of the kvs library (host side + kernel launchers).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "kvs.h"

// Device-side control block of one projection solve.  Written only by the
// single-block finalize kernels; read by every CG kernel (early exit once
// `done` is set) and copied to the host once per chunk of iterations.
struct CgState {
    double s1, s2, s3;      // finalized sums of the last reduction
    double rr, rr0, rz;     // r.r, r0.r0, r.z
    double bb;              // ||b||^2
    double pAp, alpha, beta;
    double tol2;            // tol^2 (compared with rr / bb)
    double relres_true2;    // ||-b - A phi||^2 / ||b||^2
    double net_in, net_out; // flexible PCG: network input / output scales
    double n_interior;      // interior cells (for the RMS of r)
    double h2;              // grid spacing^2 (network output scale)
    double dinv;            // 1 / diag(A)
    long long iters, max_iter, fixed_iters;
    int done, status, jacobi, flexible;
    int zjacobi;            // flexible PCG: this iteration's z is r / diag(A)
    int fallbacks;          // number of Jacobi fallbacks taken
};

// Device memory of a context or batch: the caller's allocator when kvs_opts
// names one, else hipMalloc / hipFree.  Before handing a buffer back to the
// caller's allocator the stream is synchronised, so that no queued kernel
// still uses it whatever the allocator's stream semantics (hipFree
// synchronises by itself).
struct KvsMem {
    void* (*alloc)(size_t, void*) = nullptr;
    void (*release)(void*, void*) = nullptr;
    void* user = nullptr;
    hipStream_t stream = nullptr;

    hipError_t get(void** p, size_t bytes) const {
        if (!alloc) return hipMalloc(p, bytes);
        *p = bytes ? alloc(bytes, user) : nullptr;
        return (*p || !bytes) ? hipSuccess : hipErrorOutOfMemory;
    }
    template <typename P>
    hipError_t get(P** p, size_t bytes) const {
        void* q = nullptr;
        const hipError_t e = get(&q, bytes);
        *p = static_cast<P*>(q);
        return e;
    }
    void put(void* p) const {
        if (!p) return;
        if (!alloc) {
            (void)hipFree(p);
            return;
        }
        if (stream) (void)hipStreamSynchronize(stream);
        release(p, user);
    }
};

struct kvs_ctx {
    kvs_grid grid{};
    KvsMem mem;  // where the context's device buffers come from
    int64_t N = 0;
    int prec = KVS_FP64;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;

    // sponge
    int sponge_cells = 0;
    double sigma_user = -1.0;
    double sigma_max = 0.0;

    // medium
    bool have_material = false;
    bool hetero = false;
    bool viscous = false;
    double G0 = 0, rho0 = 0, eta0 = 0;
    void* G = nullptr;     // [N] T, hetero only
    void* eta = nullptr;   // [N] T
    void* rho_t = nullptr; // [N] T: rho
    void* crho = nullptr;  // [N] T: dt^2/rho
    double dt_max = 0.0;
    double dt = 0.0;
    bool have_dt = false;

    // state: u[b], w[b] each 3N of T, b = cur or 1 - cur
    void* u[2] = {nullptr, nullptr};
    void* w[2] = {nullptr, nullptr};
    int cur = 0;
    int64_t step = 0;

    // force and projection
    double* F = nullptr;  // [3N] double
    bool have_force = false;
    void* FS = nullptr;   // [3N] T
    bool fs_current = false;
    std::vector<double> env;  // host copy of g[n]

    double* phi = nullptr;
    double* r = nullptr;
    double* r2 = nullptr;  // flexible PCG: the residual of the previous iteration (ping-pong with r)
    double* p[2] = {nullptr, nullptr};
    double* Ap = nullptr;
    double* partials = nullptr;  // 3 * npart
    int64_t npart = 0;
    CgState* cgs = nullptr;       // device
    CgState* cgs_host = nullptr;  // pinned host mirror
    bool have_phi = false;

    // probes: flat cell indices on device, traces [step][probe][ncomp] doubles
    int64_t* probe_cells = nullptr;
    int64_t nprobes = 0;
    int probe_comp = 2;
    // trace slot that the probe blocks of the step launch being issued fill
    // with the launch's input state (null: no probe blocks)
    double* probe_fused_out = nullptr;
    double* traces = nullptr;
    int64_t trace_cap = 0;    // steps of capacity
    int64_t trace_steps = 0;  // steps recorded
    // two-step launches: the probe cells by grid row, for the threads that
    // form the intermediate state (rowtab [nz][ny][ceil(nx / 64)]: the offset
    // into ptab of row (j, k) where that 64-cell segment of it holds a probe,
    // else -1; ptab: per probed row nx probe indices or -1); only when the
    // probe cells are distinct and off the planes k = 0, nz - 1 (probe_rows_ok)
    int* probe_rowtab = nullptr;
    int* probe_ptab = nullptr;
    bool probe_rows_ok = true;
    // trace slot for the intermediate state of the two-step launch being
    // issued (null: no probes)
    double* probe_mid_out = nullptr;

    // kernel timing
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<int> ev_steps;  // steps advanced by the launch of each event pair
    int64_t ev_used = 0;
    double timed_ms = 0.0;
    int64_t timed_launches = 0;  // steps advanced by the timed launches
    // the same split by kind: [0] one-step launches, [1] two-step launches
    // (summed ms and launch counts)
    double timed_ms_kind[2] = {0.0, 0.0};
    int64_t timed_n_kind[2] = {0, 0};

    // learned preconditioner (borrowed; set by kvs_set_preconditioner)
    kvs_unet* net = nullptr;
    int64_t last_fallbacks = 0;  // Jacobi fallbacks in the last flexible solve

    // tuning of the step kernel: shape variant, z planes per block (0: fill
    // whole rounds of resident blocks), XCD-contiguous tile order
    int step_variant = 0;
    int step_zchunk = 0;
    int step_remap = 1;
    // steps per launch where the two-step kernel applies (1 or 2)
    int step_block = 2;
    // storage of the projection's CG search direction (KVS_FP64 or KVS_FP32;
    // set to the state precision at creation); p_dirty: both direction
    // buffers are cleared before the next solve (after a change, the other
    // width's view would find the last solve's values on its outer planes)
    int dir_prec = 0;
    bool p_dirty = false;
    // storage of the projection's residual (with the flexible PCG, also of the
    // network's output z); r_view32: the last solve viewed r and r2 as FP32
    int res_prec = 0;
    bool r_view32 = false;
    // when set, the next step-kernel launch records its own start and end in
    // these events (the dispatch's timestamps, no extra queue packets)
    hipEvent_t launch_ev[2] = {nullptr, nullptr};

    // running peak of |u| on registered grid planes: one map of T per plane,
    // concatenated in registration order (peak_off[p] = first cell of plane p)
    int npeak = 0;
    int peak_axis[KVS_MAX_PEAK_PLANES] = {};
    int64_t peak_index[KVS_MAX_PEAK_PLANES] = {};
    int64_t peak_off[KVS_MAX_PEAK_PLANES] = {};
    int64_t peak_cells = 0;
    void* peak = nullptr;

    // acoustic radiation force: running FP64 sums over the acoustic samples,
    // [N] (plane-wave form: p^2) or [3][N] (Poynting form: p v_i)
    int arf_mode = 0;  // 0: none, KVS_ARF_PLANE, KVS_ARF_POYNTING
    double* arf_sum = nullptr;
    int64_t arf_sum_cap = 0;  // doubles allocated
    int64_t arf_samples = 0;

    // acoustic strain peaks: K (1 or N doubles, stride strain_sK), peaks [2][N]
    // (|eps|, then |grad eps|)
    double* strain_K = nullptr;
    int strain_sK = 0;
    int64_t strain_K_cap = 0;
    double* strain_peak = nullptr;
    int64_t strain_samples = 0;
    bool strain_on = false;

    // absorbing layer (C-PML): cells per face (0 = off), theoretical
    // reflection, frequency shift (< 0: default); coefficient tables [axis][4][n]
    // (rebuilt when dt, material or layer change) and the memory variables of
    // the three axes' slabs [axis][9][slab cells], in the state precision
    int pml_cells = 0;
    double pml_R = 1e-5, pml_alpha = -1.0;
    double cmax = 0.0;  // largest shear speed of the material
    bool pml_dirty = true;
    void* pml_tab = nullptr;
    void* pml_mem = nullptr;
    int64_t pml_mem_count = 0;
};

// Plane table handed to the peak kernel by value: axis, index along it, the
// in-plane extents (n1 fastest) and the map offset of every plane.
struct PeakPlanes {
    int axis[KVS_MAX_PEAK_PLANES];
    long long index[KVS_MAX_PEAK_PLANES];
    long long n1[KVS_MAX_PEAK_PLANES];
    long long n2[KVS_MAX_PEAK_PLANES];
    long long off[KVS_MAX_PEAK_PLANES];
};

inline int ncomp_of(int comp) { return comp == 3 ? 3 : 1; }

// A batch of homogeneous instances advanced together (one launch per step
// covering every instance's tiles, the step loop replayed as a hipGraph).
struct kvs_batch {
    std::vector<kvs_ctx*> inst;
    KvsMem mem;  // where the batch's own device tables come from
    int device = 0;
    int prec = KVS_FP32;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    int comp = 2;
    int64_t step = 0;  // common step index of all instances
    bool small_ok = true;  // use the persistent one-block-per-instance run when every instance fits
    int variant = 1;   // tile shape (index into the step-kernel variants), or
                       // KVS_BATCH_FIT_ROWS: each instance's tile fitted to its x rows
    int zchunk = 32;   // z planes per block

    // device tables (rebuilt when the instances' parameters change)
    void* dev_params = nullptr;  // BatchInst<T>[n], then the envelopes
    size_t params_bytes = 0;
    void* dev_work = nullptr;    // int4[nwork], instances grouped by tile shape
    int nwork = 0;
    // one launch per group: tile shape id and the group's slice of the work list
    struct Group {
        int shape, off, count;
    };
    std::vector<Group> groups;
    bool viscous = false;
    // probes: flat (instance, cell) list and traces [slot][nprobes] doubles
    std::vector<int64_t> probe_inst, probe_cell;
    std::vector<int64_t> probe_first;  // first probe of instance i (size n+1)
    void* dev_probes = nullptr;        // int64 pairs
    double* traces = nullptr;
    int64_t trace_cap = 0, trace_steps = 0;
    std::vector<double> host_traces;  // host copy of the traces, valid while
    bool host_traces_valid = false;   // no step, reset or probe change happened
    // cached graph for (start step, nsteps, first trace slot) and the per-step
    // force switch it was captured with (a step launches the force-reading
    // kernel when any instance's envelope is non-zero there)
    hipGraphExec_t graph = nullptr;
    bool graph_valid = false;
    int64_t graph_start = -1, graph_steps = 0, graph_trace0 = -1;
    std::vector<uint8_t> graph_force;  // the per-step launch plan (see kvs_batch_run)

    // two steps per launch: requested (1 or 2), and whether the batch allows
    // it (set by kvs_batch_prepare: FP32, viscous, rows <= 256 cells, probe
    // cells distinct and off the planes k = 0, nz - 1); the instances'
    // two-step arguments [parity], the work list of (instance, row pair,
    // z segment) grouped by tile width, and the probe row tables
    int step_block = 2;
    bool two_ok = false;
    void* dev_params2 = nullptr;
    size_t params2_bytes = 0;
    void* dev_work2 = nullptr;
    int nwork2 = 0;
    std::vector<Group> groups2;  // shape = wavefronts per row (2, 3 or 4)
    int* dev_ptabs2 = nullptr;   // row tables and probe tables of all instances
    std::vector<int64_t> rowtab2_off, ptab2_off;  // per instance, into dev_ptabs2 (-1: none)
    bool probes2_ok = true;      // the registered probes allow two-step launches
};

// ---- launchers (kvs_force.hip) ------------------------------------------
// Write the closed-form force pattern into c->F (3N doubles) on c's stream.
hipError_t kvs_launch_force_pattern(kvs_ctx* c, const kvs_force_pattern* p);

// ---- launchers (kvs_step.hip) -------------------------------------------
// One FDTD step from (u[cur], w[cur]) into (u[1-cur], w[1-cur]) with source
// amplitude gn (0: no force read).  Returns the launch error.
hipError_t kvs_launch_step(kvs_ctx* c, double gn);
// two steps in one launch (kvs_step2.hip), for two steps without force:
// whether the precision, medium, layer, peak maps, probes and grid allow it
bool kvs_step2_supported(const kvs_ctx* c);
hipError_t kvs_launch_step2(kvs_ctx* c);
hipError_t kvs_launch_step_variant(kvs_ctx* c, double gn, int variant);
int kvs_step_variant_count();
void kvs_step_variant_shape(int variant, int* by, int* vec, int* wx);
hipError_t kvs_launch_probe_gather(kvs_ctx* c, const void* u_new, int64_t slot);
// Fold |u_new| into the running peak maps of the registered planes.
hipError_t kvs_launch_peak_update(kvs_ctx* c, const void* u_new);
hipError_t kvs_launch_crho(kvs_ctx* c);
hipError_t kvs_launch_cast_material(kvs_ctx* c, const double* dG, const double* drho, const double* deta);
hipError_t kvs_launch_cast(kvs_ctx* c, const double* src, void* dst, int64_t n);
hipError_t kvs_launch_widen(kvs_ctx* c, const void* src, double* dst, int64_t n);
hipError_t kvs_launch_f32_to_f64(kvs_ctx* c, const float* src, double* dst, int64_t n);
hipError_t kvs_launch_zero_boundary(kvs_ctx* c, void* field3);
// stable dt: per-cell bound reduced to its minimum in *out (device double)
// acoustic radiation force (kvs_arf.hip): fold nsamp samples (dtype 0 =
// double, 1 = float; p [nsamp][N], v [nsamp][3][N] in the Poynting form) into
// c->arf_sum; then write F from the sums with coefficient maps of stride 0
// (uniform) or 1 (per cell), an optional mask and the unit beam direction d
hipError_t kvs_launch_arf_accumulate(kvs_ctx* c, const void* p, const void* v, int64_t nsamp, int dtype);
// peak strain maps (kvs_arf.hip): fold nsamp pressure samples (dtype 0 =
// double, 1 = float, [nsamp][N]) into c->strain_peak with c->strain_K
hipError_t kvs_launch_strain(kvs_ctx* c, const void* p, int64_t nsamp, int dtype);
// square roots of the gradient map (stored as squares) into out (device, N)
hipError_t kvs_launch_strain_roots(kvs_ctx* c, double* out);
// absorbing layer (kvs_pml.hip): default frequency shift, slab cells of an
// axis, coefficient tables from dt and the material, and the layer pass of
// one step (after kvs_launch_step, before the buffers flip)
double kvs_pml_default_alpha(const kvs_grid& g, double cmax, int L);
int64_t kvs_pml_slab_cells(const kvs_grid& g, int L, int axis);
hipError_t kvs_pml_build(kvs_ctx* c);
hipError_t kvs_launch_pml(kvs_ctx* c, double gn);
hipError_t kvs_launch_arf_force(kvs_ctx* c, const double* alpha, int sa, const double* cs, int sc, const double* rho,
                                int sr, const unsigned char* mask, double n_pulse, const double d[3]);
// curl-based initial state (kvs_init.hip): u[cur] = 0, w[cur] = dt curl_h A
// (A: device, 3N doubles)
hipError_t kvs_launch_curl_state(kvs_ctx* c, const double* A);
hipError_t kvs_launch_stable_dt(kvs_ctx* c, const double* dG, const double* drho, const double* deta,
                                double* partial, int64_t npartial, double* out);

// batched stepping (kvs_step.hip): refresh the device parameter table, then
// replay (or capture) the graph of nsteps steps starting at b->step
hipError_t kvs_batch_prepare(kvs_batch* b);
hipError_t kvs_batch_trial_launch(kvs_batch* b);
// Runs nsteps steps; *flips = launches that advanced the state (each swaps
// the current and next buffers once).
hipError_t kvs_batch_run(kvs_batch* b, int64_t nsteps, int64_t* flips);
// Whether the batch's instances allow two-step launches (precision, medium,
// row width, probes); the step loop also needs steps without force.
bool kvs_batch_two_step_supported(const kvs_batch* b);
// True when kvs_batch_run takes the persistent path (every instance's state
// fits one workgroup's LDS and the path is enabled).
bool kvs_batch_small_path(const kvs_batch* b);

// ---- learned preconditioner (kvs_unet.hip) ---------------------------------
// Inner products the flexible PCG needs from the preconditioned residual z,
// accumulated by the network's output kernel as it writes z (interior cells,
// FP64): partial sums z.r, z.r_old and r.r_old per block at part[block],
// part[npart + block], part[2 npart + block].  r_old = null: z.r only.
struct UnetDots {
    const void* r_old;  // the previous residual, stored as the r it comes with
    double* part;
    int npart;
};
// z = out_scale * U(in_scale * r) on the context grid, scales read from
// device memory, every kernel returns at once while *stop is set; with
// dots != null also the partial sums above, over *nblocks blocks.
hipError_t kvs_unet_precondition(kvs_unet* u, const double* r, double* z, const kvs_grid& g, const double* in_scale,
                                 const double* out_scale, const int* stop, hipStream_t s, const UnetDots* dots = nullptr,
                                 int* nblocks = nullptr);
// The same with FP32 storage: r (and dots->r_old) FP32, and z_sum the FP32
// network output before the output scale (z = out_scale * z_sum).
hipError_t kvs_unet_precondition32(kvs_unet* u, const float* r, float* z_sum, const kvs_grid& g,
                                   const double* in_scale, const double* out_scale, const int* stop, hipStream_t s,
                                   const UnetDots* dots = nullptr, int* nblocks = nullptr);
// Blocks of the network's output kernel on a grid (the partial sums above).
int64_t kvs_unet_out_blocks(const kvs_grid& g);

// ---- projection (kvs_cg.hip) ---------------------------------------------
kvs_status kvs_run_projection(kvs_ctx* c, const kvs_solve_opts* o, kvs_solve_report* rep);
int64_t kvs_cg_partials_needed(const kvs_grid& g);
