/*
 * kvs.h -- C ABI of the MI355X (gfx950) reduced Kelvin-Voigt shear-wave
 * solver.
 *
 * The library advances the reduced Kelvin-Voigt shear equation
 *     rho u_tt = div(G grad u) + eta lap(u_t) + f_S                    (1)
 * (the paper's reduced shear equation, Sec. 2.4, with spatially varying
 * G = mu, rho and eta) by the explicit leapfrog of Sec. 3.1, and makes the
 * body force solenoidal by the Helmholtz projection of Sec. 3.2:
 *     lap phi = div f,   f_S = f - grad phi,                           (2)
 * solved matrix-free by conjugate gradient (Sec. 3.2.3).  For a separable
 * force f = b0(x) g(t) the projection is computed once and scaled per step
 * (Sec. 3.3, eq. projected_separable).
 *
 * Discretisation (shared by every entry point):
 *   - Grid of nx*ny*nz cell-centred nodes with spacings hx, hy, hz [m].
 *     Scalar fields are laid out [nz][ny][nx] (x fastest, flat index
 *     i + nx*(j + ny*k)); vector fields are [3][nz][ny][nx] (x, y, z
 *     components, each a contiguous scalar field).
 *   - The outer layer of nodes (i in {0, nx-1}, same for j, k) is the
 *     Dirichlet layer of Sec. 3.5: u = 0 there at all times.
 *   - 7-point Laplacian; div(G grad u) with the harmonic mean of G on each
 *     face; viscous term eta * lap(w)/dt with w = u^n - u^{n-1} (backward
 *     difference velocity of Sec. 3.1).
 *   - State is kept in summed form (u^n, w^n = u^n - u^{n-1}):
 *       w^{n+1} = [(1 - s) w^n + (dt^2/rho)(E(u^n) + eta lap(w^n)/dt
 *                   + g_n f_S)] / (1 + s),   u^{n+1} = u^n + w^{n+1},
 *     which is the leapfrog u^{n+1} = 2u^n - u^{n-1} + dt^2 a^n plus a
 *     centred velocity damping s = sigma dt / 2 (sponge, see kvs_opts).
 *   - Projection: b = centred divergence of F on interior nodes; CG on
 *     A phi = -b with A = -lap_h (the paper's A, with the sign that makes
 *     lap phi = div f hold); f_S,a = (F_a(-a) + 2 F_a + F_a(+a))/4
 *     - (phi(+a) - phi(-a))/(2 h_a) on interior nodes, 0 on the outer layer
 *     (the cell average of the face field avg(F) - D+ phi, whose face
 *     divergence is the CG residual).
 *
 * Precision: KVS_FP64 keeps everything in double.  KVS_FP32 keeps the
 * stencil state (u, w), material and f_S in float, and the projection (F,
 * b, phi, CG vectors, inner products, residual norms, the phi-gradient
 * subtraction) in double.
 *
 * Conventions for every function:
 *   - Returns kvs_status; KVS_OK == 0.  No C++ exception crosses the ABI.
 *     On error the context (when there is one) keeps a message readable by
 *     kvs_last_error().
 *   - Host pointers are borrowed for the duration of the call only; the
 *     library copies what it needs and never frees them.
 *   - "*_device" pointers are device memory owned by the caller, read
 *     asynchronously on the context's stream; the caller keeps them alive
 *     until kvs_synchronize() returns.
 *   - The context owns every device buffer it allocates (through the
 *     allocator named in kvs_opts, else hipMalloc) and releases them in
 *     kvs_destroy().
 *   - A context is not thread-safe; distinct contexts are independent.
 *     All GPU work of a context is ordered on its stream.
 */
#ifndef KVS_H
#define KVS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kvs_ctx kvs_ctx;
typedef struct kvs_unet kvs_unet;

typedef enum {
    KVS_OK = 0,
    KVS_EINVAL = 1,      /* bad argument: sizes, non-finite / non-positive G or rho, eta < 0, probe outside grid */
    KVS_ENOMEM = 2,      /* device or host allocation failed */
    KVS_EDEVICE = 3,     /* HIP runtime error, or no GPU / wrong architecture */
    KVS_ENOTCONV = 4,    /* CG reached max_iter above tolerance (phi and f_S are still produced) */
    KVS_EBREAKDOWN = 5,  /* CG guard fired: p.Ap <= 0 or a non-finite inner product (Sec. 3.2.3) */
    KVS_EUNSTABLE = 6,   /* dt above the stability limit */
    KVS_ESTATE = 7       /* call order: material, dt, or a current projection missing */
} kvs_status;

typedef enum { KVS_FP64 = 0, KVS_FP32 = 1 } kvs_precision;
typedef enum { KVS_PC_NONE = 0, KVS_PC_JACOBI = 1, KVS_PC_UNET = 2 } kvs_precond;

typedef struct {
    int64_t nx, ny, nz; /* nodes per axis, each >= 3 */
    double hx, hy, hz;  /* spacings [m], > 0 */
} kvs_grid;

typedef struct {
    int32_t precision;       /* kvs_precision */
    int32_t sponge_cells;    /* L >= 0: linear damping ramp over L cells from every face (0 = none) */
    double sponge_sigma_max; /* ramp peak [1/s]; < 0 selects 6 ln(10) c_max / (L h_min), which makes
                                the one-way amplitude factor through the ramp about 10^-1.5 */
    int32_t device;          /* HIP device ordinal */
    void* stream;            /* hipStream_t to run on, or NULL: the context creates its own */
    /* Device-memory allocator for every buffer the context (or batch) owns, e.g. a framework's
     * caching allocator; NULL (both) selects hipMalloc / hipFree.  alloc(bytes, alloc_user)
     * returns device memory of the opts' device (NULL: KVS_ENOMEM); free(ptr, alloc_user) takes
     * back exactly what alloc returned, on the creating thread's calls, after the library has
     * synchronised its stream; every buffer is returned by kvs_destroy at the latest.  Must
     * stay callable until then.  Only one of the two set: KVS_EINVAL.  The network of
     * kvs_unet_create keeps its own buffers (hipMalloc). */
    void* (*alloc)(size_t bytes, void* user);
    void (*free)(void* ptr, void* user);
    void* alloc_user;
} kvs_opts;

typedef struct {
    double tol;          /* stop when sqrt(r.r / b.b) < tol: the relative residual of Sec. 3.2.3,
                            whose r0 = b for phi_0 = 0, kept relative to b under a warm start */
    int64_t max_iter;    /* > 0 */
    int32_t precond;     /* kvs_precond: NONE = the paper's CG; JACOBI = z = r / diag(A); UNET = flexible
                            PCG with the network set by kvs_set_preconditioner */
    int64_t fixed_iters; /* > 0: run exactly this many iterations, ignore tol (parity mode) */
    int32_t warm_start;  /* != 0: start from the previous phi instead of phi_0 = 0 */
    int32_t confirm_true; /* != 0: once the recursive residual meets tol, recompute the true residual
                             ||-b - A phi|| / ||b|| in FP64 and, while it is still >= tol, restart the
                             iteration from it (iterations keep counting up to max_iter).  Always on
                             for precond = UNET, whose recursive residual can drift from the true one;
                             0 keeps the paper's stop rule on the recursive residual alone. */
} kvs_solve_opts;

typedef struct {
    int64_t iters;           /* phi updates performed */
    double relres_recursive; /* sqrt(r.r / b.b) at exit, r the recursively updated residual */
    double relres_true;      /* ||-b - A phi|| / ||b|| recomputed from phi, FP64 */
    double ms;               /* wall time of divergence + solve + gradient subtraction */
    int32_t status;          /* kvs_status of the solve */
} kvs_solve_report;

/* ---- lifetime ---------------------------------------------------------- */

/* Create a solver for `grid` on opts->device (NULL opts: FP64, no sponge,
 * device 0, own stream).  Allocates the state (zeroed: the medium starts at
 * rest), force and projection buffers.  Fails with KVS_EDEVICE when the
 * device is not a gfx950 GPU. */
kvs_status kvs_create(const kvs_grid* grid, const kvs_opts* opts, kvs_ctx** out);
void kvs_destroy(kvs_ctx* ctx);
const char* kvs_status_string(kvs_status s);
const char* kvs_last_error(const kvs_ctx* ctx);
/* Block until all work queued on the context's stream is done. */
kvs_status kvs_synchronize(kvs_ctx* ctx);
/* The grid the context was created with (sizes and spacings). */
kvs_status kvs_get_grid(const kvs_ctx* ctx, kvs_grid* out);
/* The hipStream_t the context runs on. */
void* kvs_stream(const kvs_ctx* ctx);

/* ---- medium and time step (Sec. 2.4 coefficients, Sec. 3.1 bound) ------ */

/* Heterogeneous medium: host arrays of N = nx*ny*nz doubles each, G > 0 [Pa],
 * rho > 0 [kg/m^3], eta >= 0 [Pa s], all finite, else KVS_EINVAL.
 * Recomputes the stability limit and the default sponge strength; a time
 * step set earlier is re-checked against the new limit. */
kvs_status kvs_set_material(kvs_ctx* ctx, const double* G, const double* rho, const double* eta);
/* Homogeneous medium (no per-cell material traffic). */
kvs_status kvs_set_material_uniform(kvs_ctx* ctx, double G, double rho, double eta);
/* Largest dt with A + 2B <= 4 on every interior cell, where
 * A = 4 dt^2 (Gmax_face / rho) S, B = 4 dt (eta / rho) S, S = sum 1/h_a^2
 * and Gmax_face is the largest harmonic face modulus around the cell; for
 * eta = 0 this is the CFL bound (1/c_s)(sum 1/h_a^2)^(-1/2) of Sec. 3.1. */
kvs_status kvs_stable_dt(const kvs_ctx* ctx, double* dt_max);
/* The sponge ramp peak in use [1/s] (resolved default after set_material). */
kvs_status kvs_sponge_sigma_max(const kvs_ctx* ctx, double* sigma_max);
/* Set dt [s]; dt > dt_max (1 + 1e-12) gives KVS_EUNSTABLE and keeps the
 * previous dt. */
kvs_status kvs_set_dt(kvs_ctx* ctx, double dt);

/* ---- force and projection (Sec. 3.2, 3.3) ------------------------------ */

/* Body-force pattern b0 (or the current general force f^n): host, 3*N
 * doubles [3][nz][ny][nx] [N/m^3].  Marks the projected force stale. */
kvs_status kvs_set_force(kvs_ctx* ctx, const double* F);
/* Same from device memory: dtype 0 = double, 1 = float; copied on the
 * context's stream. */
kvs_status kvs_set_force_device(kvs_ctx* ctx, const void* F, int32_t dtype);
/* Force pattern from its closed form, generated on the device (replaces the
 * force and marks the projected force stale, like kvs_set_force): the focused
 * Gaussian push of a separable source (Sec. 3.3; the Gaussian excitation of
 * Sec. 4.4) and, with plane-wave modes, a modulated push whose parameters
 * change between re-projections (a general time-varying source f^n):
 *   F_axis = F0 exp(-lat^2 / (2 sigma_lateral^2) - ax^2 / (2 sigma_axial^2)) M,
 *   M = 1 + mod_amp sum_{m < n_modes} cos(k_m . x + phase_m),
 * other components 0; x = ((i - nx/2) hx, (j - ny/2) hy, (k - nz/2) hz) are
 * the node coordinates [m] (integer division nx/2), ax = x_axis - centre_axis,
 * lat^2 the sum of the squared offsets x_a - centre_a over the other two axes.
 * box_lateral >= 0: F = 0 where some lateral offset exceeds it in magnitude;
 * box_axial >= 0: likewise |ax|; < 0: no box.  FP64, evaluated in this order
 * without fused multiply-adds.  axis 0..2, sigmas > 0, 0 <= n_modes <=
 * KVS_MAX_FORCE_MODES, every value finite, else KVS_EINVAL.  Asynchronous on
 * the context's stream. */
#define KVS_MAX_FORCE_MODES 16
typedef struct {
    int32_t axis;          /* force component and beam axis, 0..2 */
    double F0;             /* peak [N/m^3] */
    double centre[3];      /* focus [m], node coordinates */
    double sigma_lateral;  /* [m] */
    double sigma_axial;    /* [m] */
    double box_lateral;    /* [m], < 0: none */
    double box_axial;      /* [m], < 0: none */
    int32_t n_modes;       /* plane-wave modulation modes */
    double mod_amp;        /* a in M = 1 + a sum cos(...) */
    double k[KVS_MAX_FORCE_MODES][3]; /* wave vectors [rad/m] */
    double phase[KVS_MAX_FORCE_MODES]; /* [rad] */
} kvs_force_pattern;
kvs_status kvs_set_force_pattern(kvs_ctx* ctx, const kvs_force_pattern* p);
/* Read back the force pattern (host, 3*N doubles).  No force: KVS_ESTATE.
 * Blocks. */
kvs_status kvs_get_force(const kvs_ctx* ctx, double* F);
/* Temporal envelope g[n] for steps n < n_env (absolute step index since the
 * state was last reset); steps n >= n_env use g = 0. n_env may be 0. */
kvs_status kvs_set_envelope(kvs_ctx* ctx, const double* g, int64_t n_env);
/* Project the current force: b = div F, CG solve, f_S = F - grad phi.
 * opts NULL: tol 1e-8, max_iter 10000, Jacobi-PCG.  ||b|| = 0 gives
 * 0 iterations, phi = 0.  Returns the solve status (KVS_OK, KVS_ENOTCONV,
 * KVS_EBREAKDOWN); f_S is produced in every case but EBREAKDOWN.  `report`
 * may be NULL. */
kvs_status kvs_project(kvs_ctx* ctx, const kvs_solve_opts* opts, kvs_solve_report* report);
/* Storage of the search direction p of the projection's CG (Sec. 3.2.3): KVS_FP64 or KVS_FP32
 * (other values: KVS_EINVAL); default: the context's state precision.  The residual r and phi
 * stay FP64 and are both updated with the stored direction, so r stays the residual of phi to
 * FP64 rounding and the stop rule, the inner products and the norms are as before; only the
 * direction is rounded to FP32, which the iteration absorbs like any other choice of
 * direction.  The two CG sweeps then move 52 instead of 64 B per cell and iteration.  Applies
 * from the next kvs_project. */
kvs_status kvs_set_direction_precision(kvs_ctx* ctx, int32_t prec);
/* Storage of the residual r of the projection's CG (Sec. 3.2.3): KVS_FP64 or KVS_FP32 (other
 * values: KVS_EINVAL); default: the context's state precision.  With FP32 the update's rounding
 * makes the recursive r drift from the true residual -b - A phi (phi stays FP64), so whenever
 * r.r has fallen 10^4-fold since r was last exact (checked where the host reads the solver
 * state), r is recomputed from phi in FP64 and the iteration continues with its direction
 * ("reliable update"); once the recursive residual meets tol, the true one is confirmed as with
 * confirm_true.  Inner products and norms are FP64.  In flexible PCG the network then reads the
 * FP32 r and its output z is stored as the FP32 sum before the output scale (the value is the
 * same).  With an FP32 direction the plain CG's sweeps move 40 B per cell and iteration.
 * Applies from the next kvs_project. */
kvs_status kvs_set_residual_precision(kvs_ctx* ctx, int32_t prec);
/* Network used by kvs_project with precond = KVS_PC_UNET (flexible PCG:
 * z = U(r) with the network's input scaled to unit RMS of r and its output
 * by h^2 rms(r); beta = z_{k+1}.(r_{k+1} - r_k) / (z_k.r_k); when z.r <= 0
 * or non-finite that iteration uses z = r / diag(A) instead).  The network
 * is borrowed: keep it alive while the context uses it; NULL unsets it.
 * The grid spacings must be equal. */
kvs_status kvs_set_preconditioner(kvs_ctx* ctx, kvs_unet* net);
/* Number of Jacobi fallbacks taken by the last flexible solve. */
kvs_status kvs_last_fallbacks(const kvs_ctx* ctx, int64_t* n);
/* Inject / read back the projected force f_S (host, 3*N doubles).  Setting
 * it marks it current (no projection needed before stepping). */
kvs_status kvs_set_projected_force(kvs_ctx* ctx, const double* FS);
kvs_status kvs_get_projected_force(const kvs_ctx* ctx, double* FS);
/* Read back phi of the last projection (host, N doubles). */
kvs_status kvs_get_phi(const kvs_ctx* ctx, double* phi);

/* ---- time stepping and sensors (Sec. 3.1, 4.1) ------------------------- */

/* Probe cells: ijk = n triples (i, j, k), 0 <= i < nx etc.; comp 0..2 records
 * that displacement component, 3 records all three.  Clears recorded
 * traces.  n = 0 disables probes. */
kvs_status kvs_set_probes(kvs_ctx* ctx, const int64_t* ijk, int64_t n, int32_t comp);
/* Advance nsteps >= 0 steps.  Needs material and dt; needs a current f_S
 * when the envelope is non-zero on any of these steps (else KVS_ESTATE).
 * After every step the probe values of u^{n+1} are appended to the traces. */
kvs_status kvs_step(kvs_ctx* ctx, int64_t nsteps);
/* Number of steps recorded in the traces. */
kvs_status kvs_trace_count(const kvs_ctx* ctx, int64_t* nsteps_recorded);
/* Copy the traces [step][probe][comp] (comp extent 1, or 3 for comp == 3)
 * into out (host, cap doubles); n_written = doubles written.  Blocks. */
kvs_status kvs_read_traces(const kvs_ctx* ctx, double* out, int64_t cap, int64_t* n_written);
kvs_status kvs_clear_traces(kvs_ctx* ctx);
/* State in doubles (host, 3*N each): u^n and w^n = u^n - u^{n-1}, and the
 * absolute step index n.  get blocks; set resets the outer layer to 0. */
kvs_status kvs_get_state(const kvs_ctx* ctx, double* u, double* w, int64_t* step);
kvs_status kvs_set_state(kvs_ctx* ctx, const double* u, const double* w, int64_t step);
/* Absorbing layer in place of the sponge: a convolutional perfectly matched
 * layer of `cells` cells next to every Dirichlet face (the absorbing
 * boundary the paper names for its wall reflections, Sec. 3.5 and Sec. 7).
 * Each axis is stretched, s = 1 + d / (alpha + i w), in both spatial
 * derivatives of div(G grad u) and of (eta / dt) lap(w), with memory
 * variables on the face fluxes and on each axis's cell divergence, updated
 * recursively once per step (b = exp(-(d + alpha) dt),
 * c = d / (d + alpha) (b - 1)); d = d0 q^2 over the depth q in the layer,
 * d0 = 3 c_max ln(1/R) / (2 cells h), c_max the material's largest shear
 * speed; alpha = alpha_max throughout the layer (alpha_max < 0: pi c_max /
 * (10 cells h_min), the frequency of a wave ten layer widths long).  cells = 0 switches the layer off.  Needs a context without
 * sponge and every extent >= 2 cells + 3 (else KVS_EINVAL); R in (0, 1].  The
 * memory variables (device, state precision, in slabs of cells + 1 nodes on
 * each side of every axis) belong to the state: kvs_set_state,
 * kvs_set_state_curl and kvs_reset_state zero them.  Not available to
 * batched stepping (KVS_ESTATE there). */
kvs_status kvs_set_pml(kvs_ctx* ctx, int32_t cells, double R, double alpha_max);
/* Curl-based initial state (Sec. 3.5; the source of the wavespeed validation,
 * Sec. 4.1): an initial velocity v0 = curl_h A, divergence-free by
 * construction, at rest displacement: u = 0 and w = dt v0, where curl_h
 * takes the centred first differences (f(+a) - f(-a)) / (2 h_a) on the
 * interior nodes and is 0 on the outer layer.  A: host, 3*N doubles
 * [3][nz][ny][nx] (copied); step: the absolute step index of the new state
 * (>= 0).  Needs dt (else KVS_ESTATE).  Traces and peak maps are kept, as
 * with kvs_set_state.  Blocks. */
kvs_status kvs_set_state_curl(kvs_ctx* ctx, const double* A, int64_t step);
/* Return the medium to rest (u = w = 0), reset the step index to 0 and clear
 * the traces; material, dt, force, projection and probes are kept. */
kvs_status kvs_reset_state(kvs_ctx* ctx);

/* Peak displacement maps (the |u| slices of the transcranial demonstration,
 * Sec. 5.1): after every kvs_step step, each registered plane keeps the
 * running maximum over steps of |u| = sqrt(ux^2 + uy^2 + uz^2) per cell, in
 * the state precision (a NaN, once seen, stays).  axis[p] 0..2 fixes
 * i (x), j (y) or k (z) at index[p] (0 <= index < the grid extent on that
 * axis); at most KVS_MAX_PEAK_PLANES planes, no (axis, index) pair twice.
 * Registering replaces every earlier plane and starts each map at |u| of the
 * current state; n = 0 switches the maps off.  kvs_reset_state zeroes them;
 * kvs_set_state keeps them.  Device memory: one map per plane, owned by the
 * context. */
#define KVS_MAX_PEAK_PLANES 8
kvs_status kvs_set_peak_planes(kvs_ctx* ctx, const int32_t* axis, const int64_t* index, int32_t n);
/* Copy the map of the registered plane (axis, index) into out (host):
 * axis 0 -> [nz][ny], axis 1 -> [nz][nx], axis 2 -> [ny][nx], last extent
 * fastest.  An unregistered plane is KVS_EINVAL.  Blocks. */
kvs_status kvs_peak_map(const kvs_ctx* ctx, int32_t axis, int64_t index, double* out);

/* ---- acoustic radiation force (Sec. 3.4, Eqs. isppa_norm and arf_poynting) -- */

/* The body force is derived from a time series of the acoustic field sampled
 * on the context grid, then used like kvs_set_force (project, then step).
 * The library keeps per-cell running sums over the samples in FP64, sample
 * by sample in the order given (products and sums not fused, so the sums are
 * the plain sequential ones), and turns them into the force pattern:
 *   KVS_ARF_PLANE     S = sum p^2;       F = b0 d,
 *                     b0 = (2 alpha / c) S / (rho c N_pulse)   (Eq. isppa_norm)
 *   KVS_ARF_POYNTING  S_i = sum p v_i;   F_i = (2 alpha / c) S_i / N_pulse
 *                                                           (Eq. arf_poynting)
 * alpha: absorption [Np/m] at the transmit frequency; c: sound speed [m/s];
 * rho: density [kg/m^3]; N_pulse: samples in one pulse (the sums run over
 * all samples, silent ones included, and are normalised by the pulse
 * length); d: unit beam direction.  Cells whose mask byte is 0 get F = 0
 * (regions outside the tissue of interest, Sec. 5.1).  p in Pa, v in m/s,
 * layouts [sample][nz][ny][nx] and [sample][3][nz][ny][nx]. */
typedef enum { KVS_ARF_PLANE = 1, KVS_ARF_POYNTING = 2 } kvs_arf_mode;
/* Start a time average in `mode`: zero the sums and the sample count.  The
 * sums (N doubles, or 3N in the Poynting form) are device memory owned by
 * the context.  Unknown mode: KVS_EINVAL. */
kvs_status kvs_arf_begin(kvs_ctx* ctx, int32_t mode);
/* Add nsamp >= 1 samples from device memory (dtype 0 = double, 1 = float):
 * p [nsamp][N]; v [nsamp][3][N] in the Poynting form, NULL in the plane-wave
 * form (anything else: KVS_EINVAL).  Read asynchronously on the context's
 * stream: keep the buffers alive until it synchronises.  Before
 * kvs_arf_begin: KVS_ESTATE. */
kvs_status kvs_arf_accumulate_device(kvs_ctx* ctx, const void* p, const void* v, int64_t nsamp, int32_t dtype);
/* Same from host doubles (copied sample by sample; blocks). */
kvs_status kvs_arf_accumulate(kvs_ctx* ctx, const double* p, const double* v, int64_t nsamp);
/* Samples added since kvs_arf_begin (nsamp, may be NULL) and the raw sums
 * (out: host, N doubles in the plane-wave form, 3N [3][N] in the Poynting
 * form; may be NULL).  Blocks. */
kvs_status kvs_arf_get_sums(const kvs_ctx* ctx, double* out, int64_t* nsamp);
/* Turn the sums into the force pattern F (replaces the force; the projected
 * force becomes stale, as after kvs_set_force).  alpha, c, rho: host arrays
 * of n_alpha, n_c, n_rho values, each 1 (uniform) or N (a map); alpha >= 0,
 * c > 0, rho > 0, all finite; rho and beam_dir (3 doubles, non-zero,
 * normalised here) are read in the plane-wave form only and may be NULL in
 * the Poynting form.  mask: host, N bytes, or NULL to keep every cell.
 * n_pulse > 0.  No samples yet: KVS_ESTATE.  Blocks. */
kvs_status kvs_arf_set_force(kvs_ctx* ctx, const double* alpha, int64_t n_alpha, const double* c, int64_t n_c,
                             const double* rho, int64_t n_rho, const uint8_t* mask, double n_pulse,
                             const double* beam_dir);

/* Peak acoustic strain maps (Sec. 5.2), from the pressure series alone and
 * with no pulse normalisation: per cell the running maxima over the samples
 * of |eps| with eps = -p / K (K = rho c^2 the bulk modulus), and of
 * |grad eps| = sqrt(gx^2 + gy^2 + gz^2) with the centred differences
 * g_a = (eps(+a) - eps(-a)) / (2 h_a) on the interior nodes (0 on the outer
 * layer); FP64 arithmetic, maxima in sample order (a NaN, once seen, stays).
 * kvs_strain_begin: K host, n_K = 1 (uniform) or N values, finite and > 0
 * (else KVS_EINVAL); zeroes both maps and the sample count.  Device memory
 * (K and the two maps) is owned by the context. */
kvs_status kvs_strain_begin(kvs_ctx* ctx, const double* K, int64_t n_K);
/* Add nsamp >= 1 pressure samples, p [nsamp][N] in device memory (dtype 0 =
 * double, 1 = float), read on the context's stream.  Before kvs_strain_begin:
 * KVS_ESTATE. */
kvs_status kvs_strain_accumulate_device(kvs_ctx* ctx, const void* p, int64_t nsamp, int32_t dtype);
/* Copy the maps (host, N doubles each; either may be NULL) and the sample
 * count (may be NULL).  Blocks. */
kvs_status kvs_strain_get(const kvs_ctx* ctx, double* peak_strain, double* peak_gradient, int64_t* nsamp);

/* ---- measurement -------------------------------------------------------- */

/* When on, every launch of the FDTD step kernel by kvs_step records its own
 * start and end in a pair of HIP events on the context's stream (events
 * attached to the dispatch, hipExtLaunchKernel: the kernel's duration, no
 * extra queue packets); kvs_kernel_time returns the summed duration [ms] and
 * the number of steps those launches advanced (one per launch, two per
 * two-step launch) since timing was switched on. */
kvs_status kvs_enable_kernel_timing(kvs_ctx* ctx, int32_t on);
kvs_status kvs_kernel_time(kvs_ctx* ctx, double* ms_total, int64_t* steps);
/* The same totals by launch kind: ms[0], launches[0] for one-step launches,
 * ms[1], launches[1] for two-step launches (host arrays of 2; either may be
 * NULL). */
kvs_status kvs_kernel_time_split(kvs_ctx* ctx, double* ms, int64_t* launches);
/* Streaming reference for the roofline of the FDTD step: a kernel with the
 * step's memory pattern and no stencil (per cell 9 FP32 values read, 6
 * written: 60 B; 15 contiguous streams of n floats, 16-byte accesses) run
 * reps times on `device` after one untimed launch; *gbs = 60 n bytes over
 * the median launch time (HIP events).  Allocates and frees its 15 buffers
 * (60 n bytes).  n >= 1024, reps >= 1, else KVS_EINVAL. */
kvs_status kvs_measure_stream(int32_t device, int64_t n, int32_t reps, double* gbs);
/* The same with the read/write mix of a chosen step kernel: (reads, writes)
 * = (9, 6), the heterogeneous step, or (6, 6), the homogeneous batched step
 * (u and w only, 48 B per cell); other mixes give KVS_EINVAL.  *gbs counts
 * 4 (reads + writes) n bytes; allocates and frees reads + writes buffers. */
kvs_status kvs_measure_stream_rw(int32_t device, int64_t n, int32_t reads, int32_t writes, int32_t reps,
                                 double* gbs);

/* ---- batched parameter sweeps ----------------------------------------------- */

/* A batch advances n homogeneous instances (each its own grid, medium, dt,
 * force, envelope and probes) together: every step is one kernel launch
 * covering all instances' tiles, and a run of steps is one hipGraph launch
 * (captured on first use, replayed while the start step, step count and
 * trace slot repeat, e.g. after kvs_batch_reset).  Instances are ordinary
 * contexts: configure each through kvs_batch_instance() with the functions
 * above (material must be uniform).  All instances share the batch's
 * stream. */
typedef struct kvs_batch kvs_batch;
/* grids: n grids; opts as for kvs_create (one precision and sponge for all). */
kvs_status kvs_batch_create(const kvs_grid* grids, int32_t n, const kvs_opts* opts, kvs_batch** out);
void kvs_batch_destroy(kvs_batch* b);
const char* kvs_batch_last_error(const kvs_batch* b);
/* Instance i (0 <= i < n), owned by the batch; NULL when out of range. */
kvs_ctx* kvs_batch_instance(kvs_batch* b, int32_t i);
/* Copy instance src's projected force to instance dst (same grid required):
 * the projection depends on the grid and force pattern only, not on the
 * medium. */
kvs_status kvs_batch_share_projection(kvs_batch* b, int32_t src, int32_t dst);
/* Probes of instance i (replaces its list; clears the batch traces) and the
 * recorded component for all instances (0..2). */
kvs_status kvs_batch_set_probes(kvs_batch* b, int32_t i, const int64_t* ijk, int64_t n);
kvs_status kvs_batch_set_component(kvs_batch* b, int32_t comp);
/* Advance every instance nsteps steps.  Every instance needs uniform
 * material, dt, and a current projection on steps where its envelope is
 * non-zero, and all must be at the batch's step index (else KVS_ESTATE). */
kvs_status kvs_batch_step(kvs_batch* b, int64_t nsteps);
/* All instances to rest, step index 0, traces cleared. */
kvs_status kvs_batch_reset(kvs_batch* b);
kvs_status kvs_batch_trace_count(const kvs_batch* b, int64_t* nsteps_recorded);
/* Traces of instance i, [step][probe] doubles, into out (cap doubles). */
kvs_status kvs_batch_read_traces(kvs_batch* b, int32_t i, double* out, int64_t cap, int64_t* n_written);

/* Steps per launch of kvs_batch_step: 1 or 2 (the default), else KVS_EINVAL.
 * With 2, pairs of consecutive steps in which no instance's envelope is
 * non-zero are advanced by one launch of the two-step tile over all
 * instances (the result is bitwise that of one-step launches); it applies to
 * FP32 batches with a viscous instance, rows of at most 256 cells, and probe
 * cells distinct and off each instance's planes k = 0, nz - 1
 * (kvs_batch_step_blocking_applies).  Runs that take the persistent path are
 * not affected. */
kvs_status kvs_batch_set_step_blocking(kvs_batch* b, int32_t steps);
/* 1 if two-step launches apply to the batch as it is now, else 0. */
int32_t kvs_batch_step_blocking_applies(const kvs_batch* b);
/* Persistent runs of small instances (on by default): when every instance's
 * whole state (u and w, 24 B per node in FP32, 48 B in FP64) fits in 150 KB,
 * a kvs_batch_step run is one launch with one workgroup per instance that
 * keeps the state in LDS and advances it through all the steps (two
 * workgroup barriers per step, probes written after every step), instead of
 * one launch per step.  on = 0 keeps the per-step launches.
 * kvs_batch_uses_persistent reports whether the next run takes that path. */
kvs_status kvs_batch_set_persistent(kvs_batch* b, int32_t on);
kvs_status kvs_batch_uses_persistent(const kvs_batch* b, int32_t* on);
/* Batch tile shape (a step-kernel variant, as for kvs_set_step_variant, or
 * KVS_BATCH_FIT_ROWS) and z planes per block (>= 1).  KVS_BATCH_FIT_ROWS gives
 * each instance the narrowest tile that spans its x rows (64 x 8, 128 x 8,
 * 192 x 4 or 256 x 4 cells; wider rows take several 256 x 4 tiles; FP64:
 * 64 x 8 or 128 x 4), so no tile re-reads x-halo columns of a neighbour;
 * instances of one shape share a launch (one launch per shape per step). */
#define KVS_BATCH_FIT_ROWS (-1)
kvs_status kvs_batch_set_tuning(kvs_batch* b, int32_t variant, int32_t zchunk);
/* Time every (variant, z planes in {16, 32, 64}), KVS_BATCH_FIT_ROWS included,
 * with trial_steps launches that do not advance the state, keep the fastest,
 * return it.  Needs every instance's material and dt.  ms_per_launch (cap
 * entries: one per variant, best z, then the row-fitted tiling) may be NULL. */
kvs_status kvs_batch_autotune(kvs_batch* b, int32_t trial_steps, int32_t* variant, int32_t* zchunk,
                              double* ms_per_launch, int32_t cap);

/* ---- learned preconditioner (a small linear U-Net) -------------------------- */

/* Network z = U(r): e0 = conv(r; 1 -> C0); e1 = conv(pool(e0); C0 -> C1);
 * bottleneck at 1/4 resolution: conv(pool(e1); C1 -> C2), n_bottleneck - 2
 * convs C2 -> C2 with dilations 2, 4, ..., conv(C2 -> C1);
 * g1 = conv(e1 + up(bottleneck); C1 -> C0) and gz = g1 . wp (pointwise
 * C0 -> 1) at 1/2 resolution; z = conv(e0; C0 -> 1) + up(gz), zero outside
 * the interior: a local stencil of r plus the interpolated coarse
 * correction.  conv = 3x3x3 (dilated) cross-correlation with zero padding,
 * no bias, no nonlinearity; pool = mean of the existing 2x2x2 children;
 * up = cell-centred trilinear interpolation (per axis 3/4 of the parent,
 * 1/4 of its neighbour on the fine cell's side, clamped at the edges).
 * Activations and weights are BF16, accumulation FP32 (MFMA); gz is FP32.
 * e0 is rounded to BF16 where it is pooled; the output conv takes it
 * unrounded, which on the interior equals one 5x5x5 FP32 stencil of the
 * BF16 input with the composed weights (W_out after W0).
 * Used as the preconditioner of a flexible PCG on the projection's Poisson
 * problem (not part of the paper's method; plain CG / Jacobi-PCG remain the
 * reference). */
/* channels = {C0, C1, C2} (NULL: 16, 32, 64; only these are built);
 * 2 <= n_bottleneck <= 8.  Weights start at zero. */
kvs_status kvs_unet_create(const int32_t* channels, int32_t n_bottleneck, kvs_unet** out);
void kvs_unet_destroy(kvs_unet* net);
const char* kvs_unet_last_error(const kvs_unet* net);
/* FP32 master weights, layer by layer in network order, each [co][27 * ci]
 * with k = tap * ci + c, tap = 9 (dz + 1) + 3 (dy + 1) + (dx + 1); the
 * pointwise projection is [1][ci]. */
int64_t kvs_unet_num_weights(const kvs_unet* net);
/* Layers in network order: input / output channels, dilation (0 for the
 * pointwise projection) and taps (27 or 1) of layer l. */
int32_t kvs_unet_num_layers(const kvs_unet* net);
kvs_status kvs_unet_layer(const kvs_unet* net, int32_t l, int32_t* ci, int32_t* co, int32_t* dil, int32_t* taps);
kvs_status kvs_unet_set_weights(kvs_unet* net, const float* w, int64_t n);
kvs_status kvs_unet_get_weights(const kvs_unet* net, float* w, int64_t n);
/* z = out_scale * U(in_scale * r) on an nx*ny*nz grid; r and z are FP64
 * device fields [nz][ny][nx] ordered on `stream` (hipStream_t or NULL). */
kvs_status kvs_unet_forward(kvs_unet* net, const double* r, double in_scale, double out_scale, double* z, int64_t nx,
                            int64_t ny, int64_t nz, void* stream);
/* Backward pass of the last kvs_unet_forward (same r, in_scale, grid): the
 * gradient of the raw network output (before out_scale) is dz_scale * dz
 * (dz: FP64 device field, zero outside the interior).  Writes, or with
 * accumulate != 0 adds to, the FP32 weight gradient (master layout).
 * Activation gradients are FP32; each is rounded to BF16 where it feeds a
 * transposed convolution. */
kvs_status kvs_unet_backward(kvs_unet* net, const double* r, double in_scale, const double* dz, double dz_scale,
                             int64_t nx, int64_t ny, int64_t nz, int32_t accumulate, void* stream);
kvs_status kvs_unet_get_grad(const kvs_unet* net, float* g, int64_t n);
/* One training sample at unit grid spacing: forward of b (unit RMS, scales
 * 1), loss L = (z - x)^T A (z - x) / (x^T A x) with A = -lap_1 on the
 * interior, backward; gradient written or accumulated.  b, x: FP64 device
 * fields. */
kvs_status kvs_unet_train_sample(kvs_unet* net, const double* b, const double* x, int64_t nx, int64_t ny, int64_t nz,
                                 int32_t accumulate, double* loss, void* stream);
/* Adam (beta 0.9, 0.999, eps 1e-8) on the FP32 master weights with the
 * gradient averaged over n_samples, then repack the BF16 weights. */
kvs_status kvs_unet_adam_step(kvs_unet* net, double lr, int32_t n_samples, void* stream);
/* Training pair generated by the solver itself on context ctx (FP64, force
 * set): phi* = Jacobi-PCG solution of the current force to 1e-11; x = phi*
 * (k_snapshot = 0) or the error phi* - phi_k after k_snapshot iterations of
 * the solver with preconditioner `precond` (KVS_PC_JACOBI, or KVS_PC_UNET
 * with ctx's network: the residuals the flexible PCG meets); b = A x with
 * ctx's spacing (= the residual r_k); both divided by rms(b) (returned in
 * b_rms).  b, x: device fields of N doubles. */
kvs_status kvs_unet_make_sample(kvs_ctx* ctx, int64_t k_snapshot, int32_t precond, double* b, double* x,
                                double* b_rms);
/* Verification hook: one MFMA convolution on host BF16 bit patterns,
 * out[v][co] = sum_k W[co][k] x[p][c] with W rows padded to
 * kvs_unet_conv_kpad(ci) entries; x = A, or with B (the next coarser grid,
 * (n + 1) / 2 per axis) x = bf16(A + up(B)) as the decoder forms its skip
 * input.  Blocks. */
/* Training pair from a given field: b = A x with A = -lap_1 (unit spacing)
 * on the interior of an nx*ny*nz grid, then b and x divided by rms(b)
 * (returned in b_rms).  x is read (and rescaled in place); b is written.
 * Device FP64 fields ordered on `stream`.  Blocks. */
kvs_status kvs_unet_sample_from_x(double* x, double* b, int64_t nx, int64_t ny, int64_t nz, double* b_rms,
                                  void* stream);
int64_t kvs_unet_conv_kpad(int32_t ci);
kvs_status kvs_unet_conv_check(int32_t ci, int32_t co, int32_t dil, const uint16_t* A, const uint16_t* B, int64_t nx,
                               int64_t ny, int64_t nz, const uint16_t* W, uint16_t* out);

/* ---- tuning --------------------------------------------------------------- */

/* Number of FDTD step-kernel variants (tile rows x cells per lane x
 * wavefronts per x row). */
int32_t kvs_num_step_variants(void);
/* Use variant v (0 <= v < kvs_num_step_variants()) for kvs_step.  Every
 * variant computes the same update; they differ in tile shape only. */
kvs_status kvs_set_step_variant(kvs_ctx* ctx, int32_t v);
/* Full step-kernel tuning: variant v, z planes per block zchunk (0 = split
 * z so that the blocks fill whole rounds of resident blocks), remap != 0
 * issues tiles XCD by XCD in contiguous ranges (y-adjacent tiles share L2). */
kvs_status kvs_set_step_tuning(kvs_ctx* ctx, int32_t v, int32_t zchunk, int32_t remap);
/* Steps per launch of kvs_step: 1 or 2 (the default), else KVS_EINVAL.  With
 * 2, kvs_step advances each pair of consecutive steps whose envelope values
 * g_n are both 0 in one launch (temporal blocking of the Sec. 3.1 update: the
 * intermediate state is formed on chip, with its rows next to each tile's
 * computed twice); the result is that of two one-step launches (the same
 * FP32 operations in the same order).  Applies where kvs_step_blocking_applies
 * says so: FP32 state, heterogeneous viscous medium, no absorbing layer, no
 * peak planes, nx <= 256, and probe cells (if any) distinct and off the planes
 * k = 0 and nz - 1; elsewhere, for a step with force and for the last step of
 * an odd count, kvs_step launches one step as with 1.  Traces are recorded
 * for every step either way.  Kernel timing (kvs_kernel_time) counts the
 * steps the timed launches advanced. */
kvs_status kvs_set_step_blocking(kvs_ctx* ctx, int32_t steps);
/* 1 if two-step launches apply to the context as it is now, else 0. */
int32_t kvs_step_blocking_applies(const kvs_ctx* ctx);
/* Time every variant on this context's grid, precision and medium, each with
 * the automatic z split and with 16-, 32- and 64-plane z segments
 * (trial_steps >= 1 launches each, after one untimed launch), and keep the
 * fastest.  ms_per_launch[v] is the best z split's time for variant v.  The state is not advanced: trial launches only write the
 * buffers the next real step overwrites.  Needs material and dt.  chosen and
 * ms_per_launch (cap entries, one per variant) may be NULL. */
kvs_status kvs_autotune_step(kvs_ctx* ctx, int32_t trial_steps, int32_t* chosen, double* ms_per_launch,
                             int32_t cap);

/* ---- projection without allocation ------------------------------------------ */

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * projection of kvs_project (b = div F, CG or Jacobi-PCG on A phi = -b,
 * f_S = F - grad phi, FP64 throughout) on caller-owned device buffers, with
 * the CG vectors, block partials and control block in a fixed device array
 * of KVS_NOALLOC_SCRATCH_BYTES built into the library (one per device, kept
 * until the process ends).  No hipMalloc, hipFree or event is created.
 *   grid   sizes and spacings as for kvs_create; the grid must fit the array:
 *          about 4 * 8 B per cell, so at most ~2.1e6 cells (129^3); larger
 *          grids give KVS_EINVAL with a message naming the sizes.
 *   F      device, 3N doubles [3][nz][ny][nx], read.
 *   phi    device, N doubles: the potential (written); with
 *          opts->warm_start != 0 also the initial guess (its outer layer is
 *          set to 0 first).
 *   FS     device, 3N doubles: f_S (written, 0 on the outer layer).
 *   opts   as for kvs_project (NULL: tol 1e-8, max_iter 10000, Jacobi-PCG);
 *          precond must be KVS_PC_NONE or KVS_PC_JACOBI (else KVS_EINVAL);
 *          fixed_iters and confirm_true as there.
 *   device HIP device ordinal (made current); stream: hipStream_t or NULL
 *          (the null stream); the call returns after the stream's work of
 *          the projection is done (it polls a device flag, as kvs_project).
 *   report may be NULL; ms is host wall time.
 * Returns the solve status as kvs_project does.  Calls on one device share
 * the array, so calls that overlap on one device (other threads, other
 * streams) race and must be serialised by the caller.  Error text:
 * kvs_noalloc_last_error() (per thread). */
#define KVS_NOALLOC_SCRATCH_BYTES (66u << 20)
kvs_status kvs_project_noalloc(const kvs_grid* grid, const double* F, double* phi, double* FS,
                               const kvs_solve_opts* opts, int32_t device, void* stream, kvs_solve_report* report);
const char* kvs_noalloc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KVS_H */
