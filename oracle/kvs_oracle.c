/*
 * kvs_oracle.c -- plain FP64 CPU oracle of the reduced Kelvin-Voigt shear
 * solver (Pinton, "A reduced viscoelastic FDTD formulation for
 * ultrasound-driven shear wave propagation in soft tissue").
 *
 * TEST INFRASTRUCTURE ONLY.  It is called by the tests, by the smoke check
 * and by the benchmark's CPU-baseline leg, never by the GPU library, and it
 * shares no source, header, table or helper with it.  It is deliberately
 * slow and literal: one loop nest per operator, FP64 everywhere, OpenMP only
 * on the outermost loop of each sweep.
 *
 * Layout: scalar fields are [nz][ny][nx] with x fastest,
 * index = i + nx*(j + ny*k); vector fields are [3][nz][ny][nx] (x, y, z
 * components).  The outer layer (i in {0, nx-1}, likewise j, k) is the
 * Dirichlet layer; "interior" is 1..n-2 on every axis.
 *
 * What each routine follows:
 *   ora_laplacian       7-point second-order Laplacian on cell centres
 *                       (Sec. 3.1, below the FDTD update equations).
 *   ora_elastic         div(G grad u) with harmonic face moduli: the
 *                       heterogeneous reading of the mu*lap(u) term of the
 *                       acceleration in Sec. 3.1 (equals G*lap when G is
 *                       uniform).
 *   ora_divergence      b = centred divergence of f on interior nodes
 *                       (Sec. 3.2.3, A phi = b with b = div_h f).
 *   ora_cg              the CG recurrences of Sec. 3.2.3 (interior mask after
 *                       every update, phi_0 = 0, relative-residual stop,
 *                       non-finite / non-positive guards), applied to
 *                       A = -lap_h with right-hand side -b, i.e. the Poisson
 *                       equation lap phi = div f of Sec. 3.2.1.  Optional
 *                       Jacobi preconditioning (constant diagonal).
 *   ora_grad_subtract   f_S = f - grad phi (Sec. 3.2.1), in the face-
 *                       consistent form: the cell average of the face field
 *                       H = avg_face(f) - D+ phi, i.e. (1-2-1 filter of f_a)
 *                       minus the centred difference of phi along a.
 *   ora_project         divergence -> CG -> gradient subtraction: the
 *                       pre-computation stage of Sec. 3.3.
 *   ora_run             explicit leapfrog (Sec. 3.1) in the summed form
 *                       w = u^n - u^{n-1}, u^{n+1} = u^n + w^{n+1}, with the
 *                       viscous velocity by backward difference, the source
 *                       g(t_n) f_S0 of Sec. 3.3 (time-stepping stage), a
 *                       centred velocity-damping sponge, and the Dirichlet
 *                       outer layer of Sec. 3.5.
 *   ora_stable_dt       largest dt with A + 2B <= 4 per cell (Gershgorin on
 *                       the face moduli), which reduces to the CFL bound of
 *                       Sec. 3.1 when eta = 0.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    long nx, ny, nz;
    double hx, hy, hz;
} ora_grid;

typedef struct {
    long iters;
    double relres_recursive;
    double relres_true;
    int status; /* 0 ok, 4 not converged, 5 breakdown */
} ora_report;

enum { ORA_OK = 0, ORA_EINVAL = 1, ORA_ENOMEM = 2, ORA_ENOTCONV = 4, ORA_EBREAKDOWN = 5 };

static long ncell(const ora_grid* g) { return g->nx * g->ny * g->nz; }

static long at(const ora_grid* g, long i, long j, long k) { return i + g->nx * (j + g->ny * k); }

static int inside(const ora_grid* g, long i, long j, long k) {
    return i >= 1 && i <= g->nx - 2 && j >= 1 && j <= g->ny - 2 && k >= 1 && k <= g->nz - 2;
}

static int grid_ok(const ora_grid* g) {
    return g && g->nx >= 3 && g->ny >= 3 && g->nz >= 3 && g->hx > 0 && g->hy > 0 && g->hz > 0;
}

/* ---- grid operators ---- */

/* out = lap_h q on the interior, 0 on the outer layer. */
int ora_laplacian(const ora_grid* g, const double* q, double* out) {
    if (!grid_ok(g)) return ORA_EINVAL;
    const double ax = 1.0 / (g->hx * g->hx), ay = 1.0 / (g->hy * g->hy), az = 1.0 / (g->hz * g->hz);
    const long sx = 1, sy = g->nx, sz = g->nx * g->ny;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < g->nz; ++k)
        for (long j = 0; j < g->ny; ++j)
            for (long i = 0; i < g->nx; ++i) {
                long c = at(g, i, j, k);
                if (!inside(g, i, j, k)) {
                    out[c] = 0.0;
                    continue;
                }
                out[c] = (q[c + sx] - 2.0 * q[c] + q[c - sx]) * ax
                       + (q[c + sy] - 2.0 * q[c] + q[c - sy]) * ay
                       + (q[c + sz] - 2.0 * q[c] + q[c - sz]) * az;
            }
    return ORA_OK;
}

static double harmonic(double a, double b) { return 2.0 * a * b / (a + b); }

/* E(q) = sum_a [G_{a+}(q_{+a} - q) - G_{a-}(q - q_{-a})] / h_a^2 at one
 * interior cell, G on faces = harmonic mean of the two adjacent cells. */
static double elastic_at(const ora_grid* g, const double* G, const double* q, long i, long j, long k) {
    const long c = at(g, i, j, k);
    const long st[3] = {1, g->nx, g->nx * g->ny};
    const double h[3] = {g->hx, g->hy, g->hz};
    double e = 0.0;
    for (int a = 0; a < 3; ++a) {
        const long p = c + st[a], m = c - st[a];
        const double gp = harmonic(G[c], G[p]);
        const double gm = harmonic(G[c], G[m]);
        e += (gp * (q[p] - q[c]) - gm * (q[c] - q[m])) / (h[a] * h[a]);
    }
    return e;
}

/* out = div(G grad q) for one scalar component, interior only. */
int ora_elastic(const ora_grid* g, const double* G, const double* q, double* out) {
    if (!grid_ok(g)) return ORA_EINVAL;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < g->nz; ++k)
        for (long j = 0; j < g->ny; ++j)
            for (long i = 0; i < g->nx; ++i) {
                long c = at(g, i, j, k);
                out[c] = inside(g, i, j, k) ? elastic_at(g, G, q, i, j, k) : 0.0;
            }
    return ORA_OK;
}

/* b = sum_a (F_a(+a) - F_a(-a)) / (2 h_a) on the interior, 0 outside. */
int ora_divergence(const ora_grid* g, const double* F, double* b) {
    if (!grid_ok(g)) return ORA_EINVAL;
    const long N = ncell(g);
    const double* Fx = F;
    const double* Fy = F + N;
    const double* Fz = F + 2 * N;
    const long sx = 1, sy = g->nx, sz = g->nx * g->ny;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < g->nz; ++k)
        for (long j = 0; j < g->ny; ++j)
            for (long i = 0; i < g->nx; ++i) {
                long c = at(g, i, j, k);
                if (!inside(g, i, j, k)) {
                    b[c] = 0.0;
                    continue;
                }
                b[c] = (Fx[c + sx] - Fx[c - sx]) / (2.0 * g->hx)
                     + (Fy[c + sy] - Fy[c - sy]) / (2.0 * g->hy)
                     + (Fz[c + sz] - Fz[c - sz]) / (2.0 * g->hz);
            }
    return ORA_OK;
}

/* ---- projection ---- */

/* A q = -lap_h q, masked to the interior. */
static void apply_A(const ora_grid* g, const double* q, double* out) {
    const long N = ncell(g);
    ora_laplacian(g, q, out);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < N; ++c) out[c] = -out[c];
}

static double dot(long N, const double* a, const double* b) {
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (long c = 0; c < N; ++c) s += a[c] * b[c];
    return s;
}

static void mask(const ora_grid* g, double* q) {
#pragma omp parallel for schedule(static)
    for (long k = 0; k < g->nz; ++k)
        for (long j = 0; j < g->ny; ++j)
            for (long i = 0; i < g->nx; ++i)
                if (!inside(g, i, j, k)) q[at(g, i, j, k)] = 0.0;
}

/* ||-b - A phi|| / ||b|| over the interior (= ||lap phi - b|| / ||b||). */
double ora_true_relres(const ora_grid* g, const double* b, const double* phi) {
    const long N = ncell(g);
    double* Aphi = (double*)malloc(sizeof(double) * N);
    if (!Aphi) return NAN;
    apply_A(g, phi, Aphi);
    double num = 0.0, den = 0.0;
    for (long k = 1; k < g->nz - 1; ++k)
        for (long j = 1; j < g->ny - 1; ++j)
            for (long i = 1; i < g->nx - 1; ++i) {
                long c = at(g, i, j, k);
                double r = -b[c] - Aphi[c];
                num += r * r;
                den += b[c] * b[c];
            }
    free(Aphi);
    return den > 0 ? sqrt(num / den) : 0.0;
}

/*
 * Conjugate gradient for A phi = rhs, A = -lap_h on the interior, started from
 * phi_0 = 0 (phi is overwritten).  The recurrences, the mask after every
 * update and the stop test sqrt(r.r / r0.r0) < tol follow Sec. 3.2.3; the
 * iteration stops with a breakdown status when p.Ap is not positive or a
 * reduction is not finite.  fixed_iters > 0 runs exactly that many iterations
 * and ignores tol (parity mode).  jacobi != 0 runs the preconditioned form
 * with z = r / diag(A); diag(A) = sum_a 2/h_a^2 is the same on every cell.
 * rep->iters counts phi updates.
 */
int ora_cg(const ora_grid* g, const double* rhs, double* phi, double tol, long max_iter, long fixed_iters,
           int jacobi, ora_report* rep) {
    if (!grid_ok(g) || !rhs || !phi || !rep) return ORA_EINVAL;
    const long N = ncell(g);
    double* r = (double*)malloc(sizeof(double) * N);
    double* p = (double*)malloc(sizeof(double) * N);
    double* Ap = (double*)malloc(sizeof(double) * N);
    double* z = jacobi ? (double*)malloc(sizeof(double) * N) : NULL;
    if (!r || !p || !Ap || (jacobi && !z)) {
        free(r), free(p), free(Ap), free(z);
        return ORA_ENOMEM;
    }
    const double diag = 2.0 / (g->hx * g->hx) + 2.0 / (g->hy * g->hy) + 2.0 / (g->hz * g->hz);
    int status = ORA_OK;

    memset(phi, 0, sizeof(double) * N);
    /* r_0 = (rhs - A phi_0) .* m = rhs .* m since phi_0 = 0 */
    for (long c = 0; c < N; ++c) r[c] = rhs[c];
    mask(g, r);
    if (jacobi) {
        for (long c = 0; c < N; ++c) z[c] = r[c] / diag;
        memcpy(p, z, sizeof(double) * N);
    } else {
        memcpy(p, r, sizeof(double) * N);
    }
    double rr = dot(N, r, r);
    const double rr0 = rr;
    double rz = jacobi ? dot(N, r, z) : rr;
    long k = 0;
    if (!isfinite(rr0)) status = ORA_EBREAKDOWN;
    while (status == ORA_OK && rr0 > 0.0) {
        if (fixed_iters > 0) {
            if (k >= fixed_iters) break;
        } else {
            if (sqrt(rr / rr0) < tol) break;
            if (k >= max_iter) {
                status = ORA_ENOTCONV;
                break;
            }
        }
        apply_A(g, p, Ap);
        mask(g, Ap);
        const double pAp = dot(N, p, Ap);
        if (!(pAp > 0.0) || !isfinite(pAp)) {
            status = ORA_EBREAKDOWN;
            break;
        }
        const double alpha = rz / pAp;
#pragma omp parallel for schedule(static)
        for (long c = 0; c < N; ++c) {
            phi[c] += alpha * p[c];
            r[c] -= alpha * Ap[c];
        }
        mask(g, phi);
        mask(g, r);
        ++k;
        const double rr_new = dot(N, r, r);
        if (!isfinite(rr_new) || rr_new < 0.0) {
            status = ORA_EBREAKDOWN;
            break;
        }
        double beta;
        if (jacobi) {
#pragma omp parallel for schedule(static)
            for (long c = 0; c < N; ++c) z[c] = r[c] / diag;
            const double rz_new = dot(N, r, z);
            beta = rz_new / rz;
            rz = rz_new;
#pragma omp parallel for schedule(static)
            for (long c = 0; c < N; ++c) p[c] = z[c] + beta * p[c];
        } else {
            beta = rr_new / rr;
            rz = rr_new;
#pragma omp parallel for schedule(static)
            for (long c = 0; c < N; ++c) p[c] = r[c] + beta * p[c];
        }
        mask(g, p);
        rr = rr_new;
    }
    rep->iters = k;
    rep->relres_recursive = rr0 > 0.0 ? sqrt(rr / rr0) : 0.0;
    {
        /* true residual ||rhs - A phi|| / ||rhs|| over the interior */
        apply_A(g, phi, Ap);
        double num = 0.0, den = 0.0;
        for (long kk = 1; kk < g->nz - 1; ++kk)
            for (long j = 1; j < g->ny - 1; ++j)
                for (long i = 1; i < g->nx - 1; ++i) {
                    long c = at(g, i, j, kk);
                    double d = rhs[c] - Ap[c];
                    num += d * d;
                    den += rhs[c] * rhs[c];
                }
        rep->relres_true = den > 0 ? sqrt(num / den) : 0.0;
    }
    rep->status = status;
    free(r), free(p), free(Ap), free(z);
    return status;
}

/* FS_a = (F_a(-a) + 2 F_a + F_a(+a))/4 - (phi(+a) - phi(-a))/(2 h_a) on the
 * interior, 0 on the outer layer. */
int ora_grad_subtract(const ora_grid* g, const double* F, const double* phi, double* FS) {
    if (!grid_ok(g)) return ORA_EINVAL;
    const long N = ncell(g);
    const long st[3] = {1, g->nx, g->nx * g->ny};
    const double h[3] = {g->hx, g->hy, g->hz};
    for (int a = 0; a < 3; ++a) {
        const double* Fa = F + a * N;
        double* Sa = FS + a * N;
#pragma omp parallel for schedule(static)
        for (long k = 0; k < g->nz; ++k)
            for (long j = 0; j < g->ny; ++j)
                for (long i = 0; i < g->nx; ++i) {
                    long c = at(g, i, j, k);
                    if (!inside(g, i, j, k)) {
                        Sa[c] = 0.0;
                        continue;
                    }
                    const long p = c + st[a], m = c - st[a];
                    Sa[c] = 0.25 * (Fa[m] + 2.0 * Fa[c] + Fa[p]) - (phi[p] - phi[m]) / (2.0 * h[a]);
                }
    }
    return ORA_OK;
}

/* Pre-computation stage of the separable projection: b = div F,
 * solve lap phi = b (as A phi = -b), FS = F - grad phi.  phi and FS are
 * outputs (N and 3N).  b == 0 gives phi = 0, zero iterations. */
int ora_project(const ora_grid* g, const double* F, double* FS, double* phi, double tol, long max_iter,
                long fixed_iters, int jacobi, ora_report* rep) {
    if (!grid_ok(g) || !F || !FS || !phi || !rep) return ORA_EINVAL;
    const long N = ncell(g);
    double* b = (double*)malloc(sizeof(double) * N);
    if (!b) return ORA_ENOMEM;
    ora_divergence(g, F, b);
    for (long c = 0; c < N; ++c) b[c] = -b[c];
    int st = ora_cg(g, b, phi, tol, max_iter, fixed_iters, jacobi, rep);
    ora_grad_subtract(g, F, phi, FS);
    free(b);
    return st;
}

/* ---- sponge ---- */

/* Linear ramp over L cells from each face: r = max(0, (L - d)/L) with d the
 * distance (in cells) to the nearest outer face along that axis;
 * sigma = smax * max(r_x, r_y, r_z). */
double ora_sponge_sigma(const ora_grid* g, long i, long j, long k, int L, double smax) {
    if (L <= 0) return 0.0;
    const long idx[3] = {i, j, k};
    const long n[3] = {g->nx, g->ny, g->nz};
    double rmax = 0.0;
    for (int a = 0; a < 3; ++a) {
        long d = idx[a] < n[a] - 1 - idx[a] ? idx[a] : n[a] - 1 - idx[a];
        double r = (double)(L - d) / (double)L;
        if (r > rmax) rmax = r;
    }
    return smax * rmax;
}

/* Default ramp strength: 6 ln(10) c_max / (L h_min), which makes the one-way
 * amplitude factor through the ramp about 10^-1.5. */
double ora_default_sigma_max(const ora_grid* g, const double* G, const double* rho, int L) {
    if (L <= 0) return 0.0;
    const long N = ncell(g);
    double cmax = 0.0;
    for (long c = 0; c < N; ++c) {
        double cs = sqrt(G[c] / rho[c]);
        if (cs > cmax) cmax = cs;
    }
    double hmin = g->hx;
    if (g->hy < hmin) hmin = g->hy;
    if (g->hz < hmin) hmin = g->hz;
    return 6.0 * log(10.0) * cmax / ((double)L * hmin);
}

/* ---- stable time step ---- */

/* Per cell: A = 4 dt^2 (Gmax_face/rho) S, B = 4 dt (eta/rho) S with
 * S = sum_a 1/h_a^2; dt_max solves A + 2B = 4 (positive root), minimum over
 * interior cells. */
double ora_stable_dt(const ora_grid* g, const double* G, const double* rho, const double* eta) {
    if (!grid_ok(g)) return NAN;
    const double S = 1.0 / (g->hx * g->hx) + 1.0 / (g->hy * g->hy) + 1.0 / (g->hz * g->hz);
    const long st[3] = {1, g->nx, g->nx * g->ny};
    double best = INFINITY;
    for (long k = 1; k < g->nz - 1; ++k)
        for (long j = 1; j < g->ny - 1; ++j)
            for (long i = 1; i < g->nx - 1; ++i) {
                const long c = at(g, i, j, k);
                double gmax = 0.0;
                for (int a = 0; a < 3; ++a) {
                    double gp = harmonic(G[c], G[c + st[a]]);
                    double gm = harmonic(G[c], G[c - st[a]]);
                    if (gp > gmax) gmax = gp;
                    if (gm > gmax) gmax = gm;
                }
                /* a dt^2 + b dt - 1 = 0 with a = (Gmax/rho) S, b = 2 (eta/rho) S */
                const double qa = gmax / rho[c] * S;
                const double qb = 2.0 * eta[c] / rho[c] * S;
                const double dt = (-qb + sqrt(qb * qb + 4.0 * qa)) / (2.0 * qa);
                if (dt < best) best = dt;
            }
    return best;
}

/* ---- time stepping ---- */

/* One update of cell (i,j,k), all three components:
 *   acc = E(u_c) + eta lap(w_c)/dt + gn FS_c
 *   w'  = [(1 - s) w_c + (dt^2/rho) acc] / (1 + s),  s = sigma dt / 2
 *   u'  = u_c + w'
 * This is the leapfrog u^{n+1} = 2u^n - u^{n-1} + dt^2 a^n of Sec. 3.1 with
 * u_dot = (u^n - u^{n-1})/dt and the centred damping term
 * sigma (u^{n+1} - u^{n-1}) / (2 dt). */
static void cell_update(const ora_grid* g, const double* G, const double* rho, const double* eta, int L,
                        double smax, double dt, const double* FS, double gn, const double* u, const double* w,
                        long i, long j, long k, double un[3], double wn[3]) {
    const long N = ncell(g);
    const long c = at(g, i, j, k);
    const long st[3] = {1, g->nx, g->nx * g->ny};
    const double h[3] = {g->hx, g->hy, g->hz};
    const double s = 0.5 * ora_sponge_sigma(g, i, j, k, L, smax) * dt;
    for (int comp = 0; comp < 3; ++comp) {
        const double* uc = u + comp * N;
        const double* wc = w + comp * N;
        const double E = elastic_at(g, G, uc, i, j, k);
        double lapw = 0.0;
        for (int a = 0; a < 3; ++a) lapw += (wc[c + st[a]] - 2.0 * wc[c] + wc[c - st[a]]) / (h[a] * h[a]);
        double acc = E + eta[c] * lapw / dt;
        if (FS && gn != 0.0) acc += gn * FS[comp * N + c];
        wn[comp] = ((1.0 - s) * wc[c] + dt * dt / rho[c] * acc) / (1.0 + s);
        un[comp] = uc[c] + wn[comp];
    }
}

/*
 * Advance (u, w) by nsteps from absolute step index step0.  u, w: [3][N],
 * updated in place (outer layer must be zero and stays zero).  The source at
 * step n is env[n] * FS when n < n_env, else 0 (FS may be NULL).  After each
 * step the probe values of u are written to
 * traces[(s * nprobes + p) * ncomp + c], ncomp = 3 when comp == 3 else 1.
 */
int ora_run(const ora_grid* g, const double* G, const double* rho, const double* eta, int L, double smax,
            double dt, const double* FS, const double* env, long n_env, double* u, double* w, long step0,
            long nsteps, const long* probes, long nprobes, int comp, double* traces) {
    if (!grid_ok(g) || dt <= 0 || nsteps < 0) return ORA_EINVAL;
    const long N = ncell(g);
    double* un = (double*)calloc(3 * N, sizeof(double));
    double* wn = (double*)calloc(3 * N, sizeof(double));
    if (!un || !wn) {
        free(un), free(wn);
        return ORA_ENOMEM;
    }
    const int ncomp = comp == 3 ? 3 : 1;
    for (long s = 0; s < nsteps; ++s) {
        const long n = step0 + s;
        const double gn = (env && n < n_env) ? env[n] : 0.0;
#pragma omp parallel for schedule(static)
        for (long k = 1; k < g->nz - 1; ++k)
            for (long j = 1; j < g->ny - 1; ++j)
                for (long i = 1; i < g->nx - 1; ++i) {
                    double a[3], b[3];
                    cell_update(g, G, rho, eta, L, smax, dt, FS, gn, u, w, i, j, k, a, b);
                    const long c = at(g, i, j, k);
                    for (int q = 0; q < 3; ++q) {
                        un[q * N + c] = a[q];
                        wn[q * N + c] = b[q];
                    }
                }
        memcpy(u, un, sizeof(double) * 3 * N);
        memcpy(w, wn, sizeof(double) * 3 * N);
        for (long p = 0; p < nprobes; ++p) {
            const long i = probes[3 * p], j = probes[3 * p + 1], k = probes[3 * p + 2];
            const long c = at(g, i, j, k);
            for (int q = 0; q < ncomp; ++q) {
                const int cc = ncomp == 3 ? q : comp;
                traces[(s * nprobes + p) * ncomp + q] = u[cc * N + c];
            }
        }
    }
    free(un), free(wn);
    return ORA_OK;
}

/* One step evaluated only at the listed interior cells (flattened indices),
 * from a full state (u, w): the sampled check used at sizes where the full
 * oracle run is too slow.  u_out, w_out: [ncells][3]. */
int ora_step_cells(const ora_grid* g, const double* G, const double* rho, const double* eta, int L, double smax,
                   double dt, const double* FS, double gn, const double* u, const double* w, const long* cells,
                   long ncells, double* u_out, double* w_out) {
    if (!grid_ok(g)) return ORA_EINVAL;
    for (long q = 0; q < ncells; ++q) {
        const long c = cells[q];
        const long i = c % g->nx, j = (c / g->nx) % g->ny, k = c / (g->nx * g->ny);
        if (!inside(g, i, j, k)) return ORA_EINVAL;
        cell_update(g, G, rho, eta, L, smax, dt, FS, gn, u, w, i, j, k, u_out + 3 * q, w_out + 3 * q);
    }
    return ORA_OK;
}
