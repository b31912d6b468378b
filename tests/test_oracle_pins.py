"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed-form
eigenpairs of the 7-point Laplacian, hand-computed stencil values, an exact
DST-I Poisson solve, a Kronecker-assembled dense solve, conservation of the
discrete energy, the closed-form solution of the one-mode recurrence, the
paper's printed update (three-level form), and the theoretical columns of the
paper's Kelvin-Voigt table (Sec. 4.3, Table 3).
"""
import os

import numpy as np
import pytest
import scipy.fft
import scipy.linalg
import scipy.sparse as sp

import oracle
from oracle import dispersion

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def interior(a):
    return a[..., 1:-1, 1:-1, 1:-1]


def sine_mode(grid, p, q, r):
    nx, ny, nz = grid[:3]
    i, j, k = np.arange(nx), np.arange(ny), np.arange(nz)
    sx = np.sin(p * np.pi * i / (nx - 1))
    sy = np.sin(q * np.pi * j / (ny - 1))
    sz = np.sin(r * np.pi * k / (nz - 1))
    return sz[:, None, None] * sy[None, :, None] * sx[None, None, :]


def mode_lambda(grid, p, q, r):
    nx, ny, nz, hx, hy, hz = grid
    return (4 / hx ** 2 * np.sin(p * np.pi / (2 * (nx - 1))) ** 2
            + 4 / hy ** 2 * np.sin(q * np.pi / (2 * (ny - 1))) ** 2
            + 4 / hz ** 2 * np.sin(r * np.pi / (2 * (nz - 1))) ** 2)


GRID_A = (9, 7, 11, 1.0e-3, 0.7e-3, 1.3e-3)


# ---------------------------------------------------------------- operators

@pytest.mark.parametrize("pqr", [(1, 1, 1), (2, 3, 5), (7, 5, 9)])
def test_laplacian_sine_mode_eigenpair(pqr):
    """lap_h of a Dirichlet sine mode is -lambda times the mode, with
    lambda = sum_a (4/h_a^2) sin^2(p_a pi / (2(n_a - 1)))."""
    q = sine_mode(GRID_A, *pqr)
    L = oracle.laplacian(GRID_A, q)
    lam = mode_lambda(GRID_A, *pqr)
    np.testing.assert_allclose(interior(L), -lam * interior(q), rtol=0, atol=1e-12 * lam)
    assert np.all(L[0] == 0) and np.all(L[-1] == 0)


def test_elastic_uniform_modulus_is_G_laplacian():
    G = 2.5e3
    q = sine_mode(GRID_A, 2, 1, 3)
    E = oracle.elastic(GRID_A, G, q)
    lam = mode_lambda(GRID_A, 2, 1, 3)
    np.testing.assert_allclose(interior(E), -G * lam * interior(q), rtol=0, atol=1e-12 * G * lam)


def test_elastic_hand_computed_interface():
    """5x3x3 grid, h = 1: G = 1 for i <= 1, 3 for i >= 2; u along the x line
    (j = k = 1) = (0, 1, 2, 4, 0), zero elsewhere.  At (2,1,1):
    x+ face 3*(4-2) = 6, x- face harmonic(1,3) = 1.5 -> -1.5*(2-1),
    y and z faces 3*(0-2) - 3*(2-0) = -12 each: total -19.5."""
    grid = (5, 3, 3, 1.0, 1.0, 1.0)
    G = np.ones((3, 3, 5))
    G[:, :, 2:] = 3.0
    u = np.zeros((3, 3, 5))
    u[1, 1, :] = [0, 1, 2, 4, 0]
    E = oracle.elastic(grid, G, u)
    assert E[1, 1, 2] == pytest.approx(-19.5, abs=1e-14)
    # cell (1,1,1): x+ face harmonic(1,3)(2-1) = 1.5, x- face 1*(1-0),
    # y, z faces with G = 1: -2 each
    assert E[1, 1, 1] == pytest.approx(1.5 - 1.0 - 2.0 - 2.0, abs=1e-14)


def test_elastic_operator_is_symmetric():
    rng = np.random.default_rng(7)
    grid = (10, 9, 8, 0.3e-3, 0.25e-3, 0.35e-3)
    shp = (8, 9, 10)
    G = np.exp(rng.normal(8.0, 1.0, shp))
    u = rng.standard_normal(shp)
    v = rng.standard_normal(shp)
    for a in (u, v):
        a[0], a[-1], a[:, 0], a[:, -1], a[:, :, 0], a[:, :, -1] = 0, 0, 0, 0, 0, 0
    Eu, Ev = oracle.elastic(grid, G, u), oracle.elastic(grid, G, v)
    lhs, rhs = np.vdot(v, Eu), np.vdot(Ev, u)
    assert abs(lhs - rhs) <= 1e-12 * np.sqrt(np.vdot(Eu, Eu) * np.vdot(v, v))
    assert np.vdot(u, Eu) < 0  # negative definite on interior vectors


def test_divergence_of_sines_is_exact():
    """Centred difference of sin(a x) is cos(a x) sin(a h)/h exactly."""
    grid = (12, 10, 9, 0.4e-3, 0.5e-3, 0.3e-3)
    nx, ny, nz, hx, hy, hz = grid
    x = (np.arange(nx) - nx // 2) * hx
    y = (np.arange(ny) - ny // 2) * hy
    z = (np.arange(nz) - nz // 2) * hz
    a, b, c = 900.0, 1300.0, 700.0
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    F = np.stack([np.sin(a * X), np.sin(b * Y), np.sin(c * Z)])
    expect = (np.cos(a * X) * np.sin(a * hx) / hx + np.cos(b * Y) * np.sin(b * hy) / hy
              + np.cos(c * Z) * np.sin(c * hz) / hz)
    d = oracle.divergence(grid, F)
    np.testing.assert_allclose(interior(d), interior(expect), atol=1e-9 * np.abs(expect).max())
    assert np.all(d[0] == 0) and np.all(d[:, :, -1] == 0)


# ---------------------------------------------------------------- Poisson

def dst_poisson(grid, b):
    """Exact solution of lap_h phi = b (Dirichlet box) by DST-I."""
    nx, ny, nz, hx, hy, hz = grid
    bi = interior(b)
    lam = (4 / hz ** 2 * np.sin(np.arange(1, nz - 1) * np.pi / (2 * (nz - 1))) ** 2)[:, None, None] \
        + (4 / hy ** 2 * np.sin(np.arange(1, ny - 1) * np.pi / (2 * (ny - 1))) ** 2)[None, :, None] \
        + (4 / hx ** 2 * np.sin(np.arange(1, nx - 1) * np.pi / (2 * (nx - 1))) ** 2)[None, None, :]
    bh = scipy.fft.dstn(bi, type=1)
    phi_i = scipy.fft.idstn(bh / (-lam), type=1)
    phi = np.zeros_like(b)
    phi[1:-1, 1:-1, 1:-1] = phi_i
    return phi


def kron_laplacian(grid):
    """Interior 7-point Laplacian assembled as a Kronecker sum of 1-D
    second-difference matrices (independent of the oracle's loops)."""
    nx, ny, nz, hx, hy, hz = grid

    def d2(n, h):
        m = n - 2
        return sp.diags([np.ones(m - 1), -2 * np.ones(m), np.ones(m - 1)], [-1, 0, 1]) / h ** 2

    Ix, Iy, Iz = (sp.identity(n - 2) for n in (nx, ny, nz))
    # x fastest: kron order z (slowest), y, x (fastest)
    return (sp.kron(sp.kron(Iz, Iy), d2(nx, hx)) + sp.kron(sp.kron(Iz, d2(ny, hy)), Ix)
            + sp.kron(sp.kron(d2(nz, hz), Iy), Ix)).toarray()


def random_interior(grid, rng):
    nx, ny, nz = grid[:3]
    b = np.zeros((nz, ny, nx))
    b[1:-1, 1:-1, 1:-1] = rng.standard_normal((nz - 2, ny - 2, nx - 2))
    return b


@pytest.mark.parametrize("jacobi", [False, True])
def test_cg_matches_exact_dst_solution(jacobi):
    grid = (24, 20, 28, 0.5e-3, 0.4e-3, 0.6e-3)
    b = random_interior(grid, np.random.default_rng(3))
    phi, rep = oracle.cg(grid, -b, tol=1e-13, max_iter=5000, jacobi=jacobi)
    exact = dst_poisson(grid, b)
    assert rep["status"] == 0
    assert np.linalg.norm(phi - exact) <= 1e-10 * np.linalg.norm(exact)
    assert rep["relres_true"] < 1e-12


def test_cg_matches_dense_solve_small_grid():
    grid = (9, 8, 7, 1.0, 1.3, 0.8)
    b = random_interior(grid, np.random.default_rng(11))
    A = kron_laplacian(grid)
    phi_d = scipy.linalg.solve(A, interior(b).ravel())
    phi, rep = oracle.cg(grid, -b, tol=1e-14, max_iter=1000)
    np.testing.assert_allclose(interior(phi).ravel(), phi_d, rtol=0, atol=1e-11 * np.abs(phi_d).max())


def test_cg_energy_error_decreases_monotonically():
    """CG minimises the A-norm of the error over growing Krylov spaces, so the
    A-norm error after k fixed iterations never increases with k."""
    grid = (16, 16, 16, 1.0, 1.0, 1.0)
    b = random_interior(grid, np.random.default_rng(5))
    exact = dst_poisson(grid, b)
    errs = []
    for k in range(1, 40, 3):
        phi, rep = oracle.cg(grid, -b, fixed_iters=k)
        assert rep["iters"] == k
        e = phi - exact
        errs.append(np.vdot(e, -oracle.laplacian(grid, e)))
    assert all(e2 <= e1 * (1 + 1e-12) for e1, e2 in zip(errs, errs[1:]))


def test_jacobi_pcg_equals_cg_for_constant_diagonal():
    grid = (20, 18, 22, 0.5e-3, 0.5e-3, 0.25e-3)
    b = random_interior(grid, np.random.default_rng(9))
    p1, r1 = oracle.cg(grid, -b, tol=1e-10)
    p2, r2 = oracle.cg(grid, -b, tol=1e-10, jacobi=True)
    assert r1["iters"] == r2["iters"]
    assert np.linalg.norm(p1 - p2) <= 1e-12 * np.linalg.norm(p1)


def test_cg_stop_rule_and_guards():
    grid = (10, 10, 10, 1.0, 1.0, 1.0)
    b = random_interior(grid, np.random.default_rng(1))
    # zero right-hand side: no iteration, phi = 0
    phi, rep = oracle.cg(grid, np.zeros_like(b), tol=1e-8)
    assert rep["iters"] == 0 and rep["status"] == 0 and not phi.any()
    # max_iter reached above tolerance -> not converged, phi still returned
    phi, rep = oracle.cg(grid, -b, tol=1e-12, max_iter=1)
    assert rep["iters"] == 1 and rep["status"] == oracle.ENOTCONV and phi.any()
    # non-finite right-hand side -> breakdown
    bad = b.copy()
    bad[5, 5, 5] = np.nan
    phi, rep = oracle.cg(grid, bad, tol=1e-8)
    assert rep["status"] == oracle.EBREAKDOWN
    # the stop test is on sqrt(r.r / r0.r0): the recursive residual at exit is
    # below tol and one iteration fewer is not
    phi, rep = oracle.cg(grid, -b, tol=1e-6)
    assert rep["relres_recursive"] < 1e-6
    _, rep2 = oracle.cg(grid, -b, fixed_iters=rep["iters"] - 1)
    assert rep2["relres_recursive"] >= 1e-6


# ---------------------------------------------------------------- projection

def face_field_divergence(grid, F, phi):
    """D- of the face field H_a = (F_a + F_a(+a))/2 - (phi(+a) - phi)/h_a,
    and the cell average of H, written from the face definitions."""
    nx, ny, nz, hx, hy, hz = grid
    h = (hx, hy, hz)
    axes = (2, 1, 0)  # numpy axis of x, y, z
    div = np.zeros((nz - 2, ny - 2, nx - 2))
    avg = np.zeros((3, nz - 2, ny - 2, nx - 2))
    for a in range(3):
        ax = axes[a]
        Fa = F[a]
        n = Fa.shape[ax]
        lo = [slice(1, -1)] * 3
        hi = [slice(1, -1)] * 3
        lo[ax] = slice(0, n - 1)
        hi[ax] = slice(1, n)
        H = 0.5 * (Fa[tuple(lo)] + Fa[tuple(hi)]) - (phi[tuple(hi)] - phi[tuple(lo)]) / h[a]
        s0 = [slice(None)] * 3
        s1 = [slice(None)] * 3
        s0[ax] = slice(0, -1)
        s1[ax] = slice(1, None)
        div += (H[tuple(s1)] - H[tuple(s0)]) / h[a]
        avg[a] = 0.5 * (H[tuple(s1)] + H[tuple(s0)])
    return div, avg


def test_projection_face_field_is_divergence_free_to_cg_tolerance():
    from workloads import gaussian_push
    grid = (24, 26, 22, 0.5e-3, 0.5e-3, 0.5e-3)
    rng = np.random.default_rng(2)
    F = gaussian_push(grid, 1.5e-3, 3e-3, 1e4) + 100.0 * rng.standard_normal((3, 22, 26, 24))
    FS, phi, rep = oracle.project(grid, F, tol=1e-11)
    b = oracle.divergence(grid, F)
    div, avg = face_field_divergence(grid, F, phi)
    assert np.linalg.norm(div) / np.linalg.norm(interior(b)) == pytest.approx(rep["relres_true"], rel=1e-3, abs=1e-14)
    assert rep["relres_true"] < 2e-11
    # the returned cell-centred FS is the cell average of the face field
    np.testing.assert_allclose(avg, FS[:, 1:-1, 1:-1, 1:-1], atol=1e-12 * np.abs(FS).max())
    assert not FS[:, 0].any() and not FS[:, :, :, -1].any()
    # phi equals the DST-exact solution of lap phi = div F to CG accuracy
    exact = dst_poisson(grid, b)
    assert np.linalg.norm(phi - exact) <= 1e-9 * np.linalg.norm(exact)


def test_projection_is_linear_for_separable_force():
    """P[b0 g] = g P[b0] (Sec. 3.3): with fixed iterations the projection of
    a scaled pattern is the scaled projection."""
    from workloads import gaussian_push
    grid = (20, 20, 20, 0.5e-3, 0.5e-3, 0.5e-3)
    F = gaussian_push(grid, 1e-3, 4e-3, 1e4)
    FS1, _, r1 = oracle.project(grid, F, fixed_iters=60)
    FS2, _, r2 = oracle.project(grid, 0.37 * F, fixed_iters=60)
    np.testing.assert_allclose(FS2, 0.37 * FS1, rtol=0, atol=1e-12 * np.abs(FS1).max())


def test_gaussian_push_projection_symmetry():
    """On an odd grid the z-directed Gaussian push centred on the centre node
    is even in x and y, so FS_z is even and FS_x odd in x."""
    from workloads import gaussian_push
    grid = (21, 21, 25, 0.5e-3, 0.5e-3, 0.5e-3)
    F = gaussian_push(grid, 1e-3, 3e-3, 1e4)
    FS, phi, rep = oracle.project(grid, F, tol=1e-12)
    np.testing.assert_allclose(FS[2], FS[2][:, :, ::-1], atol=1e-10 * np.abs(FS).max())
    np.testing.assert_allclose(FS[0], -FS[0][:, :, ::-1], atol=1e-10 * np.abs(FS).max())
    np.testing.assert_allclose(FS[2], FS[2][::-1, :, :], atol=1e-10 * np.abs(FS).max())


# ---------------------------------------------------------------- time stepping

def lap_numpy(q, h):
    """7-point Laplacian by array slicing (test-local, interior only)."""
    out = np.zeros_like(q)
    c = q[1:-1, 1:-1, 1:-1]
    out[1:-1, 1:-1, 1:-1] = ((q[1:-1, 1:-1, 2:] - 2 * c + q[1:-1, 1:-1, :-2]) / h[0] ** 2
                             + (q[1:-1, 2:, 1:-1] - 2 * c + q[1:-1, :-2, 1:-1]) / h[1] ** 2
                             + (q[2:, 1:-1, 1:-1] - 2 * c + q[:-2, 1:-1, 1:-1]) / h[2] ** 2)
    return out


def test_summed_form_equals_paper_three_level_update():
    """The paper's update u^{n+1} = 2u^n - u^{n-1} + dt^2 a^n with
    a^n = (mu/rho) lap u^n + (eta/rho) lap((u^n - u^{n-1})/dt) + g_n f/rho
    (Sec. 3.1, 3.3), run here in its printed three-level form for a
    homogeneous medium without sponge, equals the oracle's summed form."""
    from workloads import gaussian_push
    grid = (14, 12, 16, 0.5e-3, 0.5e-3, 0.5e-3)
    h = grid[3:]
    G, rho, eta, dt, nsteps = 3e3, 1000.0, 0.4, 2e-5, 150
    F = gaussian_push(grid, 1e-3, 2e-3, 1e4)
    FS, _, _ = oracle.project(grid, F, tol=1e-12)
    env = np.array([1.0, 1.0, 0.5, 1.0])
    probes = np.array([[i, 6, 8] for i in range(14)])
    _, _, tr = oracle.run(grid, G, rho, eta, dt, nsteps, FS=FS, env=env, probes=probes, comp=3)
    u_prev = np.zeros_like(FS)
    u = np.zeros_like(FS)
    ref = np.zeros_like(tr)
    for n in range(nsteps):
        g = env[n] if n < len(env) else 0.0
        u_next = np.empty_like(u)
        for c in range(3):
            a = (G / rho) * lap_numpy(u[c], h) + (eta / rho) * lap_numpy((u[c] - u_prev[c]) / dt, h) \
                + g * FS[c] / rho
            u_next[c] = 2 * u[c] - u_prev[c] + dt * dt * a
            u_next[c][0], u_next[c][-1] = 0, 0
            u_next[c][:, 0], u_next[c][:, -1] = 0, 0
            u_next[c][:, :, 0], u_next[c][:, :, -1] = 0, 0
        u_prev, u = u, u_next
        ref[n] = u[:, 8, 6, :].T
    assert np.linalg.norm(tr - ref) <= 1e-12 * np.linalg.norm(ref)


def test_discrete_energy_is_conserved_heterogeneous():
    """With eta = 0, no sponge and no force, the leapfrog with the
    conservative operator K = -E conserves
    E^{n+1/2} = 1/2 sum rho (w^{n+1}/dt)^2 + 1/2 (u^{n+1})^T K u^n,
    which holds only if E is symmetric and the update is the leapfrog."""
    rng = np.random.default_rng(4)
    grid = (12, 11, 13, 0.4e-3, 0.5e-3, 0.45e-3)
    shp = (13, 11, 12)
    G = np.exp(rng.uniform(np.log(1e3), np.log(1e4), shp))
    rho = rng.uniform(1000, 1100, shp)
    dt = 0.5 * oracle.stable_dt(grid, G, rho, 0.0)
    u0 = np.zeros((3,) + shp)
    w0 = np.zeros((3,) + shp)
    u0[:, 1:-1, 1:-1, 1:-1] = 1e-6 * rng.standard_normal((3, 11, 9, 10))
    w0[:, 1:-1, 1:-1, 1:-1] = 1e-7 * rng.standard_normal((3, 11, 9, 10))

    def energy(u_new, w_new, u_old):
        kin = 0.5 * np.sum(rho[None] * (w_new / dt) ** 2)
        pot = -0.5 * sum(np.vdot(u_new[c], oracle.elastic(grid, G, u_old[c])) for c in range(3))
        return kin + pot

    u, w = u0, w0
    es = []
    for _ in range(20):
        u1, w1, _ = oracle.run(grid, G, rho, 0.0, dt, 50, u=u, w=w)
        u_old = u1 - w1
        es.append(energy(u1, w1, u_old))
        u, w = u1, w1
    es = np.array(es)
    assert np.max(np.abs(es - es[0])) <= 1e-12 * abs(es[0])


@pytest.mark.parametrize("eta", [0.0, 0.3, 1.5])
def test_single_mode_follows_closed_form_recurrence(eta):
    """A Dirichlet sine mode stays a mode; its amplitude obeys the scalar
    recurrence whose characteristic roots solve
    z^2 + (a + b - 2) z + (1 - b) = 0, a = dt^2 G lam / rho,
    b = dt eta lam / rho.  Pins the viscous term (coefficient, sign, 1/dt)."""
    grid = (11, 9, 10, 0.5e-3, 0.5e-3, 0.5e-3)
    G, rho = 3e3, 1000.0
    dt = 0.6 * oracle.stable_dt(grid, G, rho, eta)
    mode = sine_mode(grid, 2, 3, 1)
    lam = mode_lambda(grid, 2, 3, 1)
    u0, wm = 1e-6, 3e-8  # u^0 and w^0 = u^0 - u^{-1}
    u = np.zeros((3,) + mode.shape)
    w = np.zeros_like(u)
    u[1], w[1] = u0 * mode, wm * mode
    nsteps = 300
    probe = np.array([[4, 3, 4]])
    _, _, tr = oracle.run(grid, G, rho, eta, dt, nsteps, u=u, w=w, probes=probe, comp=1)
    amp = tr[:, 0, 0] / mode[4, 3, 4]
    z1, z2 = dispersion.mode_roots(lam, G, rho, eta, dt)
    # u^n = c1 z1^n + c2 z2^n with u^0 = u0, u^{-1} = u0 - wm
    M = np.array([[1, 1], [1 / z1, 1 / z2]])
    c1, c2 = np.linalg.solve(M, np.array([u0, u0 - wm], dtype=complex))
    n = np.arange(1, nsteps + 1)
    pred = (c1 * z1 ** n + c2 * z2 ** n).real
    np.testing.assert_allclose(amp, pred, rtol=0, atol=1e-9 * u0)


def test_sponge_ramp_hand_values_and_single_cell_damping():
    """Ramp over L = 8 cells on a 48-cell axis: index 0 -> 1, 4 -> 0.5,
    8 -> 0, 43 -> 0.5, 47 -> 1; sigma = smax * max over axes.  On a 3^3 grid
    the single interior cell sits at distance 1 from every face (ramp 7/8)
    and is its own Laplacian eigenmode (lambda = sum 2/h^2), so its damped
    recurrence has the characteristic polynomial
    (1+s) z^2 + (a + b - 2) z + (1 - s - b) with s = sigma dt / 2."""
    g48 = (48, 48, 48, 1.0, 1.0, 1.0)
    smax = 1000.0
    assert oracle.sponge_sigma(g48, 0, 24, 24, 8, smax) == pytest.approx(1000.0)
    assert oracle.sponge_sigma(g48, 4, 24, 24, 8, smax) == pytest.approx(500.0)
    assert oracle.sponge_sigma(g48, 8, 24, 24, 8, smax) == 0.0
    assert oracle.sponge_sigma(g48, 24, 43, 24, 8, smax) == pytest.approx(500.0)
    assert oracle.sponge_sigma(g48, 24, 24, 47, 8, smax) == pytest.approx(1000.0)
    assert oracle.sponge_sigma(g48, 2, 6, 30, 8, smax) == pytest.approx(750.0)
    assert oracle.sponge_sigma(g48, 2, 6, 30, 0, smax) == 0.0

    h = 0.5e-3
    grid = (3, 3, 3, h, h, h)
    G, rho, eta, smax = 3e3, 1000.0, 0.2, 4000.0
    dt = 0.5 * oracle.stable_dt(grid, G, rho, eta)
    s = 0.5 * smax * (7 / 8) * dt
    lam = 6 / h ** 2
    u = np.zeros((3, 3, 3, 3))
    w = np.zeros_like(u)
    u[0, 1, 1, 1], w[0, 1, 1, 1] = 1.0, 0.01
    _, _, tr = oracle.run(grid, G, rho, eta, dt, 200, u=u, w=w, probes=np.array([[1, 1, 1]]), comp=0,
                          sponge_cells=8, sigma_max=smax)
    z1, z2 = dispersion.mode_roots(lam, G, rho, eta, dt, s=s)
    M = np.array([[1, 1], [1 / z1, 1 / z2]])
    c1, c2 = np.linalg.solve(M, np.array([1.0, 0.99], dtype=complex))
    n = np.arange(1, 201)
    np.testing.assert_allclose(tr[:, 0, 0], (c1 * z1 ** n + c2 * z2 ** n).real, atol=1e-12)


def test_default_sponge_strength():
    """6 ln(10) c_max / (L h_min): for G = 3 kPa, rho = 1000, L = 8,
    h = 0.5 mm this is about 5982 1/s."""
    g = (10, 10, 10, 0.5e-3, 0.5e-3, 0.5e-3)
    smax = oracle.default_sigma_max(g, 3e3, 1000.0, 8)
    assert smax == pytest.approx(6 * np.log(10) * np.sqrt(3.0) / (8 * 0.5e-3), rel=1e-14)
    assert 5970 < smax < 5990


# ---------------------------------------------------------------- stability

def test_stable_dt_reduces_to_cfl_bound_without_viscosity():
    """eta = 0: dt_max = (1/c_s)(1/dx^2 + 1/dy^2 + 1/dz^2)^(-1/2) (Sec. 3.1)."""
    grid = (8, 9, 10, 0.5e-3, 0.4e-3, 0.3e-3)
    G, rho = 3e3, 1000.0
    cs = np.sqrt(G / rho)
    expect = 1 / cs / np.sqrt(sum(1 / h ** 2 for h in grid[3:]))
    assert oracle.stable_dt(grid, G, rho, 0.0) == pytest.approx(expect, rel=1e-14)


def test_stable_dt_viscous_root_and_jury_boundary():
    """With viscosity the bound is the positive root of A + 2B = 4; at that dt
    the highest Laplacian eigenvalue 4 sum(1/h^2) gives a root of modulus 1
    of the mode recurrence (Jury boundary), and just below it all roots are
    inside the unit circle."""
    grid = (8, 8, 8, 0.25e-3, 0.25e-3, 0.25e-3)
    G, rho, eta = 2e3, 1000.0, 0.5
    dt = oracle.stable_dt(grid, G, rho, eta)
    S = 3 / 0.25e-3 ** 2
    A = 4 * dt ** 2 * G / rho * S
    B = 4 * dt * eta / rho * S
    assert A + 2 * B == pytest.approx(4.0, rel=1e-12)
    lam_max = 4 * S
    assert max(abs(dispersion.mode_roots(lam_max, G, rho, eta, dt))) == pytest.approx(1.0, abs=1e-6)
    assert max(abs(dispersion.mode_roots(lam_max, G, rho, eta, 0.999 * dt))) < 1.0
    assert max(abs(dispersion.mode_roots(lam_max, G, rho, eta, 1.001 * dt))) > 1.0


def test_run_grows_above_and_stays_bounded_below_mode_limit():
    """On a finite grid the largest eigenvalue is lam_max < 4 sum(1/h^2);
    the run blows up slightly above the dt where that mode reaches the unit
    circle and stays bounded slightly below it."""
    grid = (7, 7, 7, 0.5e-3, 0.5e-3, 0.5e-3)
    G, rho, eta = 3e3, 1000.0, 0.3
    lam_max = mode_lambda(grid, 5, 5, 5)
    dts = np.linspace(0.5, 1.5, 20001) * oracle.stable_dt(grid, G, rho, eta)
    ok = [max(abs(dispersion.mode_roots(lam_max, G, rho, eta, d))) <= 1.0 for d in dts]
    dt_lim = dts[np.argmin(ok)]  # first unstable
    rng = np.random.default_rng(0)
    u = np.zeros((3, 7, 7, 7))
    u[:, 1:-1, 1:-1, 1:-1] = rng.standard_normal((3, 5, 5, 5))
    _, _, tr_hi = oracle.run(grid, G, rho, eta, 1.01 * dt_lim, 3000, u=u, probes=np.array([[3, 3, 3]]), comp=3)
    _, _, tr_lo = oracle.run(grid, G, rho, eta, 0.99 * dt_lim, 3000, u=u, probes=np.array([[3, 3, 3]]), comp=3)
    assert np.abs(tr_hi).max() > 1e3
    assert np.abs(tr_lo).max() < 10.0


# ---------------------------------------------------------------- Kelvin-Voigt

def load_kv_table():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "kv_table.txt")) if l.strip() and not l.startswith("#")]
    return np.array(rows, dtype=float)


def test_kv_closed_form_reproduces_paper_table():
    """With c_s = 2 m/s (G = 4 kPa, rho = 1000) the drive frequency that
    gives the table's alpha_th predicts its c_th to the printed digits."""
    from scipy.optimize import brentq
    tab = load_kv_table()
    G, rho = 4e3, 1000.0
    for eta, alpha_th, c_th in tab:
        f = lambda w: dispersion.kv_attenuation_speed(w, G, rho, eta)[0] - alpha_th
        w = brentq(f, 2 * np.pi * 50, 2 * np.pi * 5000)
        _, c = dispersion.kv_attenuation_speed(w, G, rho, eta)
        assert abs(c - c_th) <= 0.0006, (eta, c, c_th)
        assert 700 < w / (2 * np.pi) < 850


def test_kv_low_loss_limit():
    """alpha -> eta w^2 / (2 rho c^3) as De_v = w eta / G -> 0."""
    G, rho, eta = 4e3, 1000.0, 0.01
    w = 2 * np.pi * 100
    a, _ = dispersion.kv_attenuation_speed(w, G, rho, eta)
    assert a == pytest.approx(dispersion.kv_low_loss_alpha(w, G, rho, eta), rel=1e-3)


def test_discrete_dispersion_converges_to_kelvin_voigt():
    """The scheme's wavenumber tends to the continuous Kelvin-Voigt one at
    second order in h (dt = 0.3 x the stability limit, tied to h)."""
    G, rho, eta = 4e3, 1000.0, 0.5
    w = 2 * np.pi * 760
    k = dispersion.kv_wavenumber(w, G, rho, eta)
    errs = []
    for h in (0.4e-3, 0.2e-3, 0.1e-3):
        S = 1 / h ** 2
        qa, qb = G / rho * S, 2 * eta / rho * S
        dt = 0.3 * (-qb + np.sqrt(qb * qb + 4 * qa)) / (2 * qa)
        errs.append(abs(dispersion.discrete_wavenumber(w, G, rho, eta, h, dt) - k) / abs(k))
    p1 = np.log(errs[0] / errs[1]) / np.log(2)
    p2 = np.log(errs[1] / errs[2]) / np.log(2)
    assert p1 > 0.9 and p2 > 0.9 and errs[-1] < 1e-2


def test_mode_recurrence_matches_discrete_dispersion():
    """For a mode with Laplacian eigenvalue K^2, the recurrence roots are
    exp(-i w dt) with w such that the discrete dispersion maps back to K."""
    G, rho, eta, h = 4e3, 1000.0, 0.3, 0.2e-3
    dt = 1e-6
    kx = 2 * np.pi / 3e-3
    K2 = 4 / h ** 2 * np.sin(kx * h / 2) ** 2
    z = dispersion.mode_roots(K2, G, rho, eta, dt)
    z = z[np.argmin(np.angle(z))]  # the root exp(-i w dt) with w > 0
    w = 1j * np.log(z) / dt  # complex frequency
    # time-decaying mode: evaluate the discrete relation at complex w
    zz = np.exp(-1j * w * dt)
    K2b = (rho / dt ** 2) * (2 - zz - 1 / zz) / (G + (eta / dt) * (1 - 1 / zz))
    assert K2b == pytest.approx(K2, rel=1e-9)


def _small_push_case(shape, seed):
    from workloads import gaussian_push, spherical_inclusions
    nx, ny, nz = shape
    h = 0.25e-3
    grid = (nx, ny, nz, h, h * 1.1, h * 0.9)
    rng = np.random.default_rng(seed)
    G, rho, eta, _ = spherical_inclusions(grid, rng, 3, (2e3, 1000.0, 0.5), (0.5e-3, 1e-3),
                                          (1e3, 1e4), (1000.0, 1100.0), (0.0, 1.5), 2)
    F = gaussian_push(grid, 0.5e-3, 1e-3, 1e4) + 50.0 * rng.standard_normal((3, nz, ny, nx))
    return grid, G, rho, eta, F


def test_peak_maps_equal_the_running_max_of_probe_traces():
    """The peak map of a plane is the largest |u| over the recorded states at
    every cell of the plane: rebuilt from all-component probe traces (the
    oracle's C sensor path, not the plane slicing) on three orthogonal planes
    of a heterogeneous viscous run with a sponge and a force switched off
    part way."""
    grid, G, rho, eta, F = _small_push_case((11, 9, 13), 5)
    nx, ny, nz = grid[:3]
    dt = 0.5 * oracle.stable_dt(grid, G, rho, eta)
    FS, _, _ = oracle.project(grid, F, tol=1e-12)
    env = np.ones(7)
    planes = [(0, 4), (1, 6), (2, 3)]
    maps, u_end, _ = oracle.peak_maps(grid, G, rho, eta, dt, 30, planes, FS=FS, env=env, sponge_cells=2,
                                      sigma_max=3e3)
    for (axis, index), m in zip(planes, maps):
        if axis == 0:
            cells = [(index, j, k) for k in range(nz) for j in range(ny)]
        elif axis == 1:
            cells = [(i, index, k) for k in range(nz) for i in range(nx)]
        else:
            cells = [(i, j, index) for j in range(ny) for i in range(nx)]
        _, _, tr = oracle.run(grid, G, rho, eta, dt, 30, FS=FS, env=env, probes=np.array(cells), comp=3,
                              sponge_cells=2, sigma_max=3e3)
        ref = np.sqrt((tr ** 2).sum(axis=2)).max(axis=0).reshape(m.shape)
        assert m.max() > 0
        np.testing.assert_allclose(m, ref, rtol=1e-15, atol=0)
        # the map dominates the final state and is zero on the Dirichlet layer
        fin = oracle.plane_view(u_end, axis, index)
        assert np.all(m >= np.sqrt((fin ** 2).sum(axis=0)))
        assert not m[0].any() and not m[-1].any() and not m[:, 0].any() and not m[:, -1].any()


def test_peak_maps_mirror_symmetry_of_a_centred_push():
    """Homogeneous odd cube, square cells, z push on the centre node: the x
    and y slices through the centre carry the same map, and the z slice is
    symmetric under x <-> y and under both mirrors."""
    from workloads import gaussian_push
    n, h = 15, 0.3e-3
    grid = (n, n, n, h, h, h)
    F = gaussian_push(grid, 0.6e-3, 1.2e-3, 1e4)
    dt = 0.5 * oracle.stable_dt(grid, 2e3, 1000.0, 0.3)
    FS, _, _ = oracle.project(grid, F, tol=1e-13)
    c = n // 2
    maps, _, _ = oracle.peak_maps(grid, 2e3, 1000.0, 0.3, dt, 25, [(0, c), (1, c), (2, c)], FS=FS,
                                  env=np.ones(5))
    mx, my, mz = maps
    assert mz.max() > 0
    np.testing.assert_allclose(mx, my, rtol=1e-12, atol=1e-12 * mx.max())
    np.testing.assert_allclose(mz, mz.T, rtol=1e-12, atol=1e-12 * mz.max())
    np.testing.assert_allclose(mz, mz[::-1, :], rtol=1e-12, atol=1e-12 * mz.max())
    np.testing.assert_allclose(mz, mz[:, ::-1], rtol=1e-12, atol=1e-12 * mz.max())


def test_peak_maps_start_from_the_given_state():
    """With a state handed in and no steps, the map is |u| of that state."""
    grid = (7, 8, 9, 1e-3, 1e-3, 1e-3)
    rng = np.random.default_rng(3)
    u = rng.standard_normal((3, 9, 8, 7))
    maps, _, _ = oracle.peak_maps(grid, 1e3, 1000.0, 0.0, 1e-5, 0, [(1, 2)], u=u, w=np.zeros_like(u))
    np.testing.assert_array_equal(maps[0], np.sqrt(u[0, :, 2, :] ** 2 + u[1, :, 2, :] ** 2 + u[2, :, 2, :] ** 2))
