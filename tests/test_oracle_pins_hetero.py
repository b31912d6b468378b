"""Further pins of the FP64 CPU oracle: the heterogeneous viscous update, the
true-residual routine, the sampled one-step routine, the default sponge
strength and the FP32 precision bar.

* The one-step map of the summed-form update (Sec. 3.1), assembled as a
  dense matrix on 5-7 node grids from the face list of the grid (harmonic face
  moduli, per-cell rho, eta and sponge), compared with the oracle's run over
  many steps; its spectral radius against the stability root A + 2B = 4.
* The paper's printed three-level update (Sec. 3.1, Sec. 3.3 source) with a
  per-cell viscosity and density and the centred sponge damping.
* Hand values of the response to a unit impulse in u or w at one cell: each
  neighbour reacts with its own eta and rho.
* ``true_relres`` on an exact DST-I Poisson solution and on the same solution
  plus a scaled Laplacian eigenmode, whose residual is known in closed form.
* ``step_cells`` against one step of ``run`` at every interior cell.
* The default sponge strength by its effect: a wave packet crossing the ramp
  twice (to the wall and back) loses 10^-3, i.e. 10^-1.5 one way.
* FP32 arithmetic of the summed form (a numpy float32 emulation) against
  the FP64 oracle at the inclusion workload's conditions: within the 2e-5
  trace bar, which the three-level form in FP32 misses.
"""
import numpy as np
import pytest
import scipy.fft

import oracle
from oracle import dispersion
from oracle.analysis import rel_l2
from workloads import gaussian_push

AXES = ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1))


def hetero_medium(shape, seed):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    G = np.exp(rng.uniform(np.log(1e3), np.log(1e4), shape))
    rho = rng.uniform(900.0, 1200.0, shape)
    eta = rng.uniform(0.0, 1.5, shape)
    return G, rho, eta


def ramp_value(a, n, L):
    d = min(a, n - 1 - a)
    return max(0.0, (L - d) / L) if L > 0 else 0.0


def assemble_step_map(grid, G, rho, eta, dt, L, smax):
    """Dense one-step map of one displacement component on the interior
    nodes, x = [u; w] -> M x + [f; f] g: the operators are built from the
    list of faces of every interior node (harmonic face modulus for the
    elastic operator, unit weight for the Laplacian, Dirichlet neighbours
    dropped), the sponge from the linear ramp.  Returns (M, fscale) with
    fscale the per-node factor of the force (dt^2 / rho / (1 + s))."""
    nx, ny, nz, hx, hy, hz = grid
    h = {0: hx, 1: hy, 2: hz}
    nodes = [(i, j, k) for k in range(1, nz - 1) for j in range(1, ny - 1) for i in range(1, nx - 1)]
    index = {c: q for q, c in enumerate(nodes)}
    m = len(nodes)
    K = np.zeros((m, m))
    Lap = np.zeros((m, m))
    for q, (i, j, k) in enumerate(nodes):
        for di, dj, dk in AXES:
            a = 0 if di else (1 if dj else 2)
            nb = (i + di, j + dj, k + dk)
            gc, gn = G[k, j, i], G[nb[2], nb[1], nb[0]]
            gf = 2.0 * gc * gn / (gc + gn)
            K[q, q] -= gf / h[a] ** 2
            Lap[q, q] -= 1.0 / h[a] ** 2
            if nb in index:
                K[q, index[nb]] += gf / h[a] ** 2
                Lap[q, index[nb]] += 1.0 / h[a] ** 2
    sig = np.array([smax * max(ramp_value(i, nx, L), ramp_value(j, ny, L), ramp_value(k, nz, L))
                    for (i, j, k) in nodes])
    s = 0.5 * sig * dt
    r = np.array([rho[k, j, i] for (i, j, k) in nodes])
    e = np.array([eta[k, j, i] for (i, j, k) in nodes])
    cr = dt * dt / r
    Bu = (cr / (1 + s))[:, None] * K
    Bw = np.diag((1 - s) / (1 + s)) + (cr * e / dt / (1 + s))[:, None] * Lap
    M = np.block([[np.eye(m) + Bu, Bw], [Bu, Bw]])
    return M, cr / (1 + s), nodes


def interior_vec(a, nodes):
    return np.array([a[k, j, i] for (i, j, k) in nodes])


@pytest.mark.parametrize("shape,L", [((5, 6, 7), 1), ((7, 7, 7), 2), ((6, 5, 5), 0)])
def test_step_map_brute_force_heterogeneous(shape, L):
    """Oracle steps equal powers of the assembled one-step map (plus the
    force) on tiny heterogeneous viscous grids with sponge, a push switched on
    and off, and a random initial state: FP64 to 1e-12."""
    nz, ny, nx = shape
    grid = (nx, ny, nz, 0.3e-3, 0.25e-3, 0.35e-3)
    G, rho, eta = hetero_medium(shape, 11 + nx)
    rng = np.random.default_rng(5)
    dt = 0.7 * oracle.stable_dt(grid, G, rho, eta)
    smax = 3000.0
    FS = np.zeros((3,) + shape)
    FS[:, 1:-1, 1:-1, 1:-1] = 1e4 * rng.standard_normal((3, nz - 2, ny - 2, nx - 2))
    env = np.array([1.0, 0.5, 0.0, 2.0, 1.0])
    u0 = np.zeros((3,) + shape)
    w0 = np.zeros((3,) + shape)
    u0[:, 1:-1, 1:-1, 1:-1] = 1e-6 * rng.standard_normal((3, nz - 2, ny - 2, nx - 2))
    w0[:, 1:-1, 1:-1, 1:-1] = 1e-8 * rng.standard_normal((3, nz - 2, ny - 2, nx - 2))
    nsteps = 40
    u, w, _ = oracle.run(grid, G, rho, eta, dt, nsteps, FS=FS, env=env, u=u0, w=w0, sponge_cells=L, sigma_max=smax)
    M, fscale, nodes = assemble_step_map(grid, G, rho, eta, dt, L, smax)
    m = len(nodes)
    for c in range(3):
        x = np.concatenate([interior_vec(u0[c], nodes), interior_vec(w0[c], nodes)])
        f = fscale * interior_vec(FS[c], nodes)
        for n in range(nsteps):
            g = env[n] if n < len(env) else 0.0
            x = M @ x + g * np.concatenate([f, f])
        ref_u, ref_w = x[:m], x[m:]
        assert np.linalg.norm(interior_vec(u[c], nodes) - ref_u) <= 1e-12 * np.linalg.norm(ref_u)
        assert np.linalg.norm(interior_vec(w[c], nodes) - ref_w) <= 1e-12 * np.linalg.norm(ref_w)
    # the outer layer stays at rest
    assert not u[:, 0].any() and not u[:, :, -1].any() and not w[:, :, :, 0].any()


def test_spectral_radius_of_step_map_and_stability_root():
    """Homogeneous viscous grid: the one-step map's spectral radius is <= 1
    exactly when A + 2B <= 4 for the largest Laplacian eigenvalue of the
    finite grid, A = dt^2 G lam / rho, B = dt eta lam / rho (the Jury
    condition of the mode recurrence).  Heterogeneous grid with sponge: the
    oracle's stable dt (per-cell bound on the face moduli) gives a map with
    spectral radius <= 1."""
    n, h = 7, 0.3e-3
    grid = (n, n, n, h, h, h)
    G, rho, eta = 3e3, 1000.0, 0.6
    lam = sum(4 / h ** 2 * np.sin((n - 2) * np.pi / (2 * (n - 1))) ** 2 for _ in range(3))
    qa, qb = G * lam / rho, 2 * eta * lam / rho
    dt_star = (-qb + np.sqrt(qb * qb + 16 * qa)) / (2 * qa)  # A + 2B = 4
    assert dt_star > oracle.stable_dt(grid, G, rho, eta)  # the finite grid is a little more stable
    shp = (n, n, n)
    Gf, rf, ef = np.full(shp, G), np.full(shp, rho), np.full(shp, eta)
    for fac, stable in ((0.999, True), (1.001, False)):
        M, _, _ = assemble_step_map(grid, Gf, rf, ef, fac * dt_star, 0, 0.0)
        radius = np.abs(np.linalg.eigvals(M)).max()
        assert (radius <= 1 + 1e-9) == stable, (fac, radius)
        assert abs(radius - 1) < 0.05
    # the mode recurrence reaches the unit circle at dt_star
    assert max(abs(dispersion.mode_roots(lam, G, rho, eta, dt_star))) == pytest.approx(1.0, abs=1e-6)
    # heterogeneous, viscous, with sponge, at the oracle's bound
    shp = (6, 7, 6)
    grid = (6, 7, 6, 0.3e-3, 0.25e-3, 0.35e-3)
    for seed in range(3):
        Gh, rh, eh = hetero_medium(shp, 40 + seed)
        dt = oracle.stable_dt(grid, Gh, rh, eh)
        M, _, _ = assemble_step_map(grid, Gh, rh, eh, dt, 1, 2000.0)
        assert np.abs(np.linalg.eigvals(M)).max() <= 1 + 1e-9


def lap_slices(q, h):
    out = np.zeros_like(q)
    c = q[1:-1, 1:-1, 1:-1]
    out[1:-1, 1:-1, 1:-1] = ((q[1:-1, 1:-1, 2:] - 2 * c + q[1:-1, 1:-1, :-2]) / h[0] ** 2
                             + (q[1:-1, 2:, 1:-1] - 2 * c + q[1:-1, :-2, 1:-1]) / h[1] ** 2
                             + (q[2:, 1:-1, 1:-1] - 2 * c + q[:-2, 1:-1, 1:-1]) / h[2] ** 2)
    return out


def test_three_level_update_with_pointwise_eta_rho_and_sponge():
    """The printed three-level update u^{n+1} = 2u^n - u^{n-1} + dt^2 a^n with
    a^n = (G lap u^n + eta(x) lap((u^n - u^{n-1}) / dt) + g_n f_S) / rho(x)
    (Sec. 3.1, 3.3), uniform G, per-cell eta and rho, and the centred sponge
    damping sigma(x) (u^{n+1} - u^{n-1}) / (2 dt) on the left-hand side, run
    in that form, equals the oracle's summed form to 1e-12."""
    shape = (15, 13, 17)
    nz, ny, nx = shape
    h = (0.3e-3, 0.25e-3, 0.35e-3)
    grid = (nx, ny, nz) + h
    _, rho, eta = hetero_medium(shape, 3)
    G = 4e3
    L, smax = 3, 2500.0
    dt = 0.6 * oracle.stable_dt(grid, G, rho, eta)
    F = gaussian_push(grid, 0.8e-3, 1.5e-3, 1e4) + 200.0 * np.random.default_rng(1).standard_normal((3,) + shape)
    FS, _, _ = oracle.project(grid, F, tol=1e-12)
    env = np.array([1.0, 1.0, 0.5, 1.0, 0.25])
    probes = np.array([[i, 6, 8] for i in range(nx)])
    nsteps = 120
    _, _, tr = oracle.run(grid, G, rho, eta, dt, nsteps, FS=FS, env=env, probes=probes, comp=3, sponge_cells=L,
                          sigma_max=smax)
    sig = np.zeros(shape)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                sig[k, j, i] = smax * max(ramp_value(i, nx, L), ramp_value(j, ny, L), ramp_value(k, nz, L))
    u_prev = np.zeros_like(FS)
    u = np.zeros_like(FS)
    ref = np.zeros_like(tr)
    for n in range(nsteps):
        g = env[n] if n < len(env) else 0.0
        u_next = np.zeros_like(u)
        for c in range(3):
            a = (G * lap_slices(u[c], h) + eta * lap_slices((u[c] - u_prev[c]) / dt, h) + g * FS[c]) / rho
            # (1 + sigma dt/2) u^{n+1} = 2 u^n - (1 - sigma dt/2) u^{n-1} + dt^2 a
            un = (2 * u[c] - (1 - 0.5 * sig * dt) * u_prev[c] + dt * dt * a) / (1 + 0.5 * sig * dt)
            u_next[c][1:-1, 1:-1, 1:-1] = un[1:-1, 1:-1, 1:-1]
        u_prev, u = u, u_next
        ref[n] = u[:, 8, 6, :].T
    assert np.linalg.norm(tr - ref) <= 1e-12 * np.linalg.norm(ref)


def test_unit_impulse_response_hand_values():
    """One step from u = 0 and w = e at cell c (one component): w' = a1 e +
    a2 (eta/dt) lap(e) cell by cell, so the cell keeps
    ((1 - s) - 2 (dt^2/rho_c)(eta_c/dt) S) / (1 + s) and a neighbour across
    axis a receives (dt^2/rho_n)(eta_n/dt) / h_a^2 / (1 + s_n) with its own
    eta and rho; from u = e and w = 0 a neighbour receives
    (dt^2/rho_n) G_f / h_a^2 / (1 + s_n), G_f the harmonic mean."""
    shape = (7, 8, 9)
    nz, ny, nx = shape
    hs = (0.3e-3, 0.25e-3, 0.35e-3)
    grid = (nx, ny, nz) + hs
    G, rho, eta = hetero_medium(shape, 21)
    dt = 0.5 * oracle.stable_dt(grid, G, rho, eta)
    L, smax = 2, 4000.0
    c = (4, 3, 3)  # (i, j, k); the x- neighbour (3, 3, 3) is in the ramp, the others are not
    i, j, k = c

    def s_at(ii, jj, kk):
        return 0.5 * dt * smax * max(ramp_value(ii, nx, L), ramp_value(jj, ny, L), ramp_value(kk, nz, L))

    e = np.zeros((3,) + shape)
    e[1, k, j, i] = 1.0
    S = sum(1 / hh ** 2 for hh in hs)
    # impulse in w
    u1, w1, _ = oracle.run(grid, G, rho, eta, dt, 1, w=e, sponge_cells=L, sigma_max=smax)
    s = s_at(i, j, k)
    assert w1[1, k, j, i] == pytest.approx(((1 - s) - 2 * dt * eta[k, j, i] / rho[k, j, i] * S) / (1 + s), rel=1e-13)
    for di, dj, dk in AXES:
        a = 0 if di else (1 if dj else 2)
        ii, jj, kk = i + di, j + dj, k + dk
        want = dt * eta[kk, jj, ii] / rho[kk, jj, ii] / hs[a] ** 2 / (1 + s_at(ii, jj, kk))
        assert w1[1, kk, jj, ii] == pytest.approx(want, rel=1e-13)
        assert u1[1, kk, jj, ii] == w1[1, kk, jj, ii]
    assert not w1[0].any() and not w1[2].any()
    # impulse in u
    u1, w1, _ = oracle.run(grid, G, rho, eta, dt, 1, u=e, sponge_cells=L, sigma_max=smax)
    for di, dj, dk in AXES:
        a = 0 if di else (1 if dj else 2)
        ii, jj, kk = i + di, j + dj, k + dk
        gf = 2 * G[k, j, i] * G[kk, jj, ii] / (G[k, j, i] + G[kk, jj, ii])
        want = dt * dt / rho[kk, jj, ii] * gf / hs[a] ** 2 / (1 + s_at(ii, jj, kk))
        assert w1[1, kk, jj, ii] == pytest.approx(want, rel=1e-13)
    assert np.count_nonzero(w1) == 7


# ---------------------------------------------------------------- true residual

def dst_poisson(grid, b):
    """Exact solution of lap_h phi = b on the interior (Dirichlet box), DST-I."""
    nx, ny, nz, hx, hy, hz = grid
    lam = (4 / hz ** 2 * np.sin(np.arange(1, nz - 1) * np.pi / (2 * (nz - 1))) ** 2)[:, None, None] \
        + (4 / hy ** 2 * np.sin(np.arange(1, ny - 1) * np.pi / (2 * (ny - 1))) ** 2)[None, :, None] \
        + (4 / hx ** 2 * np.sin(np.arange(1, nx - 1) * np.pi / (2 * (nx - 1))) ** 2)[None, None, :]
    phi = np.zeros_like(b)
    phi[1:-1, 1:-1, 1:-1] = scipy.fft.idstn(scipy.fft.dstn(b[1:-1, 1:-1, 1:-1], type=1) / (-lam), type=1)
    return phi


def test_true_relres_exact_solution_and_eigenmode_perturbation():
    """||lap phi - b|| / ||b|| over the interior: about 1e-15 for the exact
    DST-I solution; for phi = exact + eps * mode (a Dirichlet sine mode with
    eigenvalue -lam) the residual is eps lam ||mode|| exactly.  Values of b
    on the outer layer do not enter."""
    grid = (19, 17, 21, 0.4e-3, 0.3e-3, 0.5e-3)
    nx, ny, nz, hx, hy, hz = grid
    rng = np.random.default_rng(8)
    b = np.zeros((nz, ny, nx))
    b[1:-1, 1:-1, 1:-1] = rng.standard_normal((nz - 2, ny - 2, nx - 2))
    phi = dst_poisson(grid, b)
    assert oracle.true_relres(grid, b, phi) < 1e-13
    p, q, r = 3, 5, 2
    ii, jj, kk = np.arange(nx), np.arange(ny), np.arange(nz)
    mode = (np.sin(r * np.pi * kk / (nz - 1))[:, None, None] * np.sin(q * np.pi * jj / (ny - 1))[None, :, None]
            * np.sin(p * np.pi * ii / (nx - 1))[None, None, :])
    lam = (4 / hx ** 2 * np.sin(p * np.pi / (2 * (nx - 1))) ** 2 + 4 / hy ** 2 * np.sin(q * np.pi / (2 * (ny - 1))) ** 2
           + 4 / hz ** 2 * np.sin(r * np.pi / (2 * (nz - 1))) ** 2)
    for eps in (1e-9, 1e-12, 3e-15):
        want = eps * lam * np.linalg.norm(mode[1:-1, 1:-1, 1:-1]) / np.linalg.norm(b[1:-1, 1:-1, 1:-1])
        got = oracle.true_relres(grid, b, phi + eps * mode)
        assert got == pytest.approx(want, rel=1e-6 if eps > 1e-10 else 2e-2), eps
    # garbage on the outer layer of b is outside the residual
    b2 = b.copy()
    b2[0], b2[:, -1], b2[:, :, 0] = 5.0, -3.0, 7.0
    assert oracle.true_relres(grid, b2, phi) == oracle.true_relres(grid, b, phi)
    # b = 0 reports 0
    assert oracle.true_relres(grid, np.zeros_like(b), phi) == 0.0


def test_step_cells_equals_one_run_step_everywhere():
    """The sampled one-step routine gives, at every interior cell of a ragged
    heterogeneous viscous grid with sponge and a force, bit for bit what a
    full oracle step gives."""
    shape = (9, 11, 13)
    nz, ny, nx = shape
    grid = (nx, ny, nz, 0.3e-3, 0.25e-3, 0.35e-3)
    G, rho, eta = hetero_medium(shape, 31)
    rng = np.random.default_rng(4)
    dt = 0.6 * oracle.stable_dt(grid, G, rho, eta)
    FS = rng.standard_normal((3,) + shape) * 1e3
    u0 = np.zeros((3,) + shape)
    w0 = np.zeros((3,) + shape)
    u0[:, 1:-1, 1:-1, 1:-1] = rng.standard_normal((3, nz - 2, ny - 2, nx - 2)) * 1e-6
    w0[:, 1:-1, 1:-1, 1:-1] = rng.standard_normal((3, nz - 2, ny - 2, nx - 2)) * 1e-8
    gn = 0.75
    step0 = 3
    env = np.zeros(step0 + 1)
    env[step0] = gn
    u1, w1, _ = oracle.run(grid, G, rho, eta, dt, 1, FS=FS, env=env, u=u0, w=w0, step0=step0, sponge_cells=3,
                           sigma_max=2500.0)
    K, J, I = np.meshgrid(np.arange(1, nz - 1), np.arange(1, ny - 1), np.arange(1, nx - 1), indexing="ij")
    cells = (I + nx * (J + ny * K)).ravel()
    uo, wo = oracle.step_cells(grid, G, rho, eta, dt, u0, w0, cells, FS=FS, gn=gn, sponge_cells=3, sigma_max=2500.0)
    assert np.array_equal(uo, u1.reshape(3, -1)[:, cells].T)
    assert np.array_equal(wo, w1.reshape(3, -1)[:, cells].T)
    with pytest.raises(RuntimeError):
        oracle.step_cells(grid, G, rho, eta, dt, u0, w0, np.array([0]), FS=FS, gn=gn)


# ---------------------------------------------------------------- sponge strength

def test_default_sponge_strength_one_way_factor():
    """A zero-mean wave packet (carrier 4 cells, envelope 4 cells) runs along
    the centre line of an nx x (2L+1) x (2L+1) grid with transverse spacings
    of 1e6 m (the lines decouple, and the centre line sees only the x ramp)
    at Courant number ~1, crosses the L-cell ramp to the Dirichlet wall and
    back: with the default strength the round trip costs 10^-3 (10^-1.5 one
    way), as the integral of the amplitude decay rate sigma/2 over the ramp
    predicts.  Half the strength halves the exponent."""
    L, lam, env_w = 24, 4, 4
    h, G, rho = 1e-4, 4e3, 1000.0
    c = np.sqrt(G / rho)
    i0 = L + 4 * env_w
    probe = i0 + 4 * env_w
    nx = probe + 4 * env_w + L
    n = 2 * L + 1
    grid = (nx, n, n, h, 1e6, 1e6)
    smax = oracle.default_sigma_max(grid, G, rho, L)
    assert smax == pytest.approx(6 * np.log(10) * c / (L * h), rel=1e-14)
    dt = 0.999 * oracle.stable_dt(grid, G, rho, 0.0)
    assert c * dt / h == pytest.approx(0.999, rel=1e-9)
    x = (np.arange(nx) - i0) * h
    f = lambda xx: np.exp(-xx ** 2 / (2 * (env_w * h) ** 2)) * np.cos(2 * np.pi * xx / (lam * h))
    nsteps = int((2 * (nx - 1 - i0) - (probe - i0) + 6 * env_w) * h / (c * dt)) + 1
    t_inc = int((probe - i0) * h / (c * dt))
    t_ref = int((2 * (nx - 1 - i0) - (probe - i0)) * h / (c * dt))
    factors = []
    for scale in (1.0, 0.5):
        u = np.zeros((3, n, n, nx))
        w = np.zeros_like(u)
        u[2, L, L, :] = f(x)
        w[2, L, L, :] = f(x) - f(x + c * dt)
        u[:, :, :, 0] = u[:, :, :, -1] = w[:, :, :, 0] = w[:, :, :, -1] = 0.0
        _, _, tr = oracle.run(grid, G, rho, 0.0, dt, nsteps, u=u, w=w, probes=np.array([[probe, L, L]]), comp=2,
                              sponge_cells=L, sigma_max=scale * smax)
        tr = tr[:, 0, 0]
        inc = np.abs(tr[:t_inc + 4 * env_w]).max()
        ref = np.abs(tr[t_ref - 5 * env_w:]).max()
        assert inc == pytest.approx(1.0, abs=5e-3)
        factors.append(np.log10(ref / inc) / 2)
    assert factors[0] == pytest.approx(-1.5, abs=0.05), factors
    assert factors[1] == pytest.approx(-0.75, abs=0.05), factors


# ---------------------------------------------------------------- precision bar

def fp32_summed_run(grid, G, rho, eta, dt, nsteps, FS, env, L, smax, probe_line, three_level=False):
    """Homogeneous update in numpy float32: the summed form (state u, w) or
    the three-level form (state u^n, u^{n-1}); z-component traces on an x
    line (j, k)."""
    f32 = np.float32
    nx, ny, nz, hx, hy, hz = grid
    h2 = [f32(1.0 / hx ** 2), f32(1.0 / hy ** 2), f32(1.0 / hz ** 2)]
    sig = np.zeros((nz, ny, nx))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                sig[k, j, i] = smax * max(ramp_value(i, nx, L), ramp_value(j, ny, L), ramp_value(k, nz, L))
    s = 0.5 * sig * dt
    a1 = ((1 - s) / (1 + s)).astype(f32)[1:-1, 1:-1, 1:-1]
    a2 = ((dt * dt / rho) / (1 + s)).astype(f32)[1:-1, 1:-1, 1:-1]
    Gf, eta_dt = f32(G), f32(eta / dt)
    fz = FS[2].astype(f32)[1:-1, 1:-1, 1:-1]

    def lap(q):
        c2 = f32(2) * q[1:-1, 1:-1, 1:-1]
        return ((q[1:-1, 1:-1, 2:] + q[1:-1, 1:-1, :-2] - c2) * h2[0] + (q[1:-1, 2:, 1:-1] + q[1:-1, :-2, 1:-1] - c2)
                * h2[1] + (q[2:, 1:-1, 1:-1] + q[:-2, 1:-1, 1:-1] - c2) * h2[2])

    u = np.zeros((nz, ny, nx), f32)
    w = np.zeros_like(u)  # summed form: w = u^n - u^{n-1}; three-level: u^{n-1}
    j, k = probe_line
    out = np.zeros((nsteps, nx))
    for n in range(nsteps):
        g = f32(env[n]) if n < len(env) else f32(0)
        if three_level:
            um = w
            acc = Gf * lap(u) + eta_dt * lap(u - um) + g * fz
            un = np.zeros_like(u)
            # (1+s) u' = 2u - (1-s) u^{n-1} + dt^2 a, written with a1, a2
            un[1:-1, 1:-1, 1:-1] = (u[1:-1, 1:-1, 1:-1] + u[1:-1, 1:-1, 1:-1] * a1 - um[1:-1, 1:-1, 1:-1] * a1
                                    + a2 * acc)
            w, u = u, un
        else:
            acc = Gf * lap(u) + eta_dt * lap(w) + g * fz
            wn = np.zeros_like(w)
            wn[1:-1, 1:-1, 1:-1] = a1 * w[1:-1, 1:-1, 1:-1] + a2 * acc
            u = u + wn
            w = wn
        out[n] = u[k, j, :]
    return out


def _fp32_errors(n, L, dt_factor, nsteps):
    """Relative L2 of the float32 summed and three-level runs against the
    FP64 oracle on the centre-line u_z traces: h = 0.25 mm, 2 kPa,
    1000 kg/m^3, 0.5 Pa s, the 100 us push, L-cell sponge of default
    strength, dt = dt_factor x the stable limit."""
    h = 0.25e-3
    grid = (n, n, n, h, h, h)
    G, rho, eta = 2e3, 1000.0, 0.5
    dt = dt_factor * oracle.stable_dt(grid, G, rho, eta)
    smax = oracle.default_sigma_max(grid, G, rho, L)
    env = np.ones(int(round(100e-6 / dt)))
    F = gaussian_push(grid, 1e-3, 4e-3, 1e4)
    FS, _, _ = oracle.project(grid, F, tol=1e-10)
    probes = np.array([[i, n // 2, n // 2] for i in range(n)])
    _, _, tr = oracle.run(grid, G, rho, eta, dt, nsteps, FS=FS, env=env, probes=probes, comp=2, sponge_cells=L,
                          sigma_max=smax)
    ref = tr[:, :, 0]
    e_sum = rel_l2(fp32_summed_run(grid, G, rho, eta, dt, nsteps, FS, env, L, smax, (n // 2, n // 2)), ref)
    e_three = rel_l2(fp32_summed_run(grid, G, rho, eta, dt, nsteps, FS, env, L, smax, (n // 2, n // 2),
                                     three_level=True), ref)
    return e_sum, e_three


def test_fp32_summed_form_meets_trace_bar():
    """At the inclusion workload's conditions (dt = 0.4 x the stable limit,
    8-cell sponge) on a 40^3 grid over 2000 steps the summed form in float32
    stays within 2e-5 relative L2 of the FP64 oracle (measured 2.1e-7), and
    closer than the three-level form (1.3e-6).  The three-level form carries
    the viscous difference u^n - u^{n-1} of two nearly equal float32 values:
    its error per step grows like (eta / dt) eps_32 / G as dt shrinks, so at
    a ten times finer step (24^3, 0.04 x the limit, 2000 steps) it breaks the
    bar (1.7e-3) while the summed form, which stores w = u^n - u^{n-1}
    itself, stays at 3e-7.  That is why the FP32 state is (u, w)."""
    e_sum, e_three = _fp32_errors(40, 8, 0.4, 2000)
    assert e_sum < 1e-5, e_sum
    assert e_three > 2 * e_sum, (e_sum, e_three)
    e_sum, e_three = _fp32_errors(24, 6, 0.04, 2000)
    assert e_sum < 1e-5, e_sum
    assert e_three > 2e-5, e_three
