"""Pins of the C-PML oracle (an absorbing layer the paper names as future work,
Sec. 3.5 and Sec. 7; formulation in oracle/pml.py): with zero damping it is the
plain method exactly; it removes the wall reflections that a larger domain
shows to be spurious (against which the Dirichlet wall and the sponge of the
same width are checked too); the profile vanishes outside the layer and is
mirror-symmetric; a long run with viscosity, heterogeneity and force decays
and does not drift (with alpha held constant in the layer)."""
import numpy as np

import oracle
import workloads
from oracle import pml
from oracle.analysis import rel_l2
from workloads import gaussian_push, spherical_inclusions

H, G, RHO, ETA = 0.5e-3, 4e3, 1000.0, 0.2


def curl_case(n):
    return workloads.curl_wavespeed_case(n=n, h=H, sigma=1.5e-3, offsets_mm=(2.0, 3.5))


def test_zero_damping_is_the_plain_method():
    rng = np.random.default_rng(2)
    grid = (13, 11, 12, 2e-4, 2.5e-4, 3e-4)
    Gm, rho, eta, _ = spherical_inclusions(grid, rng, 3, (2e3, 1000.0, 0.5), (0.3e-3, 0.8e-3), (1e3, 1e4),
                                           (1000.0, 1100.0), (0.0, 1.5), 1)
    dt = 0.4 * oracle.stable_dt(grid, Gm, rho, eta)
    F = 10.0 * rng.standard_normal((3, 12, 11, 13))
    u0 = 1e-7 * rng.standard_normal((3, 12, 11, 13))
    env = np.array([1.0, 0.5, 0.0, 2.0])
    probes = [[i, 5, 6] for i in range(13)]
    _, _, tr = oracle.run(grid, Gm, rho, eta, dt, 40, FS=F, env=env, u=u0, probes=probes, comp=3)
    for cells, R in ((0, 1e-5), (3, 1.0)):
        u, w, tr_p = pml.run_pml(grid, Gm, rho, eta, dt, 40, cells, R=R, FS=F, env=env, u=u0, probes=probes, comp=3)
        assert rel_l2(tr_p, tr) < 1e-13, (cells, R)


def test_profile_is_zero_inside_and_mirror_symmetric():
    n, L = 30, 6
    (bc, cc), (bf, cf) = pml.profile(n, L, 2e-4, 3.0, 1e-5, 1e-5, 500.0)
    assert np.all(cc[L + 1:n - 1 - L] == 0) and np.all(cf[L:n - 2 - L + 1] == 0)
    assert np.all(cc[1:L + 1] < 0) and np.all(cf[:L] < 0)
    assert np.allclose(cc, cc[::-1], rtol=1e-14) and np.allclose(cf, cf[::-1], rtol=1e-14)
    assert np.all(np.diff(cf[:L]) > 0)  # damping grows toward the wall
    assert np.all((bc > 0) & (bc <= 1)) and np.all((bf > 0) & (bf <= 1))


def test_layer_absorbs_what_the_walls_reflect():
    """Curl source on a 32^3 grid with a 6-cell layer against the same source on
    72^3 (no reflection reaches the sensors within the window): the layer's
    trace error is below 5e-2 of the Dirichlet wall's and of a 6-cell sponge's
    (the sensors sit two cells from the layer on this small grid; the GPU test
    at 128^3 shows the layer's full effect)."""
    w = curl_case(32)
    dt = 0.4 * oracle.stable_dt(w["grid"], G, RHO, ETA)
    nsteps = int(9e-3 / dt)
    u0, w0 = oracle.curl_state(w["grid"], w["A"], dt)
    _, _, tr_p = pml.run_pml(w["grid"], G, RHO, ETA, dt, nsteps, 6, u=u0, w=w0, probes=w["probes"], comp=2)
    _, _, tr_d = oracle.run(w["grid"], G, RHO, ETA, dt, nsteps, u=u0, w=w0, probes=w["probes"], comp=2)
    smax = oracle.default_sigma_max(w["grid"], G, RHO, 6)
    _, _, tr_s = oracle.run(w["grid"], G, RHO, ETA, dt, nsteps, u=u0, w=w0, probes=w["probes"], comp=2,
                            sponge_cells=6, sigma_max=smax)
    wr = curl_case(72)
    ur, wwr = oracle.curl_state(wr["grid"], wr["A"], dt)
    _, _, tr_r = oracle.run(wr["grid"], G, RHO, ETA, dt, nsteps, u=ur, w=wwr, probes=wr["probes"], comp=2)
    e_p, e_d, e_s = rel_l2(tr_p, tr_r), rel_l2(tr_d, tr_r), rel_l2(tr_s, tr_r)
    assert e_d > 0.05 and e_s > 0.05  # the walls do reflect within the window
    assert e_p < 5e-2 * min(e_d, e_s), (e_p, e_d, e_s)


def test_long_run_decays_and_stays_bounded():
    rng = np.random.default_rng(9)
    n, L = 18, 4
    grid = (n, n, n, H, H, H)
    Gm, rho, eta, _ = spherical_inclusions(grid, rng, 3, (2e3, 1000.0, 0.5), (1e-3, 2e-3), (1e3, 1e4),
                                           (1000.0, 1100.0), (0.0, 1.5), 1)
    dt = 0.4 * oracle.stable_dt(grid, Gm, rho, eta)
    F = gaussian_push(grid, 1e-3, 2e-3, 1e4)
    FS, _, _ = oracle.project(grid, F, tol=1e-10)
    env = np.ones(10)
    c = n // 2
    u, w, tr = pml.run_pml(grid, Gm, rho, eta, dt, 2500, L, FS=FS, env=env, probes=[[c, c, c]], comp=2)
    a = np.abs(tr[:, 0, 0])
    assert np.all(np.isfinite(a))
    assert a[-300:].max() < 0.2 * a.max()
    assert a[-300:].max() <= a[600:900].max()  # no late growth
    assert np.abs(u).max() < 0.2 * a.max()
