"""Pins of the oracle's curl-based initialisation (Sec. 3.5; used by the
wavespeed-recovery validation of Sec. 4.1): the exact centred differences of
sampled sinusoids, the discrete identities div(curl) = 0 and curl(grad) = 0,
and the summed-form state built from it."""
import numpy as np

import oracle

GRID = (23, 19, 27, 2e-4, 3e-4, 2.5e-4)


def coords(grid):
    nx, ny, nz, hx, hy, hz = grid
    return (np.arange(nx) * hx)[None, None, :], (np.arange(ny) * hy)[None, :, None], (np.arange(nz) * hz)[:, None, None]


def interior(a, m=1):
    return a[..., m:-m, m:-m, m:-m]


def test_curl_of_sampled_sinusoids_is_exact():
    """A centred difference of sin(k x) is sin(k h)/h cos(k x) exactly, which
    fixes every term of the curl, its sign and its component."""
    x, y, z = coords(GRID)
    hx, hy, hz = GRID[3:]
    kx, ky, kz = 900.0, 1300.0, 700.0
    sx, cx = np.sin(kx * x), np.cos(kx * x)
    sy, cy = np.sin(ky * y), np.cos(ky * y)
    sz, cz = np.sin(kz * z), np.cos(kz * z)
    fx, fy, fz = np.sin(kx * hx) / hx, np.sin(ky * hy) / hy, np.sin(kz * hz) / hz
    shape = (3, GRID[2], GRID[1], GRID[0])
    A = np.zeros(shape)
    A[0] = sy * sz + 0 * x      # Ax: d/dz -> +cy component, d/dy -> -cz component
    A[1] = sx * cz + 0 * y      # Ay: d/dx -> +cz, d/dz -> -cx
    A[2] = cx * sy + 0 * z      # Az: d/dy -> +cx, d/dx -> -cy
    ex = fy * (cx * cy) - (-fz) * (sx * sz)
    ey = fz * (sy * cz) - (-fx) * (sx * sy)
    ez = fx * (cx * cz) - fy * (sz * cy)
    C = oracle.curl(GRID, A)
    for i, e in enumerate((ex, ey, ez)):
        e = np.broadcast_to(e, shape[1:])
        assert np.allclose(interior(C[i]), interior(e), rtol=0, atol=1e-12 * np.abs(e).max()), i
    # the outer layer is zero
    assert not C[:, 0].any() and not C[:, -1].any() and not C[:, :, 0].any() and not C[:, :, :, -1].any()


def test_divergence_of_curl_and_curl_of_gradient_vanish():
    rng = np.random.default_rng(4)
    shape = (GRID[2], GRID[1], GRID[0])
    hx, hy, hz = GRID[3:]
    A = rng.standard_normal((3,) + shape)
    C = oracle.curl(GRID, A)
    div = ((C[0][1:-1, 1:-1, 2:] - C[0][1:-1, 1:-1, :-2]) / (2 * hx)
           + (C[1][1:-1, 2:, 1:-1] - C[1][1:-1, :-2, 1:-1]) / (2 * hy)
           + (C[2][2:, 1:-1, 1:-1] - C[2][:-2, 1:-1, 1:-1]) / (2 * hz))
    # cells whose neighbours are all interior (the outer layer of C is 0)
    scale = np.abs(C).max() / min(hx, hy, hz)
    assert np.abs(div[1:-1, 1:-1, 1:-1]).max() < 1e-12 * scale
    phi = rng.standard_normal(shape)
    G = np.zeros((3,) + shape)
    G[0][:, :, 1:-1] = (phi[:, :, 2:] - phi[:, :, :-2]) / (2 * hx)
    G[1][:, 1:-1, :] = (phi[:, 2:, :] - phi[:, :-2, :]) / (2 * hy)
    G[2][1:-1, :, :] = (phi[2:, :, :] - phi[:-2, :, :]) / (2 * hz)
    CG = oracle.curl(GRID, G)
    assert np.abs(interior(CG, 2)).max() < 1e-12 * np.abs(G).max() / min(hx, hy, hz)


def test_curl_state_is_rest_plus_velocity_times_dt():
    rng = np.random.default_rng(8)
    A = rng.standard_normal((3, GRID[2], GRID[1], GRID[0]))
    u, w = oracle.curl_state(GRID, A, 2.5e-5)
    assert not u.any()
    assert np.array_equal(w, 2.5e-5 * oracle.curl(GRID, A))


def load_wavespeed_golden():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "curl_wavespeed_180.txt")
    dt = offsets = None
    for line in open(path):
        if line.startswith("# dt "):
            dt = float(line.split()[2])
        elif line.startswith("# offsets_m "):
            offsets = np.array([float(v) for v in line.split()[2:]])
    return dt, offsets, np.loadtxt(path)


def test_stored_wavespeed_traces_recover_the_shear_speed():
    """The oracle's Sec. 4.1 run (stored by tests/golden/make_curl_wavespeed.py):
    the distance-time fit of the peak arrivals gives cs = sqrt(G / rho) = 2 m/s
    within 1 % (the paper reports < 0.1 % for its own source, whose width it
    does not state; here the dipole lobes of a 1 mm Gaussian bias the near
    sensors), and the arrivals are ordered by distance."""
    from oracle.analysis import arrival_time, fit_speed
    dt, offsets, tr = load_wavespeed_golden()
    times = np.array([arrival_time(tr[:, i], dt, t0=dt) for i in range(tr.shape[1])])
    assert np.all(np.diff(times) > 0)
    c, _ = fit_speed(offsets, times)
    assert abs(c - 2.0) < 0.01 * 2.0, c


def test_stored_wavespeed_velocity_peaks_give_the_shear_speed_to_a_tenth_percent():
    """The same stored run, arrivals taken at the peaks of the centred velocity
    traces (sharper than the displacement pulses, whose dipole lobes bias the
    near sensors): the fitted speed is sqrt(G / rho) = 2 m/s within 0.1 %."""
    from oracle.analysis import arrival_time, centred_velocity, fit_speed
    dt, offsets, tr = load_wavespeed_golden()
    v = centred_velocity(tr, dt)
    times = [arrival_time(v[:, i], dt, t0=dt) for i in range(v.shape[1])]
    c, _ = fit_speed(offsets, times)
    assert abs(c - 2.0) < 1e-3 * 2.0, c
