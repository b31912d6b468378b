"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module only draws and samples inputs (grids, material maps, force
patterns, envelopes, probe lists).  It holds none of the solver's arithmetic:
no operator, no projection, no time step, no stability bound.  Where a
workload states its time step as a fraction of the stability limit, it
carries the fraction (``dt_factor``) and each side computes the limit itself.

Coordinates: node (i, j, k) sits at x = (i - nx//2) hx, y = (j - ny//2) hy,
z = (k - nz//2) hz, so the centre node of an even grid lies exactly at 0.
Arrays are [nz][ny][nx] (x fastest); vector fields [3][nz][ny][nx].
Seeds: numpy default_rng(1000 + workload index).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Workload:
    name: str
    grid: tuple                       # (nx, ny, nz, hx, hy, hz)
    G: object                         # float or [nz][ny][nx] array, Pa
    rho: object                       # kg/m^3
    eta: object                       # Pa s
    F: Optional[np.ndarray]           # [3][nz][ny][nx] body force pattern b0, N/m^3
    env: np.ndarray                   # g[n], n < len(env); 0 afterwards
    nsteps: int
    probes: np.ndarray                # [n][3] (i, j, k)
    comp: int = 2                     # recorded component (0..2) or 3 = all
    dt: Optional[float] = None        # explicit time step, s
    dt_factor: Optional[float] = None  # else dt = dt_factor * stable limit
    push_time: float = 0.0            # s; envelope length derived from dt
    sponge_cells: int = 8
    tol: float = 1e-8
    precision: str = "fp32"
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        nx, ny, nz = self.grid[:3]
        return (nz, ny, nx)

    @property
    def ncells(self):
        nx, ny, nz = self.grid[:3]
        return nx * ny * nz

    @property
    def interior_cells(self):
        nx, ny, nz = self.grid[:3]
        return (nx - 2) * (ny - 2) * (nz - 2)

    def envelope_for(self, dt):
        """Step envelope: g = 1 for n < round(push_time / dt), counted in
        whole steps."""
        n_push = int(round(self.push_time / dt))
        return np.ones(n_push)


def coords(n, h):
    return (np.arange(n) - n // 2) * h


def gaussian_push_params(sigma_l, sigma_a, F0, centre=(0.0, 0.0, 0.0), axis=2):
    """Parameters of the focused Gaussian push (a pattern dict, see
    force_from_params): no box, no modulation."""
    return dict(axis=int(axis), F0=float(F0), centre=tuple(float(c) for c in centre), sigma_lateral=float(sigma_l),
                sigma_axial=float(sigma_a), box_lateral=-1.0, box_axial=-1.0, k=np.zeros((0, 3)),
                phase=np.zeros(0), mod_amp=0.0)


def force_from_params(grid, p):
    """[3][nz][ny][nx] force of a pattern dict: F_axis = F0 exp(-lat^2 /
    (2 s_l^2) - ax^2 / (2 s_a^2)) M with M = 1 + a sum_m cos(k_m . x +
    phi_m), x the node coordinates, ax and lat^2 the axial and lateral
    offsets from the focus; 0 outside the box (when given).  Evaluated term
    by term in the order written."""
    nx, ny, nz, hx, hy, hz = grid
    axis = p["axis"]
    x = [coords(nx, hx), coords(ny, hy), coords(nz, hz)]
    off = [x[d] - p["centre"][d] for d in range(3)]
    keep = []
    for d in range(3):
        box = p["box_axial"] if d == axis else p["box_lateral"]
        keep.append(np.nonzero(np.abs(off[d]) <= box)[0] if box >= 0 else np.arange(len(off[d])))
    F = np.zeros((3, nz, ny, nx))
    ix, iy, iz = keep
    if ix.size == 0 or iy.size == 0 or iz.size == 0:
        return F
    Z, Y, X = np.meshgrid(off[2][iz], off[1][iy], off[0][ix], indexing="ij")
    O = [X, Y, Z]
    lat2 = None
    for d in range(3):
        if d != axis:
            lat2 = O[d] * O[d] if lat2 is None else lat2 + O[d] * O[d]
    ax = O[axis]
    g = np.exp(-lat2 / (2.0 * (p["sigma_lateral"] * p["sigma_lateral"]))
               - ax * ax / (2.0 * (p["sigma_axial"] * p["sigma_axial"])))
    M = np.ones_like(g)
    if len(p["phase"]):
        Za, Ya, Xa = np.meshgrid(x[2][iz], x[1][iy], x[0][ix], indexing="ij")
        for m in range(len(p["phase"])):
            k = p["k"][m]
            M = M + p["mod_amp"] * np.cos(k[0] * Xa + k[1] * Ya + k[2] * Za + p["phase"][m])
    F[axis][np.ix_(iz, iy, ix)] = p["F0"] * g * M
    return F


def gaussian_push(grid, sigma_l, sigma_a, F0, centre=(0.0, 0.0, 0.0), axis=2):
    """F along `axis` = F0 exp(-(lateral^2)/(2 sigma_l^2) - (axial - c)^2/(2 sigma_a^2)).
    Returns the [3][nz][ny][nx] force with only component `axis` non-zero."""
    return force_from_params(grid, gaussian_push_params(sigma_l, sigma_a, F0, centre, axis))


def x_line_probes(grid, j=None, k=None):
    nx, ny, nz = grid[:3]
    j = ny // 2 if j is None else j
    k = nz // 2 if k is None else k
    return np.array([[i, j, k] for i in range(nx)], dtype=np.int64)


def cfg1_homogeneous_fp64():
    """48^3, dx = 0.5 mm, G = 3 kPa, rho = 1000, eta = 0, 8-cell sponge,
    Gaussian F_z (1 mm lateral, 4 mm axial, F0 = 1e4) at the centre node,
    100 us push, dt = 5e-5 s, 200 steps, u_z on the lateral x line, FP64,
    projection tolerance 1e-10."""
    h = 0.5e-3
    grid = (48, 48, 48, h, h, h)
    F = gaussian_push(grid, 1e-3, 4e-3, 1e4)
    w = Workload(name="homogeneous 48^3 fp64", grid=grid, G=3e3, rho=1000.0, eta=0.0, F=F,
                 env=None, nsteps=200, probes=x_line_probes(grid), comp=2, dt=5e-5,
                 push_time=100e-6, sponge_cells=8, tol=1e-10, precision="fp64")
    w.env = w.envelope_for(w.dt)
    return w


def spherical_inclusions(grid, rng, n_incl, background, radius_range, G_range, rho_range, eta_range,
                         margin_cells):
    """Background (G, rho, eta) with n_incl spheres; centres uniform over the
    index box [margin, n-1-margin] on each axis, radius uniform in
    radius_range; each property uniform in its range; a cell belongs to a
    sphere when |x - c| <= r; later spheres overwrite earlier ones."""
    nx, ny, nz, hx, hy, hz = grid
    G = np.full((nz, ny, nx), float(background[0]))
    rho = np.full((nz, ny, nx), float(background[1]))
    eta = np.full((nz, ny, nx), float(background[2]))
    x, y, z = coords(nx, hx), coords(ny, hy), coords(nz, hz)
    spheres = []
    def centre(n):
        m = min(margin_cells, (n - 1) / 2.0)  # small grids: the box shrinks to the middle
        return rng.uniform(m, n - 1 - m)

    for _ in range(n_incl):
        ci, cj, ck = centre(nx), centre(ny), centre(nz)
        c = ((ci - nx // 2) * hx, (cj - ny // 2) * hy, (ck - nz // 2) * hz)
        r = rng.uniform(*radius_range)
        g_, r_, e_ = rng.uniform(*G_range), rng.uniform(*rho_range), rng.uniform(*eta_range)
        spheres.append((c, r, g_, r_, e_))
    for (c, r, g_, r_, e_) in spheres:
        dz2 = (z - c[2])[:, None, None] ** 2
        dy2 = (y - c[1])[None, :, None] ** 2
        dx2 = (x - c[0])[None, None, :] ** 2
        m = (dz2 + dy2 + dx2) <= r * r
        G[m], rho[m], eta[m] = g_, r_, e_
    return G, rho, eta, spheres


def cfg2_inclusions_fp32(n=256):
    """256^3, dx = 0.25 mm, background (2 kPa, 1000, 0.5 Pa s), 12 seeded
    spherical inclusions (radius 1.5-5 mm, G 1-10 kPa, rho 1000-1100,
    eta 0-1.5), Gaussian F_z with the same physical widths as the 48^3 case,
    100 us push, dt = 0.4 x stable limit, 4000 steps, FP32 state with FP64
    projection to 1e-8.  `n` shrinks the grid for tests (same physics)."""
    rng = np.random.default_rng(1002)
    h = 0.25e-3
    grid = (n, n, n, h, h, h)
    G, rho, eta, spheres = spherical_inclusions(grid, rng, 12, (2e3, 1000.0, 0.5), (1.5e-3, 5e-3),
                                                (1e3, 1e4), (1000.0, 1100.0), (0.0, 1.5), 8)
    F = gaussian_push(grid, 1e-3, 4e-3, 1e4)
    return Workload(name=f"inclusions {n}^3 fp32", grid=grid, G=G, rho=rho, eta=eta, F=F, env=None,
                    nsteps=4000, probes=x_line_probes(grid), comp=2, dt_factor=0.4, push_time=100e-6,
                    sponge_cells=8, tol=1e-8, precision="fp32", meta={"spheres": spheres})


def cfg3_batch_draws(n_inst=64, edges=(96, 128, 160, 192)):
    """64 homogeneous instances: edge from `edges`, G from 10 log-spaced
    values in [1, 10] kPa, eta from 16 values 0, 0.1, ..., 1.5 Pa s,
    rho = 1000, dx = 0.25 mm; returns a list of (edge, G, rho, eta)."""
    rng = np.random.default_rng(1003)
    Gs = 10.0 ** (3.0 + np.arange(10) / 9.0)
    etas = 0.1 * np.arange(16)
    out = []
    for _ in range(n_inst):
        e = int(rng.choice(edges))
        out.append((e, float(rng.choice(Gs)), 1000.0, float(rng.choice(etas))))
    return out


def random_force(grid, rng, scale=1.0):
    """Smooth-ish random 3-component force for operator tests."""
    nx, ny, nz = grid[:3]
    return scale * rng.standard_normal((3, nz, ny, nx))


def focal_focus_z(grid, epoch, dt, steps_per_epoch=10, speed=1e-3 / 20e-6):
    """Axial focus of the moving push at the start of `epoch`: it travels at
    `speed` (1 mm per 20 us) and bounces between 25 % and 75 % of the depth
    (node coordinates), starting at 25 %."""
    nz, h = grid[2], grid[5]
    zmin, zmax = -(nz // 2) * h, (nz - 1 - nz // 2) * h
    lo, hi = zmin + 0.25 * (zmax - zmin), zmin + 0.75 * (zmax - zmin)
    L = hi - lo
    s = (speed * epoch * steps_per_epoch * dt) % (2 * L)
    return lo + (s if s <= L else 2 * L - s)


def focal_modulated_params(grid, seed=1004, epoch=0, dt=1.75e-6, steps_per_epoch=10, sigma_l=1e-3, sigma_a=4e-3,
                           F0=1e4):
    """Pattern dict of the time-varying workload's push at `epoch`: a z
    Gaussian (sigma_l lateral, sigma_a axial) on the lateral centre line
    focused at the z of `focal_focus_z`, times M(x) = 1 + 0.5 / sqrt(8)
    sum_m cos(k_m . x + phi_m) with 8 plane waves, |k_m| uniform in
    [2 pi / 4 mm, 2 pi / 1 mm] with random directions (fixed by `seed`) and
    phases redrawn every epoch (seeded by (seed, epoch)); F = 0 outside the
    box where the Gaussian factor is above 1e-16 along each axis."""
    rng = np.random.default_rng(seed)
    kmag = rng.uniform(2 * np.pi / 4e-3, 2 * np.pi / 1e-3, 8)
    dirs = rng.standard_normal((8, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    kvec = kmag[:, None] * dirs
    phases = np.random.default_rng([seed, epoch]).uniform(0, 2 * np.pi, 8)
    zf = focal_focus_z(grid, epoch, dt, steps_per_epoch)
    cut = np.sqrt(2 * np.log(1e16))
    return dict(axis=2, F0=float(F0), centre=(0.0, 0.0, float(zf)), sigma_lateral=float(sigma_l),
                sigma_axial=float(sigma_a), box_lateral=float(cut * sigma_l), box_axial=float(cut * sigma_a),
                k=kvec, phase=phases, mod_amp=0.5 / np.sqrt(8))


def focal_modulated_force(grid, seed=1004, epoch=0, dt=1.75e-6, steps_per_epoch=10, sigma_l=1e-3, sigma_a=4e-3,
                          F0=1e4):
    """Non-separable push of the time-varying workload (focal_modulated_params)
    as a [3][nz][ny][nx] FP64 numpy array."""
    return force_from_params(grid, focal_modulated_params(grid, seed, epoch, dt, steps_per_epoch, sigma_l, sigma_a, F0))


def gaussian_random_field(shape, h, corr_len, rng):
    """Smooth random field on a [nz][ny][nx] grid of spacing h: white noise
    convolved (periodically, in Fourier space) with a Gaussian of standard
    deviation corr_len / sqrt(2), so the field's correlation is a Gaussian of
    standard deviation corr_len; then standardised (mean 0, variance 1)."""
    import scipy.fft
    nz, ny, nx = shape
    xi = rng.standard_normal(shape)
    spec = scipy.fft.rfftn(xi, workers=-1)
    del xi
    s2 = 0.5 * corr_len ** 2
    kz = 2 * np.pi * np.fft.fftfreq(nz, h)
    ky = 2 * np.pi * np.fft.fftfreq(ny, h)
    kx = 2 * np.pi * np.fft.rfftfreq(nx, h)
    spec *= np.exp(-0.5 * s2 * kz ** 2)[:, None, None]
    spec *= np.exp(-0.5 * s2 * ky ** 2)[None, :, None]
    spec *= np.exp(-0.5 * s2 * kx ** 2)[None, None, :]
    f = scipy.fft.irfftn(spec, s=shape, workers=-1)
    del spec
    f -= f.mean()
    f /= f.std()
    return f


def cfg4_grf_material(n=(384, 384, 512), h=0.2e-3, corr_len=3e-3, seed=1004):
    """Medium of the time-varying-source workload: G = 10^(3 + Phi(xi)) Pa
    (so 1-10 kPa) and eta = 1.5 Phi(xi') Pa s from two independent standardised
    Gaussian random fields (3 mm correlation length), Phi the standard normal
    CDF; rho = 1000.  Returns (grid, G, rho, eta) with [nz][ny][nx] arrays."""
    import scipy.special
    nx, ny, nz = n
    grid = (nx, ny, nz, h, h, h)
    xi = gaussian_random_field((nz, ny, nx), h, corr_len, np.random.default_rng([seed, 1]))
    G = 10.0 ** (3.0 + scipy.special.ndtr(xi))
    del xi
    xi = gaussian_random_field((nz, ny, nx), h, corr_len, np.random.default_rng([seed, 2]))
    eta = 1.5 * scipy.special.ndtr(xi)
    return grid, G, 1000.0, eta


def real_sph_harm_sum(coef, theta, phi):
    """sum over (l, m) of coef[(l, m)] Y_lm(theta, phi) with real, orthonormal
    spherical harmonics: Y_l0 = N_l0 P_l^0(cos theta); for m > 0 sqrt(2) N_lm
    P_l^m(cos theta) cos(m phi); for m < 0 sqrt(2) N_l|m| P_l^|m|(cos theta)
    sin(|m| phi), with N_lm^2 = (2l + 1) / (4 pi) (l - m)! / (l + m)! and P_l^m
    the associated Legendre functions with the Condon-Shortley phase, built by
    the standard three-term recurrence in l."""
    from math import factorial
    x = np.cos(theta)
    sx = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    lmax = max(l for l, _ in coef)
    out = np.zeros(np.broadcast(theta, phi).shape)
    pmm = np.ones_like(x)
    for m in range(0, lmax + 1):
        if m > 0:
            pmm = -(2 * m - 1) * sx * pmm
        cm, sm = (np.cos(m * phi), np.sin(m * phi)) if m > 0 else (None, None)
        p_prev, p = None, pmm
        for l in range(m, lmax + 1):
            if l == m + 1:
                p_prev, p = p, x * (2 * m + 1) * pmm
            elif l > m + 1:
                p_prev, p = p, ((2 * l - 1) * x * p - (l + m - 1) * p_prev) / (l - m)
            N = np.sqrt((2 * l + 1) / (4 * np.pi) * factorial(l - m) / factorial(l + m))
            if m == 0:
                if (l, 0) in coef:
                    out += coef[(l, 0)] * N * p
                continue
            if (l, m) in coef:
                out += coef[(l, m)] * np.sqrt(2) * N * p * cm
            if (l, -m) in coef:
                out += coef[(l, -m)] * np.sqrt(2) * N * p * sm
    return out


@dataclass
class ShellGeometry:
    centre: tuple       # sphere centre (x, y, z), m, node coordinates
    r_outer: float
    coef: dict          # (l, m) -> spherical-harmonic coefficient
    s_max: float        # max |s| over the 1-degree direction grid

    def thickness(self, theta, phi):
        return 6.5e-3 + 1.5e-3 * real_sph_harm_sum(self.coef, theta, phi) / self.s_max


def shell_geometry(grid, rng, r_outer=70e-3, top_depth=10e-3, lmax=4):
    """Spherical shell on the lateral centre line whose outer sphere (radius
    r_outer) reaches up to depth top_depth below the z = first-node face;
    thickness 6.5 mm + 1.5 mm s(theta, phi), s a sum of real spherical
    harmonics l = 1..lmax with N(0, 1) coefficients, scaled to max |s| = 1 over
    a 1-degree (theta, phi) grid (so 5-8 mm).  theta is measured from +z."""
    nz, hz = grid[2], grid[5]
    z_first = -(nz // 2) * hz
    centre = (0.0, 0.0, z_first + top_depth + r_outer)
    coef = {(l, m): float(rng.standard_normal()) for l in range(1, lmax + 1) for m in range(-l, l + 1)}
    th = np.deg2rad(np.arange(181.0))[:, None]
    ph = np.deg2rad(np.arange(360.0))[None, :]
    s_max = float(np.abs(real_sph_harm_sum(coef, th, ph)).max())
    return ShellGeometry(centre=centre, r_outer=r_outer, coef=coef, s_max=s_max)


def shell_material(grid, geo, shell=(100e3, 1900.0, 2.0), soft=(1.5e3, 1040.0, 0.8)):
    """(G, rho, eta) [nz][ny][nx]: `shell` properties where r_outer - T(theta,
    phi) <= |x - centre| <= r_outer, `soft` elsewhere.  Built one z plane at a
    time; the spherical harmonics are evaluated only in the radial band."""
    nx, ny, nz, hx, hy, hz = grid
    x = coords(nx, hx) - geo.centre[0]
    y = coords(ny, hy) - geo.centre[1]
    z = coords(nz, hz) - geo.centre[2]
    G = np.full((nz, ny, nx), soft[0])
    rho = np.full((nz, ny, nx), soft[1])
    eta = np.full((nz, ny, nx), soft[2])
    rxy2 = x[None, :] ** 2 + y[:, None] ** 2
    inner_min = geo.r_outer - 8.0e-3
    for k in range(nz):
        r = np.sqrt(rxy2 + z[k] ** 2)
        band = (r <= geo.r_outer) & (r >= inner_min)
        if not band.any():
            continue
        jj, ii = np.nonzero(band)
        rb = r[jj, ii]
        theta = np.arccos(np.clip(z[k] / rb, -1.0, 1.0))
        phi = np.arctan2(y[jj], x[ii])
        inside = rb >= geo.r_outer - geo.thickness(theta, phi)
        jj, ii = jj[inside], ii[inside]
        G[k, jj, ii], rho[k, jj, ii], eta[k, jj, ii] = shell
    return G, rho, eta


def cfg5_shell(n=(512, 512, 640), h=0.2e-3, seed=1005):
    """Transcranial-like case: curved shell (100 kPa, 1900, 2 Pa s, 5-8 mm
    thick) over soft tissue (1.5 kPa, 1040, 0.8 Pa s); F_z Gaussian push
    (1 mm lateral, 5 mm axial, F0 = 5e4) on the axis 20 mm below the shell's
    inner surface, 200 us; dt = 0.4 x stable limit; 6000 steps; peak |u| on
    the x, y and z planes through the push.  `n` shrinks the grid for tests
    (the shell keeps its physical size, so small grids see only its top)."""
    nx, ny, nz = n
    grid = (nx, ny, nz, h, h, h)
    geo = shell_geometry(grid, np.random.default_rng(seed))
    G, rho, eta = shell_material(grid, geo)
    t_top = float(geo.thickness(np.pi, 0.0))
    z_push = geo.centre[2] - geo.r_outer + t_top + 20e-3
    F = gaussian_push(grid, 1e-3, 5e-3, 5e4, centre=(0.0, 0.0, z_push))
    k_push = int(round(z_push / h)) + nz // 2
    planes = [(0, nx // 2), (1, ny // 2), (2, k_push)]
    return Workload(name=f"shell {nx}x{ny}x{nz}", grid=grid, G=G, rho=rho, eta=eta, F=F, env=None, nsteps=6000,
                    probes=x_line_probes(grid, k=k_push), comp=2, dt_factor=0.4, push_time=200e-6,
                    sponge_cells=8, tol=1e-8, precision="fp32",
                    meta={"geometry": geo, "z_push": z_push, "k_push": k_push, "peak_planes": planes})


def acoustic_beam_samples(grid, samples, f0=1.0e6, c=1540.0, rho=1000.0, alpha=5.8, p0=1.5e6, w0=1.5e-3,
                          focus=(0.0, 0.0, 0.0), per=20, cycles=10, s0=0, dtype=np.float32):
    """A synthetic focused tone burst standing in for an acoustic solver's
    output (the paper's Fullwave fields are not available): a Gaussian beam
    along +z focused at `focus` (waist w0, wavelength c/f0, attenuated by
    e^{-alpha (z - z_min)}), `cycles` periods of `per` samples each, silence
    after; v = p n / (rho c) with n the local direction of the phase front
    (x/R, y/R, 1), normalised.

    Returns (p, v): p [samples][nz][ny][nx], v [samples][3][nz][ny][nx] for
    sample indices s0 .. s0 + samples - 1, built in FP64 and cast to `dtype`
    (workloads.gpu.beam_samples_device draws the same samples on the device).
    """
    nx, ny, nz, hx, hy, hz = grid
    xp = np
    arange = lambda n, h: (np.arange(n) - n // 2) * h
    zeros = lambda shape: np.zeros(shape)
    cast = lambda a: a.astype(dtype)
    x = arange(nx, hx)[None, None, :] - focus[0]
    y = arange(ny, hy)[None, :, None] - focus[1]
    z = arange(nz, hz)[:, None, None]
    dz = z - focus[2]
    lam = c / f0
    k = 2 * np.pi / lam
    zr = np.pi * w0 ** 2 / lam
    w = w0 * (1 + (dz / zr) ** 2) ** 0.5
    inv_r = dz / (dz ** 2 + zr ** 2)
    rr = x ** 2 + y ** 2
    amp = p0 * (w0 / w) * xp.exp(-rr / w ** 2) * xp.exp(-alpha * (z - z.min()))
    phase = k * dz + k * rr * inv_r / 2 - xp.arctan(dz / zr)
    nxv, nyv = x * inv_r, y * inv_r
    norm = (nxv ** 2 + nyv ** 2 + 1.0) ** 0.5
    p = zeros((samples, nz, ny, nx))
    for q in range(samples):
        s = s0 + q
        if s < per * cycles:
            p[q] = amp * xp.cos(2 * np.pi * s / per - phase)
    scale = 1.0 / (rho * c)
    v = zeros((samples, 3, nz, ny, nx))
    v[:, 0] = p * (scale * nxv / norm)
    v[:, 1] = p * (scale * nyv / norm)
    v[:, 2] = p * (scale / norm)
    return cast(p), cast(v)


def curl_wavespeed_case(n=180, h=0.2e-3, cs=2.0, rho=1000.0, sigma=1.0e-3, psi0=1.0e-6, dt_factor=0.4,
                        nsteps=360, offsets_mm=(3.6, 6.0, 8.4, 10.8)):
    """Non-viscous wavespeed recovery (Sec. 4.1): a cube of n^3 nodes
    (h = 0.2 mm, 36 mm wide at n = 180), homogeneous G = rho cs^2 with
    cs = 2 m/s, eta = 0, Dirichlet walls only; the initial velocity is the
    curl of the vector potential A = psi y_hat, psi a Gaussian of width sigma
    centred on the centre node (motion in the x-z plane, u_z odd in x);
    sensors on the x (depth) axis through the centre at the given offsets,
    recording u_z.

    Returns a dict: grid, G, rho, eta, A [3][nz][ny][nx], dt_factor, nsteps,
    probes [n][3], offsets [m].
    """
    grid = (n, n, n, h, h, h)
    x = coords(n, h)
    X, Y, Z = x[None, None, :], x[None, :, None], x[:, None, None]
    A = np.zeros((3, n, n, n))
    A[1] = psi0 * np.exp(-(X ** 2 + Y ** 2 + Z ** 2) / (2 * sigma ** 2))
    c = n // 2
    steps = [int(round(o * 1e-3 / h)) for o in offsets_mm]
    probes = np.array([[c + s, c, c] for s in steps], dtype=np.int64)
    return dict(grid=grid, G=rho * cs ** 2, rho=rho, eta=0.0, A=A, dt_factor=dt_factor, nsteps=nsteps,
                probes=probes, offsets=np.array(steps) * h)


def qiba_phantoms(shape=(240, 200, 200), h=0.25e-3, G=(1e3, 2e3, 5e3, 10e3), rho=1000.0, amp=1e4,
                  x_focus=30e-3, sigma=(4.3e-3, 0.62e-3, 1.1e-3), push_time=167e-6, nsteps=400, dt_factor=0.4,
                  offsets_mm=tuple(4.0 + 0.5 * q for q in range(21))):
    """QIBA-like elastic phantoms (Sec. 4.4): an nx x ny x nz grid (x = depth,
    measured from the first node; y lateral and z elevational, centred),
    h = 0.25 mm (60 x 50 x 50 mm at the default size), homogeneous media with
    the given shear moduli, rho = 1000, eta = 0; body force along the depth
    axis with the Gaussian profile of Eq. gaussexc,
    amp exp(-((x - x_f)/s_x)^2 - (y/s_y)^2 - (z/s_z)^2) (1/e widths: axial
    4.3 mm, lateral 0.62 mm, elevational 1.1 mm; focus at 30 mm depth), on for
    167 us; sensors at the focal depth on the lateral axis at 4-14 mm from the
    push axis, recording the axial displacement.

    Returns a dict: grid, G (tuple), rho, eta, F [3][nz][ny][nx], push_time,
    dt_factor, nsteps, probes [n][3], offsets [n] (m), comp (0 = x).
    """
    nx, ny, nz = shape
    grid = (nx, ny, nz, h, h, h)
    depth = np.arange(nx) * h
    y = coords(ny, h)
    z = coords(nz, h)
    sx, sy, sz = sigma
    F = np.zeros((3, nz, ny, nx))
    F[0] = amp * np.exp(-((depth[None, None, :] - x_focus) / sx) ** 2 - (y[None, :, None] / sy) ** 2
                        - (z[:, None, None] / sz) ** 2)
    i_f = int(round(x_focus / h))
    steps = [int(round(o * 1e-3 / h)) for o in offsets_mm]
    probes = np.array([[i_f, ny // 2 + s, nz // 2] for s in steps], dtype=np.int64)
    return dict(grid=grid, G=tuple(G), rho=rho, eta=0.0, F=F, push_time=push_time, dt_factor=dt_factor,
                nsteps=nsteps, probes=probes, offsets=np.array(steps) * h, comp=0)


def pulsed_envelope(dt, on=1e-3, off=1e-3, pulses=25):
    """Pulsed forcing protocol of the TIPS demonstration (Sec. 5.2): 50 % duty
    cycle, `on` seconds on and `off` off, `pulses` pulses (50 ms at the
    defaults).  Step n is on when t_n = n dt falls in an on-interval, counted
    in whole steps like the single push (g = 1 for the first round(on / dt)
    steps of each period of round((on + off) / dt) steps).  Returns g[n] over
    the whole protocol."""
    n_on = int(round(on / dt))
    n_per = int(round((on + off) / dt))
    g = np.zeros(n_per * pulses)
    for q in range(pulses):
        g[q * n_per:q * n_per + n_on] = 1.0
    return g


def convergence_level(n, width=36e-3, sigma=3e-3, cs=2.0, rho=1000.0, Ts=120e-6, window=9.6e-3,
                      offsets_mm=(3.6, 6.0, 8.4, 10.8)):
    """One level of the grid-convergence study (Sec. 4.2): a cube `width`
    wide with n nodes (n - 1 a multiple of 30 so that the sensors, at
    multiples of 1.2 mm from the centre along x, and the centre sit on
    nodes), the curl source of the wavespeed case with a Gaussian of width
    sigma, eta = 0, Dirichlet walls; dt = Ts 30 / (n - 1), so that every
    level samples t = m Ts; `window` long.  Returns the curl_wavespeed_case
    dict plus dt, nsteps, sub (steps per Ts) and nsamp (samples at m Ts,
    m = 1 .. nsamp)."""
    assert (n - 1) % 30 == 0 and n % 2 == 1
    h = width / (n - 1)
    w = curl_wavespeed_case(n=n, h=h, cs=cs, rho=rho, sigma=sigma, offsets_mm=offsets_mm)
    sub = (n - 1) // 30
    w.update(dt=Ts / sub, sub=sub, nsteps=int(round(window / Ts)) * sub, nsamp=int(round(window / Ts)) - 1)
    return w


# Viscosity sweep of the 1-D harmonic Kelvin-Voigt benchmark (Sec. 4.3):
# eta = 0 .. 1.5 Pa s in steps of 0.1.
KV_LINE_ETAS = tuple(round(0.1 * j, 10) for j in range(16))
# Drive frequencies [Hz] at the viscosities of the benchmark's table: the ones
# at which the continuous Kelvin-Voigt law with c_s = 2 m/s (G = 4 kPa,
# rho = 1000) gives the table's theoretical attenuation; the paper names a
# smooth schedule f0(eta) without its values.
KV_LINE_F0_KNOTS = ((0.1, 800.1), (0.3, 789.9), (0.5, 761.0), (1.0, 742.0), (1.5, 742.1))


def kv_line_frequency(eta):
    """Drive frequency [Hz] for viscosity eta: linear between the knots,
    held at the end values outside them."""
    k = np.array(KV_LINE_F0_KNOTS)
    return float(np.interp(eta, k[:, 0], k[:, 1]))


def kv_line_grid(nx=301, h=1e-4, transverse=1e6):
    """A 1-D line of nx nodes (h apart, Dirichlet ends) as an nx x 3 x 3 grid
    whose y and z spacings are `transverse` metres: the line is the one
    interior row (j = k = 1), and the y and z terms of the stencil, which see
    the zero Dirichlet neighbours, scale with 1 / transverse^2 and are below
    FP64 rounding of the x terms (1e-20 of them at the defaults)."""
    return (nx, 3, 3, h, transverse, transverse)


def kv_line_case(grid, eta, dt, nsteps, alpha_expected, c_expected, amp=1e4, ramp_periods=2.0,
                 fit_periods=4.0, n_sensors=6, first_mm=0.5, source=1):
    """Inputs of one instance of the harmonic benchmark on a kv_line_grid:
    a z-directed point force on line node `source` (next to the x = 0 wall)
    driven by g^n = r(t_n) sin(w t_n), t_n = n dt, with a raised-cosine
    ramp r over `ramp_periods` periods (it keeps the start-up transient
    narrow-band), w = 2 pi f0(eta); n_sensors sensors on the line from
    first_mm past the source over a span of min(2 wavelengths, 2 e-folding
    lengths) of the expected wave (alpha_expected [Np/m], c_expected [m/s]:
    the sensors adapt to the attenuation); the fit window is the last
    fit_periods periods of the run.  The projected force is the pattern
    itself: a transverse force uniform over a plane has no divergence.
    Returns dict(f0, omega, FS [3][3][3][nx], env [nsteps], probes [s][3],
    x [s] (metres from the wall), t_from)."""
    nx, h = grid[0], grid[3]
    f0 = kv_line_frequency(eta)
    omega = 2.0 * np.pi * f0
    lam = c_expected / f0
    span = 2.0 * lam if alpha_expected <= 0 else min(2.0 * lam, 2.0 / alpha_expected)
    d = first_mm * 1e-3 + np.linspace(0.0, span, n_sensors)
    ix = source + np.round(d / h).astype(np.int64)
    assert ix[-1] < nx - 1 and len(set(ix.tolist())) == n_sensors
    FS = np.zeros((3, 3, 3, nx))
    FS[2, 1, 1, source] = amp
    t = np.arange(nsteps) * dt
    Tr = ramp_periods / f0
    r = np.where(t < Tr, 0.5 * (1.0 - np.cos(np.pi * t / Tr)), 1.0)
    env = r * np.sin(omega * t)
    probes = np.stack([ix, np.ones_like(ix), np.ones_like(ix)], axis=1)
    return dict(f0=f0, omega=omega, FS=FS, env=env, probes=probes, x=ix * h,
                t_from=nsteps * dt - fit_periods / f0)
