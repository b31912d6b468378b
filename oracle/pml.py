"""Convolutional perfectly matched layer (C-PML) for the reduced Kelvin-Voigt
shear equation: plain FP64 numpy oracle.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``; the GPU library never uses
it and it never uses the GPU library.

The paper terminates the grid with a Dirichlet layer, notes that its
reflections contaminate late arrivals, and names perfectly matched layers as
the remedy and as future work (Sec. 3.5, Sec. 6.1, Sec. 7); it gives no
formulation.  This oracle states the one the library implements: complex
coordinate stretching along each axis a, s_a = 1 + d_a(x_a) / (alpha_a + i w)
(the complex-frequency-shifted form with kappa = 1), applied to both spatial
derivatives of each term of the update of Sec. 3.1, div(G grad u_c) and
(eta / dt) lap(w_c), in recursive-convolution form (Roden and Gedney 2000;
Komatitsch and Martin 2007).  With the face fluxes of the plain method,

    F_el = G_f (u(+a) - u) / h_a,   F_w = (w(+a) - w) / h_a        (faces),

each stretched derivative adds a memory variable updated once per step from
the current value of the derivative it stretches:

    psi <- b psi + c X,   stretched X = X + psi,
    b = exp(-(d + alpha) dt),   c = d / (d + alpha) (b - 1)   (c = 0 where d = 0),

first on the face fluxes (psi_el, psi_w), then on the cell divergence of each
axis, D_a = ((F_el + psi_el)(+) - (F_el + psi_el)(-)) / h_a
      + (eta / dt) ((F_w + psi_w)(+) - (F_w + psi_w)(-)) / h_a,
stretched as D_a + phi_a.  The update is then the plain one with
acc = sum_a (D_a + phi_a) + g_n f_S (no sponge).

Profile along an axis of n nodes with an L-cell layer next to each Dirichlet
face: the layer's inner edge sits at index L + 1/2 (low side) and
n - 3/2 - L (high side); at index position x (cells at integers, faces at
half integers) the depth is q = (L + 1/2 - x) / L or (x - (n - 3/2 - L)) / L
where positive, d = d0 q^2 with d0 = 3 c_max ln(1/R) / (2 L h) (quadratic
profile, theoretical normal-incidence reflection R, c_max the largest shear
speed), alpha = alpha_max inside the layer and 0 elsewhere (default alpha_max =
pi c_max / (10 L h_min): the frequency of a wave ten layer widths long, which
the layer could not absorb anyway; a larger shift moves more of the band the
layer does absorb into the unabsorbed part).  alpha is held
constant across the layer rather than tapered to zero at the wall: at zero
frequency the stretched flux is alpha / (d + alpha) times the plain one, so a
vanishing alpha at the wall would cut the interior off from the Dirichlet
layer and leave it free to drift by a uniform displacement after a push with
net impulse (and alpha = 0 everywhere lets that drift grow linearly).

Arrays are [nz][ny][nx] per scalar field and [3][nz][ny][nx] per vector
field (x fastest).
"""
from __future__ import annotations

import math

import numpy as np


def profile(n, L, h, cmax, dt, R, alpha_max):
    """(b, c) at the cells (n values, index i) and at the faces (n - 1 values,
    face i between cells i and i + 1) of one axis."""
    d0 = 3.0 * cmax * math.log(1.0 / R) / (2.0 * L * h) if L > 0 else 0.0

    def coef(x):
        if L > 0:
            q = np.maximum((L + 0.5 - x) / L, (x - (n - 1.5 - L)) / L)
        else:
            q = np.full_like(x, -1.0)
        inside = q > 0
        q = np.where(inside, q, 0.0)
        d = d0 * q * q
        alpha = np.where(inside, alpha_max, 0.0)
        b = np.exp(-(d + alpha) * dt)
        c = np.where(d > 0, d / np.where(d > 0, d + alpha, 1.0) * (b - 1.0), 0.0)
        return b, c

    xc = np.arange(n, dtype=np.float64)
    return coef(xc), coef(xc[:-1] + 0.5)


def _field(shape, v):
    return np.broadcast_to(np.asarray(v, dtype=np.float64), shape).copy()


def _along(a, ax, ndim=4):
    """Reshape a 1-D table to broadcast along array axis ax of a [3][z][y][x] array."""
    s = [1] * ndim
    s[ax] = a.size
    return a.reshape(s)


def default_alpha_max(grid, cmax, L):
    return math.pi * cmax / (10.0 * L * min(grid[3:6]))


def run_pml(grid, G, rho, eta, dt, nsteps, pml_cells, R=1e-5, alpha_max=None, FS=None, env=None, u=None, w=None,
            probes=None, comp=2):
    """Advance the summed-form state (u, w) nsteps steps with the C-PML on every
    face (no sponge); alpha_max None takes the default.  Returns
    (u, w, traces [step][probe][ncomp])."""
    nx, ny, nz, hx, hy, hz = grid
    shape = (nz, ny, nx)
    G = _field(shape, G)
    rho = _field(shape, rho)
    eta = _field(shape, eta)
    crho = dt * dt / rho
    cmax = float(np.sqrt(np.max(G / rho)))
    if alpha_max is None:
        alpha_max = default_alpha_max(grid, cmax, max(pml_cells, 1))
    u = np.zeros((3,) + shape) if u is None else np.array(u, dtype=np.float64).reshape((3,) + shape)
    w = np.zeros((3,) + shape) if w is None else np.array(w, dtype=np.float64).reshape((3,) + shape)
    FS = None if FS is None else np.asarray(FS, dtype=np.float64).reshape((3,) + shape)
    axes = [(3, nx, hx), (2, ny, hy), (1, nz, hz)]  # (array axis of [3][z][y][x], extent, spacing)
    tabs, psi_el, psi_w, phi, Gface = [], [], [], [], []
    for ax, n, h in axes:
        (bc, cc), (bf, cf) = profile(n, pml_cells, h, cmax, dt, R, alpha_max)
        tabs.append((_along(bc, ax), _along(cc, ax), _along(bf, ax), _along(cf, ax)))
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax - 1] = slice(0, -1)
        hi[ax - 1] = slice(1, None)
        G0, G1 = G[tuple(lo)], G[tuple(hi)]
        Gface.append(2.0 * G0 * G1 / (G0 + G1))
        fshape = list((3,) + shape)
        fshape[ax] -= 1
        psi_el.append(np.zeros(fshape))
        psi_w.append(np.zeros(fshape))
        phi.append(np.zeros((3,) + shape))
    inner = np.zeros(shape, dtype=bool)
    inner[1:-1, 1:-1, 1:-1] = True
    pr = None if probes is None else np.asarray(probes, dtype=np.int64).reshape(-1, 3)
    traces = []
    for step in range(nsteps):
        gn = float(env[step]) if env is not None and step < len(env) else 0.0
        acc = np.zeros((3,) + shape)
        for a, (ax, n, h) in enumerate(axes):
            bc, cc, bf, cf = tabs[a]
            F_el = Gface[a] * (np.diff(u, axis=ax) / h)
            F_w = np.diff(w, axis=ax) / h
            psi_el[a] = bf * psi_el[a] + cf * F_el
            psi_w[a] = bf * psi_w[a] + cf * F_w
            s_el = F_el + psi_el[a]
            s_w = F_w + psi_w[a]
            D = np.zeros((3,) + shape)
            mid = [slice(None)] * 4
            mid[ax] = slice(1, -1)
            D[tuple(mid)] = np.diff(s_el, axis=ax) / h + (eta[tuple(mid[1:])] / dt) * (np.diff(s_w, axis=ax) / h)
            phi[a] = bc * phi[a] + cc * D
            acc += D + phi[a]
        if FS is not None and gn != 0.0:
            acc += gn * FS
        w = np.where(inner, w + crho * acc, 0.0)
        u = np.where(inner, u + w, 0.0)
        if pr is not None:
            vals = u[:, pr[:, 2], pr[:, 1], pr[:, 0]].T  # [probe][3]
            traces.append(vals if comp == 3 else vals[:, comp:comp + 1])
    tr = np.array(traces) if pr is not None else None
    return u, w, tr
