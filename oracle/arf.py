"""Acoustic radiation body force and acoustic strain from acoustic field time
series: plain FP64 numpy oracle.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and by the CPU-baseline leg
of ``bench.py``; the GPU library never uses it and it never uses the GPU
library.

Sec. 3.4 (sequential acoustic-elastic coupling): the acoustic pressure p and
particle velocity v are computed first, and a body force is derived from them
and handed to the shear solver as a prescribed source.  Two forms:

* plane-wave form, Eq. (isppa_norm): a scalar force b0 = (2 alpha / c) I_SPPA
  along the beam axis, with the pulse-average intensity
  I_SPPA = (1 / (rho c)) (sum over all N_total samples of p^2) / N_pulse;
* Poynting form, Eq. (arf_poynting): f_i = (2 alpha / c) I_i with the
  time-averaged Poynting vector I_i = <p v_i>, the average normalised the same
  way (sum over the samples divided by the samples in one pulse; Sec. 5.1 uses
  this form with a pulse normalisation it does not write out).

alpha is the absorption in Np/m at the transmit frequency.  Regions outside
the tissue of interest are masked to zero (Sec. 5.1).  Sec. 6.3 (Table
tab:arf_scaling) gives the frequency scaling at fixed intensity with
alpha = alpha0 f0 converted from dB/(cm MHz) to Np/m.

Sec. 5.2 also derives, from the pressure series alone and without the pulse
normalisation, the volumetric acoustic strain eps = -p / K (K = rho c^2) and
its spatial gradient, reported as their peaks over time.

Arrays are [nz][ny][nx] per scalar field and [3][nz][ny][nx] per vector field
(x fastest); a time series carries the sample index in front.
"""
from __future__ import annotations

import math

import numpy as np

# one neper is 20 log10(e) decibels (amplitude ratio e)
DB_PER_NEPER = 20.0 / math.log(10.0)


def alpha_np_per_m(alpha0_db_cm_mhz, f0_mhz):
    """Absorption at f0 in Np/m from a linear law alpha0 [dB/(cm MHz)] (Sec. 6.3)."""
    db_per_m = alpha0_db_cm_mhz * f0_mhz * 100.0
    return db_per_m / DB_PER_NEPER


def time_sums_pp(p_series):
    """Running sum over the samples, in sample order, of p^2 per cell (FP64).

    p_series: [nsamp, ...] (any float dtype; widened to FP64 before squaring).
    """
    p = np.asarray(p_series)
    S = np.zeros(p.shape[1:], dtype=np.float64)
    for t in range(p.shape[0]):
        pt = p[t].astype(np.float64)
        S = S + pt * pt
    return S


def time_sums_pv(p_series, v_series):
    """Running sums over the samples, in sample order, of p v_i per cell (FP64).

    p_series: [nsamp, ...]; v_series: [nsamp, 3, ...]; returns [3, ...].
    """
    p = np.asarray(p_series)
    v = np.asarray(v_series)
    assert v.shape[0] == p.shape[0] and v.shape[1] == 3 and v.shape[2:] == p.shape[1:]
    S = np.zeros((3,) + p.shape[1:], dtype=np.float64)
    for t in range(p.shape[0]):
        pt = p[t].astype(np.float64)
        for i in range(3):
            S[i] = S[i] + pt * v[t, i].astype(np.float64)
    return S


def _mask(mask, shape):
    if mask is None:
        return np.ones(shape, dtype=bool)
    return np.broadcast_to(np.asarray(mask) != 0, shape)


def plane_wave_force(S_pp, alpha, c, rho, n_pulse, beam_dir, mask=None):
    """Eq. (isppa_norm): F = b0 d with b0 = (2 alpha / c) I_SPPA,
    I_SPPA = S_pp / (rho c N_pulse); d = beam_dir / |beam_dir|; 0 where masked.

    S_pp: per-cell sum of p^2; alpha [Np/m], c [m/s], rho [kg/m^3]: scalars or
    per-cell arrays.  Returns [3, ...].
    """
    S_pp = np.asarray(S_pp, dtype=np.float64)
    d = np.asarray(beam_dir, dtype=np.float64)
    d = d / math.sqrt(float(d @ d))
    intensity = S_pp / (np.asarray(rho, dtype=np.float64) * np.asarray(c, dtype=np.float64) * float(n_pulse))
    b0 = (2.0 * np.asarray(alpha, dtype=np.float64) / np.asarray(c, dtype=np.float64)) * intensity
    keep = _mask(mask, S_pp.shape)
    F = np.zeros((3,) + S_pp.shape)
    for i in range(3):
        F[i] = np.where(keep, b0 * d[i], 0.0)
    return F


def poynting_force(S_pv, alpha, c, n_pulse, mask=None):
    """Eq. (arf_poynting): f_i = (2 alpha / c) I_i, I_i = S_pv,i / N_pulse; 0 where masked.

    S_pv: [3, ...] per-cell sums of p v_i.  Returns [3, ...].
    """
    S_pv = np.asarray(S_pv, dtype=np.float64)
    coef = 2.0 * np.asarray(alpha, dtype=np.float64) / np.asarray(c, dtype=np.float64)
    keep = _mask(mask, S_pv.shape[1:])
    F = np.zeros_like(S_pv)
    for i in range(3):
        F[i] = np.where(keep, coef * (S_pv[i] / float(n_pulse)), 0.0)
    return F


def strain_peaks(grid, p_series, K):
    """Peak volumetric acoustic strain and peak strain-gradient magnitude per
    cell over a pressure time series (Sec. 5.2): eps = -p / K with the bulk
    modulus K = rho c^2 (scalar or per cell), its gradient by the grid's
    centred differences (eps(+a) - eps(-a)) / (2 h_a) on the interior nodes
    (0 on the outer layer), |grad eps| = sqrt(gx^2 + gy^2 + gz^2); running
    maxima over the samples in sample order, with no pulse normalisation.  A
    NaN, once seen, stays (numpy's maximum).

    p_series: [nsamp][nz][ny][nx].  Returns (peak |eps|, peak |grad eps|).
    """
    nx, ny, nz, hx, hy, hz = grid
    p = np.asarray(p_series)
    K = np.broadcast_to(np.asarray(K, dtype=np.float64), p.shape[1:])
    pe = np.zeros(p.shape[1:])
    pg = np.zeros(p.shape[1:])
    for t in range(p.shape[0]):
        eps = -(p[t].astype(np.float64)) / K
        pe = np.maximum(pe, np.abs(eps))
        gx = (eps[1:-1, 1:-1, 2:] - eps[1:-1, 1:-1, :-2]) / (2 * hx)
        gy = (eps[1:-1, 2:, 1:-1] - eps[1:-1, :-2, 1:-1]) / (2 * hy)
        gz = (eps[2:, 1:-1, 1:-1] - eps[:-2, 1:-1, 1:-1]) / (2 * hz)
        g = np.sqrt(gx * gx + gy * gy + gz * gz)
        pg[1:-1, 1:-1, 1:-1] = np.maximum(pg[1:-1, 1:-1, 1:-1], g)
    return pe, pg
