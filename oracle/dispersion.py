"""Kelvin-Voigt dispersion relations (test infrastructure, used by the oracle
pins and by the physics checks).

Continuous law: for a plane shear wave exp(i(kx - wt)) in a Kelvin-Voigt
medium, rho w^2 = k^2 (G - i w eta), so k = w sqrt(rho / (G - i w eta)).  The
paper defines the loss parameter De_v = w eta / mu and the dimensionless
attenuation alpha c_s / w, and gives the low-loss limit
alpha ~ eta w^2 / (2 rho c_s^3) (Sec. 4.3, eq. alpha_scaling).

Discrete law of the leapfrog scheme (Sec. 3.1 update with the backward-
difference velocity): inserting u_j^n = exp(i(k x_j - w t_n)) with
z = exp(-i w dt) into the 1-D form of the update gives

    K^2 = (rho/dt^2) (2 - z - 1/z) / (G + (eta/dt)(1 - 1/z)),
    K^2 = (4/h^2) sin^2(k h / 2),

so k_h = (2/h) arcsin((h/2) K).  Both branches are chosen with Im k >= 0
(waves decaying in +x).
"""
from __future__ import annotations

import numpy as np


def _decaying(k):
    k = np.asarray(k, dtype=complex)
    return np.where(k.imag < 0, -k, k)


def kv_wavenumber(omega, G, rho, eta):
    """Continuous Kelvin-Voigt wavenumber k = w sqrt(rho / (G - i w eta))."""
    omega = np.asarray(omega, dtype=float)
    return _decaying(omega * np.sqrt(rho / (G - 1j * omega * eta)))


def kv_attenuation_speed(omega, G, rho, eta):
    """(alpha [Np/m], phase speed [m/s]) of the continuous law."""
    k = kv_wavenumber(omega, G, rho, eta)
    return k.imag, np.asarray(omega) / k.real


def kv_low_loss_alpha(omega, G, rho, eta):
    """alpha ~ eta w^2 / (2 rho c_s^3), c_s = sqrt(G/rho)."""
    cs = np.sqrt(G / rho)
    return eta * np.asarray(omega) ** 2 / (2.0 * rho * cs ** 3)


def discrete_wavenumber(omega, G, rho, eta, h, dt):
    """Wavenumber of the discrete scheme along one axis (see module doc)."""
    omega = np.asarray(omega, dtype=float)
    z = np.exp(-1j * omega * dt)
    K2 = (rho / dt ** 2) * (2.0 - z - 1.0 / z) / (G + (eta / dt) * (1.0 - 1.0 / z))
    K = np.sqrt(K2.astype(complex))
    k = (2.0 / h) * np.arcsin((h / 2.0) * K)
    return _decaying(k)


def mode_roots(lam, G, rho, eta, dt, s=0.0):
    """Roots of the one-mode recurrence of the update for a Laplacian
    eigenvalue -lam (lam > 0) and damping s = sigma dt / 2:
        (1+s) w' = (1-s) w - a u - b w,  u' = u + w',
    a = dt^2 G lam / rho, b = dt eta lam / rho.  Characteristic polynomial
    (1+s) z^2 + (a + b - 2) z + (1 - s - b) = 0."""
    a = dt * dt * G * lam / rho
    b = dt * eta * lam / rho
    return np.roots([1.0 + s, a + b - 2.0, 1.0 - s - b])
