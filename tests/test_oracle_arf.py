"""Pins of the acoustic radiation force oracle (Sec. 3.4, Eqs. isppa_norm and
arf_poynting; Sec. 6.3, Table tab:arf_scaling) against the paper's printed
table and closed forms of sampled sinusoids."""
import math
import os

import numpy as np

from oracle import arf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RHO, C_SOUND = 1000.0, 1540.0


def load_table():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "arf_table.txt")) if l.strip() and not l.startswith("#")]
    return np.array([[float(x) for x in r] for r in rows])


def tone_burst(amp, per, periods, total, phase=0.0):
    """amp cos(2 pi t / per + phase) for t < per * periods, zero after (total samples)."""
    t = np.arange(total)
    s = amp * np.cos(2 * np.pi * t / per + phase)
    s[per * periods:] = 0.0
    return s


def test_absorption_column_of_the_table():
    tab = load_table()
    for f0, alpha, _ in tab:
        assert abs(arf.alpha_np_per_m(0.5, f0) - alpha) <= 0.05 + 1e-12, f0


def test_force_column_of_the_table_both_forms():
    """A plane tone burst of intensity 1000 W/cm^2 (P0^2 = 2 rho c I, 10 periods of
    20 samples, padded with zeros) gives the printed b through either form."""
    tab = load_table()
    I = 1000.0 * 1e4
    P0 = math.sqrt(2 * RHO * C_SOUND * I)
    per, periods, total = 20, 10, 373
    p = tone_burst(P0, per, periods, total, phase=0.3).reshape(total, 1, 1, 1)
    v = np.zeros((total, 3, 1, 1, 1))
    v[:, 2] = p / (RHO * C_SOUND)  # plane-wave impedance relation, beam along z
    S_pp = arf.time_sums_pp(p)
    S_pv = arf.time_sums_pv(p, v)
    for _, alpha, b in tab:
        Fp = arf.plane_wave_force(S_pp, alpha, C_SOUND, RHO, per * periods, (0, 0, 1))
        Fv = arf.poynting_force(S_pv, alpha, C_SOUND, per * periods)
        for F in (Fp, Fv):
            assert abs(F[2].item() - b) <= 50.0, (alpha, F[2].item(), b)
            assert F[0].item() == 0.0 and F[1].item() == 0.0


def test_sums_of_sampled_sinusoids():
    """Over whole periods, sum cos^2 = n/2 and sum cos(a) cos(a + d) = n cos(d) / 2."""
    per, periods = 16, 7
    n = per * periods
    A, B, d = 3.0, 0.5, 0.9
    p = tone_burst(A, per, periods, n + 5).reshape(-1, 1, 1, 1)
    v = np.zeros((n + 5, 3, 1, 1, 1))
    v[:, 0, 0, 0, 0] = tone_burst(B, per, periods, n + 5, phase=d)
    v[:, 1, 0, 0, 0] = -2.0 * v[:, 0, 0, 0, 0]
    S_pp = arf.time_sums_pp(p)
    S_pv = arf.time_sums_pv(p, v)
    assert np.isclose(S_pp.item(), A * A * n / 2, rtol=1e-13)
    assert np.isclose(S_pv[0].item(), A * B * n * math.cos(d) / 2, rtol=1e-12)
    assert np.isclose(S_pv[1].item(), -2 * A * B * n * math.cos(d) / 2, rtol=1e-12)
    assert S_pv[2].item() == 0.0


def test_pulse_normalisation_masking_and_direction():
    rng = np.random.default_rng(5)
    shape = (3, 4, 5)
    p = rng.standard_normal((30,) + shape)
    v = rng.standard_normal((30, 3) + shape)
    pad = np.concatenate([p, np.zeros((11,) + shape)])
    vpad = np.concatenate([v, np.zeros((11, 3) + shape)])
    # trailing silence leaves the sums unchanged; the force scales as 1 / N_pulse
    assert np.array_equal(arf.time_sums_pp(pad), arf.time_sums_pp(p))
    assert np.array_equal(arf.time_sums_pv(pad, vpad), arf.time_sums_pv(p, v))
    S = arf.time_sums_pv(p, v)
    F30 = arf.poynting_force(S, 5.8, C_SOUND, 30)
    F60 = arf.poynting_force(S, 5.8, C_SOUND, 60)
    assert np.allclose(F60 * 2, F30, rtol=1e-15, atol=0)
    # per-cell coefficient 2 alpha / c
    alpha = rng.uniform(1, 40, shape)
    c = rng.uniform(1400, 3000, shape)
    F = arf.poynting_force(S, alpha, c, 30)
    assert np.allclose(F, 2 * alpha / c * S / 30, rtol=1e-14)
    # masked cells are zero, the rest untouched
    mask = rng.uniform(size=shape) < 0.5
    Fm = arf.poynting_force(S, alpha, c, 30, mask=mask)
    assert not Fm[:, ~mask].any() and np.array_equal(Fm[:, mask], F[:, mask])
    # plane-wave form: the direction is normalised and carries the whole force
    Spp = arf.time_sums_pp(p)
    F1 = arf.plane_wave_force(Spp, alpha, c, RHO, 30, (0, 3.0, 4.0))
    assert not F1[0].any()
    assert np.allclose(F1[1] / 0.6, F1[2] / 0.8, rtol=1e-14)
    assert np.allclose(np.sqrt(F1[1] ** 2 + F1[2] ** 2), 2 * alpha / c * Spp / (RHO * c * 30), rtol=1e-14)


def test_travelling_plane_wave_forms_agree():
    """An attenuated travelling plane wave p = P0 e^{-alpha z} cos(w t - k z) with
    v_z = p / (rho c): the Poynting and plane-wave forms give the same force,
    b0 = (2 alpha / c) P0^2 e^{-2 alpha z} / (2 rho c), along z."""
    nz, per, periods = 9, 24, 5
    n = per * periods
    alpha, P0, h, lam = 17.3, 1.2e6, 2e-4, 1.54e-3
    z = np.arange(nz) * h
    t = np.arange(n)
    p = (P0 * np.exp(-alpha * z)[None, :] * np.cos(2 * np.pi * t[:, None] / per - 2 * np.pi * z[None, :] / lam))
    p = p.reshape(n, nz, 1, 1)
    v = np.zeros((n, 3, nz, 1, 1))
    v[:, 2] = p / (RHO * C_SOUND)
    Fp = arf.plane_wave_force(arf.time_sums_pp(p), alpha, C_SOUND, RHO, n, (0, 0, 1))
    Fv = arf.poynting_force(arf.time_sums_pv(p, v), alpha, C_SOUND, n)
    b0 = 2 * alpha / C_SOUND * P0 ** 2 * np.exp(-2 * alpha * z) / (2 * RHO * C_SOUND)
    assert np.allclose(Fp[2, :, 0, 0], b0, rtol=1e-12)
    assert np.allclose(Fv[2, :, 0, 0], b0, rtol=1e-12)
    assert not Fv[:2].any()


def test_strain_peaks_of_a_sampled_plane_wave():
    """p = P0 cos(2 pi n / M - k x) with k h = 2 pi q / M and M divisible by 4:
    every cell's phase hits a multiple of pi/2, so the peak strain is P0 / K
    and the peak gradient the discrete closed form (P0 / K) sin(k h) / h."""
    M, q, P0, K = 16, 3, 2.0e5, 2.37e9
    grid = (20, 5, 6, 2e-4, 2e-4, 2e-4)
    h = grid[3]
    k = 2 * np.pi * q / (M * h)
    x = np.arange(grid[0]) * h
    n = np.arange(2 * M)
    p = P0 * np.cos(2 * np.pi * n[:, None] / M - k * x[None, :])
    p = np.broadcast_to(p[:, None, None, :], (2 * M, grid[2], grid[1], grid[0]))
    pe, pg = arf.strain_peaks(grid, p, K)
    assert np.allclose(pe, P0 / K, rtol=1e-13)
    assert np.allclose(pg[1:-1, 1:-1, 1:-1], P0 / K * np.sin(k * h) / h, rtol=1e-12)
    assert not pg[0].any() and not pg[:, :, -1].any()


def test_strain_gradient_is_of_p_over_k():
    """Uniform pressure over a medium whose 1/K varies linearly along y: the
    gradient is p d(1/K)/dy (exact for a linear profile), not grad(p) / K = 0;
    and silence or repeated samples do not change the peaks (no pulse
    normalisation)."""
    grid = (6, 11, 7, 2e-4, 3e-4, 2e-4)
    y = np.arange(grid[1]) * grid[4]
    invK = 1.0 / 2.0e9 + 3.0e-8 * y
    K = np.broadcast_to(1.0 / invK[None, :, None], (grid[2], grid[1], grid[0]))
    P0 = 1.5e5
    p = np.stack([np.full(K.shape, P0), np.full(K.shape, -0.5 * P0), np.zeros(K.shape)])
    pe, pg = arf.strain_peaks(grid, p, K)
    assert np.allclose(pe, P0 / K, rtol=1e-14)
    assert np.allclose(pg[1:-1, 1:-1, 1:-1], P0 * 3.0e-8, rtol=1e-6)
    pe2, pg2 = arf.strain_peaks(grid, np.concatenate([p, p[::-1], np.zeros((5,) + K.shape)]), K)
    assert np.array_equal(pe2, pe) and np.array_equal(pg2, pg)
