"""The 1-D harmonic Kelvin-Voigt benchmark (Sec. 4.3) on the oracle.

The estimators are pinned on exact synthetic phasors; the oracle's own line
runs are pinned against the closed-form dispersion relation of the discrete
scheme (the plane-wave analysis of the update, independent of the stepping
code) and against the continuous Kelvin-Voigt law within the accuracy the
paper reports for its own 16-point sweep (about 3 % in alpha, < 1 % in c)."""
import numpy as np
import pytest

import oracle
from oracle import dispersion
from oracle.analysis import harmonic_phasors, plane_wave_fit
from workloads import (KV_LINE_ETAS, KV_LINE_F0_KNOTS, kv_line_case, kv_line_frequency, kv_line_grid)

G, RHO = 4e3, 1000.0
T_RUN = 16e-3


def test_harmonic_phasors_recover_a_sinusoid_with_offset_and_trend():
    dt, w = 1e-6, 2 * np.pi * 750.0
    t = dt + np.arange(20000) * dt
    A = np.array([0.3 - 1.1j, -2.0 + 0.5j])
    tr = np.stack([(a * np.exp(-1j * w * t)).real + 0.7 * k - 30.0 * k * t for k, a in enumerate(A)], axis=1)
    got = harmonic_phasors(tr, dt, w, t_from=5e-3)
    assert np.allclose(got, A, rtol=1e-11, atol=1e-12)


def test_plane_wave_fit_recovers_alpha_and_speed():
    w = 2 * np.pi * 800.0
    k = 2600.0 + 450.0j
    x = np.linspace(0.5e-3, 6e-3, 7)
    A = (0.8 - 0.2j) * np.exp(1j * k * x)
    alpha, c = plane_wave_fit(x, A, w)
    assert alpha == pytest.approx(450.0, rel=1e-12)
    assert c == pytest.approx(w / 2600.0, rel=1e-12)


def test_frequency_schedule_reproduces_the_theoretical_table_columns():
    """At the table's viscosities the scheduled drive frequencies give the
    table's alpha_th and c_th by the continuous law (c_s = 2 m/s) to the
    printed digits (alpha to 0.1 Np/m: the knots carry one decimal)."""
    tab = np.loadtxt(__file__.replace("test_oracle_kv_line.py", "golden/kv_table.txt"))
    assert [e for e, _ in KV_LINE_F0_KNOTS] == list(tab[:, 0])
    for eta, a_th, c_th in tab:
        a, c = dispersion.kv_attenuation_speed(2 * np.pi * kv_line_frequency(eta), G, RHO, eta)
        assert abs(a - a_th) <= 0.1 and abs(c - c_th) <= 6e-4, (eta, a, c)
    assert kv_line_frequency(0.0) == 800.1 and kv_line_frequency(0.2) == pytest.approx(795.0)


def line_dt():
    grid = kv_line_grid()
    return grid, 0.3 * min(oracle.stable_dt(grid, G, RHO, e) for e in KV_LINE_ETAS)


def measure(grid, eta, dt, nsteps):
    w = 2 * np.pi * kv_line_frequency(eta)
    a_th, c_th = dispersion.kv_attenuation_speed(w, G, RHO, eta)
    case = kv_line_case(grid, eta, dt, nsteps, float(a_th), float(c_th))
    _, _, tr = oracle.run(grid, G, RHO, eta, dt, nsteps, FS=case["FS"], env=case["env"], probes=case["probes"],
                          comp=2)
    A = harmonic_phasors(tr[:, :, 0], dt, case["omega"], case["t_from"])
    alpha, c = plane_wave_fit(case["x"], A, case["omega"])
    kh = dispersion.discrete_wavenumber(case["omega"], G, RHO, eta, grid[3], dt)
    return alpha, c, float(kh.imag), float(case["omega"] / kh.real), float(a_th), float(c_th)


def test_transverse_terms_are_below_rounding():
    """The line's y and z spacings make the transverse stencil terms 1e-20 of
    the x terms: the stable step is the 1-D one to rounding."""
    grid = kv_line_grid()
    one_d = 2.0 / np.sqrt(4.0 * G / RHO / grid[3] ** 2)  # a = 4 dt^2 (G/rho) / h^2 <= 4, eta = 0
    assert oracle.stable_dt(grid, G, RHO, 0.0) == pytest.approx(one_d, rel=1e-15)


@pytest.mark.parametrize("eta", [0.0, 0.1, 0.5, 1.5])
def test_line_matches_the_discrete_dispersion_relation(eta):
    """Steady state on the line is the discrete plane wave: the measured
    alpha and c equal the scheme's closed form (1e-7; eta = 0: |alpha| below
    1e-3 Np/m)."""
    grid, dt = line_dt()
    alpha, c, a_h, c_h, _, _ = measure(grid, eta, dt, int(round(T_RUN / dt)))
    assert c == pytest.approx(c_h, rel=1e-7)
    if eta == 0.0:
        assert abs(alpha) < 1e-3
    else:
        assert alpha == pytest.approx(a_h, rel=1e-7)


def test_sweep_tracks_kelvin_voigt():
    """All 16 viscosities: alpha within 3 % of the continuous law (eta >= 0.1)
    and c within 1 %, both increasing with eta."""
    grid, dt = line_dt()
    n = int(round(T_RUN / dt))
    res = np.array([measure(grid, eta, dt, n) for eta in KV_LINE_ETAS])
    alpha, c, a_th, c_th = res[:, 0], res[:, 1], res[:, 4], res[:, 5]
    assert np.all(np.abs(alpha[1:] / a_th[1:] - 1) < 0.03), alpha / np.maximum(a_th, 1e-30)
    assert np.all(np.abs(c / c_th - 1) < 0.01), c / c_th
    assert np.all(np.diff(alpha) > 0) and np.all(np.diff(c) > 0)
