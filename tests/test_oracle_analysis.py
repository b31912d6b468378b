"""Pins of the host-side estimators used by the validation workloads: the
cross-correlation lag and the group-speed fit recover known delays of
sampled pulses (closed form: a shifted copy); the self-convergence order is
recovered from synthetic errors C h^p; the centred velocity is exact on
quadratics; the trace-L2 difference is the mean relative difference."""
import numpy as np
import pytest

from oracle.analysis import arrival_time, fit_speed, group_speed_xcorr, xcorr_lag


def pulse(t, t0, w):
    """A velocity-like (odd) pulse: derivative of a Gaussian centred at t0."""
    s = (t - t0) / w
    return -s * np.exp(-s * s / 2)


def test_xcorr_lag_recovers_known_shifts():
    dt = 1e-5
    t = np.arange(600) * dt
    ref = pulse(t, 1.0e-3, 1.2e-4)
    for shift in (0.0, 3.3e-5, 2.1e-4, 1.234e-3):
        sig = pulse(t, 1.0e-3 + shift, 1.2e-4)
        assert abs(xcorr_lag(ref, sig, dt) - shift) < 0.02 * dt, shift
        assert abs(xcorr_lag(sig, ref, dt) + shift) < 0.02 * dt, shift


def test_group_speed_from_travelling_pulses():
    dt = 2e-5
    t = np.arange(900) * dt
    c, t0 = 2.24, 4e-4
    offsets = np.arange(4e-3, 14.01e-3, 0.5e-3)
    traces = np.stack([0.1 / np.sqrt(r) * pulse(t, t0 + r / c, 3e-4) for r in offsets], axis=1)
    speed, lags = group_speed_xcorr(traces, offsets, dt)
    assert lags[0] == 0.0
    assert abs(speed - c) < 1e-3 * c
    # peak arrivals of a one-lobed pulse give the same slope (the intercept
    # absorbs t0)
    even = np.stack([np.exp(-((t - t0 - r / c) / 3e-4) ** 2 / 2) / np.sqrt(r) for r in offsets], axis=1)
    times = [arrival_time(even[:, i], dt) for i in range(len(offsets))]
    assert abs(fit_speed(offsets, times)[0] - c) < 2e-3 * c


def test_stored_qiba_speeds_are_within_two_percent():
    """The oracle's QIBA-like phantoms (Sec. 4.4; stored by
    tests/golden/make_qiba.py): each group speed is within 2 % of sqrt(G / rho)
    (the paper reports about 1 % for its runs) and the lags grow with the
    offset."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "qiba_240x200x200.txt")
    found = 0
    for line in open(path):
        f = line.split()
        if line.startswith("# phantom "):
            kv = dict(zip(f[2::2], f[3::2]))
            cs = np.sqrt(float(kv["G"]) / 1000.0)
            assert abs(float(kv["speed"]) - cs) < 0.02 * cs
            found += 1
        elif line.startswith("# lags "):
            assert np.all(np.diff([float(v) for v in f[2:]]) > 0)
    assert found == 4


def test_successive_orders_recover_known_orders():
    """Traces v_h = v + C h^p phi(t) (plus a higher-order term) on levels of
    uneven refinement give back p per interval and globally (C small, so the
    finer level's norm in the relative difference stays put)."""
    from oracle.analysis import successive_orders
    t = np.linspace(0, 1, 200)
    v = np.stack([np.sin(5 * t), np.cos(3 * t)], axis=1)
    phi = np.stack([np.cos(7 * t), np.sin(2 * t)], axis=1)
    hs = [0.6, 0.4, 0.3, 0.24, 0.2]
    for p in (1.0, 2.0, 3.0):
        traces = [v + 1e-4 * h ** p * phi for h in hs]
        d, per, glob = successive_orders(hs, traces)
        assert np.allclose(per, p, atol=1e-3) and abs(glob - p) <= 2e-3, (p, per, glob)
    traces = [v + 1e-4 * h ** 2 * phi + 2e-5 * h ** 4 * phi for h in hs]
    _, per, glob = successive_orders(hs, traces)
    assert np.all(np.abs(per - 2) < 0.15) and abs(glob - 2) < 0.1


def test_centred_velocity_is_exact_on_quadratics():
    """(u(t + dt) - u(t - dt)) / (2 dt) is the exact derivative of a quadratic;
    the end samples are left at 0."""
    from oracle.analysis import centred_velocity
    dt = 2.5e-6
    t = np.arange(40) * dt
    u = np.stack([3.0 * t ** 2 - 7.0 * t + 1.0, -2.0 * t ** 2], axis=1)
    v = centred_velocity(u, dt)
    exact = np.stack([6.0 * t - 7.0, -4.0 * t], axis=1)
    assert np.allclose(v[1:-1], exact[1:-1], rtol=1e-9, atol=1e-12)
    assert not v[0].any() and not v[-1].any()


def test_trace_l2_is_the_mean_relative_difference_over_sensors():
    """Sensor k scaled by (1 + e_k): the per-sensor relative L2 difference is
    |e_k| whatever the trace's size, and trace_l2 is their mean."""
    from oracle.analysis import trace_l2
    rng = np.random.default_rng(5)
    ref = rng.standard_normal((50, 3)) * np.array([1e-9, 1.0, 1e4])
    e = np.array([0.01, -0.03, 0.002])
    assert trace_l2(ref * (1 + e), ref) == pytest.approx(np.mean(np.abs(e)), rel=1e-12)
