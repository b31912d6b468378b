"""Pins of the host-side estimators used by the validation workloads: the
cross-correlation lag and the group-speed fit recover known delays of
sampled pulses (closed form: a shifted copy)."""
import numpy as np

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
