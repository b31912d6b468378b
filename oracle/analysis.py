"""Host-side trace analyses (test infrastructure).

* Arrival time: peak of |trace| refined by a parabola through the three
  samples around it; speed: least-squares slope of distance against arrival
  time (the estimators of Sec. 4.1).
* Trace-L2: relative L2 norm of a velocity-trace difference against a
  reference, averaged over sensors (Sec. 4.2).
* Relative L2 of two flattened arrays (parity metric).
* Two-sensor harmonic estimate of (alpha, c) from a complex amplitude ratio
  (Sec. 4.3 style measurement).
"""
from __future__ import annotations

import numpy as np


def rel_l2(a, b):
    a = np.asarray(a, dtype=float).ravel()
    b = np.asarray(b, dtype=float).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a - b))


def arrival_time(trace, dt, t0=0.0):
    """Time of max |trace| with parabolic sub-sample refinement."""
    x = np.abs(np.asarray(trace, dtype=float))
    n = int(np.argmax(x))
    frac = 0.0
    if 0 < n < len(x) - 1:
        y0, y1, y2 = x[n - 1], x[n], x[n + 1]
        den = y0 - 2.0 * y1 + y2
        if den != 0:
            frac = 0.5 * (y0 - y2) / den
    return t0 + (n + frac) * dt


def fit_speed(distances, times):
    """Least-squares slope of distance vs time (speed) and intercept."""
    d = np.asarray(distances, dtype=float)
    t = np.asarray(times, dtype=float)
    A = np.vstack([t, np.ones_like(t)]).T
    (slope, icpt), *_ = np.linalg.lstsq(A, d, rcond=None)
    return float(slope), float(icpt)


def centred_velocity(u_trace, dt):
    """v^n = (u^{n+1} - u^{n-1}) / (2 dt) for interior samples, from a
    displacement trace sampled every step (axis 0 is time)."""
    u = np.asarray(u_trace, dtype=float)
    v = np.zeros_like(u)
    v[1:-1] = (u[2:] - u[:-2]) / (2.0 * dt)
    return v


def trace_l2(v, v_ref):
    """Mean over sensors (axis 1) of ||v - v_ref|| / ||v_ref|| along time."""
    v = np.asarray(v, dtype=float)
    r = np.asarray(v_ref, dtype=float)
    num = np.linalg.norm(v - r, axis=0)
    den = np.linalg.norm(r, axis=0)
    return float(np.mean(num / den))


def harmonic_amplitude(trace, dt, omega, n0, n1):
    """Complex amplitude of exp(-i w t) in trace[n0:n1] by least squares on
    cos/sin (window chosen as whole periods by the caller)."""
    t = np.arange(n0, n1) * dt
    y = np.asarray(trace, dtype=float)[n0:n1]
    A = np.vstack([np.cos(omega * t), np.sin(omega * t)]).T
    (a, b), *_ = np.linalg.lstsq(A, y, rcond=None)
    # y = a cos wt + b sin wt = Re[(a + i b) exp(-i w t)]
    return complex(a, b)


def two_sensor_k(a1, a2, dx, k_guess):
    """Complex wavenumber from amplitudes a1, a2 at sensors dx apart
    (a2/a1 = exp(i k dx)); the phase is unwrapped against k_guess."""
    ratio = a2 / a1
    alpha = -np.log(abs(ratio)) / dx
    ph = np.angle(ratio)
    kr_guess = np.real(k_guess)
    m = np.round((kr_guess * dx - ph) / (2 * np.pi))
    kr = (ph + 2 * np.pi * m) / dx
    return complex(kr, alpha)


def xcorr_lag(ref, sig, dt):
    """Delay of `sig` relative to `ref` (positive: sig later): the lag of the
    maximum of their full cross-correlation, with parabolic sub-sample
    refinement."""
    ref = np.asarray(ref, dtype=float)
    sig = np.asarray(sig, dtype=float)
    cc = np.correlate(sig, ref, mode="full")  # entry k <-> lag k - (len(ref) - 1)
    n = int(np.argmax(cc))
    frac = 0.0
    if 0 < n < len(cc) - 1:
        y0, y1, y2 = cc[n - 1], cc[n], cc[n + 1]
        den = y0 - 2.0 * y1 + y2
        if den != 0:
            frac = 0.5 * (y0 - y2) / den
    return (n - (len(ref) - 1) + frac) * dt


def group_speed_xcorr(traces, offsets, dt):
    """Shear-wave group speed from traces [time][sensor] at lateral offsets:
    lags of every trace against the first by cross-correlation, then the
    least-squares slope of offset vs lag (Sec. 4.4 estimator).  Returns
    (speed, lags)."""
    tr = np.asarray(traces, dtype=float)
    lags = np.array([xcorr_lag(tr[:, 0], tr[:, i], dt) for i in range(tr.shape[1])])
    speed, _ = fit_speed(offsets, lags)
    return speed, lags


def successive_orders(hs, traces):
    """Self-convergence of traces sampled at common times on levels of
    spacing hs[0] > hs[1] > ...: d_k = trace_l2(v_k, v_{k+1}) (mean over
    sensors of the relative L2 difference), then for each pair of successive
    differences the order p with d_k / d_{k+1} = (h_k^p - h_{k+1}^p) /
    (h_{k+1}^p - h_{k+2}^p) (the leading error term C h^p), and a global p by
    least squares of log d_k against log(h_k^p - h_{k+1}^p) over all k.
    Returns (d, per-interval orders, global order)."""
    hs = np.asarray(hs, dtype=float)
    d = np.array([trace_l2(traces[k], traces[k + 1]) for k in range(len(traces) - 1)])

    def ratio(p, k):
        return (hs[k] ** p - hs[k + 1] ** p) / (hs[k + 1] ** p - hs[k + 2] ** p)

    def solve(target, k):
        lo, hi = 0.1, 8.0  # the ratio grows with p
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if ratio(mid, k) < target:
                lo = mid
            else:
                hi = mid
        return 0.5 * (lo + hi)

    per = np.array([solve(d[k] / d[k + 1], k) for k in range(len(d) - 1)])

    def misfit(p):
        x = np.log(hs[:-1] ** p - hs[1:] ** p)
        c = np.mean(np.log(d) - x)
        return np.sum((np.log(d) - x - c) ** 2)

    ps = np.linspace(0.5, 4.0, 3501)
    glob = float(ps[np.argmin([misfit(p) for p in ps])])
    return d, per, glob
