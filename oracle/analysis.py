"""Host-side trace analyses (test infrastructure).

* Arrival time: peak of |trace| refined by a parabola through the three
  samples around it; speed: least-squares slope of distance against arrival
  time (the estimators of Sec. 4.1).
* Trace-L2: relative L2 norm of a velocity-trace difference against a
  reference, averaged over sensors (Sec. 4.2).
* Relative L2 of two flattened arrays (parity metric).
* Peak lag by cross-correlation and group speed (Sec. 4.4); successive
  trace differences and the self-convergence order (Sec. 4.2).
* Harmonic phasors of steady traces and the plane-wave fit of attenuation
  and phase speed along a line of sensors (Sec. 4.3).
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


def harmonic_phasors(traces, dt, omega, t_from, t0=None):
    """Complex amplitudes A of steady harmonic traces (the measurement of the
    1-D harmonic Kelvin-Voigt benchmark, Sec. 4.3), u(t) = Re(A e^{-i w t})
    = Re(A) cos(w t) + Im(A) sin(w t): least squares over the samples at
    t >= t_from with a constant and a linear trend as extra columns (the
    offset a net impulse leaves on a line).  traces [step][sensor], sample k at
    t = t0 + k dt (t0 = dt: a trace row holds the state after its step).
    Returns A [sensor]."""
    tr = np.asarray(traces, dtype=float)
    t = (dt if t0 is None else t0) + np.arange(tr.shape[0]) * dt
    sel = t >= t_from
    ts = t[sel]
    M = np.stack([np.cos(omega * ts), np.sin(omega * ts), np.ones_like(ts), ts - ts.mean()], axis=1)
    coef, *_ = np.linalg.lstsq(M, tr[sel], rcond=None)
    return coef[0] + 1j * coef[1]


def plane_wave_fit(x, A, omega):
    """Attenuation and phase speed of a plane wave A(x) = A0 exp(i k x),
    k = k_r + i alpha, from phasors at positions x: alpha = minus the
    least-squares slope of ln|A| against x, k_r the slope of the unwrapped
    phase, c = w / k_r.  Returns (alpha [Np/m], c [m/s])."""
    x = np.asarray(x, dtype=float)
    A = np.asarray(A)
    alpha = -np.polyfit(x, np.log(np.abs(A)), 1)[0]
    kr = np.polyfit(x, np.unwrap(np.angle(A)), 1)[0]
    return float(alpha), float(omega / kr)
