"""Grid self-convergence of the oracle (Sec. 4.2): the curl source on three
levels of an 18 mm cube (h = 0.6, 0.3, 0.2 mm, dt proportional to h so every
level samples the same times), centred velocity traces at sensors that sit
on nodes of every level; the successive differences shrink at order 2."""
import numpy as np

import oracle
from oracle.analysis import centred_velocity, successive_orders
from workloads import convergence_level


def level_traces(n, **kw):
    w = convergence_level(n, **kw)
    u0, w0 = oracle.curl_state(w["grid"], w["A"], w["dt"])
    _, _, tr = oracle.run(w["grid"], w["G"], w["rho"], w["eta"], w["dt"], w["nsteps"], u=u0, w=w0,
                          probes=w["probes"], comp=2)
    v = centred_velocity(tr[:, :, 0], w["dt"])
    sub = w["sub"]
    # trace index k holds t = (k + 1) dt; samples t = m Ts for m = 2 .. nsamp
    return w["grid"][3], v[2 * sub - 1::sub][:w["nsamp"] - 1]


def test_velocity_traces_converge_at_second_order():
    kw = dict(width=18e-3, sigma=2e-3, window=6e-3, offsets_mm=(2.4, 3.6, 4.8))
    hs, traces = zip(*(level_traces(n, **kw) for n in (31, 61, 91)))
    assert all(t.shape == traces[0].shape for t in traces)
    d, per, _ = successive_orders(hs, traces)
    assert d[0] > d[1] > 0
    assert 1.7 <= per[0] <= 2.4, (d, per)
