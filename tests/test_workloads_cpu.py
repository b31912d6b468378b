"""Input generators (CPU): the force-pattern dicts and their numpy
evaluation against hand values of the closed form."""
import math

import numpy as np
import pytest

from workloads import (coords, focal_focus_z, focal_modulated_force, focal_modulated_params, force_from_params,
                       gaussian_push, gaussian_push_params)


def test_gaussian_push_hand_values():
    """Peak F0 on the focus node; exp(-1/2) one lateral sigma away (on a node)
    and exp(-1/2) one axial sigma away; only the axis component is set."""
    h = 0.25e-3
    grid = (33, 29, 41, h, h, h)
    F = gaussian_push(grid, 4 * h, 8 * h, 1e4, centre=(2 * h, -3 * h, 5 * h), axis=1)
    i0, j0, k0 = 33 // 2 + 2, 29 // 2 - 3, 41 // 2 + 5
    assert F[1, k0, j0, i0] == pytest.approx(1e4, rel=1e-15)
    assert F[1, k0, j0, i0 + 4] == pytest.approx(1e4 * math.exp(-0.5), rel=1e-14)
    assert F[1, k0 - 4, j0, i0] == pytest.approx(1e4 * math.exp(-0.5), rel=1e-14)
    assert F[1, k0, j0 + 8, i0] == pytest.approx(1e4 * math.exp(-0.5), rel=1e-14)
    assert not F[0].any() and not F[2].any()


@pytest.mark.parametrize("epoch", [0, 3, 57])
def test_focal_modulated_force_hand_values_and_box(epoch):
    """The modulated push at a few nodes equals the closed form evaluated with
    math.exp / math.cos; zero outside the 1e-16 box; the focus follows
    focal_focus_z."""
    grid = (48, 40, 96, 0.2e-3, 0.2e-3, 0.2e-3)
    p = focal_modulated_params(grid, epoch=epoch)
    F = focal_modulated_force(grid, epoch=epoch)
    assert np.array_equal(F, force_from_params(grid, p))
    zf = focal_focus_z(grid, epoch, 1.75e-6)
    assert p["centre"] == (0.0, 0.0, zf)
    x, y, z = coords(48, 0.2e-3), coords(40, 0.2e-3), coords(96, 0.2e-3)
    rng = np.random.default_rng(epoch)
    kz0 = int(np.argmin(np.abs(z - zf)))
    for _ in range(20):
        i, j, k = rng.integers(20, 28), rng.integers(16, 24), rng.integers(max(kz0 - 10, 0), min(kz0 + 10, 96))
        g = math.exp(-(x[i] ** 2 + y[j] ** 2) / (2 * 1e-3 ** 2) - (z[k] - zf) ** 2 / (2 * 4e-3 ** 2))
        M = 1 + 0.5 / math.sqrt(8) * sum(math.cos(p["k"][m] @ np.array([x[i], y[j], z[k]]) + p["phase"][m])
                                         for m in range(8))
        assert F[2, k, j, i] == pytest.approx(1e4 * g * M, rel=1e-12, abs=1e-12)
    cut = math.sqrt(2 * math.log(1e16))
    outside = (np.abs(x)[None, None, :] > cut * 1e-3) | (np.abs(y)[None, :, None] > cut * 1e-3) \
        | (np.abs(z - zf)[:, None, None] > cut * 4e-3)
    assert not F[2][outside].any() and not F[0].any() and not F[1].any()


def test_push_params_round_trip():
    p = gaussian_push_params(1e-3, 4e-3, 1e4)
    assert p["box_lateral"] < 0 and p["box_axial"] < 0 and len(p["phase"]) == 0 and p["axis"] == 2
