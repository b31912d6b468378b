"""Input generators: the torch path of the time-varying push builds the same
force as the numpy path (the benchmark builds each epoch's force on the GPU)."""
import numpy as np
import pytest

from workloads import focal_modulated_force


@pytest.mark.parametrize("epoch", [0, 3, 57])
def test_focal_force_torch_path_matches_numpy(epoch):
    grid = (96, 80, 120, 0.2e-3, 0.2e-3, 0.2e-3)
    a = focal_modulated_force(grid, epoch=epoch, dt=1.75e-6)
    b = focal_modulated_force(grid, epoch=epoch, dt=1.75e-6, device="cpu").numpy()
    assert np.array_equal(a != 0, b != 0)
    assert np.abs(a - b).max() <= 1e-14 * np.abs(a).max()
