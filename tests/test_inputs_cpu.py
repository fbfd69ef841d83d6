"""The two implementations of the synthetic gauge recipe agree: the NumPy
one (per-matrix eigendecompositions) and the whole-array torch one used for
large lattices on the GPU (Taylor exponential, Newton polar projection)."""
import numpy as np
import pytest

import inputs


@pytest.mark.parametrize("dims,eps,sweeps", [((4, 4, 4, 4), 0.3, 0), ((6, 4, 4, 8), 0.5, 2), ((8, 4, 4, 4), 0.5, 5)])
def test_torch_recipe_matches_numpy(dims, eps, sweeps):
    a = inputs.gauge_field(dims, eps, 1001, ape_sweeps=sweeps)
    b = inputs.gauge_field_torch(dims, eps, 1001, ape_sweeps=sweeps).numpy()
    assert a.shape == b.shape
    assert np.abs(a - b).max() < 1e-13
    u = b.reshape(-1, 3, 3)
    assert np.abs(u @ u.conj().transpose(0, 2, 1) - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(u) - 1).max() < 1e-14


def test_chunked_numpy_is_bitwise_serial():
    saved = inputs._THREADS
    try:
        inputs._THREADS = 1
        a = inputs.gauge_field((8, 8, 8, 16), 0.5, 1003, ape_sweeps=1)
        inputs._THREADS = 4
        b = inputs.gauge_field((8, 8, 8, 16), 0.5, 1003, ape_sweeps=1)
    finally:
        inputs._THREADS = saved
    assert np.array_equal(a, b)
