"""Pins Rosenbrock's gradient, used by its float32 tolerance term, against
central finite differences of the oracle's error as a function of z."""
import numpy as np
import pytest

import oracle as O
from tests.tolerance import ROSENBROCK, rosenbrock_grad_z, tolerance


def test_rosenbrock_gradient_matches_oracle_differences():
    rng = np.random.default_rng(42)
    for D in (2, 5, 12):
        for scale in (0.3, 3.0, 40.0):
            z = rng.normal(size=D) * scale
            g = rosenbrock_grad_z(z[:, None])[:, 0]
            for j in range(D):
                h = 1e-6 * max(1.0, abs(z[j]))
                zp, zm = z.copy(), z.copy()
                zp[j] += h
                zm[j] -= h
                fd = (O.error_z(ROSENBROCK, zp) - O.error_z(ROSENBROCK, zm)) / (2 * h)
                assert fd == pytest.approx(g[j], rel=2e-4, abs=1e-5 * (1 + abs(O.error_z(ROSENBROCK, z)))), (D, j)


def test_bound_is_the_stated_one_except_rosenbrock():
    D = 4
    o = np.zeros(D)
    M = np.eye(D)
    X = np.full((D, 3), 30.0)
    e = np.array([0.0, 0.05, 2e3])
    for func in (0, 2, 3, 4, 5):
        assert np.array_equal(tolerance(func, o, M, X, e), [1e-6, 1e-6, 2e-2])
    t = tolerance(ROSENBROCK, o, M, X, e)
    assert np.all(t > [1e-6, 1e-6, 2e-2])
