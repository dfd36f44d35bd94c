"""Pins the gradients used by the float32 tolerance against central finite
differences of the oracle's error as a function of z."""
import numpy as np
import pytest

import oracle as O
from tests.tolerance import grad_z


@pytest.mark.parametrize("func", range(6))
def test_gradient_matches_oracle_differences(func):
    rng = np.random.default_rng(42 + func)
    for D in (2, 5, 12):
        for scale in (0.3, 3.0, 40.0):
            z = rng.normal(size=D) * scale
            g = grad_z(func, z[:, None])[:, 0]
            for j in range(D):
                h = 1e-6 * max(1.0, abs(z[j]))
                zp, zm = z.copy(), z.copy()
                zp[j] += h
                zm[j] -= h
                fd = (O.error_z(func, zp) - O.error_z(func, zm)) / (2 * h)
                assert fd == pytest.approx(g[j], rel=2e-4, abs=1e-5 * (1 + abs(O.error_z(func, z)))), (func, D, scale, j)
