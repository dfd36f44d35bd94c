"""Pins of the oracle's instance generator (random shift o and rotation M).

M must be orthogonal to 1e-12 with |det M| = 1, and -- because the QR factor
with a positive diagonal of R is unique -- equal to LAPACK's QR of the same
Gaussian matrix after the same sign fix.  The Householder routine is also
pinned on matrices whose Q factor is known in closed form.
"""
import numpy as np
import pytest

import oracle as O

SEED = 250517431


@pytest.mark.parametrize("dim", [2, 3, 10, 30, 50, 100])
@pytest.mark.parametrize("func", [0, 3])
def test_rotation_orthogonal_and_unique(func, dim):
    o, M, G = O.instance(func, dim, 0, SEED, return_gaussian=True)
    assert np.abs(M.T @ M - np.eye(dim)).max() <= 1e-12
    assert abs(abs(np.linalg.det(M)) - 1.0) <= 1e-12
    Q, R = np.linalg.qr(G)
    Q = Q * np.sign(np.diag(R))
    assert np.abs(Q - M).max() <= 1e-12
    assert np.all((o >= -80) & (o < 80))


@pytest.mark.slow
def test_rotation_orthogonal_d1000():
    _, M = O.instance(O.ELLIPSOID, 1000, 0, SEED)
    assert np.abs(M.T @ M - np.eye(1000)).max() <= 1e-12


def test_instances_distinct_and_deterministic():
    a = O.instance(2, 10, 0, SEED)
    b = O.instance(2, 10, 0, SEED)
    c = O.instance(2, 10, 1, SEED)
    d = O.instance(3, 10, 0, SEED)
    e = O.instance(2, 10, 0, SEED + 1)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    for other in (c, d, e):
        assert not np.array_equal(a[0], other[0])
        assert not np.array_equal(a[1], other[1])


def test_householder_known_factors():
    # upper triangular with positive diagonal: Q = I
    A = np.triu(np.arange(1.0, 17.0).reshape(4, 4)) + np.eye(4)
    assert np.abs(O.householder_q(A) - np.eye(4)).max() <= 1e-15
    # A = P U with P a permutation, U upper triangular positive: Q = P
    P = np.eye(5)[[3, 0, 4, 1, 2]]
    U = np.triu(np.ones((5, 5))) + 2 * np.eye(5)
    assert np.abs(O.householder_q(P @ U) - P).max() <= 1e-14
    # negative diagonal in R flips the columns: A = -I gives Q = -I
    assert np.abs(O.householder_q(-np.eye(3)) + np.eye(3)).max() == 0.0
    # 2x2 rotation by theta times a positive diagonal
    th = 0.3
    Rt = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    assert np.abs(O.householder_q(Rt @ np.diag([2.0, 5.0])) - Rt).max() <= 1e-15
