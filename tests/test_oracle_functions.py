"""Pins of the oracle's six objective functions (e = f - f*, f* = 100).

The oracle evaluates cancellation-free rewrites of the textbook forms.  These
tests pin them against things the rewrites do not share:

* the textbook definitions themselves, evaluated in 50-digit arithmetic;
* closed-form values at M = I, o = 0 (the unrotated textbook function);
* f(o) = f* exactly, for generated instances;
* near-optimum Taylor expansions;
* brute-force grids at D = 2: nothing in the box is below f*, and the grid
  minimum sits in the cell around o.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle as O

SEED = 250517431
mp.mp.dps = 50


# --- textbook definitions in high precision (independent of the oracle's forms) ---
def mp_textbook(func, z):
    z = [mp.mpf(float(v)) for v in z]
    D = len(z)
    if func == O.ELLIPSOID:
        return mp.fsum(mp.power(10, mp.mpf(6) * i / (D - 1)) * z[i] ** 2 for i in range(D))
    if func == O.ROSENBROCK:
        w = [v + 1 for v in z]
        return mp.fsum(100 * (w[i] ** 2 - w[i + 1]) ** 2 + (w[i] - 1) ** 2 for i in range(D - 1))
    if func == O.RASTRIGIN:
        return mp.fsum(v ** 2 - 10 * mp.cos(2 * mp.pi * v) + 10 for v in z)
    if func == O.SCHWEFEL:
        s = mp.mpf(O.schwefel_constants()[0])
        c = s * mp.sin(mp.sqrt(s))
        lam = mp.mpf("0.01")

        def g(u):
            if u > 500:
                return c - 500 * mp.sin(mp.sqrt(500)) + lam * (u - 500) ** 2
            if u < -500:
                return c + 500 * mp.sin(mp.sqrt(500)) + lam * (u + 500) ** 2
            return c - u * mp.sin(mp.sqrt(abs(u)))
        return mp.fsum(g(v + s) for v in z)
    if func == O.GRIEWANK:
        prod = mp.mpf(1)
        for i, v in enumerate(z):
            prod *= mp.cos(v / mp.sqrt(i + 1))
        return 1 + mp.fsum(v ** 2 for v in z) / 4000 - prod
    if func == O.ACKLEY:
        a = -20 * mp.exp(-mp.mpf("0.2") * mp.sqrt(mp.fsum(v ** 2 for v in z) / D))
        b = -mp.exp(mp.fsum(mp.cos(2 * mp.pi * v) for v in z) / D)
        return a + b + 20 + mp.e
    raise ValueError(func)


@pytest.mark.parametrize("func", range(6))
@pytest.mark.parametrize("scale", [1e-7, 1e-4, 1e-2, 0.7, 30.0, 150.0])
def test_identity_forms_match_textbook(func, scale):
    rng = np.random.default_rng(1000 + func)
    for D in (2, 5, 10):
        for _ in range(3):
            z = rng.normal(size=D) * scale
            want = mp_textbook(func, z)
            got = O.error_z(func, z)
            # relative to the value, or absolute at the level the FP64 forms can reach
            tol = 1e-12 * abs(float(want)) + 1e-13 * (1 + float(np.sum(np.abs(z))))
            if func == O.SCHWEFEL:
                tol = 1e-12 * abs(float(want)) + 1e-13 * D * (1 + scale ** 2)
            assert abs(got - float(want)) <= tol, (func, D, scale, got, float(want))


@pytest.mark.parametrize("func", range(6))
@pytest.mark.parametrize("dim", [2, 3, 10, 30, 50, 100])
def test_value_at_optimum_is_exact(func, dim):
    for inst in (0, 7):
        o, M = O.instance(func, dim, inst, SEED)
        assert O.error(func, o, M, o) == 0.0


def _identity(dim):
    return np.zeros(dim), np.eye(dim)


@pytest.mark.parametrize("dim", [2, 7, 10, 30])
def test_closed_forms_unrotated(dim):
    o, M = _identity(dim)
    D = dim
    for k in range(D):
        e_k = np.zeros(D); e_k[k] = 1.0
        assert O.error(O.ELLIPSOID, o, M, e_k) == pytest.approx(10 ** (6 * k / (D - 1)), rel=1e-14)
    assert O.error(O.RASTRIGIN, o, M, np.full(D, 0.5)) == pytest.approx(20.25 * D, rel=1e-14)
    assert O.error(O.ROSENBROCK, o, M, np.full(D, -1.0)) == pytest.approx(D - 1, rel=1e-14)
    assert O.error(O.ACKLEY, o, M, np.ones(D)) == pytest.approx(20 * (1 - math.exp(-0.2)), rel=1e-13)
    zg = math.pi * np.sqrt(np.arange(1, D + 1))
    want = 1 + math.pi ** 2 * D * (D + 1) / 8000 - (-1) ** D
    assert O.error(O.GRIEWANK, o, M, zg) == pytest.approx(want, rel=1e-13)
    # Schwefel: u = z + s = 0 gives c per term; u = +-500 the boundary values
    s, c, lam = O.schwefel_constants()
    assert O.error(O.SCHWEFEL, o, M, np.full(D, -s)) == pytest.approx(c * D, rel=1e-13)
    g500 = c - 500 * math.sin(math.sqrt(500))
    assert O.error(O.SCHWEFEL, o, M, np.full(D, 500 - s)) == pytest.approx(g500 * D, rel=1e-12)
    assert O.error(O.SCHWEFEL, o, M, np.full(D, 510 - s)) == pytest.approx((g500 + lam * 100) * D, rel=1e-12)


def test_schwefel_constants():
    s, c, lam = O.schwefel_constants()
    # s is a stationary point of u sin(sqrt u): sin(sqrt s) + sqrt(s)/2 cos(sqrt s) = 0
    assert abs(math.sin(math.sqrt(s)) + math.sqrt(s) / 2 * math.cos(math.sqrt(s))) < 1e-13
    assert c == pytest.approx(418.98288727243370, rel=1e-15)
    assert 418.9829 - c == pytest.approx(1.273e-5, rel=1e-3)
    assert lam > 0


def test_near_optimum_taylor():
    rng = np.random.default_rng(5)
    D = 10
    z = rng.normal(size=D) * 1e-6
    n2 = float(z @ z)
    assert O.error_z(O.RASTRIGIN, z) == pytest.approx((1 + 20 * math.pi ** 2) * n2, rel=1e-9)
    i = np.arange(1, D + 1)
    assert O.error_z(O.GRIEWANK, z) == pytest.approx(float(np.sum(z ** 2 * (1 / 4000 + 1 / (2 * i)))), rel=1e-9)
    w = 10.0 ** (6 * np.arange(D) / (D - 1))
    assert O.error_z(O.ELLIPSOID, z) == pytest.approx(float(np.sum(w * z * z)), rel=1e-15)
    # Schwefel: second derivative of g at s over 2
    s, c, _ = O.schwefel_constants()
    a = math.sqrt(s)
    g2 = -3 * math.cos(a) / (4 * a) + math.sin(a) / 4   # d2/du2 of -u sin(sqrt u) at u = s
    assert O.error_z(O.SCHWEFEL, z) == pytest.approx(0.5 * g2 * n2, rel=1e-6)
    assert 0.5 * g2 == pytest.approx(0.1262, rel=1e-3)


@pytest.mark.parametrize("func", range(6))
def test_rotation_and_shift_are_applied(func):
    o, M = O.instance(func, 10, 2, SEED)
    x = np.random.default_rng(func).uniform(-100, 100, size=10)
    assert O.error(func, o, M, x) == O.error_z(func, M @ (x - o)) or \
        abs(O.error(func, o, M, x) - O.error_z(func, M @ (x - o))) <= 1e-12 * abs(O.error(func, o, M, x))


@pytest.mark.parametrize("func", range(6))
def test_grid_d2_nothing_below_optimum(func):
    o, M = O.instance(func, 2, 0, SEED)
    h = 0.25
    g = np.arange(-100, 100 + h / 2, h)
    XX, YY = np.meshgrid(g, g, indexing="ij")
    X = np.stack([XX.ravel(), YY.ravel()], axis=1)
    e = O.errors(func, o, M, X)
    assert e.min() >= -1e-12
    far = np.abs(X - o).max(axis=1) > 2.0
    assert e[far].min() > 1e-3
    # fine grid in the +-2 window around o: the error grows at least
    # quadratically away from o, so o is the unique minimiser in the box
    hf = 0.01
    gx = o[0] + np.arange(-2, 2 + hf / 2, hf) + 0.37 * hf
    gy = o[1] + np.arange(-2, 2 + hf / 2, hf) + 0.61 * hf
    XX, YY = np.meshgrid(gx, gy, indexing="ij")
    Xf = np.stack([XX.ravel(), YY.ravel()], axis=1)
    ef = O.errors(func, o, M, Xf)
    r2 = np.sum((Xf - o) ** 2, axis=1)
    assert ef.min() >= 0.0
    assert (ef / r2).min() >= 0.05
