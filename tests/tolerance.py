"""Tolerance of single-precision evaluation against the FP64 oracle.

Target bound per point: |e_gpu - e_oracle| <= max(1e-6, 1e-5 e_oracle).

A float32 rotation cannot always meet it: each z_j carries an absolute
rounding error of order eps32 ||d|| (d = x - o; the products and the
accumulation over D coordinates are rounded), and the objective turns that
into |de| ~ sum_j |de/dz_j| |dz_j|.  Where the function is ill-conditioned at
the point -- Rosenbrock's curved valley, where q = z_j^2 + 2 z_j - z_{j+1}
cancels; large-D Ellipsoid, whose weights span 1e6 -- the first-order term
exceeds 1e-5 e.  The stated tolerance is therefore

    tol = max(1e-6, 1e-5 e) + 4 eps32 ||d||_2 ||grad_z e||_1

with eps32 = 2^-24.  The conditioning term is an upper bound of the rounding
error the float32 arithmetic is allowed to make; a defect in the method
(a wrong term, sign, index or operand) produces errors of order e itself.
The gradients below are the textbook derivatives; tests/test_tolerance.py
pins them against finite differences of the oracle.
"""
import math

import numpy as np

EPS32 = 2.0 ** -24
S_SCHWEFEL = 420.96874635998202731
LAMBDA = 0.01


def grad_z(func, Z):
    """Gradient of e with respect to z for the columns of Z (D, n), float64."""
    Z = np.asarray(Z, dtype=np.float64)
    D = Z.shape[0]
    if func == 0:
        w = 10.0 ** (6 * np.arange(D) / (D - 1))
        return 2 * w[:, None] * Z
    if func == 1:
        G = np.zeros_like(Z)
        q = Z[:-1] ** 2 + 2 * Z[:-1] - Z[1:]
        G[:-1] += 200 * q * (2 * Z[:-1] + 2) + 2 * Z[:-1]
        G[1:] += -200 * q
        return G
    if func == 2:
        return 2 * Z + 20 * math.pi * np.sin(2 * math.pi * Z)
    if func == 3:
        U = Z + S_SCHWEFEL
        A = np.abs(U)
        r = np.sqrt(np.maximum(A, 1e-300))
        inner = -np.sin(r) - 0.5 * r * np.cos(r)           # d/du of -u sin sqrt|u|
        out = np.where(U > 500, 2 * LAMBDA * (U - 500), np.where(U < -500, 2 * LAMBDA * (U + 500), inner))
        return out
    if func == 4:
        i = np.arange(1, D + 1)[:, None]
        C = np.cos(Z / np.sqrt(i))
        Sn = np.sin(Z / np.sqrt(i))
        G = Z / 2000.0
        for j in range(D):
            others = np.prod(np.delete(C, j, axis=0), axis=0)
            G[j] += Sn[j] / math.sqrt(j + 1) * others
        return G
    if func == 5:
        r = np.sqrt(np.sum(Z * Z, axis=0) / D)
        c = np.mean(np.cos(2 * math.pi * Z), axis=0)
        safe = np.where(r > 0, r, 1.0)
        g1 = np.where(r > 0, 4.0 * np.exp(-0.2 * r) * Z / (D * safe), 0.0)
        g2 = np.exp(c) * 2 * math.pi * np.sin(2 * math.pi * Z) / D
        return g1 + g2
    raise ValueError(func)


def tolerance(func, o, M, X, e_oracle, rel=1e-5, abs_=1e-6):
    """Per-point tolerance for float32 evaluation of the columns of X."""
    d = np.asarray(X, dtype=np.float64) - np.asarray(o, dtype=np.float64)[:, None]
    Z = np.asarray(M) @ d
    cond = 4 * EPS32 * np.linalg.norm(d, axis=0) * np.sum(np.abs(grad_z(func, Z)), axis=0)
    return np.maximum(abs_, rel * np.abs(e_oracle)) + cond


def strict_tolerance(e_oracle, rel=1e-5, abs_=1e-6):
    return np.maximum(abs_, rel * np.abs(e_oracle))
