"""Tolerance of single-precision evaluation against the FP64 oracle, stated
per function.

Relative to the error value e = f - f* (not to f, whose bias of 100 would
hide everything below 1e-5), for Ellipsoid, Rastrigin, Schwefel, Griewank
and Ackley, at every dimension and in both single precisions (FP32
rotation, split-bf16 rotation):

    |e_gpu - e_oracle| <= max(1e-6, 1e-5 |e_oracle|)

that is relative 1e-5, or absolute 1e-6 near the optimum.  The oracle
evaluates at the same float32 point the GPU was given (widened exactly).

Rosenbrock adds one term.  The method rounds the double shift d = x - o to
float once before the rotation, which moves each z_i by up to about
eps32 ||d||_2 (M has unit rows; the float products and accumulation add a
small multiple of that).  To first order e then moves by
sum_i |de/dz_i| |dz_i|.  Rosenbrock's terms 100 q_i^2 with
q_i = z_i^2 + 2 z_i - z_{i+1} cancel inside q on the walls of its curved
valley, where |de/dz_i| = |200 q_i (2 z_i + 2) + 2 z_i - 200 q_{i-1}| is
large against e itself; there that shift costs more than 1e-5 e (measured:
1.03e-5 relative at one of 650 uniform points at D = 2).  Its bound is

    max(1e-6, 1e-5 |e|) + 4 eps32 ||x - o||_2 ||grad_z e||_1

with eps32 = 2^-24; the factor 4 covers the float rotation's products and
accumulation.  A defect (a wrong term, sign, index or operand) moves e by an
amount of the order of e itself, far outside either bound.
"""
import numpy as np

REL, ABS = 1e-5, 1e-6
EPS32 = 2.0 ** -24
ROSENBROCK = 1


def rosenbrock_grad_z(Z):
    """Gradient of Rosenbrock's e with respect to z for the columns of Z (D, n)."""
    Z = np.asarray(Z, dtype=np.float64)
    G = np.zeros_like(Z)
    q = Z[:-1] ** 2 + 2 * Z[:-1] - Z[1:]
    G[:-1] += 200 * q * (2 * Z[:-1] + 2) + 2 * Z[:-1]
    G[1:] += -200 * q
    return G


def tolerance(func, o, M, X, e_oracle, rel=REL, abs_=ABS):
    """Per-point bound for float evaluation of the columns of X (D, n)."""
    e = np.asarray(e_oracle, dtype=np.float64)
    tol = np.maximum(abs_, rel * np.abs(e))
    if func == ROSENBROCK:
        d = np.asarray(X, dtype=np.float64) - np.asarray(o, dtype=np.float64)[:, None]
        Z = np.asarray(M) @ d
        tol = tol + 4 * EPS32 * np.linalg.norm(d, axis=0) * np.sum(np.abs(rosenbrock_grad_z(Z)), axis=0)
    return tol
