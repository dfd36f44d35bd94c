"""Seeded synthetic inputs shared by the tests and the benchmark.

This module holds no arithmetic of the method: only the workload recipes
(which runs use which function, dimension and instance) and seeded random
points drawn with numpy.  Both the GPU path and the oracle receive the same
arrays from here.

Workloads (synthetic stand-ins: no benchmark-suite data is used):
  C1  plain DE rand/1/bin: Rastrigin, D=10, NP=50, F=0.5, CR=0.9, 1000 generations
  C2  batched evaluation: 6 functions x D in {10,30,50,100} x 10 instances,
      51 runs x 100 points each, points uniform in [-100, 100]^D
  C3  batched PSO: 4096 swarms x 40 particles, swarm s -> function s mod 6,
      D = (10,30,50)[(s div 6) mod 3], instance (s div 18) mod 10, 2000 iterations
  C4  batched SHADE: 2048 runs, run r -> D = (10,30,50,100)[r mod 4],
      function (r div 4) mod 6, instance (r div 24) mod 10, NP = min(18 D, 200),
      budget 10000 D
  C5  large scale: D = 1000, Ellipsoid and Rastrigin, instance 0, 64 runs x 100 points
  CSO  the large-scale study's shape: 30 runs, run r -> function r mod 6, D = 1000,
      instance (r div 6) mod 5, swarm 300, 1e6 evaluations, phi = 0.1
  PSODE  the case study's hybrid, batched: 4096 runs, run r -> Rosenbrock, D = 30,
      instance r mod 10, NP = 100, budget 1000 D; PSO half spherical with ring
      topology (SPSO-2011 constants), DE half SHADE (p = 0.1, H = 6)
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 250517430
INSTANCE_SEED = 250517431
LB, UB = -100.0, 100.0
F_STAR = 100.0
FUNCS = list(range(6))

C2_DIMS = (10, 30, 50, 100)
C2_INSTANCES = 10
C2_RUNS = 51
C2_POINTS_PER_RUN = 100


def c2_groups(dims=C2_DIMS, instances=C2_INSTANCES, runs=C2_RUNS, points=C2_POINTS_PER_RUN):
    """(func, dim, instance, n_points) of every evaluation group of the sweep."""
    return [(f, d, k, runs * points) for d in dims for f in FUNCS for k in range(instances)]


def uniform_points(seed, dim, n, lb=LB, ub=UB, dtype=np.float32):
    """Structure-of-arrays block (dim, n) of points uniform in the box."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lb, ub, size=(dim, n)).astype(dtype)


def group_seed(func, dim, inst, salt=0):
    return (BASE_SEED * 1_000_003 + func * 10_007 + dim * 101 + inst * 7 + salt) % (2**63)


def near_points(o, rhos=(1e-1, 1e-3, 1e-5), per_rho=8, seed=0, dtype=np.float32):
    """Points round(o + rho N(0, 1)) for each rho, plus round(o) itself:
    the accuracy set around an optimum o (given by the caller)."""
    rng = np.random.default_rng(seed)
    cols = [np.asarray(o, dtype=np.float64)]
    for r in rhos:
        for _ in range(per_rho):
            cols.append(np.asarray(o) + r * rng.standard_normal(len(o)))
    X = np.stack(cols, axis=1)
    return np.clip(X, LB, UB).astype(dtype)


def c3_swarm(s):
    """(func, dim, instance) of swarm s of the batched PSO workload."""
    return s % 6, (10, 30, 50)[(s // 6) % 3], (s // 18) % 10


def c4_run(r):
    """(func, dim, instance, np) of run r of the batched SHADE workload."""
    d = (10, 30, 50, 100)[r % 4]
    return (r // 4) % 6, d, (r // 24) % 10, min(18 * d, 200)


def psode_run(r):
    """(func, dim, instance, np) of run r of the batched PSODE workload."""
    return 1, 30, r % 10, 100


CSO_RUNS = 30
CSO_PHI = 0.1


def cso_run(r):
    """(func, dim, instance, swarm, budget) of run r of the large-scale CSO workload."""
    return r % 6, 1000, (r // 6) % 5, 300, 1_000_000
