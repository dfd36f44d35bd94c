"""MI355X (gfx950) batched shifted-rotated evaluation with fused DE / PSO /
SHADE generation steps: the data-parallel hot path of SEvoBench
(arXiv 2505.17430), behind the C ABI in ``include/sevo.h``.

``paper_2505_17430_amd.sevo`` is the Python binding; ``...build`` compiles
``libsevo.so``.
"""
from . import sevo  # noqa: F401
from .sevo import (ACKLEY, ELLIPSOID, FP32, FP64, GRIEWANK, RASTRIGIN, ROSENBROCK,  # noqa: F401
                   SCHWEFEL, SPLIT_BF16, Context, SevoError, problem)
