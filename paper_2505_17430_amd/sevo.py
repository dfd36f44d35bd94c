"""Thin Python binding of ``libsevo.so`` (the C ABI in ``include/sevo.h``).

Argument marshalling only: every step of the evaluation and of the DE / PSO /
SHADE generations runs in the library's HIP kernels.  Buffers are passed as
device pointers (anything with ``data_ptr()``, e.g. torch tensors on the GPU,
or plain integers); streams as ``hipStream_t`` handles (a torch stream's
``cuda_stream``) or None for the default stream.

There is no fallback: if the library is not built, importing the binding's
entry points raises.
"""
from __future__ import annotations

import ctypes as C
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsevo.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "sevo.h")

OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED, ESTATE = 0, -1, -2, -3, -4, -5
ELLIPSOID, ROSENBROCK, RASTRIGIN, SCHWEFEL, GRIEWANK, ACKLEY = range(6)
FUNC_NAMES = ["ellipsoid", "rosenbrock", "rastrigin", "schwefel", "griewank", "ackley"]
FP64, FP32, SPLIT_BF16 = 0, 1, 2
ALGO_DE, ALGO_PSO, ALGO_SHADE, ALGO_LSHADE, ALGO_PSODE, ALGO_CSO, ALGO_JADE, ALGO_LSHADE_RS = range(8)
TRACE_EVERY = 200


class SevoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sevo error {code}: {msg}")
        self.code = code


class Problem(C.Structure):
    _fields_ = [("func", C.c_int32), ("dim", C.c_int32), ("lb", C.c_double),
                ("ub", C.c_double), ("f_star", C.c_double)]


class EvalItem(C.Structure):
    _fields_ = [("prob", Problem), ("instance", C.c_uint32), ("n", C.c_int32),
                ("ld", C.c_int64), ("x", C.c_void_p), ("err_out", C.c_void_p)]


class DEState(C.Structure):
    _fields_ = [("n_runs", C.c_int32), ("np", C.c_int32), ("ld", C.c_int64),
                ("run_stride", C.c_int64), ("run_uid0", C.c_uint32), ("generation", C.c_uint32),
                ("x", C.c_void_p), ("ex", C.c_void_p), ("u", C.c_void_p), ("eu", C.c_void_p),
                ("donors", C.c_void_p), ("replaced", C.c_void_p)]


class DEParams(C.Structure):
    _fields_ = [("F", C.c_double), ("CR", C.c_double)]


class PSOState(C.Structure):
    _fields_ = [("n_runs", C.c_int32), ("np", C.c_int32), ("ld", C.c_int64),
                ("run_stride", C.c_int64), ("run_uid0", C.c_uint32), ("iteration", C.c_uint32),
                ("x", C.c_void_p), ("v", C.c_void_p), ("p", C.c_void_p),
                ("ex", C.c_void_p), ("ep", C.c_void_p), ("gbest", C.c_void_p)]


class PSOParams(C.Structure):
    _fields_ = [("w", C.c_double), ("c1", C.c_double), ("c2", C.c_double), ("vmax", C.c_double)]


class RunDesc(C.Structure):
    _fields_ = [("prob", Problem), ("instance", C.c_uint32), ("run_uid", C.c_uint32),
                ("algo", C.c_int32), ("np", C.c_int32), ("budget", C.c_int64),
                ("F", C.c_double), ("CR", C.c_double),
                ("w", C.c_double), ("c1", C.c_double), ("c2", C.c_double), ("vmax", C.c_double),
                ("p", C.c_double), ("H", C.c_int32),
                ("r_arc", C.c_double), ("np_min", C.c_int32), ("topology", C.c_int32),
                ("velocity", C.c_int32), ("max_generations", C.c_int32), ("c", C.c_double),
                ("restart_tol", C.c_double)]


class RunResult(C.Structure):
    _fields_ = [("best_e", C.c_double), ("best_e32", C.c_float), ("success", C.c_int32),
                ("fes", C.c_int64), ("generations", C.c_int32), ("restarts", C.c_int32)]


class RunState(C.Structure):
    _fields_ = [("max_np", C.c_int32), ("max_dim", C.c_int32), ("max_arc", C.c_int32),
                ("reserved", C.c_int32),
                ("x", C.c_void_p), ("e", C.c_void_p), ("u", C.c_void_p), ("eu", C.c_void_p),
                ("v", C.c_void_p), ("p", C.c_void_p), ("ep", C.c_void_p), ("memory", C.c_void_p),
                ("archive", C.c_void_p), ("counts", C.c_void_p)]


def header_functions():
    """Names of the functions declared in include/sevo.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(sevo_\w+)\s*\(", text, re.M)))


_lib = None


def lib():
    """Load libsevo.so (raises ImportError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2505_17430_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, u32, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64
    L.sevo_create.argtypes = [C.POINTER(vp), i32, u64, u64]
    L.sevo_destroy.argtypes = [vp]
    L.sevo_last_error.argtypes = [vp]
    L.sevo_last_error.restype = C.c_char_p
    L.sevo_sync.argtypes = [vp, vp]
    L.sevo_instance.argtypes = [vp, C.POINTER(Problem), u32, vp, vp]
    L.sevo_set_instance.argtypes = [vp, C.POINTER(Problem), u32, vp, vp]
    L.sevo_generate_instance.argtypes = [i32, i32, u32, u64, vp, vp]
    L.sevo_evaluate.argtypes = [vp, C.POINTER(Problem), u32, vp, i64, i32, vp, i32, vp]
    L.sevo_evaluate_batch.argtypes = [vp, C.POINTER(EvalItem), i32, i32, vp]
    L.sevo_evaluate_batch_noalloc.argtypes = [vp, C.POINTER(EvalItem), i32, i32, vp]
    L.sevo_tune_evaluate.argtypes = [vp, C.POINTER(EvalItem), i32, i32, vp, C.POINTER(i32)]
    L.sevo_de_step.argtypes = [vp, C.POINTER(Problem), u32, C.POINTER(DEState),
                               C.POINTER(DEParams), i32, vp]
    L.sevo_pso_step.argtypes = [vp, C.POINTER(Problem), u32, C.POINTER(PSOState),
                                C.POINTER(PSOParams), i32, vp]
    L.sevo_run.argtypes = [vp, C.POINTER(RunDesc), i32, i32, vp, vp, i64, vp, i32, vp]
    L.sevo_run_observed.argtypes = [vp, C.POINTER(RunDesc), i32, i32, vp, vp, i64, vp, i32, vp, i64, vp]
    L.sevo_run_snapshot.argtypes = [vp, C.POINTER(RunDesc), i32, i32, vp, vp, i64, vp, i32,
                                    C.POINTER(RunState), vp]
    L.sevo_plan_evaluate.argtypes = [vp, C.POINTER(EvalItem), i32, i32, C.POINTER(vp)]
    L.sevo_plan_run.argtypes = [vp, C.POINTER(RunDesc), i32, i32, vp, vp, i64, vp, i32, C.POINTER(vp)]
    L.sevo_plan_launch.argtypes = [vp, vp]
    L.sevo_plan_destroy.argtypes = [vp]
    for f in header_functions():
        if f != "sevo_last_error":
            getattr(L, f).restype = C.c_int
    _lib = L
    return L


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(s):
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


def generate_instance(func, dim, inst, instance_seed=250517431):
    """(o, M) of (func, dim, inst) from the library's host generator (no GPU)."""
    import numpy as np
    L = lib()
    o = np.zeros(dim)
    M = np.zeros((dim, dim))
    rc = L.sevo_generate_instance(func, dim, inst, instance_seed, o.ctypes.data, M.ctypes.data)
    if rc != OK:
        raise SevoError(rc, L.sevo_last_error(None).decode())
    return o, M


def problem(func, dim, lb=-100.0, ub=100.0, f_star=100.0):
    return Problem(func, dim, lb, ub, f_star)


class Plan:
    """A prepared evaluation or set of runs (sevo_plan_*): launch() enqueues
    kernels only, so it can be captured into a graph and replayed."""

    def __init__(self, ctx, handle):
        self._ctx = ctx
        self._h = handle

    def launch(self, stream=None):
        self._ctx._check(self._ctx._L.sevo_plan_launch(self._h, _stream(stream)))

    def close(self):
        if getattr(self, "_h", None):
            self._ctx._L.sevo_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """Owns a library context (instance cache, workspaces) on one GPU."""

    def __init__(self, device=0, base_seed=250517430, instance_seed=250517431):
        L = lib()
        h = C.c_void_p()
        rc = L.sevo_create(C.byref(h), device, base_seed, instance_seed)
        if rc != OK:
            raise SevoError(rc, L.sevo_last_error(None).decode())
        self._h = h
        self._L = L

    def close(self):
        if getattr(self, "_h", None):
            self._L.sevo_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc):
        if rc != OK:
            raise SevoError(rc, self._L.sevo_last_error(self._h).decode())

    def last_error(self):
        return self._L.sevo_last_error(self._h).decode()

    def sync(self, stream=None):
        self._check(self._L.sevo_sync(self._h, _stream(stream)))

    def instance(self, prob, inst):
        import numpy as np
        o = np.zeros(prob.dim)
        M = np.zeros((prob.dim, prob.dim))
        self._check(self._L.sevo_instance(self._h, C.byref(prob), inst, o.ctypes.data, M.ctypes.data))
        return o, M

    def set_instance(self, prob, inst, o, M):
        import numpy as np
        o = np.ascontiguousarray(o, dtype=np.float64)
        M = np.ascontiguousarray(M, dtype=np.float64)
        self._check(self._L.sevo_set_instance(self._h, C.byref(prob), inst, o.ctypes.data, M.ctypes.data))

    def evaluate(self, prob, inst, x, err, n=None, ld=None, precision=FP32, stream=None):
        """x: device [dim][ld] (float or double), err: device [n]."""
        ld = x.stride(0) if ld is None else ld
        n = x.shape[1] if n is None else n
        self._check(self._L.sevo_evaluate(self._h, C.byref(prob), inst, _ptr(x), ld, n, _ptr(err),
                                          precision, _stream(stream)))

    @staticmethod
    def prepare_batch(items):
        """Marshal a list of (prob, inst, x, err[, n, ld]) once; the result can
        be passed to evaluate_batch any number of times."""
        arr = (EvalItem * len(items))()
        for k, it in enumerate(items):
            prob, inst, x, err = it[:4]
            n = it[4] if len(it) > 4 else x.shape[1]
            ld = it[5] if len(it) > 5 else x.stride(0)
            arr[k] = EvalItem(prob, inst, n, ld, _ptr(x), _ptr(err))
        return arr

    def evaluate_batch(self, items, precision=FP32, stream=None):
        """items: list of (prob, inst, x, err[, n, ld]) or a prepare_batch() result."""
        arr = items if isinstance(items, C.Array) else self.prepare_batch(items)
        self._check(self._L.sevo_evaluate_batch(self._h, arr, len(arr), precision, _stream(stream)))

    def evaluate_batch_noalloc(self, items, precision=FP32, stream=None):
        """sevo_evaluate_batch_noalloc: the same evaluation with no device
        allocation (instances must be resident; D <= 120 in single precision)."""
        arr = items if isinstance(items, C.Array) else self.prepare_batch(items)
        self._check(self._L.sevo_evaluate_batch_noalloc(self._h, arr, len(arr), precision, _stream(stream)))

    def tune_evaluate(self, items, precision=FP32, stream=None):
        """Autotune the evaluation launch shape on these items; returns
        {k-step class: tiles per workgroup (0 = resident grid)}."""
        arr = items if isinstance(items, C.Array) else self.prepare_batch(items)
        chosen = (C.c_int32 * 64)()
        self._check(self._L.sevo_tune_evaluate(self._h, arr, len(arr), precision, _stream(stream), chosen))
        return {k: chosen[k] for k in range(64) if chosen[k] >= 0}

    def plan_evaluate(self, items, precision=FP32):
        arr = items if isinstance(items, C.Array) else self.prepare_batch(items)
        h = C.c_void_p()
        self._check(self._L.sevo_plan_evaluate(self._h, arr, len(arr), precision, C.byref(h)))
        return Plan(self, h)

    def plan_run(self, descs, results, trace=None, trace_len=0, best_x=None, max_dim=0, precision=FP32):
        arr = (RunDesc * len(descs))(*descs)
        h = C.c_void_p()
        self._check(self._L.sevo_plan_run(self._h, arr, len(descs), precision, _ptr(results), _ptr(trace),
                                          trace_len, _ptr(best_x), max_dim, C.byref(h)))
        return Plan(self, h)

    def de_step(self, prob, inst, state: DEState, F, CR, precision=FP32, stream=None):
        self._check(self._L.sevo_de_step(self._h, C.byref(prob), inst, C.byref(state),
                                         C.byref(DEParams(F, CR)), precision, _stream(stream)))

    def pso_step(self, prob, inst, state: PSOState, w, c1, c2, vmax, precision=FP32, stream=None):
        self._check(self._L.sevo_pso_step(self._h, C.byref(prob), inst, C.byref(state),
                                          C.byref(PSOParams(w, c1, c2, vmax)), precision,
                                          _stream(stream)))

    def run(self, descs, results, trace=None, trace_len=0, best_x=None, max_dim=0,
            precision=FP32, stream=None):
        arr = (RunDesc * len(descs))(*descs)
        self._check(self._L.sevo_run(self._h, arr, len(descs), precision, _ptr(results),
                                     _ptr(trace), trace_len, _ptr(best_x), max_dim,
                                     _stream(stream)))

    def run_observed(self, descs, results, mu, mu_len, trace=None, trace_len=0, best_x=None, max_dim=0,
                     precision=FP32, stream=None):
        """sevo_run_observed: `mu` a device float buffer of n_runs * mu_len * 2."""
        arr = (RunDesc * len(descs))(*descs)
        self._check(self._L.sevo_run_observed(self._h, arr, len(descs), precision, _ptr(results),
                                              _ptr(trace), trace_len, _ptr(best_x), max_dim, _ptr(mu),
                                              mu_len, _stream(stream)))

    def run_snapshot(self, descs, results, state, trace=None, trace_len=0, best_x=None, max_dim=0,
                     precision=FP32, stream=None):
        """sevo_run_snapshot: `state` a dict with max_np, max_dim, max_arc and
        device buffers x, e (required), u, eu, v, p, ep, memory, archive,
        counts (optional)."""
        arr = (RunDesc * len(descs))(*descs)
        st = RunState(state["max_np"], state["max_dim"], state.get("max_arc", 0), 0,
                      *[_ptr(state.get(k)) for k in ("x", "e", "u", "eu", "v", "p", "ep", "memory",
                                                     "archive", "counts")])
        self._check(self._L.sevo_run_snapshot(self._h, arr, len(descs), precision, _ptr(results),
                                              _ptr(trace), trace_len, _ptr(best_x), max_dim, C.byref(st),
                                              _stream(stream)))
