"""FP64 CPU oracle: ctypes wrapper over ``liboracle.so`` (built from oracle.c).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` import this package.  The product library
(``paper_2505_17430_amd``) never imports it, and it never imports the product.

Arrays are numpy; populations are individual-major ``(np, dim)`` float64 here,
converted from/to the GPU's structure-of-arrays layout by the caller.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ELLIPSOID, ROSENBROCK, RASTRIGIN, SCHWEFEL, GRIEWANK, ACKLEY = range(6)
FUNC_NAMES = ["ellipsoid", "rosenbrock", "rastrigin", "schwefel", "griewank", "ackley"]
ALGO_DE, ALGO_PSO, ALGO_SHADE, ALGO_LSHADE, ALGO_PSODE, ALGO_CSO, ALGO_JADE, ALGO_LSHADE_RS = range(8)
TRACE_EVERY = 200


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C99, FP64, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
        os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "oracle.h"))
    ):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=gnu99", "-Wall",
             "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [("func", C.c_int32), ("dim", C.c_int32), ("lb", C.c_double), ("ub", C.c_double)]


class RunDesc(C.Structure):
    _fields_ = [
        ("algo", C.c_int32), ("func", C.c_int32), ("dim", C.c_int32),
        ("lb", C.c_double), ("ub", C.c_double),
        ("instance", C.c_uint32), ("run_uid", C.c_uint32), ("np", C.c_int32),
        ("budget", C.c_int64),
        ("F", C.c_double), ("CR", C.c_double),
        ("w", C.c_double), ("c1", C.c_double), ("c2", C.c_double), ("vmax", C.c_double),
        ("p", C.c_double), ("H", C.c_int32),
        ("r_arc", C.c_double), ("np_min", C.c_int32),
        ("topology", C.c_int32), ("velocity", C.c_int32),
        ("c", C.c_double), ("restart_tol", C.c_double),
    ]


class _LShadeState(C.Structure):
    _fields_ = [("np", C.c_int32), ("na", C.c_int32), ("acap", C.c_int32), ("H", C.c_int32),
                ("pos", C.c_int32), ("X", C.POINTER(C.c_double)), ("eX", C.POINTER(C.c_double)),
                ("A", C.POINTER(C.c_double)), ("MF", C.c_double * 64), ("MCR", C.c_double * 64)]


class RunResult(C.Structure):
    _fields_ = [("best_e", C.c_double), ("fes", C.c_int64), ("generations", C.c_int32),
                ("success", C.c_int32), ("restarts", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        fp = C.POINTER(C.c_float)
        ip = C.POINTER(C.c_int32)
        up = C.POINTER(C.c_uint32)
        bp = C.POINTER(C.c_uint8)
        pp = C.POINTER(_Problem)
        L.orc_philox4x32_10.argtypes = [up, up, up]
        L.orc_u24.restype = C.c_double
        L.orc_u24.argtypes = [C.c_uint32]
        L.orc_u53.restype = C.c_double
        L.orc_u53.argtypes = [C.c_uint32, C.c_uint32]
        L.orc_range.restype = C.c_uint32
        L.orc_range.argtypes = [C.c_uint32, C.c_uint32]
        L.orc_cr_threshold.restype = C.c_uint32
        L.orc_cr_threshold.argtypes = [C.c_double]
        L.orc_instance.argtypes = [C.c_int32, C.c_int32, C.c_uint32, C.c_uint64, dp, dp, dp]
        L.orc_householder_q.argtypes = [C.c_int32, dp, dp]
        L.orc_error.restype = C.c_double
        L.orc_error.argtypes = [C.c_int32, C.c_int32, dp, dp, dp]
        L.orc_error_z.restype = C.c_double
        L.orc_error_z.argtypes = [C.c_int32, C.c_int32, dp]
        L.orc_error_soa_f32.argtypes = [C.c_int32, C.c_int32, dp, dp, fp, C.c_int64, C.c_int32, dp]
        L.orc_error_aos.argtypes = [C.c_int32, C.c_int32, dp, dp, dp, C.c_int32, dp]
        L.orc_init_population.argtypes = [pp, C.c_int32, C.c_uint32, C.c_uint64, dp]
        L.orc_donors_from_words.argtypes = [C.c_int32, C.c_int32, C.c_int32, up, ip]
        L.orc_de_donors.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_uint32, C.c_uint64,
                                    C.c_uint32, ip]
        L.orc_de_generation.argtypes = [pp, dp, dp, C.c_int32, C.c_double, C.c_double,
                                        C.c_uint32, C.c_uint64, C.c_uint32, dp, dp, dp, dp,
                                        dp, dp, ip, bp, bp]
        L.orc_pso_init.argtypes = [pp, dp, dp, C.c_int32, C.c_uint32, C.c_uint64, dp, dp, dp,
                                   dp, dp, ip]
        L.orc_pso_iteration.argtypes = [pp, dp, dp, C.c_int32, C.c_double, C.c_double,
                                        C.c_double, C.c_double, C.c_uint32, C.c_uint64,
                                        C.c_uint32, dp, dp, dp, dp, dp, ip]
        L.orc_shade_generation.argtypes = [pp, dp, dp, C.c_int32, C.c_double, C.c_int32, dp,
                                           dp, ip, C.c_uint32, C.c_uint64, C.c_uint32, dp, dp,
                                           dp, dp, dp, dp, ip, dp, dp, dp, bp, bp, ip]
        L.orc_shade_memory_update.argtypes = [C.c_int32, dp, dp, ip, C.c_int32, dp, dp, dp]
        L.orc_shade_pnum.restype = C.c_int32
        L.orc_shade_pnum.argtypes = [C.c_double, C.c_int32]
        L.orc_lshade_np.restype = C.c_int32
        L.orc_lshade_np.argtypes = [C.c_int32, C.c_int32, C.c_int64, C.c_int64]
        L.orc_lshade_archive_max.restype = C.c_int32
        L.orc_lshade_archive_max.argtypes = [C.c_double, C.c_int32]
        L.orc_lshade_memory_update.argtypes = [C.c_int32, dp, dp, ip, C.c_int32, dp, dp, dp]
        L.orc_lshade_generation.argtypes = [pp, dp, dp, C.POINTER(_LShadeState), C.c_double, C.c_double,
                                            C.c_int32, C.c_uint32, C.c_uint64, C.c_uint32, dp, dp, ip]
        L.orc_pso_variant_iteration.argtypes = [pp, dp, dp, C.c_int32, C.c_int32, C.c_int32, C.c_double,
                                                C.c_double, C.c_double, C.c_double, C.c_uint32, C.c_uint64,
                                                C.c_uint32, dp, dp, dp, dp, dp, ip]
        L.orc_psode_generation.argtypes = [pp, dp, dp, C.c_int32, C.c_int32, C.c_int32, C.c_double,
                                           C.c_double, C.c_double, C.c_double, C.c_double, C.c_int32,
                                           dp, dp, ip, C.c_uint32, C.c_uint64, C.c_uint32, dp, dp, dp,
                                           dp, dp, dp, dp, C.POINTER(C.c_uint8)]
        L.orc_cso_iteration.argtypes = [pp, dp, dp, C.c_int32, C.c_double, C.c_uint32, C.c_uint64,
                                        C.c_uint32, dp, dp, dp, dp, dp, ip, ip]
        L.orc_run.argtypes = [C.POINTER(RunDesc), C.c_uint64, C.c_uint64, C.POINTER(RunResult),
                              dp, C.c_int64, dp]
        L.orc_run_observed.argtypes = [C.POINTER(RunDesc), C.c_uint64, C.c_uint64, C.POINTER(RunResult),
                                       dp, C.c_int64, dp, dp, C.c_int64]
        L.orc_restart_population.argtypes = [pp, C.c_int32, C.c_uint32, C.c_uint64, C.c_uint32, dp]
        L.orc_restart_population.restype = None
        L.orc_converged.argtypes = [dp, C.c_int32, C.c_double]
        L.orc_jade_update.argtypes = [C.c_double, dp, dp, C.c_int32, dp, dp]
        L.orc_jade_update.restype = None
        L.orc_jade_generation.argtypes = [pp, dp, dp, C.POINTER(_LShadeState), C.c_double, C.c_double,
                                          C.c_double, C.c_uint32, C.c_uint64, C.c_uint32, dp, dp, ip]
        for name in ("orc_schwefel_s", "orc_schwefel_c", "orc_schwefel_lambda"):
            getattr(L, name).restype = C.c_double
            getattr(L, name).argtypes = []
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct)) if a is not None else None


def _d(a):
    return _p(a, C.c_double)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# Random numbers

def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c, C.c_uint32), _p(k, C.c_uint32), _p(out, C.c_uint32))
    return out


def u24(w):
    return lib().orc_u24(int(w))


def u53(a, b):
    return lib().orc_u53(int(a), int(b))


def rng_range(w, n):
    return int(lib().orc_range(int(w), int(n)))


def cr_threshold(cr):
    return int(lib().orc_cr_threshold(float(cr)))


# --------------------------------------------------------------------------
# Instances and objective functions

def instance(func, dim, inst, inst_seed, return_gaussian=False):
    o = np.zeros(dim)
    M = np.zeros((dim, dim))
    G = np.zeros((dim, dim)) if return_gaussian else None
    rc = lib().orc_instance(func, dim, inst, inst_seed, _d(o), _d(M), _d(G))
    if rc != 0:
        raise ValueError("orc_instance failed")
    return (o, M, G) if return_gaussian else (o, M)


def householder_q(A):
    A = _f64(A)
    n = A.shape[0]
    Q = np.zeros((n, n))
    if lib().orc_householder_q(n, _d(A), _d(Q)) != 0:
        raise ValueError("householder failed")
    return Q


def error(func, o, M, x):
    o, M, x = _f64(o), _f64(M), _f64(x)
    return lib().orc_error(func, o.shape[0], _d(o), _d(M), _d(x))


def error_z(func, z):
    z = _f64(z)
    return lib().orc_error_z(func, z.shape[0], _d(z))


def errors(func, o, M, X):
    """Errors of the rows of X (n, dim), float64."""
    o, M, X = _f64(o), _f64(M), _f64(X)
    n = X.shape[0]
    e = np.zeros(n)
    lib().orc_error_aos(func, o.shape[0], _d(o), _d(M), _d(X), n, _d(e))
    return e


def errors_soa_f32(func, o, M, Xsoa, n=None):
    """Errors of the columns of a float32 (dim, ld) structure-of-arrays block."""
    o, M = _f64(o), _f64(M)
    X = np.ascontiguousarray(Xsoa, dtype=np.float32)
    dim, ld = X.shape
    n = ld if n is None else n
    e = np.zeros(n)
    lib().orc_error_soa_f32(func, dim, _d(o), _d(M), _p(X, C.c_float), ld, n, _d(e))
    return e


def schwefel_constants():
    L = lib()
    return L.orc_schwefel_s(), L.orc_schwefel_c(), L.orc_schwefel_lambda()


# --------------------------------------------------------------------------
# Algorithm steps

def _problem(func, dim, lb, ub):
    return _Problem(func, dim, lb, ub)


def init_population(func, dim, lb, ub, np_, run_uid, seed):
    X = np.zeros((np_, dim))
    pb = _problem(func, dim, lb, ub)
    lib().orc_init_population(C.byref(pb), np_, run_uid, seed, _d(X))
    return X


def de_donors(np_, dim, i, run_uid, seed, t):
    out = np.zeros(4, dtype=np.int32)
    lib().orc_de_donors(np_, dim, i, run_uid, seed, t, _p(out, C.c_int32))
    return out


def donors_from_words(np_, dim, i, words):
    w = np.ascontiguousarray(words, dtype=np.uint32)
    out = np.zeros(4, dtype=np.int32)
    lib().orc_donors_from_words(np_, dim, i, _p(w, C.c_uint32), _p(out, C.c_int32))
    return out


def de_generation(func, lb, ub, o, M, X, eX, F, CR, run_uid, seed, t):
    """One synchronous rand/1/bin generation.  Returns a dict of every output."""
    o, M, X, eX = _f64(o), _f64(M), _f64(X), _f64(eX)
    np_, dim = X.shape
    U = np.zeros_like(X)
    eU = np.zeros(np_)
    Xn = np.zeros_like(X)
    eXn = np.zeros(np_)
    donors = np.zeros((np_, 4), dtype=np.int32)
    mask = np.zeros((np_, dim), dtype=np.uint8)
    rep = np.zeros(np_, dtype=np.uint8)
    pb = _problem(func, dim, lb, ub)
    rc = lib().orc_de_generation(C.byref(pb), _d(o), _d(M), np_, F, CR, run_uid, seed, t,
                                 _d(X), _d(eX), _d(U), _d(eU), _d(Xn), _d(eXn),
                                 _p(donors, C.c_int32), _p(mask, C.c_uint8), _p(rep, C.c_uint8))
    if rc != 0:
        raise ValueError("orc_de_generation failed")
    return dict(U=U, eU=eU, X=Xn, eX=eXn, donors=donors, mask=mask.astype(bool),
                replaced=rep.astype(bool))


def pso_init(func, lb, ub, o, M, np_, run_uid, seed):
    o, M = _f64(o), _f64(M)
    dim = o.shape[0]
    X = np.zeros((np_, dim)); V = np.zeros_like(X); P = np.zeros_like(X)
    eX = np.zeros(np_); eP = np.zeros(np_)
    g = np.zeros(1, dtype=np.int32)
    pb = _problem(func, dim, lb, ub)
    lib().orc_pso_init(C.byref(pb), _d(o), _d(M), np_, run_uid, seed, _d(X), _d(V), _d(P),
                       _d(eX), _d(eP), _p(g, C.c_int32))
    return dict(X=X, V=V, P=P, eX=eX, eP=eP, g=int(g[0]))


def pso_iteration(func, lb, ub, o, M, state, w, c1, c2, vmax, run_uid, seed, t):
    """One synchronous PSO iteration on a copy of ``state``; returns the new state."""
    o, M = _f64(o), _f64(M)
    X = _f64(state["X"]).copy(); V = _f64(state["V"]).copy(); P = _f64(state["P"]).copy()
    eX = np.zeros(X.shape[0]); eP = _f64(state["eP"]).copy()
    g = np.array([state["g"]], dtype=np.int32)
    np_, dim = X.shape
    pb = _problem(func, dim, lb, ub)
    rc = lib().orc_pso_iteration(C.byref(pb), _d(o), _d(M), np_, w, c1, c2, vmax, run_uid, seed,
                                 t, _d(X), _d(V), _d(P), _d(eX), _d(eP), _p(g, C.c_int32))
    if rc != 0:
        raise ValueError("orc_pso_iteration failed")
    return dict(X=X, V=V, P=P, eX=eX, eP=eP, g=int(g[0]))


def shade_pnum(p, np_):
    return int(lib().orc_shade_pnum(p, np_))


def shade_generation(func, lb, ub, o, M, X, eX, MF, MCR, pos, p, run_uid, seed, t):
    """One SHADE generation; memory arrays are copied, updated copies returned."""
    o, M, X, eX = _f64(o), _f64(M), _f64(X), _f64(eX)
    MF = _f64(MF).copy(); MCR = _f64(MCR).copy()
    H = MF.shape[0]
    posa = np.array([pos], dtype=np.int32)
    np_, dim = X.shape
    U = np.zeros_like(X); eU = np.zeros(np_); Xn = np.zeros_like(X); eXn = np.zeros(np_)
    idx = np.zeros((np_, 6), dtype=np.int32)
    F = np.zeros(np_); CR = np.zeros(np_); margin = np.zeros((np_, 2))
    mask = np.zeros((np_, dim), dtype=np.uint8); rep = np.zeros(np_, dtype=np.uint8)
    srt = np.zeros(np_, dtype=np.int32)
    pb = _problem(func, dim, lb, ub)
    rc = lib().orc_shade_generation(C.byref(pb), _d(o), _d(M), np_, p, H, _d(MF), _d(MCR),
                                    _p(posa, C.c_int32), run_uid, seed, t, _d(X), _d(eX),
                                    _d(U), _d(eU), _d(Xn), _d(eXn), _p(idx, C.c_int32), _d(F),
                                    _d(CR), _d(margin), _p(mask, C.c_uint8), _p(rep, C.c_uint8),
                                    _p(srt, C.c_int32))
    if rc != 0:
        raise ValueError("orc_shade_generation failed")
    return dict(U=U, eU=eU, X=Xn, eX=eXn, idx=idx, F=F, CR=CR, margin=margin,
                mask=mask.astype(bool), replaced=rep.astype(bool), sorted=srt,
                MF=MF, MCR=MCR, pos=int(posa[0]))


def shade_memory_update(MF, MCR, pos, SF, SCR, dS):
    MF = _f64(MF).copy(); MCR = _f64(MCR).copy()
    SF, SCR, dS = _f64(SF), _f64(SCR), _f64(dS)
    posa = np.array([pos], dtype=np.int32)
    lib().orc_shade_memory_update(MF.shape[0], _d(MF), _d(MCR), _p(posa, C.c_int32),
                                  SF.shape[0], _d(SF), _d(SCR), _d(dS))
    return MF, MCR, int(posa[0])


def pso_variant_iteration(func, lb, ub, o, M, X, V, P, eX, eP, topology, velocity, w, c1, c2, vmax,
                          run_uid, seed, t):
    """One PSO iteration with the given topology (0 global, 1 ring) and
    velocity update (0 inertia, 1 spherical); returns the new (X, V, P, eX,
    eP) and the neighbourhood bests used."""
    X, V, P = (np.ascontiguousarray(a, dtype=np.float64).copy() for a in (X, V, P))
    eX, eP = (np.ascontiguousarray(a, dtype=np.float64).copy() for a in (eX, eP))
    np_, dim = X.shape
    pb = _Problem(func, dim, lb, ub)
    lbest = np.zeros(np_, dtype=np.int32)
    rc = lib().orc_pso_variant_iteration(C.byref(pb), _d(np.ascontiguousarray(o, dtype=np.float64)),
                                         _d(np.ascontiguousarray(M, dtype=np.float64)), np_, topology, velocity,
                                         w, c1, c2, vmax, run_uid, C.c_uint64(seed), t, _d(X), _d(V), _d(P),
                                         _d(eX), _d(eP), _p(lbest, C.c_int32))
    if rc != 0:
        raise ValueError("orc_pso_variant_iteration failed")
    return X, V, P, eX, eP, lbest


def psode_generation(func, lb, ub, o, M, X, eX, V, MF, MCR, pos, topology, velocity, w, c1, c2, vmax,
                     p, run_uid, seed, t):
    """One PSODE generation (pairwise/3 selection); returns a dict with the
    new X, eX, V, the PSO moves Y / eY, the DE trials U / eU, the SHADE
    memory and the choice per individual (0 parent, 1 DE trial, 2 PSO move)."""
    X, eX, V = (np.ascontiguousarray(a, dtype=np.float64).copy() for a in (X, eX, V))
    MF = _f64(MF).copy(); MCR = _f64(MCR).copy()
    posa = np.array([pos], dtype=np.int32)
    np_, dim = X.shape
    Y = np.zeros_like(X); eY = np.zeros(np_); U = np.zeros_like(X); eU = np.zeros(np_)
    choice = np.zeros(np_, dtype=np.uint8)
    pb = _Problem(func, dim, lb, ub)
    rc = lib().orc_psode_generation(C.byref(pb), _d(_f64(o)), _d(_f64(M)), np_, topology, velocity,
                                    w, c1, c2, vmax, p, MF.shape[0], _d(MF), _d(MCR), _p(posa, C.c_int32),
                                    run_uid, C.c_uint64(seed), t, _d(X), _d(eX), _d(V), _d(Y), _d(eY),
                                    _d(U), _d(eU), _p(choice, C.c_uint8))
    if rc != 0:
        raise ValueError("orc_psode_generation failed")
    return dict(X=X, eX=eX, V=V, Y=Y, eY=eY, U=U, eU=eU, MF=MF, MCR=MCR, pos=int(posa[0]),
                choice=choice)


def cso_iteration(func, lb, ub, o, M, X, V, e, phi, run_uid, seed, t):
    """One CSO iteration; returns a dict with the new X, V, e, the losers' new
    positions G / errors eG in pair order and the pairs (winner, loser)."""
    X, V, e = (np.ascontiguousarray(a, dtype=np.float64).copy() for a in (X, V, e))
    m, dim = X.shape
    G = np.zeros((m // 2, dim)); eG = np.zeros(m // 2)
    win = np.zeros(m // 2, dtype=np.int32); los = np.zeros(m // 2, dtype=np.int32)
    pb = _Problem(func, dim, lb, ub)
    rc = lib().orc_cso_iteration(C.byref(pb), _d(_f64(o)), _d(_f64(M)), m, phi, run_uid, C.c_uint64(seed), t,
                                 _d(X), _d(V), _d(e), _d(G), _d(eG), _p(win, C.c_int32), _p(los, C.c_int32))
    if rc != 0:
        raise ValueError("orc_cso_iteration failed")
    return dict(X=X, V=V, e=e, G=G, eG=eG, winner=win, loser=los)


def lshade_np(np_init, np_min, budget, fe):
    return int(lib().orc_lshade_np(np_init, np_min, C.c_int64(budget), C.c_int64(fe)))


def lshade_archive_max(r_arc, np_):
    return int(lib().orc_lshade_archive_max(C.c_double(r_arc), np_))


def lshade_memory_update(MF, MCR, pos, SF, SCR, dS):
    MF = np.ascontiguousarray(MF, dtype=np.float64).copy()
    MCR = np.ascontiguousarray(MCR, dtype=np.float64).copy()
    SF, SCR, dS = (np.ascontiguousarray(a, dtype=np.float64) for a in (SF, SCR, dS))
    posa = np.array([pos], dtype=np.int32)
    lib().orc_lshade_memory_update(MF.shape[0], _d(MF), _d(MCR), _p(posa, C.c_int32),
                                   SF.shape[0], _d(SF), _d(SCR), _d(dS))
    return MF, MCR, int(posa[0])


class LShade:
    """One L-SHADE run's state in the oracle, advanced a generation at a time."""

    def __init__(self, func, dim, lb, ub, o, M, X, eX, H=6, r_arc=2.6):
        self.pb = _Problem(func, dim, lb, ub)
        self.o = np.ascontiguousarray(o, dtype=np.float64)
        self.M = np.ascontiguousarray(M, dtype=np.float64)
        np_ = X.shape[0]
        self.X = np.ascontiguousarray(X, dtype=np.float64).copy()
        self.eX = np.ascontiguousarray(eX, dtype=np.float64).copy()
        self.acap = lshade_archive_max(r_arc, np_) + 1
        self.A = np.zeros((self.acap, dim))
        self.r_arc = r_arc
        self.st = _LShadeState(np_, 0, self.acap, H, 0, _d(self.X), _d(self.eX), _d(self.A))
        for k in range(H):
            self.st.MF[k] = 0.5
            self.st.MCR[k] = 0.5

    @property
    def np(self):
        return self.st.np

    @property
    def na(self):
        return self.st.na

    def memory(self):
        H = self.st.H
        return np.array(self.st.MF[:H]), np.array(self.st.MCR[:H]), self.st.pos

    def archive(self):
        return self.A[: self.st.na].copy()

    def set_state(self, A, MF, MCR, pos):
        """Take over an archive ([na, dim]) and a memory (H slots, next slot
        pos) from elsewhere, e.g. another implementation's run state."""
        A = np.asarray(A, dtype=np.float64)
        if A.shape[0] > self.acap - 1:
            raise ValueError("archive larger than its bound")
        self.A[: A.shape[0]] = A
        self.st.na = A.shape[0]
        for k in range(self.st.H):
            self.st.MF[k] = float(MF[k])
            self.st.MCR[k] = float(MCR[k])
        self.st.pos = int(pos)

    def generation(self, p, np_next, run_uid, seed, t):
        """Returns (trials U, their errors eU, number of successes)."""
        n = self.st.np
        D = self.pb.dim
        U = np.zeros((n, D))
        eU = np.zeros(n)
        ns = np.zeros(1, dtype=np.int32)
        rc = lib().orc_lshade_generation(C.byref(self.pb), _d(self.o), _d(self.M), C.byref(self.st),
                                        C.c_double(p), C.c_double(self.r_arc), np_next, run_uid,
                                        C.c_uint64(seed), t, _d(U), _d(eU), _p(ns, C.c_int32))
        if rc != 0:
            raise ValueError("orc_lshade_generation failed")
        return U, eU, int(ns[0])

    def jade_generation(self, p, c, run_uid, seed, t):
        """JADE's generation (the state must have H = 1); returns (trials U,
        their errors eU, number of successes)."""
        n = self.st.np
        D = self.pb.dim
        U = np.zeros((n, D))
        eU = np.zeros(n)
        ns = np.zeros(1, dtype=np.int32)
        rc = lib().orc_jade_generation(C.byref(self.pb), _d(self.o), _d(self.M), C.byref(self.st),
                                      C.c_double(p), C.c_double(self.r_arc), C.c_double(c), run_uid,
                                      C.c_uint64(seed), t, _d(U), _d(eU), _p(ns, C.c_int32))
        if rc != 0:
            raise ValueError("orc_jade_generation failed")
        return U, eU, int(ns[0])


def run(desc: dict, seed, inst_seed, trace_len=0, mu_len=None):
    """Whole run; returns (result dict, trace array, best x), and with
    mu_len also the observer's [mu_len, 2] array of (muF, muCR) after each
    generation (orc_run_observed)."""
    d = RunDesc(**{k: v for k, v in desc.items()})
    res = RunResult()
    trace = np.full(max(trace_len, 0), np.nan)
    best_x = np.zeros(desc["dim"])
    tr = _d(trace) if trace_len > 0 else None
    if mu_len is None:
        rc = lib().orc_run(C.byref(d), seed, inst_seed, C.byref(res), tr, trace_len, _d(best_x))
    else:
        mu = np.zeros((max(mu_len, 0), 2))
        rc = lib().orc_run_observed(C.byref(d), seed, inst_seed, C.byref(res), tr, trace_len, _d(best_x),
                                    _d(mu) if mu_len > 0 else None, mu_len)
    if rc != 0:
        raise ValueError("orc_run failed")
    out = (dict(best_e=res.best_e, fes=res.fes, generations=res.generations,
                success=bool(res.success), restarts=res.restarts), trace, best_x)
    return out if mu_len is None else out + (mu,)


def jade_update(c, muF, muCR, SF, SCR):
    """JADE's parameter update from the successful F and CR values."""
    f = np.array([muF], dtype=np.float64)
    cr = np.array([muCR], dtype=np.float64)
    SF, SCR = (np.ascontiguousarray(a, dtype=np.float64) for a in (SF, SCR))
    lib().orc_jade_update(c, _d(f), _d(cr), SF.shape[0], _d(SF), _d(SCR))
    return float(f[0]), float(cr[0])


def restart_population(func, dim, lb, ub, np_, run_uid, seed, k):
    """Population of restart k ([np, dim]); k = 0 is the initial one."""
    X = np.zeros((np_, dim))
    lib().orc_restart_population(C.byref(_Problem(func, dim, lb, ub)), np_, run_uid, C.c_uint64(seed), k, _d(X))
    return X


def converged(e, tol):
    e = np.ascontiguousarray(e, dtype=np.float64)
    return bool(lib().orc_converged(_d(e), e.shape[0], tol))
