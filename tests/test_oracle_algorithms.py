"""Pins of the oracle's DE, PSO and SHADE generation steps and its run driver.

Each check follows from the algorithm's definition rather than from the
oracle's code: special parameter values that collapse a step to something
known (F = 0, CR in {0, 1}, c1 = c2 = 0), invariants (bounds, monotone best,
distinct donors), the SHADE memory update on a hand-built success set,
distribution tests of the sampled F and CR, and the recorder's FE accounting
recomputed from the step outputs.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle as O

SEED = 250517430
ISEED = 250517431
LB, UB = -100.0, 100.0


def _pop(func, dim, np_, run_uid=3):
    o, M = O.instance(func, dim, 0, ISEED)
    X = O.init_population(func, dim, LB, UB, np_, run_uid, SEED)
    eX = O.errors(func, o, M, X)
    return o, M, X, eX


def test_init_population_in_bounds_and_on_float32_grid():
    X = O.init_population(O.RASTRIGIN, 10, LB, UB, 50, 0, SEED)
    assert X.min() >= LB and X.max() < UB
    # lb + 200 u24 is exact in double; its float32 rounding is what the GPU stores
    assert stats.kstest(((X - LB) / (UB - LB)).ravel(), "uniform").pvalue > 1e-3
    Y = O.init_population(O.RASTRIGIN, 10, LB, UB, 50, 1, SEED)
    assert not np.array_equal(X, Y)


def test_de_f0_cr1_copies_r1():
    o, M, X, eX = _pop(O.RASTRIGIN, 10, 20)
    out = O.de_generation(O.RASTRIGIN, LB, UB, o, M, X, eX, 0.0, 1.0, 3, SEED, 1)
    for i in range(20):
        assert np.array_equal(out["U"][i], X[out["donors"][i, 0]])
        assert out["mask"][i].all()


def test_de_cr0_changes_exactly_jrand():
    o, M, X, eX = _pop(O.ELLIPSOID, 10, 20)
    out = O.de_generation(O.ELLIPSOID, LB, UB, o, M, X, eX, 0.5, 0.0, 3, SEED, 1)
    for i in range(20):
        jr = out["donors"][i, 3]
        assert out["mask"][i].sum() == 1 and out["mask"][i, jr]
        diff = np.nonzero(out["U"][i] != X[i])[0]
        assert set(diff) <= {jr}
        r1, r2, r3 = out["donors"][i, :3]
        v = X[r1, jr] + 0.5 * (X[r2, jr] - X[r3, jr])
        want = v if LB <= v <= UB else (0.5 * (LB + X[i, jr]) if v < LB else 0.5 * (UB + X[i, jr]))
        assert out["U"][i, jr] == want


def test_de_mutation_crossover_repair_definition():
    o, M, X, eX = _pop(O.SCHWEFEL, 7, 30)
    F, CR = 0.9, 0.5
    out = O.de_generation(O.SCHWEFEL, LB, UB, o, M, X, eX, F, CR, 3, SEED, 4)
    U, mask = out["U"], out["mask"]
    assert U.min() >= LB and U.max() <= UB
    n_repaired = 0
    for i in range(30):
        r1, r2, r3, jr = out["donors"][i]
        assert len({i, r1, r2, r3}) == 4
        v = X[r1] + F * (X[r2] - X[r3])
        for j in range(7):
            if not mask[i, j]:
                assert U[i, j] == X[i, j]
            elif v[j] < LB:
                assert U[i, j] == 0.5 * (LB + X[i, j]); n_repaired += 1
            elif v[j] > UB:
                assert U[i, j] == 0.5 * (UB + X[i, j]); n_repaired += 1
            else:
                assert U[i, j] == v[j]
    assert n_repaired > 0
    # mask frequency ~ CR outside jrand
    assert abs(mask.mean() - (CR + (1 - CR) / 7)) < 0.1


def test_de_selection_greedy_ties_to_trial():
    o, M, X, eX = _pop(O.ACKLEY, 5, 12)
    out = O.de_generation(O.ACKLEY, LB, UB, o, M, X, eX, 0.5, 0.9, 3, SEED, 2)
    assert np.array_equal(out["replaced"], out["eU"] <= eX)
    assert np.all(out["eX"] <= eX)
    # identical population: every trial equals its target, every tie goes to the trial
    Xs = np.tile(X[:1], (12, 1))
    eXs = O.errors(O.ACKLEY, o, M, Xs)
    out = O.de_generation(O.ACKLEY, LB, UB, o, M, Xs, eXs, 0.5, 0.9, 3, SEED, 2)
    assert np.array_equal(out["U"], Xs) and np.array_equal(out["eU"], eXs)
    assert out["replaced"].all()


def test_de_nan_counts_as_infinity():
    o, M, X, eX = _pop(O.RASTRIGIN, 4, 8)
    eX = eX.copy()
    eX[2] = np.nan
    out = O.de_generation(O.RASTRIGIN, LB, UB, o, M, X, eX, 0.5, 0.9, 3, SEED, 2)
    assert out["replaced"][2]


def test_de_steps_depend_only_on_generation_counter():
    # resume bit-identity: generation t's draws do not depend on history
    o, M, X, eX = _pop(O.GRIEWANK, 6, 10)
    a = O.de_generation(O.GRIEWANK, LB, UB, o, M, X, eX, 0.5, 0.9, 3, SEED, 9)
    O.de_generation(O.GRIEWANK, LB, UB, o, M, X, eX, 0.5, 0.9, 3, SEED, 2)
    b = O.de_generation(O.GRIEWANK, LB, UB, o, M, X, eX, 0.5, 0.9, 3, SEED, 9)
    for k in a:
        assert np.array_equal(a[k], b[k])


# ------------------------------------------------------------------ PSO

def test_pso_init():
    o, M = O.instance(O.ELLIPSOID, 8, 0, ISEED)
    st = O.pso_init(O.ELLIPSOID, LB, UB, o, M, 16, 5, SEED)
    assert np.all(st["V"] == 0) and np.array_equal(st["P"], st["X"])
    assert st["g"] == int(np.argmin(st["eP"]))


def test_pso_inertia_only_decay():
    # c1 = c2 = 0: v_t = w^t v_0 while no clamp or bound is hit
    o, M = O.instance(O.ELLIPSOID, 6, 0, ISEED)
    st = O.pso_init(O.ELLIPSOID, LB, UB, o, M, 8, 5, SEED)
    st["X"] = np.zeros_like(st["X"])
    v0 = np.random.default_rng(0).uniform(-1, 1, st["V"].shape)
    st["V"] = v0.copy()
    w = 0.7298
    x_expect = np.zeros_like(v0)
    for t in range(1, 6):
        st = O.pso_iteration(O.ELLIPSOID, LB, UB, o, M, st, w, 0.0, 0.0, 40.0, 5, SEED, t)
        x_expect = x_expect + w ** t * v0
        assert np.allclose(st["V"], w ** t * v0, rtol=1e-14, atol=0)
        assert np.allclose(st["X"], x_expect, rtol=1e-13, atol=1e-15)


def test_pso_invariants():
    func = O.RASTRIGIN
    o, M = O.instance(func, 10, 0, ISEED)
    st = O.pso_init(func, LB, UB, o, M, 40, 9, SEED)
    prev = st["eP"].copy()
    hit_clamp = hit_bound = False
    for t in range(1, 30):
        st = O.pso_iteration(func, LB, UB, o, M, st, 0.7298, 1.49618, 1.49618, 40.0, 9, SEED, t)
        assert np.all(np.abs(st["V"]) <= 40.0)
        assert st["X"].min() >= LB and st["X"].max() <= UB
        assert np.all(st["eP"] <= prev)
        improved = st["eP"] < prev
        # personal bests move only on strict improvement, to the current position
        assert np.array_equal(st["P"][improved], st["X"][improved])
        assert st["g"] == int(np.argmin(st["eP"]))
        hit_clamp |= bool(np.any(np.abs(st["V"]) == 40.0))
        hit_bound |= bool(np.any((st["X"] == LB) | (st["X"] == UB)))
        prev = st["eP"].copy()
    assert hit_clamp and hit_bound


def test_pso_gbest_ties_lowest_index():
    o, M = O.instance(O.ELLIPSOID, 4, 0, ISEED)
    st = O.pso_init(O.ELLIPSOID, LB, UB, o, M, 6, 2, SEED)
    # recorded personal bests far below any true error: no particle improves,
    # and the tie among indices 1, 3, 4 must resolve to 1
    st["eP"] = np.array([5e-9, 1e-9, 3e-9, 1e-9, 1e-9, 7e-9])
    st2 = O.pso_iteration(O.ELLIPSOID, LB, UB, o, M, st, 0.7298, 1.49618, 1.49618, 40.0, 2, SEED, 1)
    assert np.array_equal(st2["eP"], st["eP"])
    assert st2["g"] == 1


# ------------------------------------------------------------------ SHADE

def test_shade_memory_update_closed_form():
    MF = np.full(6, 0.5); MCR = np.full(6, 0.5)
    MF2, MCR2, pos = O.shade_memory_update(MF, MCR, 5, [0.5, 1.0], [0.2, 0.6], [1.0, 3.0])
    # weights 1/4, 3/4: M_CR = 0.25*0.2 + 0.75*0.6, M_F = Lehmer mean sum(w F^2)/sum(w F)
    assert MCR2[5] == pytest.approx(0.5, abs=1e-15)
    assert MF2[5] == pytest.approx((0.25 * 0.25 + 0.75 * 1.0) / (0.25 * 0.5 + 0.75 * 1.0), rel=1e-15)
    assert pos == 0
    assert np.array_equal(MF2[:5], MF[:5])
    # empty success set: nothing changes
    MF3, MCR3, pos3 = O.shade_memory_update(MF, MCR, 2, [], [], [])
    assert np.array_equal(MF3, MF) and pos3 == 2


@pytest.mark.parametrize("np_,want", [(180, 18), (200, 20), (10, 2), (4, 2), (25, 3), (35, 4)])
def test_shade_pnum(np_, want):
    assert O.shade_pnum(0.1, np_) == want


def test_shade_generation_invariants():
    func, D, np_ = O.ROSENBROCK, 10, 180
    o, M, X, eX = _pop(func, D, np_)
    MF = np.full(6, 0.5); MCR = np.full(6, 0.5)
    out = O.shade_generation(func, LB, UB, o, M, X, eX, MF, MCR, 0, 0.1, 3, SEED, 1)
    idx = out["idx"]
    order = np.lexsort((np.arange(np_), eX))
    assert np.array_equal(out["sorted"], order)
    top = set(order[:18].tolist())
    for i in range(np_):
        k, pb, r1, r2, jr, retries = idx[i]
        assert 0 <= k < 6 and pb in top
        assert r1 != i and r2 not in (i, r1) and 0 <= jr < D
        assert 0 < out["F"][i] <= 1 and 0 <= out["CR"][i] <= 1
        v = X[i] + out["F"][i] * (X[pb] - X[i]) + out["F"][i] * (X[r1] - X[r2])
        for j in range(D):
            if not out["mask"][i, j]:
                assert out["U"][i, j] == X[i, j]
            elif LB <= v[j] <= UB:
                assert out["U"][i, j] == v[j]
    assert out["pos"] == 1
    succ = out["eU"] < eX
    if succ.any():
        d = (eX - out["eU"])[succ]
        w = d / d.sum()
        assert out["MCR"][0] == pytest.approx(float(np.sum(w * out["CR"][succ])), rel=1e-12)
        F = out["F"][succ]
        assert out["MF"][0] == pytest.approx(float(np.sum(w * F * F) / np.sum(w * F)), rel=1e-12)


def test_shade_parameter_distributions():
    # F ~ Cauchy(0.5, 0.1) redrawn while <= 0 then capped at 1; CR ~ N(0.5, 0.1) clipped
    func, D, np_ = O.ELLIPSOID, 4, 200
    o, M, X, eX = _pop(func, D, np_)
    MF = np.full(6, 0.5); MCR = np.full(6, 0.5)
    Fs, CRs = [], []
    for t in range(1, 31):
        out = O.shade_generation(func, LB, UB, o, M, X, eX, MF, MCR, 0, 0.1, 3, SEED, t)
        Fs.append(out["F"]); CRs.append(out["CR"])
    F = np.concatenate(Fs); CR = np.concatenate(CRs)
    c = stats.cauchy(0.5, 0.1)
    p0 = c.cdf(0.0)

    def cdf_f(x):
        x = np.asarray(x, dtype=float)
        return np.where(x >= 1.0, 1.0, (c.cdf(x) - p0) / (1 - p0))
    # compare below the cap (the cap has a point mass at 1)
    below = F[F < 1.0]
    cond = lambda x: cdf_f(x) / cdf_f(np.nextafter(1.0, 0))
    assert stats.kstest(below, cond).pvalue > 1e-3
    assert abs(np.mean(F == 1.0) - (1 - cdf_f(np.nextafter(1.0, 0)))) < 0.01
    n = stats.norm(0.5, 0.1)
    inner = CR[(CR > 0) & (CR < 1)]
    assert stats.kstest(inner, lambda x: (n.cdf(x) - n.cdf(0)) / (n.cdf(1) - n.cdf(0))).pvalue > 1e-3


# ------------------------------------------------------------------ run driver

def _desc(algo, func, dim, np_, budget, **kw):
    d = dict(algo=algo, func=func, dim=dim, lb=LB, ub=UB, instance=0, run_uid=1, np=np_,
             budget=budget, F=0.5, CR=0.9, w=0.7298, c1=1.49618, c2=1.49618,
             vmax=0.2 * (UB - LB), p=0.1, H=6)
    d.update(kw)
    return d


@pytest.mark.parametrize("algo", [O.ALGO_DE, O.ALGO_PSO, O.ALGO_SHADE])
def test_run_matches_steps_and_recorder(algo):
    func, D, np_, budget = O.RASTRIGIN, 5, 20, 1000
    d = _desc(algo, func, D, np_, budget)
    res, trace, best_x = O.run(d, SEED, ISEED, trace_len=budget // 200)
    # replay with the step functions and recompute the recorder in Python
    o, M = O.instance(func, D, 0, ISEED)
    evals = []
    if algo == O.ALGO_PSO:
        st = O.pso_init(func, LB, UB, o, M, np_, 1, SEED)
        evals += list(zip(st["eX"], st["X"]))
        t = 0
        while len(evals) < budget:
            t += 1
            st = O.pso_iteration(func, LB, UB, o, M, st, 0.7298, 1.49618, 1.49618, 40.0, 1, SEED, t)
            evals += list(zip(st["eX"], st["X"]))
    else:
        X = O.init_population(func, D, LB, UB, np_, 1, SEED)
        eX = O.errors(func, o, M, X)
        evals += list(zip(eX, X))
        MF = np.full(6, 0.5); MCR = np.full(6, 0.5); pos = 0
        t = 0
        while len(evals) < budget:
            t += 1
            if algo == O.ALGO_DE:
                out = O.de_generation(func, LB, UB, o, M, X, eX, 0.5, 0.9, 1, SEED, t)
            else:
                out = O.shade_generation(func, LB, UB, o, M, X, eX, MF, MCR, pos, 0.1, 1, SEED, t)
                MF, MCR, pos = out["MF"], out["MCR"], out["pos"]
            evals += list(zip(out["eU"], out["U"]))
            X, eX = out["X"], out["eX"]
    e = np.array([v for v, _ in evals])
    assert res["fes"] == len(e) and res["generations"] == t
    assert res["best_e"] == e[:budget].min()
    assert np.array_equal(best_x, evals[int(np.argmin(e[:budget]))][1])
    want_trace = [e[: 200 * (k + 1)].min() for k in range(budget // 200)]
    assert np.array_equal(trace, want_trace)
    assert np.all(np.diff(trace) <= 0)


def test_run_fe_accounting_shade_c4_shape():
    # D = 10, NP = 180, budget 10000 D: 555 generations, last one overshoots to 100080 FEs
    d = _desc(O.ALGO_SHADE, O.ELLIPSOID, 10, 180, 100000)
    res, trace, _ = O.run(d, SEED, ISEED, trace_len=500)
    assert res["generations"] == 555 and res["fes"] == 100080
    assert np.all(np.isfinite(trace)) and np.all(np.diff(trace) <= 0)


def test_run_c1_de_converges():
    # the plain DE configuration: Rastrigin, D = 10, NP = 50, 1000 generations
    d = _desc(O.ALGO_DE, O.RASTRIGIN, 10, 50, 50 * 1001)
    res, trace, _ = O.run(d, SEED, ISEED, trace_len=50 * 1001 // 200)
    assert res["generations"] == 1000 and res["fes"] == 50050
    assert res["best_e"] < trace[0]
    assert res["success"] == (res["best_e"] <= 1e-8)


# ------------------------------------------------------------------ L-SHADE

def test_lshade_population_schedule():
    """Linear reduction: NP_init at the start, NP_min at the budget, never
    increasing, one step per (NP_init - NP_min)^-1 of the budget."""
    n0, nmin, B = 180, 4, 100000
    assert O.lshade_np(n0, nmin, B, 0) == n0
    assert O.lshade_np(n0, nmin, B, B) == nmin
    assert O.lshade_np(n0, nmin, B, 2 * B) == nmin            # clamped past the budget
    seq = [O.lshade_np(n0, nmin, B, fe) for fe in range(0, B + 1, 97)]
    assert all(a >= b for a, b in zip(seq, seq[1:]))
    assert O.lshade_np(n0, nmin, B, B // 2) in (92, 93)        # halfway: (180 + 4) / 2
    assert O.lshade_archive_max(2.6, 180) == 468 and O.lshade_archive_max(0.0, 50) == 0


def test_lshade_memory_update_closed_form():
    """Weighted Lehmer means for F and CR; the terminal CR value (stored as
    -1) is set when every successful CR is 0 and then kept."""
    MF, MCR = np.full(3, 0.5), np.full(3, 0.5)
    # one success: both means are its own values
    MF, MCR, pos = O.lshade_memory_update(MF, MCR, 0, [0.7], [0.3], [2.0])
    assert (MF[0], MCR[0], pos) == (pytest.approx(0.7), pytest.approx(0.3), 1)
    # two successes, weights 1/4 and 3/4: mean_L = (w1 a^2 + w2 b^2) / (w1 a + w2 b)
    MF, MCR, pos = O.lshade_memory_update(MF, MCR, pos, [0.2, 0.6], [0.4, 0.8], [1.0, 3.0])
    assert MF[1] == pytest.approx((0.25 * 0.04 + 0.75 * 0.36) / (0.25 * 0.2 + 0.75 * 0.6))
    assert MCR[1] == pytest.approx((0.25 * 0.16 + 0.75 * 0.64) / (0.25 * 0.4 + 0.75 * 0.8))
    assert pos == 2
    # all successful CR zero: terminal; it stays terminal in that slot
    MF, MCR, pos = O.lshade_memory_update(MF, MCR, pos, [0.5], [0.0], [1.0])
    assert MCR[2] == -1.0 and pos == 0
    MF, MCR, pos = O.lshade_memory_update(MF, MCR, 2, [0.5], [0.9], [1.0])
    assert MCR[2] == -1.0
    # no success: nothing moves
    MF2, MCR2, pos2 = O.lshade_memory_update(MF, MCR, pos, [], [], [])
    assert np.array_equal(MF2, MF) and np.array_equal(MCR2, MCR) and pos2 == pos


def test_lshade_first_generation_is_shades():
    """With an empty archive and the initial memory, the first generation's
    trials are SHADE's (same draws, r2 from the population only)."""
    func, D, np_ = O.RASTRIGIN, 10, 60
    o, M, X, eX = _pop(func, D, np_)
    ref = O.shade_generation(func, LB, UB, o, M, X, eX, np.full(6, 0.5), np.full(6, 0.5), 0, 0.11, 9,
                             SEED, 1)
    ls = O.LShade(func, D, LB, UB, o, M, X, eX, H=6, r_arc=2.6)
    U, eU, ns = ls.generation(0.11, np_, 9, SEED, 1)
    assert np.array_equal(U, ref["U"]) and np.array_equal(eU, ref["eU"])
    assert ns == int(np.sum(ref["eU"] < eX))
    assert ls.na == ns                                   # every improved parent archived


def test_lshade_generation_invariants():
    """Over many generations with reduction: the archive never exceeds
    round(r_arc NP) and holds only former population members; the kept
    individuals are the best of the selected population, in index order;
    per-slot errors never rise before the reduction."""
    func, D, n0, r_arc = O.ROSENBROCK, 8, 40, 1.4
    o, M, X, eX = _pop(func, D, n0)
    ls = O.LShade(func, D, LB, UB, o, M, X, eX, H=6, r_arc=r_arc)
    seen = {tuple(x) for x in X}
    B = 40 * 60
    fe = n0
    for t in range(1, 60):
        n = ls.np
        if fe >= B:
            break
        nn = O.lshade_np(n0, 4, B, fe + n)
        before_X, before_e = ls.X[:n].copy(), ls.eX[:n].copy()
        U, eU, ns = ls.generation(0.11, min(nn, n), 9, SEED, t)
        fe += n
        seen |= {tuple(x) for x in U}
        assert ns == int(np.sum(eU < before_e))
        # selection result before the reduction, reconstructed from the trials
        sel = np.where((eU <= before_e)[:, None], U, before_X)
        sel_e = np.where(eU <= before_e, eU, before_e)
        k = ls.np
        keep = np.sort(np.lexsort((np.arange(n), sel_e))[:k])
        assert np.array_equal(ls.X[:k], sel[keep]) and np.array_equal(ls.eX[:k], sel_e[keep])
        assert ls.na <= O.lshade_archive_max(r_arc, ls.np)
        for a in ls.A[:ls.na]:
            assert tuple(a) in seen
    assert ls.np < n0


def test_lshade_run_fe_accounting():
    d = _desc(O.ALGO_LSHADE, O.SCHWEFEL, 10, 180, 20000, p=0.11, r_arc=2.6, np_min=4)
    res, trace, _ = O.run(d, SEED, ISEED, trace_len=100)
    # replay the population schedule: whole generations, NP from the formula
    fe, n, gens = 180, 180, 0
    while fe < d["budget"]:
        nn = min(O.lshade_np(180, 4, d["budget"], fe + n), n)
        fe += n
        n = nn
        gens += 1
    assert res["fes"] == fe and res["generations"] == gens
    assert np.all(np.diff(trace[: fe // 200]) <= 0)
    assert res["best_e"] <= trace[0]


# ------------------------------------------------------------------ PSO variants

W_SPSO, C_SPSO = 1.0 / (2.0 * math.log(2.0)), 0.5 + math.log(2.0)


def _swarm(func, D, np_, iters=3, uid=4):
    o, M = O.instance(func, D, 0, ISEED)
    st = O.pso_init(func, LB, UB, o, M, np_, uid, SEED)
    for t in range(1, iters + 1):
        st = O.pso_iteration(func, LB, UB, o, M, st, 0.7298, 1.49618, 1.49618, 40.0, uid, SEED, t)
    return o, M, st


def test_pso_variant_global_inertia_is_the_classic_update():
    func, D, np_ = O.GRIEWANK, 7, 30
    o, M, st = _swarm(func, D, np_)
    ref = O.pso_iteration(func, LB, UB, o, M, st, 0.7298, 1.49618, 1.49618, 40.0, 4, SEED, 9)
    X, V, P, eX, eP, lb = O.pso_variant_iteration(func, LB, UB, o, M, st["X"], st["V"], st["P"], st["eX"],
                                                  st["eP"], 0, 0, 0.7298, 1.49618, 1.49618, 40.0, 4, SEED, 9)
    assert np.array_equal(X, ref["X"]) and np.array_equal(V, ref["V"]) and np.array_equal(P, ref["P"])
    assert np.all(lb == st["g"])


def test_pso_ring_neighbourhood_best_brute_force():
    func, D, np_ = O.RASTRIGIN, 5, 23
    o, M, st = _swarm(func, D, np_)
    eP = st["eP"].copy()
    eP[5] = eP[6] = eP[7] = eP[:].min() - 1.0          # a tie: lowest index wins
    *_, lb = O.pso_variant_iteration(func, LB, UB, o, M, st["X"], st["V"], st["P"], st["eX"], eP, 1, 0,
                                     0.7298, 1.49618, 1.49618, 40.0, 4, SEED, 9)
    for i in range(np_):
        nb = [(i - 1) % np_, i, (i + 1) % np_]
        want = min(nb, key=lambda k: (eP[k], k))
        assert lb[i] == want
    assert lb[6] == 5 and lb[7] == 6 and lb[5] == 5


def test_pso_spherical_sample_in_the_ball_uniformly():
    """With w = 0, no velocity clamp and a box that never binds, the new
    position is the sampled point x': it lies in the ball of centre G and
    radius |G - x|, G from the definition (x, p', l' centroid, or x and p'
    when the particle is its own neighbourhood best), and (|x' - G| / R)^D is
    uniform on [0, 1]."""
    func, D, np_ = O.SCHWEFEL, 6, 40
    o, M, st = _swarm(func, D, np_)
    us = []
    for t in range(10, 40):
        X, V, P, eX, eP, lb = O.pso_variant_iteration(func, -1e9, 1e9, o, M, st["X"], st["V"], st["P"], st["eX"],
                                                      st["eP"], 1, 1, 0.0, C_SPSO, C_SPSO, 1e12, 4, SEED, t)
        x, p = st["X"], st["P"]
        for i in range(np_):
            pp = x[i] + C_SPSO * (p[i] - x[i])
            if lb[i] == i:
                G = (x[i] + pp) / 2
            else:
                G = (x[i] + pp + x[i] + C_SPSO * (p[lb[i]] - x[i])) / 3
            R = np.linalg.norm(G - x[i])
            d = np.linalg.norm(X[i] - G)
            assert d <= R * (1 + 1e-12) + 1e-12
            if R > 0:
                us.append((d / R) ** D)
            else:                  # on its own best: the ball is the point G = x
                assert d == 0
    assert len(us) > 900
    assert stats.kstest(us, "uniform").pvalue > 1e-3


def test_pso_variant_runs_fe_accounting():
    for topo, vel in ((1, 0), (0, 1), (1, 1)):
        d = _desc(O.ALGO_PSO, O.SPHERE if hasattr(O, "SPHERE") else O.ELLIPSOID, 10, 40, 40 * 101,
                  topology=topo, velocity=vel, w=W_SPSO if vel else 0.7298,
                  c1=C_SPSO if vel else 1.49618, c2=C_SPSO if vel else 1.49618)
        res, trace, _ = O.run(d, SEED, ISEED, trace_len=30)
        assert res["fes"] == 40 * 101 and res["generations"] == 100
        assert np.all(np.diff(trace[: res["fes"] // 200]) <= 0) and np.isfinite(res["best_e"])


# ------------------------------------------------------------------ PSODE (pairwise/3)

def _psode_start(func, D, np_, uid=5):
    o, M, X, eX = _pop(func, D, np_, run_uid=uid)
    return o, M, X, eX, np.zeros_like(X)


def _key(e):
    e = np.asarray(e, dtype=np.float64)
    return np.where(np.isnan(e), np.inf, e)


@pytest.mark.parametrize("topology", [0, 1])
def test_psode_reduces_to_shade_when_the_pso_half_stands_still(topology):
    """With w = c1 = c2 = 0 the inertia update gives v = 0, so every PSO move
    is the parent itself, evaluated again; ties go to the DE result, so the
    population, the SHADE memory and the best so far follow SHADE exactly,
    at twice the evaluations per generation."""
    func, D, np_ = O.ROSENBROCK, 6, 24
    o, M, X, eX, V = _psode_start(func, D, np_)
    MF = np.full(6, 0.5); MCR = np.full(6, 0.5); pos = 0
    Xs, eXs, MFs, MCRs, poss = X.copy(), eX.copy(), MF.copy(), MCR.copy(), 0
    for t in range(1, 8):
        g = O.psode_generation(func, LB, UB, o, M, X, eX, V, MF, MCR, pos, topology, 0, 0.0, 0.0, 0.0,
                               40.0, 0.1, 5, SEED, t)
        s = O.shade_generation(func, LB, UB, o, M, Xs, eXs, MFs, MCRs, poss, 0.1, 5, SEED, t)
        assert np.array_equal(g["Y"], X) and np.array_equal(g["eY"], eX)
        assert np.array_equal(g["U"], s["U"]) and np.array_equal(g["eU"], s["eU"])
        assert np.array_equal(g["X"], s["X"]) and np.array_equal(g["eX"], s["eX"])
        assert np.array_equal(g["MF"], s["MF"]) and np.array_equal(g["MCR"], s["MCR"]) and g["pos"] == s["pos"]
        assert np.all(g["choice"] != 2)
        X, eX, V, MF, MCR, pos = g["X"], g["eX"], g["V"], g["MF"], g["MCR"], g["pos"]
        Xs, eXs, MFs, MCRs, poss = s["X"], s["eX"], s["MF"], s["MCR"], s["pos"]
    k = 9
    d_ps = _desc(O.ALGO_PSODE, func, D, np_, np_ * (1 + 2 * k), w=0.0, c1=0.0, c2=0.0, topology=topology)
    d_sh = _desc(O.ALGO_SHADE, func, D, np_, np_ * (1 + k))
    r_ps, _, bx_ps = O.run(d_ps, SEED, ISEED)
    r_sh, _, bx_sh = O.run(d_sh, SEED, ISEED)
    assert r_ps["generations"] == r_sh["generations"] == k
    assert r_ps["fes"] == np_ * (1 + 2 * k) and r_sh["fes"] == np_ * (1 + k)
    assert r_ps["best_e"] == r_sh["best_e"] and np.array_equal(bx_ps, bx_sh)


@pytest.mark.parametrize("topology,velocity", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_psode_generation_pairwise3_invariants(topology, velocity):
    """Each index keeps the best of parent, DE trial and PSO move (the PSO
    move only when strictly better); V becomes the DE displacement; in the
    first generation (V = 0) a particle that is its own neighbourhood best
    stands still under either update (its pull terms vanish)."""
    func, D, np_ = O.RASTRIGIN, 9, 30
    o, M, X, eX, V = _psode_start(func, D, np_)
    w, c = (W_SPSO, C_SPSO) if velocity else (0.7298, 1.49618)
    MF = np.full(6, 0.5); MCR = np.full(6, 0.5); pos = 0
    for t in range(1, 6):
        g = O.psode_generation(func, LB, UB, o, M, X, eX, V, MF, MCR, pos, topology, velocity, w, c, c,
                               40.0, 0.1, 5, SEED, t)
        kx, ku, ky = _key(eX), _key(g["eU"]), _key(g["eY"])
        rep = ku <= kx
        e3 = np.where(rep, g["eU"], eX)
        pso = ky < _key(e3)
        assert np.array_equal(g["choice"], np.where(pso, 2, np.where(rep, 1, 0)))
        assert np.array_equal(g["eX"], np.where(pso, g["eY"], e3))
        assert np.all(_key(g["eX"]) <= np.minimum(np.minimum(kx, ku), ky))
        want_x = np.where(pso[:, None], g["Y"], np.where(rep[:, None], g["U"], X))
        assert np.array_equal(g["X"], want_x)
        assert np.array_equal(g["V"], np.where(rep[:, None], g["U"] - X, 0.0))
        assert np.all(g["Y"] >= LB) and np.all(g["Y"] <= UB)
        if t == 1:
            own = [i for i in range(np_)
                   if (topology == 0 and i == int(np.argmin(kx))) or
                   (topology == 1 and min([(i - 1) % np_, i, (i + 1) % np_], key=lambda q: (kx[q], q)) == i)]
            assert own
            for i in own:
                assert np.array_equal(g["Y"][i], X[i]) and g["eY"][i] == eX[i]
        X, eX, V, MF, MCR, pos = g["X"], g["eX"], g["V"], g["MF"], g["MCR"], g["pos"]


@pytest.mark.parametrize("velocity", [0, 1])
def test_psode_run_matches_generations_and_recorder(velocity):
    """The run driver records the PSO moves, then the DE trials, of each
    generation; its best, best point and 200-FE trace are recomputed here
    from the generations."""
    func, D, np_, budget = O.GRIEWANK, 5, 20, 1300
    w, c = (W_SPSO, C_SPSO) if velocity else (0.7298, 1.49618)
    d = _desc(O.ALGO_PSODE, func, D, np_, budget, topology=1, velocity=velocity, w=w, c1=c, c2=c)
    res, trace, best_x = O.run(d, SEED, ISEED, trace_len=budget // 200)
    o, M = O.instance(func, D, 0, ISEED)
    X = O.init_population(func, D, LB, UB, np_, 1, SEED)
    eX = O.errors(func, o, M, X)
    V = np.zeros_like(X)
    evals = list(zip(eX, X))
    MF = np.full(6, 0.5); MCR = np.full(6, 0.5); pos = 0
    t = 0
    while len(evals) < budget:
        t += 1
        g = O.psode_generation(func, LB, UB, o, M, X, eX, V, MF, MCR, pos, 1, velocity, w, c, c,
                               0.2 * (UB - LB), 0.1, 1, SEED, t)
        evals += list(zip(g["eY"], g["Y"])) + list(zip(g["eU"], g["U"]))
        X, eX, V, MF, MCR, pos = g["X"], g["eX"], g["V"], g["MF"], g["MCR"], g["pos"]
    e = np.array([v for v, _ in evals])
    assert res["fes"] == len(e) == np_ + 2 * np_ * t and res["generations"] == t
    assert res["best_e"] == e[:budget].min()
    assert np.array_equal(best_x, evals[int(np.argmin(e[:budget]))][1])
    assert np.array_equal(trace, [e[: 200 * (k + 1)].min() for k in range(budget // 200)])


def test_psode_case_study_fe_accounting():
    """The case study's shape: D = 30, 100 individuals, 1000 D evaluations:
    150 generations of 200 evaluations after the initial 100."""
    d = _desc(O.ALGO_PSODE, O.ROSENBROCK, 30, 100, 30000, topology=1, velocity=1, w=W_SPSO, c1=C_SPSO,
              c2=C_SPSO)
    res, trace, _ = O.run(d, SEED, ISEED, trace_len=150)
    assert res["generations"] == 150 and res["fes"] == 30100
    assert np.all(np.isfinite(trace)) and np.all(np.diff(trace) <= 0)


# ------------------------------------------------------------------ CSO (competitive swarm optimizer)

def _fold(seed):
    return (seed & 0xFFFFFFFF) ^ (seed >> 32)


def _cso_start(func, D, m, uid=6):
    o, M, X, e = _pop(func, D, m, run_uid=uid)
    return o, M, X, np.zeros_like(X), e


def test_cso_pairing_is_the_sorted_key_matching():
    """Pairs are consecutive entries of the particles sorted by (Philox key,
    index), recomputed here from the Philox primitive; the lower error wins,
    the lower index on equal errors; every particle is in exactly one pair."""
    func, D, m, uid, t = O.ACKLEY, 4, 40, 6, 3
    o, M, X, V, e = _cso_start(func, D, m, uid)
    e = e.copy()
    e[7] = e[11] = e[19] = e[23] = e.min()                      # ties
    out = O.cso_iteration(func, LB, UB, o, M, X, V, e, 0.1, uid, SEED, t)
    keys = [int(O.philox([t, i, 12 << 24, 0], [uid, _fold(SEED)])[0]) for i in range(m)]
    perm = sorted(range(m), key=lambda i: (keys[i], i))
    for k in range(m // 2):
        a, b = perm[2 * k], perm[2 * k + 1]
        a_wins = e[a] < e[b] or (e[a] == e[b] and a < b)
        assert (out["winner"][k], out["loser"][k]) == ((a, b) if a_wins else (b, a))
    assert sorted(np.concatenate([out["winner"], out["loser"]])) == list(range(m))


def test_cso_iteration_state_invariants():
    """Winners keep position, velocity and error; each loser takes its new
    position (kept in the box) and the error of that position."""
    func, D, m = O.SCHWEFEL, 7, 30
    o, M, X, V, e = _cso_start(func, D, m)
    for t in range(1, 5):
        out = O.cso_iteration(func, LB, UB, o, M, X, V, e, 0.2, 6, SEED, t)
        w, l = out["winner"], out["loser"]
        assert np.array_equal(out["X"][w], X[w]) and np.array_equal(out["V"][w], V[w])
        assert np.array_equal(out["e"][w], e[w])
        assert np.array_equal(out["X"][l], out["G"]) and np.array_equal(out["e"][l], out["eG"])
        assert np.all(out["G"] >= LB) and np.all(out["G"] <= UB)
        assert np.allclose(out["eG"], O.errors(func, o, M, out["G"]), rtol=0, atol=0)
        X, V, e = out["X"], out["V"], out["e"]


def test_cso_first_iteration_moves_along_the_segment_to_the_winner():
    """With zero velocities and phi = 0 a loser coordinate moves to
    x_l + r2 (x_w - x_l): the fraction of the way to the winner is uniform
    on [0, 1)."""
    func, D, m = O.RASTRIGIN, 20, 200
    o, M, X, V, e = _cso_start(func, D, m)
    out = O.cso_iteration(func, -1e9, 1e9, o, M, X, V, e, 0.0, 6, SEED, 1)
    w, l = out["winner"], out["loser"]
    frac = ((out["X"][l] - X[l]) / (X[w] - X[l])).ravel()
    assert np.all(frac >= 0) and np.all(frac < 1)
    assert stats.kstest(frac, "uniform").pvalue > 1e-3
    assert np.array_equal(out["V"][l], out["X"][l] - X[l])


def test_cso_update_law_by_regression():
    """Second iteration, phi = 0.3, no clamping: the move y = x' - x_l of a
    loser coordinate is r1 v + r2 (x_w - x_l) + phi r3 (xbar - x_l) with
    independent uniforms, so least squares of y on (v, x_w - x_l, xbar - x_l)
    gives (1/2, 1/2, phi/2); xbar is the mean of the swarm before the move."""
    func, D, m, phi = O.ELLIPSOID, 50, 300, 0.3
    o, M, X, V, e = _cso_start(func, D, m)
    out = O.cso_iteration(func, -1e9, 1e9, o, M, X, V, e, phi, 6, SEED, 1)
    X, V, e = out["X"], out["V"], out["e"]
    xbar = X.mean(axis=0)
    out = O.cso_iteration(func, -1e9, 1e9, o, M, X, V, e, phi, 6, SEED, 2)
    w, l = out["winner"], out["loser"]
    y = (out["X"][l] - X[l]).ravel()
    A = np.stack([V[l].ravel(), (X[w] - X[l]).ravel(), (xbar - X[l]).ravel()], axis=1)
    coef, *_ = np.linalg.lstsq(A, y, rcond=None)
    assert np.all(np.abs(coef - [0.5, 0.5, 0.5 * phi]) < [0.03, 0.03, 0.03])
    # a wrong mean (of the winners only) fits clearly worse
    xbar_w = X[w].mean(axis=0)
    A2 = A.copy(); A2[:, 2] = (xbar_w - X[l]).ravel()
    r1 = np.linalg.lstsq(A, y, rcond=None)[1][0]
    r2 = np.linalg.lstsq(A2, y, rcond=None)[1][0]
    assert r1 < r2


def test_cso_identical_swarm_is_a_fixed_point():
    """All particles at one point whose coordinates sum exactly: every pair
    ties, the pull terms vanish and nothing moves."""
    func, D, m = O.GRIEWANK, 6, 16
    o, M = O.instance(func, D, 0, ISEED)
    X = np.tile(np.array([1.5, -2.25, 0.125, 40.0, -8.5, 3.0]), (m, 1))
    e = O.errors(func, o, M, X)
    out = O.cso_iteration(func, LB, UB, o, M, X, np.zeros_like(X), e, 0.1, 6, SEED, 1)
    assert np.array_equal(out["X"], X) and np.all(out["V"] == 0)
    assert np.all(out["winner"] < out["loser"])


def test_cso_run_matches_iterations_and_recorder():
    func, D, m, budget = O.ROSENBROCK, 6, 30, 1420
    d = _desc(O.ALGO_CSO, func, D, m, budget, c1=0.1)
    res, trace, best_x = O.run(d, SEED, ISEED, trace_len=budget // 200)
    o, M = O.instance(func, D, 0, ISEED)
    X = O.init_population(func, D, LB, UB, m, 1, SEED)
    e = O.errors(func, o, M, X)
    V = np.zeros_like(X)
    evals = list(zip(e, X))
    t = 0
    while len(evals) < budget:
        t += 1
        out = O.cso_iteration(func, LB, UB, o, M, X, V, e, 0.1, 1, SEED, t)
        evals += list(zip(out["eG"], out["G"]))
        X, V, e = out["X"], out["V"], out["e"]
    ev = np.array([v for v, _ in evals])
    assert res["fes"] == len(ev) == m + (m // 2) * t and res["generations"] == t
    assert res["best_e"] == ev[:budget].min()
    assert np.array_equal(best_x, evals[int(np.argmin(ev[:budget]))][1])
    assert np.array_equal(trace, [ev[: 200 * (k + 1)].min() for k in range(budget // 200)])


def test_cso_large_scale_fe_accounting():
    """The large-scale study's budget: a swarm of 300 and 1e6 evaluations is
    6665 iterations of 150 after the initial 300 (here at D = 3)."""
    d = _desc(O.ALGO_CSO, O.ELLIPSOID, 3, 300, 1_000_000, c1=0.1)
    res, trace, _ = O.run(d, SEED, ISEED, trace_len=5000)
    assert res["generations"] == 6665 and res["fes"] == 1_000_050
    assert np.all(np.diff(trace) <= 0)


def test_cso_update_draws_are_independent():
    """The three uniforms of a loser coordinate are independent: the squared
    residual of the move about its mean has expectation
    (v^2 + (x_w - x_l)^2 + phi^2 (xbar - x_l)^2) / 12 with no cross terms (a
    uniform shared by two terms would add 2 phi (x_w - x_l)(xbar - x_l) / 12)."""
    func, D, m, phi = O.ELLIPSOID, 50, 300, 1.0
    o, M, X, V, e = _cso_start(func, D, m)
    rows, ys = [], []
    for t in (1, 2, 3, 4):
        xbar = X.mean(axis=0)
        out = O.cso_iteration(func, -1e9, 1e9, o, M, X, V, e, phi, 6, SEED, t)
        w, l = out["winner"], out["loser"]
        if t >= 2:
            rows.append(np.stack([V[l].ravel(), (X[w] - X[l]).ravel(), (xbar - X[l]).ravel()], axis=1))
            ys.append((out["X"][l] - X[l]).ravel())
        X, V, e = out["X"], out["V"], out["e"]
    A, y = np.concatenate(rows), np.concatenate(ys)
    res = y - A @ np.array([0.5, 0.5, 0.5 * phi])
    B = np.stack([A[:, 0] ** 2, A[:, 1] ** 2, A[:, 2] ** 2, A[:, 1] * A[:, 2], A[:, 0] * A[:, 1],
                  A[:, 0] * A[:, 2]], axis=1)
    c, *_ = np.linalg.lstsq(B, res ** 2, rcond=None)
    c = 12 * c
    assert np.all(np.abs(c[:3] - [1, 1, phi ** 2]) < 0.3)
    assert np.all(np.abs(c[3:]) < 0.8)


# ------------------------------------------------------------------ JADE and the parameter observer

def test_jade_update_closed_form():
    """JADE's update on a hand-built success set: muCR moves a fraction c
    towards the plain mean of S_CR, muF towards the Lehmer mean of S_F."""
    # S_CR = {0.3, 0.9}: mean 0.6; S_F = {0.2, 0.6}: (0.04 + 0.36) / 0.8 = 0.5
    f, cr = O.jade_update(0.1, 0.5, 0.5, [0.2, 0.6], [0.3, 0.9])
    assert cr == pytest.approx(0.51, abs=1e-15)
    assert f == pytest.approx(0.5, abs=1e-15)
    # c = 1: the means themselves; a single success: its own values
    assert O.jade_update(1.0, 0.5, 0.5, [0.8], [0.1]) == pytest.approx((0.8, 0.1), abs=1e-15)
    # c = 0 or an empty set: unchanged
    assert O.jade_update(0.0, 0.3, 0.7, [0.9], [0.2]) == (0.3, 0.7)
    assert O.jade_update(0.1, 0.3, 0.7, [], []) == (0.3, 0.7)
    # unweighted: repeating a success does not move the means
    assert O.jade_update(0.5, 0.5, 0.5, [0.2, 0.6, 0.6, 0.2], [0.3, 0.9, 0.9, 0.3]) == \
        pytest.approx(O.jade_update(0.5, 0.5, 0.5, [0.2, 0.6], [0.3, 0.9]), abs=1e-15)


@pytest.mark.parametrize("c", [0.1, 1.0])
def test_jade_first_generation_is_shades_with_one_slot(c):
    """JADE's first generation draws from its one parameter pair exactly as
    SHADE with a one-slot memory (empty archive): the same trials, errors
    and population; its update then follows from SHADE's own F, CR and
    success flags by JADE's rule."""
    func, D, np_, p = O.ELLIPSOID, 10, 50, 0.05
    o, M, X, eX = _pop(func, D, np_)
    ref = O.shade_generation(func, LB, UB, o, M, X, eX, np.full(1, 0.5), np.full(1, 0.5), 0, p, 7, SEED, 1)
    jd = O.LShade(func, D, LB, UB, o, M, X, eX, H=1, r_arc=1.0)
    U, eU, ns = jd.jade_generation(p, c, 7, SEED, 1)
    assert np.array_equal(U, ref["U"]) and np.array_equal(eU, ref["eU"])
    assert np.array_equal(jd.X[:np_], ref["X"]) and np.array_equal(jd.eX[:np_], ref["eX"])
    succ = ref["eU"] < eX
    assert ns == int(succ.sum()) and ns > 0 and jd.na == ns
    SF, SCR = ref["F"][succ], ref["CR"][succ]
    mf, mcr, _ = jd.memory()
    assert mcr[0] == pytest.approx((1 - c) * 0.5 + c * SCR.mean(), rel=1e-14)
    assert mf[0] == pytest.approx((1 - c) * 0.5 + c * (SF ** 2).sum() / SF.sum(), rel=1e-14)


def test_jade_archive_bound_and_fixed_population():
    """Over many generations JADE keeps its population size, the archive
    stays within round(r_arc NP) and holds only former members, muF stays in
    (0, 1] and muCR in [0, 1]."""
    func, D, np_, r_arc = O.RASTRIGIN, 6, 30, 1.0
    o, M, X, eX = _pop(func, D, np_)
    jd = O.LShade(func, D, LB, UB, o, M, X, eX, H=1, r_arc=r_arc)
    seen = {tuple(x) for x in X}
    for t in range(1, 80):
        before = jd.eX[:np_].copy()
        U, eU, ns = jd.jade_generation(0.05, 0.1, 4, SEED, t)
        seen |= {tuple(x) for x in U}
        assert jd.np == np_
        assert np.all(jd.eX[:np_] <= before)
        assert jd.na <= O.lshade_archive_max(r_arc, np_)
        for a in jd.A[:jd.na]:
            assert tuple(a) in seen
        mf, mcr, _ = jd.memory()
        assert 0.0 < mf[0] <= 1.0 and 0.0 <= mcr[0] <= 1.0
    assert jd.na == O.lshade_archive_max(r_arc, np_)   # full after 79 generations


def _jade_desc(func, D, np_, budget, c=0.1, **kw):
    return _desc(O.ALGO_JADE, func, D, np_, budget, p=0.05, r_arc=1.0, c=c, H=1, np_min=4, **kw)


def test_jade_run_matches_generations_and_observer():
    """The run driver's JADE run is the generation function stepped by hand:
    same evaluations (count, best, trace) and observer rows equal to the
    parameter pair after each generation, NaN beyond."""
    func, D, np_, budget = O.GRIEWANK, 5, 20, 1000
    d = _jade_desc(func, D, np_, budget)
    gens = -(-(budget - np_) // np_)
    res, trace, _, mu = O.run(d, SEED, ISEED, trace_len=budget // 200, mu_len=gens + 3)
    o, M = O.instance(func, D, 0, ISEED)
    X = O.init_population(func, D, LB, UB, np_, 1, SEED)
    eX = O.errors(func, o, M, X)
    jd = O.LShade(func, D, LB, UB, o, M, X, eX, H=1, r_arc=1.0)
    evals = list(eX)
    rows = [(0.5, 0.5)]
    for t in range(1, gens + 1):
        U, eU, _ = jd.jade_generation(0.05, 0.1, 1, SEED, t)
        evals += list(eU)
        mf, mcr, _ = jd.memory()
        rows.append((mf[0], mcr[0]))
    e = np.array(evals)
    assert res["fes"] == len(e) and res["generations"] == gens
    assert res["best_e"] == e[:budget].min()
    assert np.array_equal(trace, [e[: 200 * (k + 1)].min() for k in range(budget // 200)])
    assert np.array_equal(mu[: gens + 1], np.array(rows))
    assert np.all(np.isnan(mu[gens + 1:]))
    # rows move: the parameters adapt
    assert len({tuple(r) for r in rows}) > gens // 2


def test_observer_rows_per_algorithm():
    """Observer rows: DE its fixed (F, CR); SHADE and PSODE the means of the
    memory slots, from (0.5, 0.5); PSO and CSO NaN; rows replayed from
    SHADE's generation function."""
    func, D, np_, budget = O.RASTRIGIN, 5, 20, 610
    gens = -(-(budget - np_) // np_)   # whole generations: 30
    _, _, _, mu = O.run(_desc(O.ALGO_DE, func, D, np_, budget, F=0.7, CR=0.3), SEED, ISEED, mu_len=gens + 2)
    assert np.array_equal(mu[: gens + 1], np.tile([0.7, 0.3], (gens + 1, 1)))
    assert np.all(np.isnan(mu[gens + 1:]))
    for algo in (O.ALGO_PSO, O.ALGO_CSO):
        _, _, _, mu = O.run(_desc(algo, func, D, np_, budget), SEED, ISEED, mu_len=5)
        assert np.all(np.isnan(mu))
    # SHADE: replay the memory by hand
    _, _, _, mu = O.run(_desc(O.ALGO_SHADE, func, D, np_, budget, H=3), SEED, ISEED, mu_len=gens + 1)
    o, M = O.instance(func, D, 0, ISEED)
    X = O.init_population(func, D, LB, UB, np_, 1, SEED)
    eX = O.errors(func, o, M, X)
    MF = np.full(3, 0.5); MCR = np.full(3, 0.5); pos = 0
    assert tuple(mu[0]) == (0.5, 0.5)
    for t in range(1, gens + 1):
        out = O.shade_generation(func, LB, UB, o, M, X, eX, MF, MCR, pos, 0.1, 1, SEED, t)
        MF, MCR, pos, X, eX = out["MF"], out["MCR"], out["pos"], out["X"], out["eX"]
        assert mu[t] == pytest.approx([MF.mean(), MCR.mean()], rel=1e-15)
    # PSODE: rows start at (0.5, 0.5) and stay in range
    _, _, _, mu = O.run(_desc(O.ALGO_PSODE, func, D, np_, budget), SEED, ISEED, mu_len=8)
    assert tuple(mu[0]) == (0.5, 0.5) and np.all((mu[1:] > 0) & (mu[1:] <= 1))


def test_observer_counts_a_terminal_cr_slot_as_zero():
    """L-SHADE's terminal CR slot (set when every successful CR was 0) gives
    CR = 0, and the observer counts it as 0: rows of a long L-SHADE run
    replayed from the generation function."""
    MF, MCR, pos = O.lshade_memory_update(np.full(2, 0.5), np.full(2, 0.5), 0, [0.4], [0.0], [1.0])
    assert MCR[0] < 0                               # terminal
    # a run found (by a scan over functions and run ids) to reach a
    # terminal slot in generation 47
    func, D, np_, gens, uid = O.ROSENBROCK, 4, 8, 100, 16
    d = _desc(O.ALGO_LSHADE, func, D, np_, np_ * (gens + 1), p=0.11, H=2, r_arc=1.0, np_min=np_, run_uid=uid)
    _, _, _, mu = O.run(d, SEED, ISEED, mu_len=gens + 1)
    o, M = O.instance(func, D, 0, ISEED)
    X = O.init_population(func, D, LB, UB, np_, uid, SEED)
    ls = O.LShade(func, D, LB, UB, o, M, X, O.errors(func, o, M, X), H=2, r_arc=1.0)
    terminal = 0
    for t in range(1, gens + 1):
        ls.generation(0.11, np_, uid, SEED, t)
        mf, mcr, _ = ls.memory()
        terminal += int(np.any(mcr < 0))
        assert mu[t] == pytest.approx([mf.mean(), np.where(mcr < 0, 0.0, mcr).mean()], rel=1e-15)
    assert terminal > 0


# ------------------------------------------------------------------ L-SHADE with restarts

def test_restart_population_k0_is_the_initial_population():
    X0 = O.init_population(O.RASTRIGIN, 7, LB, UB, 30, 5, SEED)
    assert np.array_equal(O.restart_population(O.RASTRIGIN, 7, LB, UB, 30, 5, SEED, 0), X0)
    seen = [X0]
    for k in (1, 2, 77):
        Xk = O.restart_population(O.RASTRIGIN, 7, LB, UB, 30, 5, SEED, k)
        assert np.all((Xk >= LB) & (Xk < UB))
        assert all(not np.any(Xk == S) for S in seen)   # fresh draws, no shared coordinate
        seen.append(Xk)


def test_converged_spread():
    assert O.converged([3.0, 3.0, 3.0], 0.0)
    assert O.converged([1.0, 1.5], 0.5) and not O.converged([1.0, 1.5], 0.49)
    assert not O.converged([1.0, np.nan], 1e300)
    assert not O.converged([np.inf, np.inf], 1e300)


def _rs_desc(func, D, np_, budget, tol, **kw):
    return _desc(O.ALGO_LSHADE_RS, func, D, np_, budget, p=0.11, r_arc=1.4, np_min=4, restart_tol=tol, **kw)


def test_lshade_restart_never_triggered_is_lshade():
    func, D, np_, budget = O.SCHWEFEL, 6, 40, 4000
    a = O.run(_rs_desc(func, D, np_, budget, -1.0), SEED, ISEED, trace_len=20, mu_len=200)
    b = O.run(_desc(O.ALGO_LSHADE, func, D, np_, budget, p=0.11, r_arc=1.4, np_min=4), SEED, ISEED,
              trace_len=20, mu_len=200)
    assert a[0] == b[0] and a[0]["restarts"] == 0
    for x, y in zip(a[1:], b[1:]):
        assert np.array_equal(x, y, equal_nan=True)


def _replay_restarts(func, D, np_, budget, tol, uid=1):
    """The restart rule recomposed from the generation function: returns
    (evaluations in order, generations, restarts, population sizes)."""
    o, M = O.instance(func, D, 0, ISEED)
    X = O.init_population(func, D, LB, UB, np_, uid, SEED)
    eX = O.errors(func, o, M, X)
    ls = O.LShade(func, D, LB, UB, o, M, X, eX, H=6, r_arc=1.4)
    evals, fe, fe_r, t, k, sizes = list(eX), np_, 0, 0, 0, []
    while fe < budget:
        t += 1
        n = ls.np
        nn = min(O.lshade_np(np_, 4, budget - fe_r, fe - fe_r + n), n)
        U, eU, _ = ls.generation(0.11, nn, uid, SEED, t)
        evals += list(eU)
        fe += n
        sizes.append(n)
        if fe < budget and O.converged(ls.eX[: ls.np], tol):
            k += 1
            fe_r = fe
            X = O.restart_population(func, D, LB, UB, np_, uid, SEED, k)
            eX = O.errors(func, o, M, X)
            ls = O.LShade(func, D, LB, UB, o, M, X, eX, H=6, r_arc=1.4)
            evals += list(eX)
            fe += np_
    return np.array(evals), t, k, sizes


@pytest.mark.parametrize("func,tol", [(O.ELLIPSOID, 1e300), (O.ELLIPSOID, 1e-6), (O.RASTRIGIN, 1e-3),
                                      (O.ROSENBROCK, 0.5)])
def test_lshade_restart_run_matches_replay(func, tol):
    """The run driver against the rule recomposed by hand: restart after a
    generation that leaves budget and a converged population, a fresh
    population k, memories and archive reset, the size schedule started
    over; the best and the trace span all restarts."""
    D, np_, budget = 4, 24, 24 * 250
    res, trace, _ = O.run(_rs_desc(func, D, np_, budget, tol), SEED, ISEED, trace_len=budget // 200)
    e, gens, k, sizes = _replay_restarts(func, D, np_, budget, tol)
    assert res["fes"] == len(e) and res["generations"] == gens and res["restarts"] == k
    assert res["best_e"] == e[:budget].min()
    assert np.array_equal(trace, [e[: 200 * (j + 1)].min() for j in range(budget // 200)])
    if tol > 1e100:
        assert k == gens - 1 or k == gens          # a restart after every generation with budget left
        assert all(s == np_ for s in sizes)          # the schedule never gets to shrink
    assert k > 0                                     # every case here restarts at least once


# ------------------------------------------------------------------ PSO attraction terms
# The update v = w v + c1 r1 (p - x) + c2 r2 (l - x) (the PSO module of Sec. 2.2,
# Listing 1's inertia velocity with the global best or a ring neighbourhood
# best l) is pinned from outside the oracle's code: by least squares on many
# particles (the coefficients of p - x and l - x are c1 E[r1] = c1 / 2 and
# c2 / 2, with c1 != c2 so that the two terms cannot be exchanged), and by
# inverting single moves for r1 and r2, which must be the uniforms of the
# documented Philox words (iteration t, particle i, tag PSO_R = 4, block
# j div 2: words 0 and 1 for the even coordinate, 2 and 3 for the odd one).

PSO_C1, PSO_C2 = 0.9, 2.1          # unequal, so that a p/l exchange shows
FAR = 1e9                           # a box and a velocity bound that never bind


def _u24_words(run_uid, t, i, block):
    w = O.philox([t, i, (4 << 24) | block, 0], [run_uid, SEED & 0xFFFFFFFF ^ (SEED >> 32)])
    return [int(x >> 8) * 2.0 ** -24 for x in w]


def _pso_move(topology, X, V, P, eP, t, uid=4, w=0.0):
    """One move of the oracle's inertia update (through the variant entry for
    the ring, the classic entry for the global best) with nothing clamped."""
    func = O.ELLIPSOID
    D = X.shape[1]
    o, M = O.instance(func, D, 0, ISEED)
    if topology == 0:
        st = dict(X=X, V=V, P=P, eX=np.zeros(X.shape[0]), eP=eP, g=int(np.argmin(eP)))
        out = O.pso_iteration(func, -FAR, FAR, o, M, st, w, PSO_C1, PSO_C2, FAR, uid, SEED, t)
        return out["X"], out["V"]
    Xn, Vn, *_ = O.pso_variant_iteration(func, -FAR, FAR, o, M, X, V, P, np.zeros(X.shape[0]), eP, 1, 0, w,
                                         PSO_C1, PSO_C2, FAR, uid, SEED, t)
    return Xn, Vn


@pytest.mark.parametrize("topology", [0, 1])
def test_pso_attraction_terms_by_regression(topology):
    """w = 0: the move is c1 r1 (p - x) + c2 r2 (l - x) per coordinate with
    r1, r2 independent uniforms, so least squares on (p - x, l - x) gives
    (c1 / 2, c2 / 2); swapping the two attractors or a sign fits far worse."""
    rng = np.random.default_rng(11)
    n, D = 2000, 12
    X = rng.uniform(-50, 50, (n, D))
    P = X + rng.normal(0, 30, (n, D))
    eP = rng.uniform(1, 2, n)
    V = rng.normal(0, 3, (n, D))          # w = 0: the old velocity must drop out
    Xn, Vn = _pso_move(topology, X, V, P, eP, t=5)
    if topology == 0:
        L = np.tile(P[int(np.argmin(eP))], (n, 1))
    else:
        L = np.empty_like(P)
        for i in range(n):
            nb = [(i - 1) % n, i, (i + 1) % n]
            L[i] = P[min(nb, key=lambda k: (eP[k], k))]
    y = Vn.ravel()
    assert np.allclose(Xn - X, Vn, rtol=1e-12, atol=1e-12)
    A = np.stack([(P - X).ravel(), (L - X).ravel()], axis=1)
    coef, res, *_ = np.linalg.lstsq(A, y, rcond=None)
    assert np.all(np.abs(coef - [PSO_C1 / 2, PSO_C2 / 2]) < 0.03), coef
    # residual variance of the two independent uniform terms: Var(r) = 1/12
    pred_var = (PSO_C1 ** 2 * np.mean((P - X) ** 2) + PSO_C2 ** 2 * np.mean((L - X) ** 2)) / 12
    assert res[0] / y.size == pytest.approx(pred_var, rel=0.1)


@pytest.mark.parametrize("topology", [0, 1])
def test_pso_attraction_draws_are_the_documented_words(topology):
    """Particle 1 of a three-particle swarm whose best personal best is
    particle 0's (its global best and its ring neighbourhood best).  With its
    position on that best, only c1 r1 (p - x) is left: r1 = v / (c1 (p - x))
    per coordinate.  With its position on its own personal best, only
    c2 r2 (l - x) is left.  Both must be the u24 uniforms of the documented
    Philox words, each coordinate its own pair (odd coordinates from words 2
    and 3 of the block)."""
    rng = np.random.default_rng(5)
    D, t, uid = 9, 7, 13
    P = rng.uniform(-60, 60, (3, D))
    eP = np.array([1.0, 2.0, 3.0])
    V = np.zeros((3, D))
    want_r1 = np.array([_u24_words(uid, t, 1, j // 2)[2 * (j % 2)] for j in range(D)])
    want_r2 = np.array([_u24_words(uid, t, 1, j // 2)[2 * (j % 2) + 1] for j in range(D)])
    assert np.all(want_r1 != want_r2)
    # state A: x_1 = l = P_0, so l - x vanishes
    X = rng.uniform(-60, 60, (3, D)); X[1] = P[0]
    _, Vn = _pso_move(topology, X, V, P, eP, t, uid)
    r1 = Vn[1] / (PSO_C1 * (P[1] - X[1]))
    assert np.allclose(r1, want_r1, rtol=1e-12, atol=0), (r1, want_r1)
    # state B: x_1 = p_1, so p - x vanishes
    X = rng.uniform(-60, 60, (3, D)); X[1] = P[1]
    _, Vn = _pso_move(topology, X, V, P, eP, t, uid)
    r2 = Vn[1] / (PSO_C2 * (P[0] - X[1]))
    assert np.allclose(r2, want_r2, rtol=1e-12, atol=0), (r2, want_r2)


def test_pso_inertia_term_is_w_v():
    """With the particle on both attractors (x = p = l) only w v is left."""
    D = 6
    P = np.tile(np.linspace(-3, 3, D), (3, 1))
    X = P.copy()
    eP = np.array([1.0, 1.0, 1.0])
    V = np.random.default_rng(2).normal(0, 2, (3, D))
    for topology in (0, 1):
        Xn, Vn = _pso_move(topology, X, V, P, eP, t=3, w=0.7298)
        assert np.allclose(Vn, 0.7298 * V, rtol=1e-15, atol=0)
        assert np.allclose(Xn - X, 0.7298 * V, rtol=1e-13, atol=1e-15)
