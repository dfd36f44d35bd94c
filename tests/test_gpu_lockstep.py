"""Point-by-point parity of the fused run kernels with the FP64 oracle, one
generation at a time.

Every fused family (DE rand/1/bin; SHADE; L-SHADE, JADE and L-SHADE-Restart
with archive and population reduction; PSO with the global-best and ring
topologies and the inertia and spherical updates; PSODE) runs in one
sevo_run_snapshot call per (team, placement): for each case a run stopped
after t - 1 generations and the same run stopped after t generations
(max_generations), both writing their final state.  The oracle then makes
generation t from the GPU's state after t - 1 (the population widened
exactly to double, its float errors, memories, archive, velocities and
personal bests) with the same Philox draws (Sec. 2.2 Listing 1's modules,
Sec. 4 Listing 4's hybrid; Sec. 2.4's independent runs), and the GPU's state
after t is compared with it:

* trials and moves: every coordinate to float rounding (a wrong donor,
  pbest, archive member or attraction term moves it by O(1) or more);
  coordinates the crossover leaves to the parent are the parent's bits;
* errors: within the evaluation tolerance of the oracle's error at the
  GPU's own point;
* decisions (selection, personal bests, global best, ranking ties): the
  GPU's own rule on its own errors, bit for bit, and the oracle's decision
  the same except where the two errors lie within the evaluation tolerance
  of each other (none of the cases here has such a near tie; the test
  reports it if one appears);
* archive members bit for bit (they are copies of parents), memory slots to
  1e-3 (the weights are improvements, computed from float errors on the GPU
  and from the oracle's double errors), the next memory slot, population
  size, archive size and global-best index exactly.

Also here: runs on a constant function (M = 0, every error exactly 0),
where every decision is a tie -- DE trials replace their parents, SHADE's
ranking and L-SHADE's reduction follow the index, pbest stays, gbest is 0 --
and free runs of three generations against the oracle's own run (best
point, its error, the trace).
"""
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.tolerance import tolerance

torch = pytest.importorskip("torch")
from paper_2505_17430_amd import sevo as S  # noqa: E402

pytestmark = pytest.mark.gpu
SEED, ISEED = W.BASE_SEED, W.INSTANCE_SEED
LB, UB = W.LB, W.UB
W_SPSO, C_SPSO = 1.0 / (2.0 * math.log(2.0)), 0.5 + math.log(2.0)

# generations compared one at a time (runs stopped after t - 1 and t)
GENS = (1, 2, 3, 8)
CAPS = sorted({c for t in GENS for c in (t - 1, t)})

# family name -> run settings (algorithm, and what differs from the defaults)
FAMILIES = {
    "de": dict(algo=S.ALGO_DE),
    "shade": dict(algo=S.ALGO_SHADE),
    "lshade": dict(algo=S.ALGO_LSHADE, p=0.11, r_arc=2.6),
    "jade": dict(algo=S.ALGO_JADE, p=0.05, r_arc=1.0, c=0.1),
    "lshade_rs": dict(algo=S.ALGO_LSHADE_RS, p=0.11, r_arc=2.6, restart_tol=-1.0),
    "pso": dict(algo=S.ALGO_PSO),
    "pso_ring": dict(algo=S.ALGO_PSO, topology=1),
    "pso_sph": dict(algo=S.ALGO_PSO, velocity=1),
    "pso_sph_ring": dict(algo=S.ALGO_PSO, velocity=1, topology=1),
    "psode": dict(algo=S.ALGO_PSODE, velocity=1, topology=1),
    "psode_gbest": dict(algo=S.ALGO_PSODE),
}
DIMS = (10, 30, 50, 100)
# (team, placement) forced through the library's environment switches; the
# default placement keeps a population on chip when it fits
CONFIGS = {"wave_onchip": ("wave", None), "wave_ws": ("wave", "workspace"),
           "block_onchip": ("block", None), "block_ws": ("block", "workspace")}
FUNC_OF_DIM = {10: S.RASTRIGIN, 30: S.SCHWEFEL, 50: S.ELLIPSOID, 100: S.ACKLEY}
OTHER_FUNC = {10: S.GRIEWANK, 30: S.ROSENBROCK, 50: S.ACKLEY, 100: S.ELLIPSOID}


def say(*a):
    print(*a, flush=True)


def settings(fam):
    d = dict(F=0.5, CR=0.9, w=0.7298, c1=1.49618, c2=1.49618, vmax=0.2 * (UB - LB), p=0.1, H=6,
             r_arc=2.6, np_min=4, topology=0, velocity=0, c=0.1, restart_tol=0.0)
    d.update({k: v for k, v in FAMILIES[fam].items() if k != "algo"})
    if d["velocity"] == 1:     # SPSO-2011 constants
        d["w"], d["c1"], d["c2"] = W_SPSO, C_SPSO, C_SPSO
    return FAMILIES[fam]["algo"], d


def run_desc(fam, func, dim, np_, budget, uid, cap, inst=0):
    """A run stopped after `cap` generations; cap 0 is the initial
    population alone (budget NP: max_generations 0 means no limit); cap
    None runs to the budget."""
    algo, d = settings(fam)
    if cap == 0:
        budget = np_
    cap = cap or 0
    return S.RunDesc(S.problem(func, dim), inst, uid, algo, np_, budget, d["F"], d["CR"], d["w"], d["c1"],
                     d["c2"], d["vmax"], d["p"], d["H"], d["r_arc"], d["np_min"], d["topology"], d["velocity"],
                     cap, d["c"], d["restart_tol"])


def odesc(d):
    return dict(algo=d.algo, func=d.prob.func, dim=d.prob.dim, lb=d.prob.lb, ub=d.prob.ub, instance=d.instance,
                run_uid=d.run_uid, np=d.np, budget=d.budget, F=d.F, CR=d.CR, w=d.w, c1=d.c1, c2=d.c2,
                vmax=d.vmax, p=d.p, H=d.H, r_arc=d.r_arc, np_min=d.np_min, topology=d.topology,
                velocity=d.velocity, c=d.c, restart_tol=d.restart_tol)


def sizes(fam, dim, team):
    """(np, budget) of a case: wave teams carry at most 64 individuals;
    L-SHADE's budget is short so that its population shrinks every
    generation."""
    np_ = {10: 40, 30: 60, 50: 48, 100: 64}[dim] if team == "wave" else {10: 100, 30: 64, 50: 130, 100: 90}[dim]
    if fam in ("lshade", "lshade_rs"):
        return np_, 16 * np_
    return np_, 50 * np_


def gpu_snapshot(ctx, descs, trace_len=0):
    n = len(descs)
    mnp = max(d.np for d in descs)
    mdim = max(d.prob.dim for d in descs)
    marc = max([int(math.floor(d.r_arc * d.np + 0.5)) for d in descs if d.algo in (S.ALGO_LSHADE, S.ALGO_JADE,
                                                                         S.ALGO_LSHADE_RS)] + [1])
    f = dict(device="cuda")
    st = dict(max_np=mnp, max_dim=mdim, max_arc=marc,
              x=torch.full((n, mdim, mnp), float("nan"), **f), e=torch.full((n, mnp), float("nan"), **f),
              u=torch.full((n, mdim, mnp), float("nan"), **f), eu=torch.full((n, mnp), float("nan"), **f),
              v=torch.full((n, mdim, mnp), float("nan"), **f), p=torch.full((n, mdim, mnp), float("nan"), **f),
              ep=torch.full((n, mnp), float("nan"), **f), memory=torch.full((n, 32), float("nan"), **f),
              archive=torch.full((n, mdim, marc), float("nan"), **f),
              counts=torch.full((n, 4), -1, dtype=torch.int32, **f))
    res = torch.zeros((n, 32), dtype=torch.uint8, **f)
    tr = torch.full((max(n * trace_len, 1),), -7.0, **f)
    bx = torch.zeros((n, mdim), dtype=torch.float64, **f)
    ctx.run_snapshot(descs, res, st, trace=tr if trace_len else None, trace_len=trace_len, best_x=bx,
                     max_dim=mdim)
    torch.cuda.synchronize()
    out = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in st.items()}
    raw = res.cpu().numpy().tobytes()
    out["res"] = []
    for r in range(n):
        rr = S.RunResult.from_buffer_copy(raw[r * 32:(r + 1) * 32])
        out["res"].append(dict(best_e=rr.best_e, best_e32=rr.best_e32, success=rr.success, fes=rr.fes,
                               generations=rr.generations, restarts=rr.restarts))
    out["trace"] = tr.cpu().numpy()[: n * trace_len].reshape(n, trace_len)
    out["best_x"] = bx.cpu().numpy()
    return out


def run_state(snap, r, d):
    """The state of run r of a snapshot, individual-major, in double."""
    D = d.prob.dim
    c = snap["counts"][r]
    n = int(c[0])
    s = dict(np=n, na=int(c[1]), pos=int(c[2]), g=int(c[3]), res=snap["res"][r],
             X=snap["x"][r, :D, :n].T.astype(np.float64), e=snap["e"][r, :n].astype(np.float64),
             U=snap["u"][r, :D, :].T.astype(np.float64), eu=snap["eu"][r].astype(np.float64),
             V=snap["v"][r, :D, :n].T.astype(np.float64), P=snap["p"][r, :D, :n].T.astype(np.float64),
             eP=snap["ep"][r, :n].astype(np.float64),
             MF=snap["memory"][r, :16].astype(np.float64), MCR=snap["memory"][r, 16:].astype(np.float64),
             A=snap["archive"][r, :D, :int(c[1])].T.astype(np.float64))
    return s


def key(e):
    e = np.asarray(e, dtype=np.float64)
    return np.where(np.isnan(e), np.inf, e)


# ---------------------------------------------------------------------------
# the GPU side: one call per (team, placement), every family and dimension

def cases(team):
    out = []
    uid = 9000
    for fam in FAMILIES:
        for dim in DIMS:
            np_, budget = sizes(fam, dim, team)
            out.append((fam, dim, FUNC_OF_DIM[dim], np_, budget, uid))
            uid += 1
    return out


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    c = S.Context(0, SEED, ISEED)
    yield c
    c.close()


_SNAPS = {}


def snapshots(ctx, cfg):
    """Run (once per module) every case of a configuration at every cap."""
    if cfg in _SNAPS:
        return _SNAPS[cfg]
    team, place = CONFIGS[cfg]
    old = {k: os.environ.get(k) for k in ("SEVO_RUN_TEAM", "SEVO_RUN_PLACEMENT")}
    os.environ["SEVO_RUN_TEAM"] = team
    if place:
        os.environ["SEVO_RUN_PLACEMENT"] = place
    else:
        os.environ.pop("SEVO_RUN_PLACEMENT", None)
    try:
        descs, index = [], {}
        for (fam, dim, func, np_, budget, uid) in cases(team):
            for cap in CAPS:
                index[(fam, dim, cap)] = len(descs)
                descs.append(run_desc(fam, func, dim, np_, budget, uid, cap))
        say(f"  lockstep snapshot {cfg}: {len(descs)} runs")
        snap = gpu_snapshot(ctx, descs)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    _SNAPS[cfg] = (descs, index, snap)
    return _SNAPS[cfg]


# ---------------------------------------------------------------------------
# the oracle's generation t from the GPU's state after t - 1

def oracle_step(fam, d, prev, o, M, t):
    func, D = d.prob.func, d.prob.dim
    algo = d.algo
    X, e = prev["X"], prev["e"]
    if algo == S.ALGO_DE:
        out = O.de_generation(func, LB, UB, o, M, X, e, d.F, d.CR, d.run_uid, SEED, t)
        return dict(U=out["U"], eU=out["eU"], X=out["X"], e=out["eX"], mask=out["mask"], rep=out["replaced"])
    if algo == S.ALGO_SHADE:
        H = d.H
        out = O.shade_generation(func, LB, UB, o, M, X, e, prev["MF"][:H], prev["MCR"][:H], prev["pos"], d.p,
                                 d.run_uid, SEED, t)
        return dict(U=out["U"], eU=out["eU"], X=out["X"], e=out["eX"], mask=out["mask"], rep=out["replaced"],
                    MF=out["MF"], MCR=out["MCR"], pos=out["pos"])
    if algo in (S.ALGO_LSHADE, S.ALGO_JADE, S.ALGO_LSHADE_RS):
        H = 1 if algo == S.ALGO_JADE else d.H
        L = O.LShade(func, D, LB, UB, o, M, X, e, H=H, r_arc=d.r_arc)
        L.set_state(prev["A"], prev["MF"][:H], prev["MCR"][:H], prev["pos"])
        n = prev["np"]
        if algo == S.ALGO_JADE:
            U, eU, _ = L.jade_generation(d.p, d.c, d.run_uid, SEED, t)
        else:
            fe = prev["res"]["fes"]
            nn = min(O.lshade_np(d.np, d.np_min, d.budget, fe + n), n)
            U, eU, _ = L.generation(d.p, nn, d.run_uid, SEED, t)
        MF, MCR, pos = L.memory()
        return dict(U=U, eU=eU, X=L.X[: L.np].copy(), e=L.eX[: L.np].copy(), np=L.np, A=L.archive(), na=L.na,
                    MF=MF, MCR=MCR, pos=pos)
    if algo == S.ALGO_PSO:
        if d.topology == 0 and d.velocity == 0:
            out = O.pso_iteration(func, LB, UB, o, M, dict(X=X, V=prev["V"], P=prev["P"], eP=prev["eP"],
                                                           g=prev["g"]), d.w, d.c1, d.c2, d.vmax, d.run_uid,
                                  SEED, t)
            return dict(X=out["X"], V=out["V"], P=out["P"], e=out["eX"], eP=out["eP"], g=out["g"])
        Xn, Vn, Pn, eXn, ePn, _ = O.pso_variant_iteration(func, LB, UB, o, M, X, prev["V"], prev["P"], e,
                                                          prev["eP"], d.topology, d.velocity, d.w, d.c1, d.c2,
                                                          d.vmax, d.run_uid, SEED, t)
        g = int(np.argmin(key(ePn)))
        return dict(X=Xn, V=Vn, P=Pn, e=eXn, eP=ePn, g=g)
    if algo == S.ALGO_PSODE:
        H = d.H
        out = O.psode_generation(func, LB, UB, o, M, X, e, prev["V"], prev["MF"][:H], prev["MCR"][:H],
                                 prev["pos"], d.topology, d.velocity, d.w, d.c1, d.c2, d.vmax, d.p, d.run_uid,
                                 SEED, t)
        return dict(U=out["U"], eU=out["eU"], X=out["X"], e=out["eX"], V=out["V"], MF=out["MF"],
                    MCR=out["MCR"], pos=out["pos"], g=int(np.argmin(key(out["eX"]))))
    raise ValueError(algo)


def pos_tol(fam):
    """Per-coordinate bound for positions computed from the same float
    inputs in float (GPU) and double (oracle): a few roundings of values up
    to a few hundred (ulp(256) = 3.1e-5), more for the spherical update's
    sqrt/log/sincos chain."""
    if "sph" in fam or fam == "psode":
        return 2e-3
    if fam.startswith("pso"):
        return 5e-4
    return 2e-4


def check_errors(func, o, M, Xg, eg, what):
    """GPU errors of its own points against the oracle's error there."""
    if Xg.shape[0] == 0:
        return
    eo = O.errors(func, o, M, Xg)
    tol = tolerance(func, o, M, Xg.T, eo)
    bad = np.abs(eg - eo) > tol
    assert not bad.any(), (what, np.flatnonzero(bad)[:5], eg[bad][:5], eo[bad][:5])


def compare_generation(fam, d, prev, cur, want, o, M, lb=LB, ub=UB, tol_fn=check_errors):
    func, D = d.prob.func, d.prob.dim
    n_old = prev["np"]
    ptol = pos_tol(fam)
    near = []
    assert cur["res"]["generations"] == prev["res"]["generations"] + 1
    has_trials = d.algo != S.ALGO_PSO
    if has_trials:
        Ug, eUg = cur["U"][:n_old], cur["eu"][:n_old]
        dU = np.abs(Ug - want["U"])
        assert dU.max() <= ptol, (fam, "trials", dU.max(), np.unravel_index(dU.argmax(), dU.shape))
        if "mask" in want:
            # coordinates left to the parent (and not repaired) are its bits
            keep = ~want["mask"] & (want["U"] == prev["X"])
            assert np.array_equal(Ug[keep], prev["X"][keep]), fam
        tol_fn(func, o, M, Ug, eUg, (fam, "trial errors"))
    if d.algo in (S.ALGO_DE, S.ALGO_SHADE):
        # selection on the GPU's own errors: e(u) <= e(x), ties to the trial
        rep = key(eUg) <= key(prev["e"])
        assert np.array_equal(cur["X"], np.where(rep[:, None], Ug, prev["X"])), fam
        assert np.array_equal(cur["e"], np.where(rep, eUg, prev["e"])), fam
        diff = rep != want["rep"]
        for i in np.flatnonzero(diff):
            t_i = tolerance(func, o, M, Ug[i][:, None], np.array([want["eU"][i]]))[0]
            assert abs(eUg[i] - prev["e"][i]) <= 2 * t_i, (fam, "selection", i)
            near.append(i)
    if d.algo == S.ALGO_PSO:
        # personal bests on the GPU's own errors (strict), global best the
        # lowest index of the least error
        dX = np.abs(cur["X"] - want["X"])
        assert dX.max() <= ptol, (fam, "positions", dX.max())
        at_bound = (np.minimum(np.abs(cur["X"] - lb), np.abs(cur["X"] - ub)) <= 1e-3) | \
                   (np.minimum(np.abs(want["X"] - lb), np.abs(want["X"] - ub)) <= 1e-3)
        dV = np.where(at_bound, 0.0, np.abs(cur["V"] - want["V"]))
        assert dV.max() <= ptol, (fam, "velocities", dV.max())
        tol_fn(func, o, M, cur["X"], cur["e"], (fam, "errors"))
        imp = key(cur["e"]) < key(prev["eP"])
        assert np.array_equal(cur["P"], np.where(imp[:, None], cur["X"], prev["P"])), fam
        assert np.array_equal(cur["eP"], np.where(imp, cur["e"], prev["eP"])), fam
        oimp = key(want["e"]) < key(prev["eP"])
        for i in np.flatnonzero(imp != oimp):
            t_i = tolerance(func, o, M, cur["X"][i][:, None], np.array([want["e"][i]]))[0]
            assert abs(cur["e"][i] - prev["eP"][i]) <= 2 * t_i, (fam, "pbest", i)
            near.append(i)
        if d.topology == 0:
            assert cur["g"] == int(np.argmin(key(cur["eP"]))), fam
            if not near:
                assert cur["g"] == want["g"], fam
        return near
    if d.algo == S.ALGO_PSODE:
        dX = np.abs(cur["X"] - want["X"])
        assert dX.max() <= ptol, (fam, "population", dX.max())
        dV = np.abs(cur["V"] - want["V"])
        assert dV.max() <= ptol, (fam, "velocities", dV.max())
        tol_fn(func, o, M, cur["X"], cur["e"], (fam, "errors"))
        if d.topology == 0:
            assert cur["g"] == int(np.argmin(key(cur["e"]))), fam
    if d.algo in (S.ALGO_LSHADE, S.ALGO_JADE, S.ALGO_LSHADE_RS):
        assert cur["np"] == want["np"], (fam, cur["np"], want["np"])
        assert cur["na"] == want["na"], (fam, cur["na"], want["na"])
        # archive members are copies of parents: bit for bit
        assert np.array_equal(cur["A"], want["A"]), fam
        dX = np.abs(cur["X"] - want["X"])
        assert dX.max() <= ptol, (fam, "population", dX.max())
        tol_fn(func, o, M, cur["X"], cur["e"], (fam, "errors"))
    if d.algo == S.ALGO_DE:
        dX = np.abs(cur["X"] - want["X"])
        assert dX.max() <= ptol, fam
    if d.algo in (S.ALGO_SHADE, S.ALGO_LSHADE, S.ALGO_JADE, S.ALGO_LSHADE_RS, S.ALGO_PSODE):
        H = 1 if d.algo == S.ALGO_JADE else d.H
        assert cur["pos"] == want["pos"], (fam, "memory slot")
        assert np.allclose(cur["MF"][:H], want["MF"], rtol=1e-3, atol=1e-5), (fam, cur["MF"][:H], want["MF"])
        assert np.allclose(cur["MCR"][:H], want["MCR"], rtol=1e-3, atol=1e-5), (fam, cur["MCR"][:H], want["MCR"])
    return near


@pytest.mark.parametrize("cfg", list(CONFIGS))
@pytest.mark.parametrize("fam", list(FAMILIES))
def test_lockstep_generations_match_oracle(ctx, cfg, fam):
    descs, index, snap = snapshots(ctx, cfg)
    near_all = 0
    for dim in DIMS:
        for t in GENS:
            dp = descs[index[(fam, dim, t - 1)]]
            dc = descs[index[(fam, dim, t)]]
            prev = run_state(snap, index[(fam, dim, t - 1)], dp)
            cur = run_state(snap, index[(fam, dim, t)], dc)
            assert prev["res"]["generations"] == t - 1 and cur["res"]["generations"] == t, (dim, t)
            o, M = O.instance(dc.prob.func, dim, dc.instance, ISEED)
            want = oracle_step(fam, dc, prev, o, M, t)
            near = compare_generation(fam, dc, prev, cur, want, o, M)
            near_all += len(near)
    say(f"  {cfg} {fam}: generations {GENS} at D = {DIMS} match; near ties {near_all}")


# ---------------------------------------------------------------------------
# every decision a tie: a constant function (M = 0)

TIE_FAMS = ("de", "shade", "lshade", "jade", "pso", "pso_ring", "psode_gbest")


@pytest.mark.parametrize("team", ["wave", "block"])
def test_ties_on_a_constant_function(ctx, team, monkeypatch):
    monkeypatch.setenv("SEVO_RUN_TEAM", team)
    dim, func, inst = 10, S.RASTRIGIN, 7
    prob = S.problem(func, dim)
    o = np.zeros(dim)
    M = np.zeros((dim, dim))
    c = S.Context(0, SEED, ISEED)
    try:
        c.set_instance(prob, inst, o, M)
        descs, index = [], {}
        for k, fam in enumerate(TIE_FAMS):
            np_ = 40 if fam != "lshade" else 48
            for cap in (0, 1, 2):
                index[(fam, cap)] = len(descs)
                descs.append(run_desc(fam, func, dim, np_, 12 * np_, 9500 + k, cap, inst=inst))
        snap = gpu_snapshot(c, descs)
    finally:
        c.close()
    for fam in TIE_FAMS:
        for t in (1, 2):
            dp, dc = descs[index[(fam, t - 1)]], descs[index[(fam, t)]]
            prev = run_state(snap, index[(fam, t - 1)], dp)
            cur = run_state(snap, index[(fam, t)], dc)
            assert np.all(cur["e"] == 0.0) and np.all(prev["e"] == 0.0), fam
            want = oracle_step(fam, dc, prev, o, M, t)

            def zero_errors(func_, o_, M_, Xg, eg, what):
                assert np.all(eg == 0.0), what

            near = compare_generation(fam, dc, prev, cur, want, o, M, tol_fn=zero_errors)
            assert not near, fam
            if fam in ("de", "shade", "psode_gbest"):
                # every trial ties its parent and replaces it
                n = prev["np"]
                assert np.array_equal(cur["X"] if fam != "psode_gbest" else cur["X"], cur["U"][:n]), fam
            if fam in ("shade", "lshade", "jade", "psode_gbest"):
                # no strict improvement: the memory and its slot stay
                H = 1 if fam == "jade" else dc.H
                assert np.array_equal(cur["MF"][:H], prev["MF"][:H]) and cur["pos"] == prev["pos"], fam
            if fam == "lshade":
                # the reduction keeps the lowest indices, in order; no archive
                assert cur["na"] == 0
                assert np.array_equal(cur["X"], cur["U"][: cur["np"]]), fam
            if fam in ("pso", "pso_ring"):
                assert np.array_equal(cur["P"], prev["P"]) and cur["g"] == 0, fam
    say(f"  {team}: ties resolved as the rules say for {TIE_FAMS}")


# ---------------------------------------------------------------------------
# free runs of three generations against the oracle's own run

@pytest.mark.parametrize("fam", list(FAMILIES))
def test_free_runs_follow_oracle(ctx, fam):
    """Budget NP (1 + 3): the GPU and the oracle each run three generations
    (L-SHADE: as many as its shrinking population fits in that budget)
    from the same initial population (the oracle in double throughout): the
    best point agrees to float rounding, the GPU's error of its best point
    is within the evaluation tolerance of the oracle's error there and the
    oracle's best, and the trace follows."""
    descs = []
    for k, dim in enumerate(DIMS):
        func = OTHER_FUNC[dim]
        np_ = {10: 30, 30: 50, 50: 64, 100: 120}[dim]
        mult = 2 if fam == "psode" or fam == "psode_gbest" else 1
        descs.append(run_desc(fam, func, dim, np_, np_ * (1 + 3 * mult), 9700 + k, None))
    tl = max(d.budget for d in descs) // 200
    snap = gpu_snapshot(ctx, descs, trace_len=tl)
    for r, d in enumerate(descs):
        g = snap["res"][r]
        o_res, otr, obx = O.run(odesc(d), SEED, ISEED, trace_len=tl)
        assert g["fes"] == o_res["fes"] and g["generations"] == o_res["generations"], (fam, d.prob.dim)
        if fam not in ("lshade", "lshade_rs"):   # their shrinking population makes more generations
            assert g["generations"] == 3, (fam, d.prob.dim)
        D = d.prob.dim
        bx = snap["best_x"][r][:D]
        oi, oM = O.instance(d.prob.func, D, d.instance, ISEED)
        e_at = O.error(d.prob.func, oi, oM, bx)
        tol = tolerance(d.prob.func, oi, oM, bx[:, None], np.array([e_at]))[0]
        assert abs(g["best_e32"] - e_at) <= tol, (fam, D, g["best_e32"], e_at, tol)
        assert e_at == pytest.approx(o_res["best_e"], rel=1e-4, abs=1e-6), (fam, D)
        assert np.allclose(bx, obx, rtol=0, atol=2e-3), (fam, D, np.abs(bx - obx).max())
        n_rec = min(g["fes"] // 200, tl)
        assert np.allclose(snap["trace"][r][:n_rec], otr[:n_rec], rtol=1e-4, atol=1e-6), (fam, D)
