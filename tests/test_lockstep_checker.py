"""The power of the generation-by-generation comparison in
test_gpu_lockstep.py, shown on the CPU: the oracle plays the GPU.

A state after generation t - 1 comes from the oracle's initial population.
The oracle makes generation t from it; that result, rounded to float the way
the GPU stores it and with the GPU's own selection on its own float errors,
must pass the comparison.  The same result with one planted mistake must
fail it:

* DE: one individual's trial built from the donor after r1 (an off-by-one
  in the donor gather), or one selection decision flipped;
* SHADE: the next memory slot off by one, or one trial's pbest member
  replaced by another individual;
* PSO: one particle moved with its velocity's sign flipped.

Each mistake is planted in the oracle's output, never in GPU code
(Sec. 2.2 Listing 1's modules; Sec. 2.4's independent runs).
"""
import numpy as np
import pytest

import oracle as O
from tests.test_gpu_lockstep import (ISEED, LB, SEED, UB, compare_generation, key, oracle_step, run_desc,
                                     S)

F32 = np.float32


def f32(a):
    return np.asarray(a, dtype=np.float64).astype(F32).astype(np.float64)


def start(fam, func, dim, np_, uid):
    """The state after generation 0 (the initial population and its errors)
    and the descriptor of a run stopped after generation 1."""
    d = run_desc(fam, func, dim, np_, 50 * np_, uid, 1)
    o, M = O.instance(func, dim, 0, ISEED)
    X = f32(O.init_population(func, dim, LB, UB, np_, uid, SEED))
    e = f32(O.errors(func, o, M, X))
    prev = dict(np=np_, X=X, e=e, res=dict(generations=0, fes=np_), MF=np.full(16, 0.5), MCR=np.full(16, 0.5),
                pos=0)
    if d.algo == S.ALGO_PSO:
        prev.update(V=np.zeros_like(X), P=X.copy(), eP=e.copy(), g=int(np.argmin(key(e))))
    return d, o, M, prev


def gpu_like_de(fam, d, o, M, prev, want, U=None):
    """What the fused kernel stores after the generation: float trials,
    float errors of its own points, and its selection on them."""
    Ug = f32(want["U"] if U is None else U)
    eUg = f32(O.errors(d.prob.func, o, M, Ug))
    rep = key(eUg) <= key(prev["e"])
    cur = dict(np=prev["np"], res=dict(generations=1, fes=2 * prev["np"]), U=Ug, eu=eUg,
               X=np.where(rep[:, None], Ug, prev["X"]), e=np.where(rep, eUg, prev["e"]))
    if fam == "shade":
        cur.update(MF=np.concatenate([want["MF"], np.zeros(16 - len(want["MF"]))]),
                   MCR=np.concatenate([want["MCR"], np.zeros(16 - len(want["MCR"]))]), pos=want["pos"])
    return cur


def test_de_comparison_passes_the_oracle_and_catches_planted_mistakes():
    d, o, M, prev = start("de", S.RASTRIGIN, 10, 40, 4101)
    want = oracle_step("de", d, prev, o, M, 1)
    compare_generation("de", d, prev, gpu_like_de("de", d, o, M, prev, want), want, o, M)

    # the donor after r1 for one individual whose trial takes mutant coordinates
    out = O.de_generation(d.prob.func, LB, UB, o, M, prev["X"], prev["e"], d.F, d.CR, d.run_uid, SEED, 1)
    i = int(np.flatnonzero(out["mask"].any(axis=1))[0])
    r1, r2, r3 = out["donors"][i, :3]
    bad_r1 = (r1 + 1) % d.np
    U = want["U"].copy()
    X = prev["X"]
    for j in np.flatnonzero(out["mask"][i]):
        v = X[bad_r1, j] + d.F * (X[r2, j] - X[r3, j])
        U[i, j] = (X[i, j] + LB) / 2 if v < LB else (X[i, j] + UB) / 2 if v > UB else v
    with pytest.raises(AssertionError):
        compare_generation("de", d, prev, gpu_like_de("de", d, o, M, prev, want, U), want, o, M)

    # one selection flipped: a parent kept although its trial is no worse
    cur = gpu_like_de("de", d, o, M, prev, want)
    rep = key(cur["eu"]) <= key(prev["e"])
    k = int(np.flatnonzero(rep)[0])
    cur["X"][k], cur["e"][k] = prev["X"][k], prev["e"][k]
    with pytest.raises(AssertionError):
        compare_generation("de", d, prev, cur, want, o, M)


def test_shade_comparison_catches_a_wrong_memory_slot_and_a_wrong_pbest():
    d, o, M, prev = start("shade", S.SCHWEFEL, 30, 60, 4102)
    want = oracle_step("shade", d, prev, o, M, 1)
    compare_generation("shade", d, prev, gpu_like_de("shade", d, o, M, prev, want), want, o, M)

    cur = gpu_like_de("shade", d, o, M, prev, want)
    cur["pos"] = (want["pos"] + 1) % d.H
    with pytest.raises(AssertionError):
        compare_generation("shade", d, prev, cur, want, o, M)

    # one trial whose mutant coordinates moved by (x_q - x_pbest) F for a
    # wrong pbest member q: current-to-pbest/1 takes F (x_pbest - x_i)
    mask = want["mask"]
    i = int(np.flatnonzero(mask.any(axis=1))[0])
    best = int(np.argmin(key(prev["e"])))
    q = (best + 1) % d.np
    U = want["U"].copy()
    shift = 0.5 * (prev["X"][q] - prev["X"][best])
    U[i] = np.where(mask[i], np.clip(U[i] + shift, LB, UB), U[i])
    assert np.abs(U[i] - want["U"][i]).max() > 1.0
    with pytest.raises(AssertionError):
        compare_generation("shade", d, prev, gpu_like_de("shade", d, o, M, prev, want, U), want, o, M)


def test_pso_comparison_catches_a_flipped_velocity():
    d, o, M, prev = start("pso", S.ELLIPSOID, 30, 40, 4103)
    # generation 1 from a state with nonzero velocities: run the oracle's
    # first iteration, then compare the second
    s1 = oracle_step("pso", d, prev, o, M, 1)
    prev2 = dict(np=prev["np"], res=dict(generations=1, fes=2 * prev["np"]), X=f32(s1["X"]), e=f32(s1["e"]),
                 V=f32(s1["V"]), P=f32(s1["P"]), eP=f32(s1["eP"]), g=s1["g"])
    want = oracle_step("pso", d, prev2, o, M, 2)

    def gpu_like(Xn, Vn):
        Xg, Vg = f32(Xn), f32(Vn)
        eg = f32(O.errors(d.prob.func, o, M, Xg))
        imp = key(eg) < key(prev2["eP"])
        eP = np.where(imp, eg, prev2["eP"])
        return dict(np=prev["np"], res=dict(generations=2, fes=3 * prev["np"]), X=Xg, V=Vg, e=eg,
                    P=np.where(imp[:, None], Xg, prev2["P"]), eP=eP, g=int(np.argmin(key(eP))))

    compare_generation("pso", d, prev2, gpu_like(want["X"], want["V"]), want, o, M)
    k = int(np.argmax(np.abs(want["V"]).max(axis=1)))
    Vb, Xb = want["V"].copy(), want["X"].copy()
    Xb[k] = np.clip(prev2["X"][k] - want["V"][k], LB, UB)
    Vb[k] = -want["V"][k]
    with pytest.raises(AssertionError):
        compare_generation("pso", d, prev2, gpu_like(Xb, Vb), want, o, M)
