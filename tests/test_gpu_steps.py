"""GPU parity of the one-generation steps (sevo_de_step, sevo_pso_step)
against the FP64 oracle, through the C ABI.

Bit-exact: the initial population (its float rounding of the oracle's double
values), the DE donor indices r1, r2, r3 and jrand, the unchanged (masked
out) trial coordinates, the selection decision on equal errors, the PSO
global-best index given the same personal-best errors.  Float arithmetic
(mutation, velocity update) is compared with a bound of a few float32
roundings of the operands; errors with the evaluation tolerance.
"""
import sys

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
EPS = 2.0 ** -24


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    c = S.Context(0, SEED, ISEED)
    yield c
    c.close()


class DEBufs:
    def __init__(self, R, np_, dim, pad=3, rpad=5, dtype=torch.float32):
        self.R, self.np, self.dim = R, np_, dim
        self.ld = np_ + pad
        self.rs = dim * self.ld + rpad
        n = R * self.rs
        self.x = torch.full((n,), float("nan"), dtype=dtype, device="cuda")
        self.u = torch.full((n,), float("nan"), dtype=dtype, device="cuda")
        self.ex = torch.full((R * self.ld,), float("nan"), dtype=dtype, device="cuda")
        self.eu = torch.full((R * self.ld,), float("nan"), dtype=dtype, device="cuda")
        self.donors = torch.full((R * 4 * self.ld,), -1, dtype=torch.int32, device="cuda")
        self.rep = torch.full((R * self.ld,), 7, dtype=torch.uint8, device="cuda")

    def state(self, t, uid0):
        return S.DEState(self.R, self.np, self.ld, self.rs, uid0, t, self.x.data_ptr(),
                         self.ex.data_ptr(), self.u.data_ptr(), self.eu.data_ptr(),
                         self.donors.data_ptr(), self.rep.data_ptr())

    def pop(self, buf, r):
        """(np, dim) individual-major copy of run r of a population buffer."""
        a = buf.cpu().numpy()[r * self.rs: r * self.rs + self.dim * self.ld].reshape(self.dim, self.ld)
        return a[:, : self.np].T.astype(np.float64)

    def vals(self, buf, r):
        return buf.cpu().numpy()[r * self.ld: r * self.ld + self.np].astype(np.float64)


# the variation stages a run's population in LDS: (10, 50) in one slab,
# (100, 200) in three slabs of at most 36 rows, (30, 2048) in eight slabs of
# 4 rows; (13, 4096) does not fit and gathers its donors from global memory.
# With ld = np and runs on 16-byte boundaries (pad 0, run stride a multiple
# of 4 floats) a whole population stages as 16-byte vectors: (10, 50) with
# no tail, (7, 5) with 35 elements, three after the last whole vector.
@pytest.mark.parametrize("func,dim,np_,pad,rpad", [(2, 10, 50, 3, 5), (0, 30, 37, 3, 5), (3, 7, 4, 3, 5),
                                                   (1, 100, 200, 3, 5), (5, 2, 5, 3, 5), (2, 30, 2048, 3, 5),
                                                   (4, 13, 4096, 3, 5), (2, 10, 50, 0, 0), (0, 7, 5, 0, 1)])
def test_de_steps_parity(ctx, func, dim, np_, pad, rpad):
    R, uid0, F, CR = 3, 40, 0.5, 0.9
    o, M = O.instance(func, dim, 0, ISEED)
    b = DEBufs(R, np_, dim, pad=pad, rpad=rpad)
    prob = S.problem(func, dim)
    say(f"  de func={func} dim={dim} np={np_} t=0")
    ctx.de_step(prob, 0, b.state(0, uid0), F, CR)
    torch.cuda.synchronize()
    for r in range(R):
        X = b.pop(b.x, r)
        want = O.init_population(func, dim, LB, UB, np_, uid0 + r, SEED).astype(np.float32)
        assert np.array_equal(X, want.astype(np.float64)), "initial population must be bit-exact"
        eX = b.vals(b.ex, r)
        eo = O.errors(func, o, M, X)
        assert np.all(np.abs(eX - eo) <= tolerance(func, o, M, X.T, eo))
    # padding between ld and np, and between runs, is never written
    xa = b.x.cpu().numpy()
    for r in range(R):
        blk = xa[r * b.rs: r * b.rs + dim * b.ld].reshape(dim, b.ld)
        assert np.all(np.isnan(blk[:, np_:]))
        assert np.all(np.isnan(xa[r * b.rs + dim * b.ld: (r + 1) * b.rs]))
    for t in (1, 2, 3):
        prev = [(b.pop(b.x, r), b.vals(b.ex, r)) for r in range(R)]
        say(f"  de t={t}")
        ctx.de_step(prob, 0, b.state(t, uid0), F, CR)
        torch.cuda.synchronize()
        dn = b.donors.cpu().numpy()
        rep = b.rep.cpu().numpy()
        for r in range(R):
            X, eX = prev[r]
            out = O.de_generation(func, LB, UB, o, M, X, eX, F, CR, uid0 + r, SEED, t)
            got_dn = dn[r * 4 * b.ld: (r + 1) * 4 * b.ld].reshape(4, b.ld)[:, :np_].T
            assert np.array_equal(got_dn, out["donors"]), "donor indices must be bit-exact"
            U = b.pop(b.u, r)
            mask = out["mask"]
            assert np.array_equal(U[~mask], X[~mask]), "unmasked coordinates are the parent's"
            r1, r2, r3 = (out["donors"][:, k] for k in range(3))
            scale = np.abs(X[r1]) + F * (np.abs(X[r2]) + np.abs(X[r3])) + 1e-30
            v = X[r1] + F * (X[r2] - X[r3])
            inside = mask & (v >= LB) & (v <= UB) & (np.abs(v - LB) > 8 * EPS * scale) & \
                (np.abs(v - UB) > 8 * EPS * scale)
            assert np.all(np.abs(U - out["U"])[inside] <= 4 * EPS * scale[inside])
            outside = mask & ((v < LB) | (v > UB)) & (np.abs(v - LB) > 8 * EPS * scale) & \
                (np.abs(v - UB) > 8 * EPS * scale)
            assert np.all(np.abs(U - out["U"])[outside] <= 2 * EPS * (np.abs(X) + 100)[outside])
            assert U.min() >= LB and U.max() <= UB
            eU = b.vals(b.eu, r)
            eo = O.errors(func, o, M, U)
            assert np.all(np.abs(eU - eo) <= tolerance(func, o, M, U.T, eo))
            # selection decided on the GPU's own errors, ties to the trial
            want_rep = np.where(np.isnan(eU), np.inf, eU) <= np.where(np.isnan(eX), np.inf, eX)
            assert np.array_equal(rep[r * b.ld: r * b.ld + np_].astype(bool), want_rep)
            Xn = b.pop(b.x, r)
            assert np.array_equal(Xn[want_rep], U[want_rep]) and np.array_equal(Xn[~want_rep], X[~want_rep])


def test_de_tie_goes_to_trial(ctx):
    """Identical population: every trial equals its parent bit for bit, the
    errors tie exactly and every decision must be 'replace'."""
    func, dim, np_, R = 2, 10, 16, 1
    b = DEBufs(R, np_, dim)
    row = W.uniform_points(3, dim, 1)[:, 0]
    xa = b.x.cpu().numpy()
    for j in range(dim):
        xa[j * b.ld: j * b.ld + np_] = row[j]
    b.x.copy_(torch.from_numpy(xa))
    ctx.evaluate(S.problem(func, dim), 0, b.x, b.ex, n=np_, ld=b.ld)
    ctx.de_step(S.problem(func, dim), 0, b.state(1, 9), 0.5, 0.9)
    torch.cuda.synchronize()
    assert np.array_equal(b.pop(b.u, 0), b.pop(b.x, 0))
    assert np.array_equal(b.vals(b.eu, 0), b.vals(b.ex, 0))
    assert np.all(b.rep.cpu().numpy()[:np_] == 1)


def test_de_nan_error_counts_as_infinity(ctx):
    func, dim, np_ = 0, 10, 8
    b = DEBufs(1, np_, dim)
    ctx.de_step(S.problem(func, dim), 0, b.state(0, 3), 0.5, 0.9)
    ex = b.ex.cpu().numpy()
    ex[2] = np.nan
    b.ex.copy_(torch.from_numpy(ex))
    ctx.de_step(S.problem(func, dim), 0, b.state(1, 3), 0.5, 0.9)
    torch.cuda.synchronize()
    assert b.rep.cpu().numpy()[2] == 1
    assert np.isfinite(b.vals(b.ex, 0)).all()


def test_de_step_rejects_bad_arguments(ctx):
    b = DEBufs(1, 8, 10)
    st = b.state(1, 0)
    with pytest.raises(S.SevoError):
        ctx.de_step(S.problem(0, 10), 0, st, 0.5, 1.5)
    bad = b.state(1, 0)
    bad.np = 3
    with pytest.raises(S.SevoError):
        ctx.de_step(S.problem(0, 10), 0, bad, 0.5, 0.9)
    bad = b.state(1, 0)
    bad.run_stride = 5
    with pytest.raises(S.SevoError):
        ctx.de_step(S.problem(0, 10), 0, bad, 0.5, 0.9)


class PSOBufs:
    def __init__(self, R, np_, dim, dtype=torch.float32):
        self.R, self.np, self.dim = R, np_, dim
        self.ld = np_ + 1
        self.rs = dim * self.ld
        n = R * self.rs
        mk = lambda m: torch.full((m,), float("nan"), dtype=dtype, device="cuda")
        self.x, self.v, self.p = mk(n), mk(n), mk(n)
        self.ex, self.ep = mk(R * self.ld), mk(R * self.ld)
        self.g = torch.full((R,), -1, dtype=torch.int32, device="cuda")

    def state(self, t, uid0):
        return S.PSOState(self.R, self.np, self.ld, self.rs, uid0, t, self.x.data_ptr(),
                          self.v.data_ptr(), self.p.data_ptr(), self.ex.data_ptr(),
                          self.ep.data_ptr(), self.g.data_ptr())

    def pop(self, buf, r):
        a = buf.cpu().numpy()[r * self.rs:(r + 1) * self.rs].reshape(self.dim, self.ld)
        return a[:, : self.np].T.astype(np.float64)

    def vals(self, buf, r):
        return buf.cpu().numpy()[r * self.ld: r * self.ld + self.np].astype(np.float64)


# the personal-best kernel takes eight particles per thread and pass: 600
# particles fill part of a pass, 2100 need a second one
@pytest.mark.parametrize("func,dim,np_", [(2, 10, 40), (4, 30, 40), (0, 50, 17), (3, 3, 1), (1, 6, 600),
                                          (5, 4, 2100)])
def test_pso_steps_parity(ctx, func, dim, np_):
    R, uid0 = 2, 100
    w, c1, c2, vmax = 0.7298, 1.49618, 1.49618, 40.0
    o, M = O.instance(func, dim, 1, ISEED)
    b = PSOBufs(R, np_, dim)
    prob = S.problem(func, dim)
    say(f"  pso func={func} dim={dim} np={np_}")
    ctx.pso_step(prob, 1, b.state(0, uid0), w, c1, c2, vmax)
    torch.cuda.synchronize()
    for r in range(R):
        X = b.pop(b.x, r)
        want = O.init_population(func, dim, LB, UB, np_, uid0 + r, SEED).astype(np.float32)
        assert np.array_equal(X, want.astype(np.float64))
        assert np.all(b.pop(b.v, r) == 0) and np.array_equal(b.pop(b.p, r), X)
        ex = b.vals(b.ex, r)
        assert np.array_equal(b.vals(b.ep, r), ex)
        assert int(b.g.cpu().numpy()[r]) == int(np.argmin(ex))
    for t in (1, 2, 3, 4):
        prev = [dict(X=b.pop(b.x, r), V=b.pop(b.v, r), P=b.pop(b.p, r), eP=b.vals(b.ep, r),
                     g=int(b.g.cpu().numpy()[r])) for r in range(R)]
        ctx.pso_step(prob, 1, b.state(t, uid0), w, c1, c2, vmax)
        torch.cuda.synchronize()
        for r in range(R):
            st = prev[r]
            out = O.pso_iteration(func, LB, UB, o, M, st, w, c1, c2, vmax, uid0 + r, SEED, t)
            X, V = b.pop(b.x, r), b.pop(b.v, r)
            scale = w * np.abs(st["V"]) + c1 * np.abs(st["P"] - st["X"]) + c2 * np.abs(st["P"][st["g"]] - st["X"]) + np.abs(st["X"])
            tol = 8 * EPS * (scale + 1e-30)
            # velocity clamp and bound decisions close to their threshold may differ
            near = (np.abs(np.abs(out["V"]) - vmax) < tol) | (np.abs(out["X"] - LB) < tol) | \
                (np.abs(out["X"] - UB) < tol) | ((V == 0) != (out["V"] == 0))
            assert np.all((np.abs(V - out["V"]) <= tol) | near)
            assert np.all((np.abs(X - out["X"]) <= tol) | near)
            assert np.all(np.abs(V) <= vmax) and X.min() >= LB and X.max() <= UB
            # personal / global bests from the GPU's own errors
            ex, ep = b.vals(b.ex, r), b.vals(b.ep, r)
            improved = ex < st["eP"]
            assert np.array_equal(ep, np.where(improved, ex, st["eP"]))
            P = b.pop(b.p, r)
            assert np.array_equal(P[improved], X[improved]) and np.array_equal(P[~improved], st["P"][~improved])
            assert int(b.g.cpu().numpy()[r]) == int(np.argmin(ep))
            eo = O.errors(func, o, M, X)
            assert np.all(np.abs(ex - eo) <= tolerance(func, o, M, X.T, eo))


def test_pso_fp64_step_matches_oracle_closely(ctx):
    func, dim, np_ = 2, 10, 12
    o, M = O.instance(func, dim, 0, ISEED)
    b = PSOBufs(1, np_, dim, dtype=torch.float64)
    prob = S.problem(func, dim)
    ctx.pso_step(prob, 0, b.state(0, 5), 0.7298, 1.49618, 1.49618, 40.0, precision=S.FP64)
    st = O.pso_init(func, LB, UB, o, M, np_, 5, SEED)
    for t in range(1, 6):
        ctx.pso_step(prob, 0, b.state(t, 5), 0.7298, 1.49618, 1.49618, 40.0, precision=S.FP64)
        st = O.pso_iteration(func, LB, UB, o, M, st, 0.7298, 1.49618, 1.49618, 40.0, 5, SEED, t)
    torch.cuda.synchronize()
    assert np.allclose(b.pop(b.x, 0), st["X"], rtol=1e-12, atol=1e-11)
    assert np.allclose(b.vals(b.ep, 0), st["eP"], rtol=1e-10, atol=1e-12)
    assert int(b.g.cpu().numpy()[0]) == st["g"]
