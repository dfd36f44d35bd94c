"""GPU parity of the batched evaluation (sevo_evaluate / sevo_evaluate_batch)
against the FP64 oracle, through the C ABI.

Inputs come from ``workloads`` (seeded numpy) and the oracle's own instance
generator; nothing the oracle sees comes from the GPU path.  The bound for
the single-precision paths (FP32 MFMA rotation, split-bf16 rotation) is the
one stated per function in tests/tolerance.py, relative to the error value
e = f - f* (not to f, whose bias 100 would hide 1e-6):
    |e_gpu - e_oracle| <= max(1e-6, 1e-5 e)
for Ellipsoid, Rastrigin, Schwefel, Griewank and Ackley, plus for Rosenbrock
the first-order effect of rounding the shifted point to float on the walls
of its valley.  Each check prints the worst deviation as a fraction of the
bound.
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
ISEED = W.INSTANCE_SEED


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = S.Context(0, W.BASE_SEED, ISEED)
    yield c
    c.close()


def gpu_eval(ctx, func, dim, inst, X, precision=S.FP32, pad=5):
    dt = torch.float64 if precision == S.FP64 else torch.float32
    n = X.shape[1]
    ld = n + pad
    xd = torch.zeros((dim, ld), dtype=dt, device="cuda")
    xd[:, :n] = torch.from_numpy(np.ascontiguousarray(X)).to(dt)
    err = torch.full((n + 3,), float("nan"), dtype=dt, device="cuda")
    say(f"  eval func={func} dim={dim} inst={inst} n={n} prec={precision}")
    ctx.evaluate(S.problem(func, dim), inst, xd, err, n=n, ld=ld, precision=precision)
    torch.cuda.synchronize()
    out = err.cpu().numpy()
    assert np.all(np.isnan(out[n:])), "kernel wrote past n"
    return out[:n].astype(np.float64)


def check(e_gpu, e_ora, what, tol):
    dev = np.abs(e_gpu - e_ora)
    bad = np.nonzero(~(dev <= tol))[0]
    worst = float(np.max(dev / tol)) if len(dev) else 0.0
    say(f"  {what}: n={len(e_ora)} worst |de| / bound = {worst:.3g}")
    assert len(bad) == 0, (what, bad[:5], e_gpu[bad[:5]], e_ora[bad[:5]])


def check_f32(e_gpu, func, o, M, X, e_ora, what):
    """Single precision against the bound stated for the function."""
    check(e_gpu, e_ora, what, tolerance(func, o, M, X, e_ora))


SMALL_DIMS = [2, 3, 7, 10, 16, 30, 50, 64, 100, 120]
LARGE_DIMS = [121, 200, 1000]


@pytest.mark.parametrize("dim", [10, 30, 100, 200])
def test_identity_instance_textbook_values(ctx, dim):
    """M = I, o = 0 (a user-defined instance): the unrotated textbook functions,
    whose values at these points are known in closed form."""
    o, M = np.zeros(dim), np.eye(dim)
    inst = 900
    D = dim
    for func in range(6):
        ctx.set_instance(S.problem(func, dim), inst, o, M)
    cols = [np.eye(D)[:, k] for k in range(D)]                      # ellipsoid: e_k
    e = gpu_eval(ctx, S.ELLIPSOID, D, inst, np.stack(cols, 1).astype(np.float32))
    want = 10.0 ** (6 * np.arange(D) / (D - 1))
    assert np.allclose(e, want, rtol=2e-6)
    X = np.stack([np.full(D, 0.5), np.full(D, -1.0), np.ones(D)], 1).astype(np.float32)
    assert gpu_eval(ctx, S.RASTRIGIN, D, inst, X)[0] == pytest.approx(20.25 * D, rel=2e-6)
    assert gpu_eval(ctx, S.ROSENBROCK, D, inst, X)[1] == pytest.approx(D - 1, rel=2e-6)
    assert gpu_eval(ctx, S.ACKLEY, D, inst, X)[2] == pytest.approx(20 * (1 - np.exp(-0.2)), rel=2e-6)
    # every function, random points, identity instance: oracle parity
    Xr = W.uniform_points(11 + dim, dim, 200)
    for func in range(6):
        eo = O.errors_soa_f32(func, o, M, Xr)
        check_f32(gpu_eval(ctx, func, D, inst, Xr), func, o, M, Xr, eo, f"identity f{func} D{dim}")


def _points(func, dim, inst, n=300):
    o, M = O.instance(func, dim, inst, ISEED)
    X = np.concatenate([W.uniform_points(W.group_seed(func, dim, inst), dim, n),
                        W.near_points(o, seed=dim + func)], axis=1)
    return o, M, X


@pytest.mark.parametrize("dim", SMALL_DIMS + LARGE_DIMS)
def test_parity_fp32(ctx, dim):
    for func in range(6):
        for inst in (0, 3):
            o, M, X = _points(func, dim, inst, n=300 if dim < 500 else 150)
            eo = O.errors_soa_f32(func, o, M, X)
            check_f32(gpu_eval(ctx, func, dim, inst, X), func, o, M, X, eo, f"fp32 f{func} D{dim} i{inst}")


# 65 .. 112: the small path's split-bf16 kernel (65 and 112 its ends; 96
# whole bf16 steps only, 100 a float k-step after them); 33 .. 64 and
# 113 .. 120: the float kernel serves the precision; above 120 the tiled GEMM
@pytest.mark.parametrize("dim", [33, 50, 64, 65, 96, 100, 112, 113, 121, 200, 1000])
def test_parity_split_bf16(ctx, dim):
    for func in range(6):
        o, M, X = _points(func, dim, 1, n=150)
        eo = O.errors_soa_f32(func, o, M, X)
        check_f32(gpu_eval(ctx, func, dim, 1, X, precision=S.SPLIT_BF16), func, o, M, X, eo,
                  f"bf16 f{func} D{dim}")


@pytest.mark.parametrize("dim", [2, 10, 50, 130])
def test_parity_fp64(ctx, dim):
    for func in range(6):
        o, M, X = _points(func, dim, 2, n=100)
        eo = O.errors_soa_f32(func, o, M, X)
        check(gpu_eval(ctx, func, dim, 2, X.astype(np.float64), precision=S.FP64), eo, f"fp64 f{func} D{dim}",
              np.maximum(1e-12, 1e-11 * np.abs(eo)))


@pytest.mark.parametrize("dim", [2, 10, 30, 100, 120, 200, 1000])
def test_exact_zero_at_optimum(ctx, dim):
    """With o on the float32 grid, x = o gives d = 0 and e = 0 exactly on every path."""
    for func in range(6):
        o, M = O.instance(func, dim, 0, ISEED)
        o32 = o.astype(np.float32).astype(np.float64)
        ctx.set_instance(S.problem(func, dim), 901, o32, M)
        X = np.stack([o32, o32], 1).astype(np.float32)
        for prec in (S.FP32, S.SPLIT_BF16, S.FP64):
            e = gpu_eval(ctx, func, dim, 901, X, precision=prec)
            assert np.all(e == 0.0), (func, dim, prec, e)


def test_batch_equals_single_and_is_deterministic(ctx):
    groups = [(f, d, k, n) for (f, d, k, n) in
              [(0, 10, 0, 257), (2, 30, 1, 130), (5, 50, 2, 1), (3, 100, 3, 500), (1, 200, 0, 129),
               (4, 10, 4, 0), (2, 1000, 0, 70)]]
    xs, errs, items = [], [], []
    for (f, d, k, n) in groups:
        X = W.uniform_points(W.group_seed(f, d, k, 9), d, max(n, 1))
        xd = torch.from_numpy(X).cuda()
        e = torch.full((max(n, 1),), float("nan"), device="cuda")
        xs.append(xd); errs.append(e)
        items.append((S.problem(f, d), k, xd, e, n, xd.stride(0)))
    say("  batch of", len(items))
    ctx.evaluate_batch(items)
    torch.cuda.synchronize()
    batch = [e.cpu().numpy().copy() for e in errs]
    ctx.evaluate_batch(items)
    torch.cuda.synchronize()
    again = [e.cpu().numpy().copy() for e in errs]
    for (f, d, k, n), xd, b, a in zip(groups, xs, batch, again):
        assert np.array_equal(b[:n], a[:n])                       # bit-identical repeat
        if n == 0:
            assert np.isnan(b[0])                                  # n = 0 writes nothing
            continue
        single = gpu_eval(ctx, f, d, k, xd.cpu().numpy()[:, :n], pad=0)
        assert np.array_equal(single, b[:n].astype(np.float64))   # same kernel, same bits


def test_launch_shape_and_autotune_do_not_change_results(ctx, monkeypatch):
    """Every tiles-per-workgroup choice (and the autotuner's) computes the same
    bits; the tuner reports a choice for each dimension class present."""
    groups = [(0, 10, 0, 5100), (2, 30, 1, 777), (3, 50, 2, 5100), (5, 100, 3, 2049), (1, 100, 4, 33)]
    errs, items = [], []
    for (f, d, k, n) in groups:
        xd = torch.from_numpy(W.uniform_points(W.group_seed(f, d, k, 11), d, n)).cuda()
        e = torch.zeros(n, device="cuda")
        errs.append(e)
        items.append((S.problem(f, d), k, xd, e))
    arr = S.Context.prepare_batch(items)

    def outputs():
        for e in errs:
            e.fill_(float("nan"))
        ctx.evaluate_batch(arr)
        torch.cuda.synchronize()
        return [e.cpu().numpy().copy() for e in errs]

    ref = outputs()
    for tpb in ("1", "2", "3", "8"):
        monkeypatch.setenv("SEVO_TILES_PER_BLOCK", tpb)
        # the override is read when a context is created
        c2 = S.Context(0, W.BASE_SEED, W.INSTANCE_SEED)
        for e in errs:
            e.fill_(float("nan"))
        c2.evaluate_batch(arr)
        torch.cuda.synchronize()
        say("  tiles per block", tpb)
        for a, b in zip(ref, [e.cpu().numpy() for e in errs]):
            assert np.array_equal(a, b)
        c2.close()
    monkeypatch.delenv("SEVO_TILES_PER_BLOCK")
    chosen = ctx.tune_evaluate(arr)
    say("  tuned", chosen)
    assert set(chosen) == {3, 8, 13, 25}
    assert all(v in (0, 1, 2, 3, 4, 6, 8) for v in chosen.values())
    for a, b in zip(ref, outputs()):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("precision", [S.FP32, S.SPLIT_BF16])
def test_large_d_workgroup_width_does_not_change_results(ctx, monkeypatch, precision):
    """The D > 120 GEMM gives the same bits with 64 or 128 points per
    workgroup (one batch of several items, ragged point counts, Rosenbrock's
    neighbours across row blocks); both agree with the oracle."""
    groups = [(1, 200, 0, 333), (4, 1000, 1, 130), (5, 129, 2, 64), (3, 300, 3, 257)]
    errs, items, pts = [], [], []
    for (f, d, k, n) in groups:
        X = W.uniform_points(W.group_seed(f, d, k, 12), d, n)
        pts.append(X)
        e = torch.zeros(n, device="cuda")
        errs.append(e)
        items.append((S.problem(f, d), k, torch.from_numpy(X).cuda(), e))
    arr = S.Context.prepare_batch(items)
    got = {}
    for width in ("64", "128"):
        monkeypatch.setenv("SEVO_LARGE_POINTS", width)
        c2 = S.Context(0, W.BASE_SEED, W.INSTANCE_SEED)
        for e in errs:
            e.fill_(float("nan"))
        c2.evaluate_batch(arr, precision=precision)
        torch.cuda.synchronize()
        got[width] = [e.cpu().numpy().copy() for e in errs]
        c2.close()
        say("  points per workgroup", width)
    monkeypatch.delenv("SEVO_LARGE_POINTS")
    for (f, d, k, n), X, a, b in zip(groups, pts, got["64"], got["128"]):
        assert np.array_equal(a, b), (f, d, n)
        o, M = O.instance(f, d, k, ISEED)
        check_f32(a, f, o, M, X, O.errors_soa_f32(f, o, M, X), f"width f{f} D{d} n{n}")


def test_invalid_arguments(ctx):
    x = torch.zeros((10, 4), device="cuda")
    e = torch.zeros(4, device="cuda")
    with pytest.raises(S.SevoError) as ei:
        ctx.evaluate(S.problem(0, 10), 0, x, e, precision=7)
    assert ei.value.code == S.EINVAL
    with pytest.raises(S.SevoError):
        ctx.evaluate(S.problem(9, 10), 0, x, e)
    with pytest.raises(S.SevoError):
        ctx.evaluate(S.problem(0, 10), 0, x, e, n=4, ld=3)
    with pytest.raises(S.SevoError):
        ctx.evaluate(S.problem(0, 10, lb=1.0, ub=-1.0), 0, x, e)
    with pytest.raises(S.SevoError):
        ctx.evaluate(S.problem(0, 10), 0, 0, e, n=4, ld=4)
    ctx.evaluate(S.problem(0, 10), 0, x, e, n=0, ld=4)           # no-op
    ctx.sync()


@pytest.mark.parametrize("precision", [S.FP32, S.SPLIT_BF16])
def test_c2_full_size_sampled(ctx, precision):
    """The full batched-evaluation workload (6 functions x D in {10,30,50,100}
    x 10 instances x 51 runs x 100 points) in one batch call, in the launch
    configuration the benchmark times, in both single precisions; a seeded
    sample of points per group is checked one by one against the oracle."""
    groups = W.c2_groups()
    items, keep = [], []
    for (f, d, k, n) in groups:
        X = W.uniform_points(W.group_seed(f, d, k), d, n)
        xd = torch.from_numpy(X).cuda()
        e = torch.full((n,), float("nan"), device="cuda")
        items.append((S.problem(f, d), k, xd, e))
        keep.append((f, d, k, X, e))
    say("  c2 items", len(items), "precision", precision)
    ctx.evaluate_batch(items, precision=precision)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    for (f, d, k, X, e) in keep:
        eg = e.cpu().numpy().astype(np.float64)
        assert np.all(np.isfinite(eg)) and eg.min() >= -1e-6
        idx = rng.choice(X.shape[1], size=12, replace=False)
        o, M = O.instance(f, d, k, ISEED)
        Xs = X[:, idx]
        check_f32(eg[idx], f, o, M, Xs, O.errors_soa_f32(f, o, M, Xs), f"c2 f{f} D{d} i{k}")
