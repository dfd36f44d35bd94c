"""Plans (sevo_plan_*): prepared evaluations and runs whose launch enqueues
kernels only, so that it can be captured into a HIP graph and replayed.

* A plan's launch gives the same bits as the eager call it was made from.
* Captured into a graph (torch.cuda.CUDAGraph over the plan's launch) and
  replayed several times, with new inputs written eagerly and the device
  synchronised between replays, every replay matches the eager call on the
  same inputs bit for bit.
"""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
from paper_2505_17430_amd import sevo as S  # noqa: E402

pytestmark = pytest.mark.gpu
LB, UB = W.LB, W.UB


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    c = S.Context(0, W.BASE_SEED, W.INSTANCE_SEED)
    yield c
    c.close()


def snapshot(ts):
    torch.cuda.synchronize()
    return [t.cpu().numpy().copy() for t in ts]


def same(a, b):
    return all(np.array_equal(x, y, equal_nan=True) for x, y in zip(a, b))


@pytest.mark.parametrize("precision", [S.FP32, S.SPLIT_BF16, S.FP64])
def test_plan_evaluate_matches_eager_and_replays_in_graph(ctx, precision):
    groups = [(0, 10, 0, 5100), (3, 30, 1, 777), (5, 100, 2, 2049), (2, 200, 0, 300), (4, 50, 3, 1)]
    dt = torch.float64 if precision == S.FP64 else torch.float32
    xs, errs, items = [], [], []
    for (f, d, k, n) in groups:
        x = torch.from_numpy(W.uniform_points(W.group_seed(f, d, k, 21), d, n)).to("cuda", dt)
        e = torch.zeros(n, device="cuda", dtype=dt)
        xs.append(x)
        errs.append(e)
        items.append((S.problem(f, d), k, x, e))
    say(f"  plan evaluate precision={precision}")
    ctx.evaluate_batch(items, precision=precision)
    ref = snapshot(errs)
    plan = ctx.plan_evaluate(items, precision=precision)
    for e in errs:
        e.fill_(float("nan"))
    plan.launch(torch.cuda.current_stream())
    assert same(ref, snapshot(errs))

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.launch(torch.cuda.current_stream())
    gen = torch.Generator(device="cuda")
    for rep in range(3):
        gen.manual_seed(100 + rep)
        for x in xs:
            x.uniform_(LB, UB, generator=gen)
        for e in errs:
            e.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        got = snapshot(errs)
        ctx.evaluate_batch(items, precision=precision)
        eager = snapshot(errs)
        say(f"  replay {rep}")
        assert same(got, eager)
        assert not same(got, ref)   # the inputs did change
    plan.close()


def run_descs():
    def desc(algo, func, dim, np_, budget, uid, inst=0):
        d = S.RunDesc(S.problem(func, dim), inst, uid, algo, np_, budget, 0.5, 0.9, 0.7298, 1.49618,
                      1.49618, 0.2 * (UB - LB), 0.1, 6, 1.4, 4)
        d.c = 0.1
        d.restart_tol = 1e-2
        return d
    return [desc(S.ALGO_DE, S.RASTRIGIN, 10, 50, 5000, 1),
            desc(S.ALGO_PSO, S.GRIEWANK, 30, 40, 4000, 2, inst=1),
            desc(S.ALGO_SHADE, S.SCHWEFEL, 50, 100, 5000, 3, inst=2),
            desc(S.ALGO_SHADE, S.ELLIPSOID, 100, 200, 4000, 4),
            desc(S.ALGO_PSO, S.ACKLEY, 10, 40, 3000, 5, inst=3),
            desc(S.ALGO_PSO, S.ACKLEY, 10, 40, 3000, 6, inst=3),
            desc(S.ALGO_JADE, S.RASTRIGIN, 30, 60, 4000, 7, inst=1),
            # restarts happen (Rosenbrock D = 10 converges to 1e-2 spread well within the budget)
            desc(S.ALGO_LSHADE_RS, S.ROSENBROCK, 10, 50, 20000, 8, inst=2)]


@pytest.mark.parametrize("team", ["", "wave"])
def test_plan_run_matches_eager_and_replays_in_graph(ctx, monkeypatch, team):
    if team:
        monkeypatch.setenv("SEVO_RUN_TEAM", team)
    descs = run_descs()
    n, tl, md = len(descs), 30, 100
    res = torch.zeros((n, 32), dtype=torch.uint8, device="cuda")
    tr = torch.zeros(n * tl, device="cuda")
    bx = torch.zeros((n, md), dtype=torch.float64, device="cuda")
    outs = [res, tr, bx]
    say(f"  plan run team={team or 'default'}")
    ctx.run(descs, res, tr, tl, bx, md)
    ref = snapshot(outs)
    plan = ctx.plan_run(descs, res, tr, tl, bx, md)
    for t in outs:
        t.zero_()
    plan.launch(torch.cuda.current_stream())
    assert same(ref, snapshot(outs))

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.launch(torch.cuda.current_stream())
    for rep in range(2):
        for t in outs:
            t.zero_()
        torch.cuda.synchronize()
        g.replay()
        got = snapshot(outs)
        say(f"  replay {rep}")
        assert same(got, ref)
    plan.close()


def test_plan_rejects_double_precision_runs(ctx):
    res = torch.zeros((1, 32), dtype=torch.uint8, device="cuda")
    with pytest.raises(S.SevoError) as ei:
        ctx.plan_run(run_descs()[:1], res, precision=S.FP64)
    assert ei.value.code == -4
