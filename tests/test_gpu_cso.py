"""CSO runs on the GPU (update kernels + batched evaluation) against the FP64
oracle: FE accounting, the first iterations point by point (positions are
computed from the same draws, so the best point agrees to float rounding and
its error to the evaluation tolerance), final-error distributions, split-bf16
against FP32, mixed calls, determinism and graph replays of a plan."""
import numpy as np
import pytest
import torch
from scipy import stats

import oracle as O
from paper_2505_17430_amd import sevo as S
from tests.tolerance import tolerance

pytestmark = pytest.mark.gpu

SEED = 250517430
ISEED = 250517431
LB, UB = -100.0, 100.0


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    c = S.Context(0, SEED, ISEED)
    yield c
    c.close()


def cso(func, dim, m, budget, uid, inst=0, phi=0.1):
    return S.RunDesc(S.problem(func, dim), inst, uid, S.ALGO_CSO, m, budget, 0.5, 0.9, 0.7298, phi, 1.49618,
                     40.0, 0.1, 6, 2.6, 4, 0, 0)


def shade(func, dim, np_, budget, uid):
    return S.RunDesc(S.problem(func, dim), 0, uid, S.ALGO_SHADE, np_, budget, 0.5, 0.9, 0.7298, 1.49618,
                     1.49618, 40.0, 0.1, 6, 2.6, 4, 0, 0)


def odesc(d):
    return dict(algo=d.algo, func=d.prob.func, dim=d.prob.dim, lb=d.prob.lb, ub=d.prob.ub, instance=d.instance,
                run_uid=d.run_uid, np=d.np, budget=d.budget, F=d.F, CR=d.CR, w=d.w, c1=d.c1, c2=d.c2,
                vmax=d.vmax, p=d.p, H=d.H, r_arc=d.r_arc, np_min=d.np_min, topology=d.topology,
                velocity=d.velocity)


def gpu_run(ctx, descs, precision=S.FP32, trace_len=0):
    n = len(descs)
    md = max(d.prob.dim for d in descs)
    res = torch.zeros((n, 32), dtype=torch.uint8, device="cuda")
    tr = torch.full((max(n * trace_len, 1),), -7.0, device="cuda")
    bx = torch.zeros((n, md), dtype=torch.float64, device="cuda")
    say(f"  cso run n={n} prec={precision} dims={sorted(set(d.prob.dim for d in descs))}")
    ctx.run(descs, res, tr if trace_len else None, trace_len, bx, md, precision=precision)
    torch.cuda.synchronize()
    raw = res.cpu().numpy().tobytes()
    out = []
    for r in range(n):
        rr = S.RunResult.from_buffer_copy(raw[r * 32:(r + 1) * 32])
        out.append(dict(best_e=rr.best_e, best_e32=rr.best_e32, success=rr.success, fes=rr.fes,
                        generations=rr.generations))
    return out, tr.cpu().numpy()[: n * trace_len].reshape(n, trace_len), bx.cpu().numpy()


@pytest.mark.parametrize("m,budget", [(40, 40 + 20 * 25 + 7), (30, 30), (300, 300 + 150 * 4)])
def test_cso_fe_accounting_and_trace(ctx, m, budget):
    d = cso(S.RASTRIGIN, 10, m, budget, uid=3)
    tl = budget // 200 + 2
    (g,), tr, _ = gpu_run(ctx, [d], trace_len=tl)
    o, _, _ = O.run(odesc(d), SEED, ISEED)
    assert g["fes"] == o["fes"] and g["generations"] == o["generations"]
    n_rec = min(g["fes"] // 200, tl)
    assert np.all(np.isfinite(tr[0][:n_rec])) and np.all(np.diff(tr[0][:n_rec]) <= 0)
    assert np.all(tr[0][n_rec:] == -7.0)
    assert g["best_e32"] <= (tr[0][0] if n_rec else np.inf)


@pytest.mark.parametrize("func,dim,m,iters", [(S.GRIEWANK, 10, 40, 1), (S.RASTRIGIN, 200, 64, 1),
                                              (S.ELLIPSOID, 1000, 300, 1), (S.SCHWEFEL, 30, 100, 3),
                                              (S.RASTRIGIN, 1000, 300, 3)])
def test_cso_first_iterations_match_oracle(ctx, func, dim, m, iters):
    """Same initial swarm (bit for bit), same draws and pairings: the best
    point agrees to float rounding, its FP32 error is within the evaluation
    tolerance of the oracle's error at that point, and the trace follows."""
    budget = m + iters * (m // 2)
    d = cso(func, dim, m, budget, uid=11 + dim)
    tl = budget // 200
    (g,), tr, bx = gpu_run(ctx, [d], trace_len=tl)
    o, otr, obx = O.run(odesc(d), SEED, ISEED, trace_len=tl)
    assert g["fes"] == o["fes"] == budget and g["generations"] == iters
    assert np.allclose(bx[0][:dim], obx, rtol=0, atol=2e-3), np.abs(bx[0][:dim] - obx).max()
    oi, oM = O.instance(func, dim, 0, ISEED)
    e_at = O.error(func, oi, oM, bx[0][:dim])
    tol = tolerance(func, oi, oM, bx[0][:dim, None], np.array([e_at]))[0]
    assert abs(g["best_e32"] - e_at) <= tol, (g["best_e32"], e_at, tol)
    assert e_at == pytest.approx(o["best_e"], rel=1e-4, abs=1e-6)
    assert np.allclose(tr[0], otr, rtol=1e-4, atol=1e-6)


def test_cso_distribution_vs_oracle(ctx):
    descs = [cso(S.RASTRIGIN, 10, 40, 40 * 101, uid=500 + r, inst=r % 3) for r in range(32)]
    gres, _, _ = gpu_run(ctx, descs)
    ores = [O.run(odesc(d), SEED, ISEED)[0] for d in descs]
    for g, o in zip(gres, ores):
        assert g["fes"] == o["fes"] and g["generations"] == o["generations"]
    ge = np.array([g["best_e"] for g in gres])
    oe = np.array([o["best_e"] for o in ores])
    p = stats.ks_2samp(np.log10(ge + 1e-12), np.log10(oe + 1e-12)).pvalue
    say(f"  median gpu {np.median(ge):.3e} oracle {np.median(oe):.3e} KS p={p:.3g}")
    assert p > 1e-3


def test_cso_split_bf16_follows_fp32(ctx):
    """Split-bf16 evaluation changes errors by its tolerance only: over a few
    iterations the pairings and moves are the same, so the best error
    agrees closely and the evaluation count exactly."""
    descs = [cso(f, 1000, 300, 300 + 150 * 3, uid=40 + f) for f in (S.ELLIPSOID, S.RASTRIGIN, S.ACKLEY)]
    r32, _, b32 = gpu_run(ctx, descs, precision=S.FP32)
    rbf, _, bbf = gpu_run(ctx, descs, precision=S.SPLIT_BF16)
    for a, b in zip(r32, rbf):
        assert a["fes"] == b["fes"]
        assert b["best_e"] == pytest.approx(a["best_e"], rel=1e-3)
    assert np.allclose(b32, bbf, atol=2e-3)


def test_cso_mixed_call_and_determinism(ctx):
    """CSO runs beside fused runs in one call give the same bits as alone, and
    a repeated call gives the same bits."""
    c = [cso(S.ACKLEY, 30, 50, 2000, uid=61), cso(S.GRIEWANK, 200, 20, 1500, uid=62, inst=1)]
    f = [shade(S.RASTRIGIN, 10, 40, 2000, uid=63)]
    mixed, trm, bxm = gpu_run(ctx, [c[0], f[0], c[1]], trace_len=8)
    alone_c, trc, bxc = gpu_run(ctx, c, trace_len=8)
    alone_f, trf, _ = gpu_run(ctx, f, trace_len=8)
    assert mixed[0] == alone_c[0] and mixed[2] == alone_c[1] and mixed[1] == alone_f[0]
    assert np.array_equal(trm[[0, 2]], trc) and np.array_equal(trm[1], trf[0])
    assert np.array_equal(bxm[[0, 2]], bxc)
    again, tra, bxa = gpu_run(ctx, c, trace_len=8)
    assert again == alone_c and np.array_equal(tra, trc) and np.array_equal(bxa, bxc)


def test_cso_plan_replays_in_graph(ctx):
    descs = [cso(S.SCHWEFEL, 30, 20, 20 + 10 * 40, uid=71), cso(S.ELLIPSOID, 150, 40, 40 + 20 * 20, uid=72)]
    n, tl, md = len(descs), 2, 150
    res = torch.zeros((n, 32), dtype=torch.uint8, device="cuda")
    tr = torch.zeros(n * tl, device="cuda")
    bx = torch.zeros((n, md), dtype=torch.float64, device="cuda")
    outs = [res, tr, bx]
    ctx.run(descs, res, tr, tl, bx, md)
    torch.cuda.synchronize()
    ref = [t.clone() for t in outs]
    plan = ctx.plan_run(descs, res, tr, tl, bx, md)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.launch(torch.cuda.current_stream())
    for rep in range(2):
        for t in outs:
            t.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        say(f"  replay {rep}")
        assert all(torch.equal(a, b) for a, b in zip(outs, ref))
    plan.close()


def test_cso_rejects_bad_arguments(ctx):
    res = torch.zeros(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(S.SevoError):
        ctx.run([cso(S.RASTRIGIN, 10, 31, 1000, 1)], res)              # odd swarm
    with pytest.raises(S.SevoError):
        ctx.run([cso(S.RASTRIGIN, 10, 1026, 5000, 1)], res)            # swarm > 1024
    with pytest.raises(S.SevoError):
        ctx.run([cso(S.RASTRIGIN, 10, 30, 1000, 1)], res, precision=S.FP64)
    with pytest.raises(S.SevoError):
        ctx.run([shade(S.RASTRIGIN, 10, 30, 1000, 1)], res, precision=S.SPLIT_BF16)
