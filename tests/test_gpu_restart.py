"""GPU parity of L-SHADE-Restart runs (sevo_run, SEVO_ALGO_LSHADE_RS)
against the FP64 oracle.

* A threshold that is never met: the runs are L-SHADE's, bit for bit.
* A threshold that is always met: a restart after every generation that
  leaves budget, so the run is a fixed sequence of fresh populations (drawn
  bit-exactly as the oracle's) and first generations: evaluations,
  generations and restarts exactly the oracle's, the best error to the
  evaluation tolerance.
* A threshold met on convergence: every run restarts, about as often as
  the oracle's runs; FE accounting and the recorder stay consistent.
* Team and placement choices do not change the results.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

torch = pytest.importorskip("torch")
from paper_2505_17430_amd import sevo as S  # noqa: E402

from .test_gpu_run import ctx, desc, gpu_run, odesc, say  # noqa: F401,E402

pytestmark = pytest.mark.gpu
SEED, ISEED = W.BASE_SEED, W.INSTANCE_SEED


def rdesc(func, dim, np_, budget, uid, tol, inst=0, **kw):
    kw.setdefault("p", 0.11)   # L-SHADE's
    d = desc(S.ALGO_LSHADE_RS, func, dim, np_, budget, uid=uid, inst=inst, **kw)
    d.restart_tol = tol
    return d


def ordesc(d):
    o = odesc(d)
    o["restart_tol"] = d.restart_tol
    return o


def restarts_of(ctx, descs):
    """Results with the restart counts (sevo_run_result.restarts)."""
    n = len(descs)
    res = torch.zeros((n, 32), dtype=torch.uint8, device="cuda")
    ctx.run(descs, res)
    torch.cuda.synchronize()
    raw = res.cpu().numpy().tobytes()
    return [S.RunResult.from_buffer_copy(raw[r * 32:(r + 1) * 32]) for r in range(n)]


def test_restart_never_triggered_is_lshade(ctx):
    descs = [rdesc(S.SCHWEFEL, 30, 100, 8000, uid=120, tol=-1.0),
             rdesc(S.RASTRIGIN, 10, 40, 4000, uid=121, tol=-1.0),
             rdesc(S.ELLIPSOID, 100, 200, 6000, uid=122, tol=-1.0)]
    plain = [desc(S.ALGO_LSHADE, d.prob.func, d.prob.dim, d.np, d.budget, uid=d.run_uid) for d in descs]
    a = gpu_run(ctx, descs, trace_len=40, max_dim=100)
    b = gpu_run(ctx, plain, trace_len=40, max_dim=100)
    assert a[0] == b[0]
    assert np.array_equal(a[1], b[1], equal_nan=True) and np.array_equal(a[2], b[2])
    assert all(r.restarts == 0 for r in restarts_of(ctx, descs))


@pytest.mark.parametrize("func,dim,np_,budget", [(S.RASTRIGIN, 10, 40, 4000), (S.GRIEWANK, 30, 100, 6000),
                                                 (S.ACKLEY, 50, 64, 5000), (S.ELLIPSOID, 100, 200, 6000)])
def test_restart_every_generation_matches_oracle(ctx, func, dim, np_, budget):
    d = rdesc(func, dim, np_, budget, uid=130, tol=1e300)
    (g,), tr, _ = gpu_run(ctx, [d], trace_len=budget // 200)
    (r,) = restarts_of(ctx, [d])
    o, otr, _ = O.run(ordesc(d), SEED, ISEED, trace_len=budget // 200)
    say(f"  gens {g['generations']} restarts {r.restarts} best gpu {g['best_e']:.6e} oracle {o['best_e']:.6e}")
    assert g["fes"] == o["fes"] and g["generations"] == o["generations"] and r.restarts == o["restarts"]
    assert o["restarts"] >= g["generations"] - 1
    assert g["best_e"] == pytest.approx(o["best_e"], rel=1e-4)
    n_rec = g["fes"] // 200
    assert np.allclose(tr[0][:n_rec], otr[:n_rec], rtol=1e-4)


def test_restart_on_convergence(ctx):
    """Rosenbrock D = 10, threshold 1e-2: every oracle run restarts once or
    twice in 20,000 evaluations; so do the GPU's, as often on average."""
    n, budget = 24, 50 * 400
    descs = [rdesc(S.ROSENBROCK, 10, 50, budget, uid=500 + r, tol=1e-2, inst=r % 3) for r in range(n)]
    rr = restarts_of(ctx, descs)
    gres, tr, _ = gpu_run(ctx, descs, trace_len=budget // 200)
    ores = [O.run(ordesc(d), SEED, ISEED)[0] for d in descs]
    gk = np.array([r.restarts for r in rr])
    ok = np.array([o["restarts"] for o in ores])
    say(f"  restarts gpu {gk.tolist()} oracle {ok.tolist()}")
    assert np.all(gk >= 1) and np.all(ok >= 1)
    assert abs(gk.mean() - ok.mean()) <= 0.5
    for k, g in enumerate(gres):
        assert budget <= g["fes"] < budget + 50
        n_rec = g["fes"] // 200
        assert np.all(np.diff(tr[k][:n_rec]) <= 0)
        assert g["best_e"] <= tr[k][min(n_rec, budget // 200) - 1] * (1 + 1e-6) + 1e-12


def test_restart_team_and_placement_do_not_change_results(ctx, monkeypatch):
    descs = [rdesc(S.ROSENBROCK, 10, 50, 8000, uid=140, tol=1e-2), rdesc(S.ROSENBROCK, 10, 20, 8000, uid=141, tol=1e-2),
             rdesc(S.RASTRIGIN, 30, 150, 9000, uid=142, tol=1e300), rdesc(S.ELLIPSOID, 100, 200, 4000, uid=143, tol=1e300)]
    base = gpu_run(ctx, descs, trace_len=40, max_dim=100)
    for var, val in (("SEVO_RUN_TEAM", "wave"), ("SEVO_RUN_TEAM", "block"), ("SEVO_RUN_PLACEMENT", "workspace")):
        monkeypatch.setenv(var, val)
        other = gpu_run(ctx, descs, trace_len=40, max_dim=100)
        monkeypatch.delenv(var)
        assert other[0] == base[0], (var, val)
        assert np.array_equal(other[1], base[1], equal_nan=True) and np.array_equal(other[2], base[2])


def test_restart_rejects_nan_threshold(ctx):
    res = torch.zeros((1, 32), dtype=torch.uint8, device="cuda")
    with pytest.raises(S.SevoError):
        ctx.run([rdesc(S.RASTRIGIN, 10, 50, 1000, 1, tol=float("nan"))], res)
    with pytest.raises(S.SevoError):
        ctx.run([rdesc(S.RASTRIGIN, 10, 50, 1000, 1, tol=1e-3)], res, precision=S.FP64)
