"""GPU parity of JADE runs and of the muF/muCR parameter observer
(sevo_run_observed) against the FP64 oracle.

* JADE's evaluations and generations exactly the oracle's.
* Observer row 0 is the initial pair exactly; row 1 (the first generation,
  drawn from the same Philox stream on the same initial population) the
  oracle's to float rounding of F and CR; rows beyond the run NaN.
* c = 0 keeps JADE's pair at (0.5, 0.5) for the whole run, bit for bit.
* DE rows are its fixed (F, CR); PSO rows NaN; SHADE / L-SHADE / PSODE rows
  the memory means, checked in generation 1 against the oracle.
* Final errors of many JADE runs distributed as the oracle's (two-sample
  KS); the observer's mean trajectory over runs (the quantity plotted in
  the case study) close to the oracle's over the first generations.
* Team and placement choices do not change JADE's results or observer rows.
"""
import numpy as np
import pytest
from scipy import stats

import oracle as O
import workloads as W

torch = pytest.importorskip("torch")
from paper_2505_17430_amd import sevo as S  # noqa: E402

from .test_gpu_run import ctx, desc, odesc, say  # noqa: F401,E402

pytestmark = pytest.mark.gpu
SEED, ISEED = W.BASE_SEED, W.INSTANCE_SEED


def jdesc(func, dim, np_, budget, uid, inst=0, c=0.1, p=0.05, r_arc=1.0):
    d = desc(S.ALGO_JADE, func, dim, np_, budget, uid=uid, inst=inst, p=p, r_arc=r_arc, H=1)
    d.c = c
    return d


def ojdesc(d):
    o = odesc(d)
    o["c"] = d.c
    return o


def gpu_observed(ctx, descs, mu_len, max_dim=None):
    n = len(descs)
    max_dim = max_dim or max(d.prob.dim for d in descs)
    res = torch.zeros((n, 32), dtype=torch.uint8, device="cuda")
    mu = torch.full((n * mu_len * 2,), -7.0, device="cuda")
    bx = torch.zeros((n, max_dim), dtype=torch.float64, device="cuda")
    say(f"  observed run n={n} mu_len={mu_len} algos={sorted(set(d.algo for d in descs))}")
    ctx.run_observed(descs, res, mu, mu_len, best_x=bx, max_dim=max_dim)
    torch.cuda.synchronize()
    raw = res.cpu().numpy().tobytes()
    out = []
    for r in range(n):
        rr = S.RunResult.from_buffer_copy(raw[r * 32:(r + 1) * 32])
        out.append(dict(best_e=rr.best_e, best_e32=rr.best_e32, fes=rr.fes, generations=rr.generations))
    return out, mu.cpu().numpy().reshape(n, mu_len, 2), bx.cpu().numpy()


@pytest.mark.parametrize("func,dim,np_,budget", [(S.RASTRIGIN, 10, 100, 20000), (S.SCHWEFEL, 30, 60, 9000),
                                                 (S.ELLIPSOID, 100, 200, 12000), (S.ACKLEY, 50, 33, 5000)])
def test_jade_fe_accounting_and_observer_rows(ctx, func, dim, np_, budget):
    d = jdesc(func, dim, np_, budget, uid=71)
    mu_len = budget // np_ + 3
    (g,), mu, _ = gpu_observed(ctx, [d], mu_len)
    o, _, _, omu = O.run(ojdesc(d), SEED, ISEED, mu_len=mu_len)
    assert g["fes"] == o["fes"] and g["generations"] == o["generations"]
    gens = g["generations"]
    assert tuple(mu[0, 0]) == (0.5, 0.5)
    assert np.all(np.isfinite(mu[0, : gens + 1])) and np.all(np.isnan(mu[0, gens + 1:]))
    assert np.all((mu[0, : gens + 1, 0] > 0) & (mu[0, : gens + 1, 0] <= 1))
    assert np.all((mu[0, : gens + 1, 1] >= 0) & (mu[0, : gens + 1, 1] <= 1))
    # generation 1: same population, same draws; F and CR in float
    assert mu[0, 1] == pytest.approx(omu[1], abs=2e-6)


def test_jade_first_generation_rows_many_runs(ctx):
    """Row 1 of 64 runs over the six functions and three dimensions against
    the oracle, each to float rounding."""
    descs = [jdesc(r % 6, (10, 30, 50)[r // 6 % 3], 50 + r % 7, 400, uid=300 + r, inst=r % 4)
             for r in range(64)]
    _, mu, _ = gpu_observed(ctx, descs, 4)
    for k, d in enumerate(descs):
        _, _, _, omu = O.run(ojdesc(d), SEED, ISEED, mu_len=4)
        assert mu[k, 1] == pytest.approx(omu[1], abs=2e-6), k


def test_jade_c0_keeps_the_pair(ctx):
    d = jdesc(S.GRIEWANK, 30, 40, 4000, uid=72, c=0.0)
    (g,), mu, _ = gpu_observed(ctx, [d], 120)
    gens = g["generations"]
    assert np.all(mu[0, : gens + 1] == 0.5) and np.all(np.isnan(mu[0, gens + 1:]))


def test_observer_rows_of_the_other_algorithms(ctx):
    descs = [desc(S.ALGO_DE, S.RASTRIGIN, 10, 50, 3000, uid=81, F=0.7, CR=0.3),
             desc(S.ALGO_PSO, S.RASTRIGIN, 10, 40, 3000, uid=82),
             desc(S.ALGO_SHADE, S.ROSENBROCK, 30, 100, 3000, uid=83),
             desc(S.ALGO_LSHADE, S.ROSENBROCK, 30, 100, 6000, uid=84),
             desc(S.ALGO_PSODE, S.ACKLEY, 10, 40, 3000, uid=85)]
    gres, mu, _ = gpu_observed(ctx, descs, 80)
    de = gres[0]["generations"]
    assert np.array_equal(mu[0, : de + 1], np.tile(np.float32([0.7, 0.3]), (de + 1, 1)))
    assert np.all(np.isnan(mu[0, de + 1:]))
    assert np.all(np.isnan(mu[1]))
    for k in (2, 3, 4):
        _, _, _, omu = O.run(odesc(descs[k]), SEED, ISEED, mu_len=80)
        gk = gres[k]["generations"]
        assert tuple(mu[k, 0]) == (0.5, 0.5)
        assert mu[k, 1] == pytest.approx(omu[1], abs=2e-6), k
        assert np.all(np.isfinite(mu[k, : gk + 1])) and np.all(np.isnan(mu[k, gk + 1:]))


def test_jade_distribution_and_mean_trajectory(ctx):
    """Final errors of 40 runs against the oracle's (KS), and the mean
    (muF, muCR) over the runs -- the case study's plotted quantity -- close to
    the oracle's mean through the first 20 generations."""
    n, np_, budget = 40, 60, 60 * 151
    descs = [jdesc(S.RASTRIGIN, 10, np_, budget, uid=2000 + r, inst=r % 3) for r in range(n)]
    gres, mu, _ = gpu_observed(ctx, descs, 152)
    ores = [O.run(ojdesc(d), SEED, ISEED, mu_len=152) for d in descs]
    for g, o in zip(gres, ores):
        assert g["fes"] == o[0]["fes"] and g["generations"] == o[0]["generations"]
    ge = np.array([g["best_e"] for g in gres])
    oe = np.array([o[0]["best_e"] for o in ores])
    p = stats.ks_2samp(np.log10(ge + 1e-12), np.log10(oe + 1e-12)).pvalue
    say(f"  median gpu {np.median(ge):.3e} oracle {np.median(oe):.3e} KS p={p:.3g}")
    assert p > 1e-3
    omu = np.stack([o[3] for o in ores])
    gm, om = mu[:, :21].mean(axis=0), omu[:, :21].mean(axis=0)
    say(f"  mean muF/muCR after 20 generations: gpu {gm[20]} oracle {om[20]}")
    assert np.max(np.abs(gm - om)) < 0.02


def test_jade_team_and_placement_do_not_change_results(ctx, monkeypatch):
    descs = [jdesc(S.RASTRIGIN, 30, 64, 3000, uid=90), jdesc(S.RASTRIGIN, 30, 20, 3000, uid=91),
             jdesc(S.SCHWEFEL, 10, 150, 6000, uid=92, r_arc=2.6), jdesc(S.ELLIPSOID, 100, 200, 4000, uid=93)]
    base = gpu_observed(ctx, descs, 40, max_dim=100)
    for var, val in (("SEVO_RUN_TEAM", "wave"), ("SEVO_RUN_TEAM", "block"), ("SEVO_RUN_PLACEMENT", "workspace")):
        monkeypatch.setenv(var, val)
        other = gpu_observed(ctx, descs, 40, max_dim=100)
        monkeypatch.delenv(var)
        assert other[0] == base[0], (var, val)
        assert np.array_equal(other[1], base[1], equal_nan=True), (var, val)
        assert np.array_equal(other[2], base[2]), (var, val)


def test_observed_rejects_bad_arguments(ctx):
    res = torch.zeros((1, 32), dtype=torch.uint8, device="cuda")
    mu = torch.zeros(16, device="cuda")
    with pytest.raises(S.SevoError):
        ctx.run_observed([jdesc(S.RASTRIGIN, 10, 50, 1000, 1, c=1.5)], res, mu, 8)
    with pytest.raises(S.SevoError):
        ctx.run_observed([jdesc(S.RASTRIGIN, 10, 50, 1000, 1)], res, mu, 8, precision=S.FP64)
    with pytest.raises(S.SevoError):
        ctx.run_observed([desc(S.ALGO_CSO, S.RASTRIGIN, 10, 50, 1000, 1)], res, mu, 8)
    with pytest.raises(S.SevoError):
        ctx.run_observed([jdesc(S.RASTRIGIN, 10, 50, 1000, 1)], res, None, 8)
