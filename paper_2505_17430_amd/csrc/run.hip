// run.hip -- host side of whole runs: validation, placement and team
// choices, workspace, grouping into launches (one per dimension class,
// algorithm family, placement and team), plans, and the sevo_run entry
// point.  The kernels are in run_kernel.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <vector>

#include "../../include/sevo.h"
#include "run_kernel.h"
#include "state.h"

namespace sevo {

void release_state(sevo_ctx *) {}

}  // namespace sevo

using namespace sevo;

namespace {

int32_t shade_pnum(double p, int32_t np)
{
    long k = std::lround(p * (double)np);
    k = std::max<long>(2, std::min<long>(k, np));
    return (int32_t)k;
}

// Archive slots of an L-SHADE or JADE run (its bound at the initial
// population, plus one); 0 for the other algorithms.
int archive_cap(const sevo_run_desc &d)
{
    if (d.algo != SEVO_ALGO_LSHADE && d.algo != SEVO_ALGO_JADE && d.algo != SEVO_ALGO_LSHADE_RS) return 0;
    return (int)std::lround(d.r_arc * (double)d.np) + 1;
}

int validate_runs(sevo_ctx *ctx, const sevo_run_desc *runs, int n, int precision, int64_t trace_len,
                  const float *trace, const double *best_x, int max_dim)
{
    if (n < 1 || !runs) return set_error(ctx, SEVO_EINVAL, "no runs");
    if (precision != SEVO_FP32 && precision != SEVO_FP64 && precision != SEVO_SPLIT_BF16)
        return set_error(ctx, SEVO_EINVAL, "runs take precision FP32, SPLIT_BF16 (CSO) or FP64");
    if (trace_len < 0 || (trace_len > 0 && !trace)) return set_error(ctx, SEVO_EINVAL, "bad trace");
    for (int r = 0; r < n; ++r) {
        const sevo_run_desc &d = runs[r];
        const sevo_problem &p = d.prob;
        if (p.func < 0 || p.func >= NFUNC || p.dim < 2 || p.dim > MAX_DIM || !(p.lb < p.ub))
            return set_error(ctx, SEVO_EINVAL, "run has an invalid problem");
        if (d.algo != SEVO_ALGO_DE && d.algo != SEVO_ALGO_PSO && d.algo != SEVO_ALGO_SHADE &&
            d.algo != SEVO_ALGO_LSHADE && d.algo != SEVO_ALGO_PSODE && d.algo != SEVO_ALGO_CSO &&
            d.algo != SEVO_ALGO_JADE && d.algo != SEVO_ALGO_LSHADE_RS)
            return set_error(ctx, SEVO_EINVAL, "unknown algorithm");
        if (d.algo == SEVO_ALGO_CSO) {
            // CSO: the update kernels and the batched evaluation, any D
            if (d.np < 2 || d.np > 1024 || d.np % 2 != 0)
                return set_error(ctx, SEVO_EINVAL, "CSO needs an even swarm size in [2, 1024]");
            if (d.budget < 1) return set_error(ctx, SEVO_EINVAL, "budget < 1");
            if (d.max_generations < 0) return set_error(ctx, SEVO_EINVAL, "max_generations < 0");
            if (!std::isfinite(d.c1)) return set_error(ctx, SEVO_EINVAL, "CSO needs a finite phi (c1)");
            if (precision == SEVO_FP64)
                return set_error(ctx, SEVO_EUNSUPPORTED, "CSO runs take precision FP32 or SPLIT_BF16");
            if (best_x && max_dim < p.dim) return set_error(ctx, SEVO_EINVAL, "max_dim < dim");
            continue;
        }
        if (precision == SEVO_SPLIT_BF16)
            return set_error(ctx, SEVO_EINVAL, "precision SPLIT_BF16 is for CSO runs only");
        const bool pso_like = d.algo == SEVO_ALGO_PSO || d.algo == SEVO_ALGO_PSODE;
        const int min_np = d.algo == SEVO_ALGO_PSO ? 1 : 4;
        if (d.np < min_np || d.np > RUN_MAX_NP) return set_error(ctx, SEVO_EINVAL, "np outside [4 (1 for PSO), 256]");
        if (d.budget < 1) return set_error(ctx, SEVO_EINVAL, "budget < 1");
        if (d.max_generations < 0) return set_error(ctx, SEVO_EINVAL, "max_generations < 0");
        if (d.algo == SEVO_ALGO_DE && (!std::isfinite(d.F) || !(d.CR >= 0 && d.CR <= 1)))
            return set_error(ctx, SEVO_EINVAL, "DE needs finite F and CR in [0, 1]");
        if (pso_like && !(d.vmax > 0))
            return set_error(ctx, SEVO_EINVAL, "PSO needs vmax > 0");
        const bool lshade_like = d.algo == SEVO_ALGO_LSHADE || d.algo == SEVO_ALGO_LSHADE_RS;
        if ((d.algo == SEVO_ALGO_SHADE || lshade_like || d.algo == SEVO_ALGO_PSODE) &&
            (d.H < 1 || d.H > 16 || !(d.p > 0 && d.p <= 1)))
            return set_error(ctx, SEVO_EINVAL, "SHADE needs H in [1, 16] and p in (0, 1]");
        if (lshade_like && (d.np_min < 4 || d.np_min > d.np || !(d.r_arc >= 0 && d.r_arc <= 2.9)))
            return set_error(ctx, SEVO_EINVAL, "L-SHADE needs np_min in [4, np] and r_arc in [0, 2.9]");
        if (d.algo == SEVO_ALGO_LSHADE_RS && std::isnan(d.restart_tol))
            return set_error(ctx, SEVO_EINVAL, "L-SHADE-Restart needs a restart_tol that is not NaN");
        if (d.algo == SEVO_ALGO_JADE &&
            (!(d.p > 0 && d.p <= 1) || !(d.r_arc >= 0 && d.r_arc <= 2.9) || !(d.c >= 0 && d.c <= 1)))
            return set_error(ctx, SEVO_EINVAL, "JADE needs p in (0, 1], r_arc in [0, 2.9] and c in [0, 1]");
        if (best_x && max_dim < p.dim) return set_error(ctx, SEVO_EINVAL, "max_dim < dim");
        if (precision == SEVO_FP32 && p.dim > SMALL_D_MAX)
            return set_error(ctx, SEVO_EUNSUPPORTED, "fused runs support D <= 120");
        if (pso_like && (d.topology < 0 || d.topology > 1 || d.velocity < 0 || d.velocity > 1))
            return set_error(ctx, SEVO_EINVAL, "PSO topology and velocity are 0 or 1");
        if (precision == SEVO_FP64 && d.algo == SEVO_ALGO_PSO && (d.topology != 0 || d.velocity != 0))
            return set_error(ctx, SEVO_EUNSUPPORTED, "the double-precision PSO is global-best inertia");
        if (precision == SEVO_FP64 && (d.algo == SEVO_ALGO_SHADE || lshade_like ||
                                       d.algo == SEVO_ALGO_PSODE || d.algo == SEVO_ALGO_JADE))
            return set_error(ctx, SEVO_EUNSUPPORTED, "the double-precision run path has DE and PSO");
    }
    return SEVO_OK;
}

// Dynamic LDS that a workgroup of k_run<ks, on chip, team, family> may take: what
// the device allows beside the kernel's own arrays, capped so that two
// workgroups still fit a CU's 160 KB.  0 when not available.  Computed once
// per process and kernel.
static size_t onchip_limit(int ks, bool wave, int fam)
{
    static size_t cache[64][2][NFAM][2] = {};   // [ks][wave][family] = {done, limit}
    constexpr size_t CAP = 80 * 1024;
    if (ks < 1 || ks >= 64) return 0;
    size_t *c = cache[ks][wave ? 1 : 0][fam];
    if (c[0]) return c[1];
    size_t lim = 0;
    int dev = 0, maxblk = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&maxblk, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess) {
        const void *k = (const void *)run_table(fam, ks, true, wave);
        hipFuncAttributes fa;
        const size_t total = std::min((size_t)maxblk, CAP);
        // an on-chip variant that spills registers to scratch (at the largest
        // k-step counts of some families) is never used: its runs take the
        // workspace variant, which does not spill
        if (k && hipFuncGetAttributes(&fa, k) == hipSuccess && fa.localSizeBytes == 0 &&
            total > fa.sharedSizeBytes) {
            const size_t want = total - fa.sharedSizeBytes;
            if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)want) == hipSuccess)
                lim = want;
        }
    }
    (void)hipGetLastError();
    c[0] = 1;
    c[1] = lim;
    return lim;
}

int run_fused(sevo_ctx *ctx, const sevo_run_desc *runs, int n, sevo_run_result *results, float *trace,
              int64_t trace_len, double *best_x, int max_dim, float *mu, int64_t mu_len, const sevo_run_state *st,
              hipStream_t stream)
{
    // Team: runs of up to 64 individuals get one wave each (four runs of
    // one instance per workgroup), larger ones a whole workgroup.
    // Placement: a population that fits in the LDS left beside the kernel's
    // own arrays stays on chip, the others use the workspace.  Results do
    // not depend on either choice (the tests compare them); the variables
    // SEVO_RUN_TEAM=block|wave and SEVO_RUN_PLACEMENT=workspace force the
    // alternatives.
    const char *tv = std::getenv("SEVO_RUN_TEAM");
    const bool force_block = tv && std::strcmp(tv, "block") == 0;
    const char *pl = std::getenv("SEVO_RUN_PLACEMENT");
    const bool force_ws = pl && std::strcmp(pl, "workspace") == 0;
    // Wave teams pay off once a dimension class has enough small runs to
    // fill the GPU with four-run workgroups; a few runs go faster with a
    // whole workgroup each (SEVO_RUN_TEAM=wave forces wave teams).
    const bool force_wave = tv && std::strcmp(tv, "wave") == 0;
    int cus = 256, dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    std::map<int, int> small_in_class;
    for (int r = 0; r < n; ++r)
        if (runs[r].algo != SEVO_ALGO_CSO && runs[r].np <= 64) ++small_in_class[ks_of(runs[r].prob.dim)];
    std::vector<char> onchip(n), wave(n);
    std::vector<size_t> dyn(n), off(n);
    size_t total = 0;
    for (int r = 0; r < n; ++r) {
        if (runs[r].algo == SEVO_ALGO_CSO) continue;   // cso.hip runs those
        const int npp = (runs[r].np + 15) & ~15;
        const size_t D = runs[r].prob.dim;
        const size_t nbuf = runs[r].algo == SEVO_ALGO_PSODE ? 4 : runs[r].algo == SEVO_ALGO_PSO ? 3 : 2;
        const bool many = small_in_class[ks_of((int)D)] >= 4 * cus;
        wave[r] = !force_block && runs[r].np <= 64 && (many || force_wave) ? 1 : 0;
        dyn[r] = nbuf * D * npp;   // floats
        const size_t per_wg = (wave[r] ? 4 : 1) * dyn[r] * sizeof(float);
        onchip[r] = !force_ws && per_wg <= onchip_limit(ks_of((int)D), wave[r], family_of(runs[r].algo)) ? 1 : 0;
        off[r] = total;
        total += (onchip[r] ? 0 : 4 * D * npp) + D + D * (size_t)archive_cap(runs[r]);
        total = (total + 63) & ~(size_t)63;
    }
    float *ws = nullptr;
    int rc = ctx_ws(ctx).get(ctx, WS_RUN, total * sizeof(float), (void **)&ws);
    if (rc) return rc;
    // one launch per (dimension class, family, placement, team)
    struct Group {
        std::vector<RunDev> runs;
        std::vector<double> cost;
        size_t stride = 0;
    };
    std::map<int, Group> groups;
    for (int r = 0; r < n; ++r) {
        const sevo_run_desc &d = runs[r];
        if (d.algo == SEVO_ALGO_CSO) continue;
        InstanceView I;
        if ((rc = lookup_instance(ctx, &d.prob, d.instance, &I))) return rc;
        RunDev R{};
        R.algo = d.algo;
        R.func = d.prob.func;
        R.dim = d.prob.dim;
        R.np = d.np;
        R.npp = (d.np + 15) & ~15;
        R.run_uid = d.run_uid;
        R.H = d.algo == SEVO_ALGO_JADE ? 1 : d.H;
        R.pnum = d.algo == SEVO_ALGO_SHADE || d.algo == SEVO_ALGO_PSODE ? shade_pnum(d.p, d.np) : 0;
        R.budget = d.budget;
        R.F = (float)d.F;
        R.w = (float)d.w;
        R.c1 = (float)d.c1;
        R.c2 = (float)d.c2;
        R.vmax = (float)d.vmax;
        R.thr = cr_threshold(d.CR);
        R.lb = (float)d.prob.lb;
        R.ub = (float)d.prob.ub;
        R.o = I.o;
        R.Mfrag = I.Mfrag;
        R.tab = I.tab;
        R.M64 = I.M64;
        float *b = ws + off[r];
        if (onchip[r]) {
            R.X = R.U = R.V = R.P = nullptr;
            R.bestx = b;
        } else {
            const size_t DN = (size_t)R.dim * R.npp;
            R.X = b; R.U = b + DN; R.V = b + 2 * DN; R.P = b + 3 * DN;
            R.bestx = b + 4 * DN;
        }
        const bool pso_like = d.algo == SEVO_ALGO_PSO || d.algo == SEVO_ALGO_PSODE;
        R.topology = pso_like ? d.topology : 0;
        R.velocity = pso_like ? d.velocity : 0;
        R.p = d.p;
        R.r_arc = d.r_arc;
        R.np_min = d.algo == SEVO_ALGO_JADE ? d.np : d.np_min;
        R.acap = archive_cap(d);
        R.Arc = R.acap > 0 ? R.bestx + R.dim : nullptr;
        R.res = results;
        R.trace = trace;
        R.trace_len = trace_len;
        R.best_x_out = best_x;
        R.max_dim = max_dim;
        R.out_index = r;
        R.mu = mu_len > 0 ? mu : nullptr;
        R.mu_len = mu_len;
        R.c_adapt = d.c;
        R.CR = (float)d.CR;
        R.restart = d.algo == SEVO_ALGO_LSHADE_RS ? 1 : 0;
        R.restart_tol = d.restart_tol;
        R.gen_cap = d.max_generations;
        if (st) {
            R.st_np = st->max_np;
            R.st_dim = st->max_dim;
            R.st_arc = st->max_arc;
            R.st_x = st->x;
            R.st_e = st->e;
            R.st_u = st->u;
            R.st_eu = st->eu;
            R.st_v = st->v;
            R.st_p = st->p;
            R.st_ep = st->ep;
            R.st_mem = st->memory;
            R.st_arc_out = st->archive;
            R.st_cnt = st->counts;
        }
        Group &G = groups[(ks_of(R.dim) * NFAM + family_of(d.algo)) * 4 + onchip[r] * 2 + wave[r]];
        G.runs.push_back(R);
        G.cost.push_back((double)d.budget * R.dim * R.dim);
        if (onchip[r]) G.stride = std::max(G.stride, dyn[r]);
    }
    // Launch order and streams.  Groups go longest run first.  A group
    // whose workgroups fill every slot the GPU holds for its kernel runs
    // alone: such groups follow one another on the caller's stream, since
    // beside another group part of its workgroups would wait for a slot and
    // finish a whole run length late (measured: 2048 L-SHADE runs at
    // D = 10, 30, 50, 100, 1.39 s one class after another against 1.89 s
    // together).  Smaller groups get an internal stream each and run beside
    // the others (4096 PSO swarms in three classes of 360 workgroups:
    // 105 ms together against 139 ms).  A plan records each launch's stream index
    // and forks when it is launched.  SEVO_RUN_GROUPS=serial|concurrent
    // forces one way for all groups.
    struct Prepared {
        std::vector<RunDev> launch;
        unsigned grid;
        bool on, wave;
        int key;
        size_t stride;
        int lane;
    };
    std::vector<std::pair<double, std::map<int, Group>::iterator>> byc;
    for (auto itg = groups.begin(); itg != groups.end(); ++itg)
        byc.emplace_back(*std::max_element(itg->second.cost.begin(), itg->second.cost.end()), itg);
    std::stable_sort(byc.begin(), byc.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
    std::vector<Prepared> prep;
    for (auto &bc : byc) {
        auto &kv = *bc.second;
        const bool gon = (kv.first & 2) != 0, gwave = (kv.first & 1) != 0;
        Group &G = kv.second;
        std::vector<RunDev> launch;
        std::vector<int> order(G.runs.size());
        for (size_t i = 0; i < G.runs.size(); ++i) order[i] = (int)i;
        if (!gwave) {
            // longest runs first, so the tail is short
            std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return G.cost[a] > G.cost[b]; });
            for (int i : order) launch.push_back(G.runs[i]);
        } else {
            // workgroups of four runs of one instance (empty slots have np = 0),
            // workgroups with the longest runs first
            std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
                if (G.runs[a].Mfrag != G.runs[b].Mfrag) return G.runs[a].Mfrag < G.runs[b].Mfrag;
                return G.cost[a] > G.cost[b];
            });
            std::vector<std::pair<double, std::vector<int>>> wgs;
            for (size_t i = 0; i < order.size();) {
                std::vector<int> m;
                const float *inst = G.runs[order[i]].Mfrag;
                while (i < order.size() && m.size() < 4 && G.runs[order[i]].Mfrag == inst) m.push_back(order[i++]);
                wgs.emplace_back(G.cost[m[0]], m);
            }
            std::stable_sort(wgs.begin(), wgs.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
            for (const auto &w : wgs)
                for (int k = 0; k < 4; ++k) {
                    if (k < (int)w.second.size()) {
                        launch.push_back(G.runs[w.second[k]]);
                    } else {
                        RunDev E = G.runs[w.second[0]];   // same instance, no work
                        E.np = 0;
                        launch.push_back(E);
                    }
                }
        }
        const unsigned grid = (unsigned)(gwave ? launch.size() / 4 : launch.size());
        prep.push_back({std::move(launch), grid, gon, gwave, kv.first, G.stride, 0});
    }
    const char *gm = std::getenv("SEVO_RUN_GROUPS");
    const bool all_serial = gm && std::strcmp(gm, "serial") == 0;
    const bool all_conc = gm && std::strcmp(gm, "concurrent") == 0;
    int ng = 1;   // lane 0: the caller's stream, for the groups that run alone
    for (auto &P : prep) {
        bool alone = all_serial;
        if (!all_serial && !all_conc) {
            int per_cu = 0;
            const size_t shm = P.on ? (P.wave ? 4 : 1) * P.stride * sizeof(float) : 0;
            RunKernel k = run_table(P.key / 4 % NFAM, P.key / 4 / NFAM, P.on, P.wave);
            if (k && hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 256, shm) == hipSuccess && per_cu > 0)
                alone = (long)P.grid >= (long)per_cu * cus;
            (void)hipGetLastError();
        }
        P.lane = alone ? 0 : ng++;
    }
    const bool recording = ctx_recording(ctx) != nullptr;
    std::vector<hipStream_t> ss(ng, stream);
    if (!recording && ng > 1) {
        if ((rc = fork_streams(ctx, stream, ng - 1, ss.data() + 1))) return rc;
    }
    for (auto &P : prep) {
        const int g = P.lane;
        std::vector<char> blob(P.launch.size() * sizeof(RunDev));
        std::memcpy(blob.data(), P.launch.data(), blob.size());
        const void *d = nullptr;
        int slot;
        if ((rc = stage_blob(ctx, blob, ss[g], &d, &slot))) return rc;
        const size_t shm = P.on ? (P.wave ? 4 : 1) * P.stride * sizeof(float) : 0;
        const Launch L{L_RUN, d, (int)P.launch.size(), P.key / 4 / NFAM, 0, (int)P.grid, P.on, P.wave, shm,
                       (int)P.stride, g, P.key / 4 % NFAM};
        if ((rc = emit_launch(ctx, L, ss[g]))) return rc;
        if ((rc = finish_slot(ctx, slot, ss[g]))) return rc;
    }
    return recording || ng == 1 ? SEVO_OK : join_streams(ctx, stream, ng - 1, ss.data() + 1);
}

// Single-precision runs: the fused kernels for DE, SHADE, L-SHADE, PSO and
// PSODE, the update-and-evaluate loop for CSO.
int run_single(sevo_ctx *ctx, const sevo_run_desc *runs, int n, int precision, sevo_run_result *results,
               float *trace, int64_t trace_len, double *best_x, int max_dim, hipStream_t stream,
               float *mu = nullptr, int64_t mu_len = 0, const sevo_run_state *st = nullptr)
{
    bool fused = false;
    for (int r = 0; r < n; ++r) fused |= runs[r].algo != SEVO_ALGO_CSO;
    int rc = SEVO_OK;
    if (fused &&
        (rc = run_fused(ctx, runs, n, results, trace, trace_len, best_x, max_dim, mu, mu_len, st, stream)))
        return rc;
    return cso_runs(ctx, runs, n, precision, results, trace, trace_len, best_x, max_dim, stream);
}

}  // namespace

hipError_t sevo::exec_run_launch(const Launch &L, hipStream_t stream, uint32_t seed32, const Consts &k)
{
    RunKernel kern = run_table(L.fam, L.ks, L.flag, L.wave);
    if (!kern) return hipErrorInvalidValue;
    hipLaunchKernelGGL(kern, dim3((unsigned)L.grid), dim3(256), L.shm, stream, (const RunDev *)L.d, seed32, k,
                       L.stride);
    return hipGetLastError();
}

extern "C" int sevo_plan_run(sevo_ctx *ctx, const sevo_run_desc *runs, int32_t n_runs, int32_t precision,
                             sevo_run_result *results, float *trace, int64_t trace_len, double *best_x,
                             int32_t max_dim, sevo_plan **out)
{
    if (!ctx) return set_error(nullptr, SEVO_EINVAL, "ctx is NULL");
    if (!out) return set_error(ctx, SEVO_EINVAL, "out is NULL");
    *out = nullptr;
    if (!results) return set_error(ctx, SEVO_EINVAL, "results is NULL");
    int rc = validate_runs(ctx, runs, n_runs, precision, trace_len, trace, best_x, max_dim);
    if (rc) return rc;
    if (precision == SEVO_FP64) return set_error(ctx, SEVO_EUNSUPPORTED, "plans run single-precision runs only");
    DeviceScope dg(ctx);
    for (int r = 0; r < n_runs; ++r) {   // instances are made before recording
        InstanceView I;
        if ((rc = lookup_instance(ctx, &runs[r].prob, runs[r].instance, &I))) return rc;
    }
    if ((rc = plan_begin(ctx))) return rc;
    rc = run_single(ctx, runs, n_runs, precision, results, trace, trace_len, best_x, max_dim, nullptr);
    return plan_finish(ctx, rc, out);
}

extern "C" int sevo_run(sevo_ctx *ctx, const sevo_run_desc *runs, int32_t n_runs, int32_t precision,
                        sevo_run_result *results, float *trace, int64_t trace_len, double *best_x,
                        int32_t max_dim, void *stream)
{
    if (!ctx) return set_error(nullptr, SEVO_EINVAL, "ctx is NULL");
    if (!results) return set_error(ctx, SEVO_EINVAL, "results is NULL");
    int rc = validate_runs(ctx, runs, n_runs, precision, trace_len, trace, best_x, max_dim);
    if (rc) return rc;
    DeviceScope dg(ctx);
    if (precision != SEVO_FP64)
        return run_single(ctx, runs, n_runs, precision, results, trace, trace_len, best_x, max_dim,
                          (hipStream_t)stream);
    return run_plain_f64(ctx, runs, n_runs, results, trace, trace_len, best_x, max_dim, (hipStream_t)stream);
}

extern "C" int sevo_run_observed(sevo_ctx *ctx, const sevo_run_desc *runs, int32_t n_runs, int32_t precision,
                                 sevo_run_result *results, float *trace, int64_t trace_len, double *best_x,
                                 int32_t max_dim, float *mu, int64_t mu_len, void *stream)
{
    if (!ctx) return set_error(nullptr, SEVO_EINVAL, "ctx is NULL");
    if (!results) return set_error(ctx, SEVO_EINVAL, "results is NULL");
    if (mu_len < 0 || (mu_len > 0 && !mu)) return set_error(ctx, SEVO_EINVAL, "bad observer buffer");
    int rc = validate_runs(ctx, runs, n_runs, precision, trace_len, trace, best_x, max_dim);
    if (rc) return rc;
    if (mu_len > 0) {
        if (precision != SEVO_FP32)
            return set_error(ctx, SEVO_EUNSUPPORTED, "the parameter observer records FP32 runs");
        for (int r = 0; r < n_runs; ++r)
            if (runs[r].algo == SEVO_ALGO_CSO)
                return set_error(ctx, SEVO_EUNSUPPORTED, "the parameter observer records no CSO runs");
    }
    DeviceScope dg(ctx);
    if (precision != SEVO_FP64)
        return run_single(ctx, runs, n_runs, precision, results, trace, trace_len, best_x, max_dim,
                          (hipStream_t)stream, mu, mu_len);
    return run_plain_f64(ctx, runs, n_runs, results, trace, trace_len, best_x, max_dim, (hipStream_t)stream);
}

extern "C" int sevo_run_snapshot(sevo_ctx *ctx, const sevo_run_desc *runs, int32_t n_runs, int32_t precision,
                                 sevo_run_result *results, float *trace, int64_t trace_len, double *best_x,
                                 int32_t max_dim, const sevo_run_state *state, void *stream)
{
    if (!ctx) return set_error(nullptr, SEVO_EINVAL, "ctx is NULL");
    if (!results) return set_error(ctx, SEVO_EINVAL, "results is NULL");
    if (!state || !state->x || !state->e) return set_error(ctx, SEVO_EINVAL, "state needs x and e");
    int rc = validate_runs(ctx, runs, n_runs, precision, trace_len, trace, best_x, max_dim);
    if (rc) return rc;
    if (precision != SEVO_FP32) return set_error(ctx, SEVO_EUNSUPPORTED, "run states come from FP32 runs");
    for (int r = 0; r < n_runs; ++r) {
        const sevo_run_desc &d = runs[r];
        if (d.algo == SEVO_ALGO_CSO) return set_error(ctx, SEVO_EUNSUPPORTED, "no run state for CSO runs");
        if (d.np > state->max_np || d.prob.dim > state->max_dim)
            return set_error(ctx, SEVO_EINVAL, "state rows shorter than a run's np or dim");
        if (state->archive && archive_cap(d) > 0 && archive_cap(d) - 1 > state->max_arc)
            return set_error(ctx, SEVO_EINVAL, "state archive narrower than a run's archive bound");
    }
    DeviceScope dg(ctx);
    return run_single(ctx, runs, n_runs, precision, results, trace, trace_len, best_x, max_dim,
                      (hipStream_t)stream, nullptr, 0, state);
}
