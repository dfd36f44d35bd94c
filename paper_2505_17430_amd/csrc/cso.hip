// cso.hip -- CSO runs (the competitive swarm optimizer of Cheng and Jin, the
// optimiser of the paper's large-scale study, Sec. 3.3: a swarm of 300 and
// 1e6 evaluations at D = 1000).
//
// An iteration evaluates only the m/2 losers of one swarm, too little work to
// fill the GPU with one run, so the runs advance together:
//   k_cso_pair(t)    one workgroup per run: takes in the previous iteration's
//                    loser errors, records them, pairs the swarm and writes
//                    the winner and loser lists;
//   k_cso_update(t)  one workgroup per (run, slice of 16 dimensions): the
//                    swarm mean of each coordinate and the losers' moves,
//                    their new positions also into the gather buffer G;
//   evaluation       the batched evaluation of every run's G (small- or
//                    large-D kernels, FP32 or split-bf16), launches prepared
//                    once per buffer parity.
// The error list E, the loser list L and G alternate between two buffers by
// the parity of t, so no kernel overwrites what the next one still reads.
// Runs that need fewer iterations than the longest stop recording after
// their last one (their later evaluations are not used).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/sevo.h"
#include "algo.h"
#include "objective.h"
#include "runtime.h"
#include "state.h"

namespace sevo {
namespace {

constexpr int CSO_MAX_M = 1024;   // swarm size limit (pairing in LDS)
constexpr int CSO_SLICE = 16;     // dimensions per update workgroup
constexpr int CSO_THREADS = 256;

enum { CSO_INIT = 0, CSO_BEGIN = 1, CSO_PAIR = 2, CSO_UPDATE = 3, CSO_FINISH = 4 };

// One CSO run as the kernels see it.  X, V: [dim][ldx]; G[p]: [dim][ldg];
// E[p]: [ldx]; EG: [ldg]; L[p]: [ldg] (loser of each pair).
struct CsoDev {
    int32_t func, dim, m, h, ldx, ldg;
    uint32_t run_uid;
    int32_t iters;            // iterations to run
    int64_t budget;
    float lb, ub, phi;
    float *X, *V, *G[2], *E[2], *EG;
    int32_t *L[2], *W;        // losers (by parity of t) and winners of the pairs
    float *bestx;             // [dim]
    float *best;              // [0]: best of all evaluations, [1]: of the first `budget`
    const double *o, *M64;
    sevo_run_result *res;
    float *trace;
    int64_t trace_len;
    double *best_x_out;
    int32_t max_dim, out_index;
};

// Record n evaluations e[0..n) (in LDS, in evaluation order) that follow fe0
// earlier ones: the best so far, the best of the first `budget` (lowest
// position among equal values) and its point (column c of P, leading
// dimension ld), the trace entry at every 200th evaluation (the best so far
// there).  Wave 0 takes the items lane-strided and combines lanes by
// butterflies; the whole workgroup calls it.
__device__ void record_batch(const CsoDev &R, const float *e, int n, int64_t fe0, const float *P, int ld,
                             int *sIdx)
{
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const int64_t left = R.budget - fe0;
        const int lim = left < n ? (int)max<int64_t>(left, 0) : n;   // items within the budget
        float mn = INFINITY, bk = INFINITY;
        int bi = 0x7fffffff;
        for (int c = lane; c < n; c += 64) {
            const float k = err_key(e[c]);
            mn = fminf(mn, k);
            if (c < lim && k < bk) {
                bk = k;
                bi = c;
            }
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            mn = fminf(mn, __shfl_xor(mn, o, 64));
            const float ok = __shfl_xor(bk, o, 64);
            const int oi = __shfl_xor(bi, o, 64);
            if (ok < bk || (ok == bk && oi < bi)) {
                bk = ok;
                bi = oi;
            }
        }
        const float before = R.best[0], beforeB = R.best[1];
        if (R.trace) {
            // positions c with (fe0 + c + 1) a multiple of 200
            for (int cp = TRACE_EVERY - 1 - (int)(fe0 % TRACE_EVERY); cp < n; cp += TRACE_EVERY) {
                float pm = INFINITY;
                for (int c = lane; c <= cp; c += 64) pm = fminf(pm, err_key(e[c]));
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1) pm = fminf(pm, __shfl_xor(pm, o, 64));
                const int64_t q = (fe0 + cp + 1) / TRACE_EVERY - 1;
                if (lane == 0 && q < R.trace_len) R.trace[(int64_t)R.out_index * R.trace_len + q] = fminf(before, pm);
            }
        }
        if (lane == 0) {
            const bool imp = bk < beforeB;
            R.best[0] = fminf(before, mn);
            if (imp) R.best[1] = bk;
            *sIdx = imp ? bi : -1;
        }
    }
    __syncthreads();
    const int kb = *sIdx;
    if (kb >= 0)
        for (int j = threadIdx.x; j < R.dim; j += CSO_THREADS) R.bestx[j] = P[(int64_t)j * ld + kb];
    __syncthreads();
}

// Generation 0: x uniform in the box (double, then rounded to float), v = 0.
__global__ __launch_bounds__(CSO_THREADS) void k_cso_init(const CsoDev *__restrict__ runs, uint32_t seed32)
{
    const CsoDev R = runs[blockIdx.x];   // by value: stores through its pointers cannot alias it
    const int j0 = blockIdx.y * CSO_SLICE;
    if (j0 >= R.dim) return;
    const int j1 = min(R.dim, j0 + CSO_SLICE);
    for (int q = threadIdx.x; q < (j1 - j0) * R.m; q += CSO_THREADS) {
        const int j = j0 + q / R.m, i = q % R.m;
        const u32x4 w = draw(R.run_uid, seed32, 0, (uint32_t)i, TAG_INIT_X, (uint32_t)(j / 4));
        R.X[(int64_t)j * R.ldx + i] =
            (float)((double)R.lb + ((double)R.ub - (double)R.lb) * u24d(word(w, j % 4)));
        R.V[(int64_t)j * R.ldx + i] = 0.f;
    }
}

// After the initial evaluation: record it, in index order.
__global__ __launch_bounds__(CSO_THREADS) void k_cso_begin(const CsoDev *__restrict__ runs)
{
    const CsoDev R = runs[blockIdx.x];   // by value: stores through its pointers cannot alias it
    __shared__ float sE[CSO_MAX_M];
    __shared__ int sIdx;
    if (threadIdx.x == 0) {
        R.best[0] = INFINITY;
        R.best[1] = INFINITY;
    }
    for (int i = threadIdx.x; i < R.m; i += CSO_THREADS) sE[i] = R.E[0][i];
    __syncthreads();
    record_batch(R, sE, R.m, 0, R.X, R.ldx, &sIdx);
}

// Iteration t (1-based), one workgroup per run: take in and record
// iteration t - 1's evaluations, then (t <= iters) pair the swarm.
__global__ __launch_bounds__(CSO_THREADS) void k_cso_pair(const CsoDev *__restrict__ runs, uint32_t seed32, int t)
{
    const CsoDev R = runs[blockIdx.x];   // by value: stores through its pointers cannot alias it
    if (t > R.iters + 1) return;
    const int tid = threadIdx.x, m = R.m, h = R.h;
    __shared__ float sE[CSO_MAX_M];
    __shared__ unsigned long long sK[CSO_MAX_M];
    __shared__ float sEG[CSO_MAX_M / 2];
    __shared__ int sIdx;

    const float *Eprev = R.E[(t - 1) & 1];
    for (int i = tid; i < m; i += CSO_THREADS) sE[i] = Eprev[i];
    if (t >= 2)
        for (int k = tid; k < h; k += CSO_THREADS) sEG[k] = R.EG[k];
    __syncthreads();
    if (t >= 2) {
        // the losers of iteration t - 1 take their new errors
        const int32_t *Lp = R.L[(t - 1) & 1];
        for (int k = tid; k < h; k += CSO_THREADS) sE[Lp[k]] = sEG[k];
        __syncthreads();
        record_batch(R, sEG, h, (int64_t)m + (int64_t)(t - 2) * h, R.G[(t - 1) & 1], R.ldg, &sIdx);
    }
    if (t > R.iters) return;
    for (int i = tid; i < m; i += CSO_THREADS) R.E[t & 1][i] = sE[i];

    // pairing: the particles in ascending order of (key, index), two at a
    // time; the distinct 64-bit values key << 32 | index sorted by a bitonic
    // network over the next power of two (padding sorts last)
    int N = 2;
    while (N < m) N <<= 1;
    for (int i = tid; i < N; i += CSO_THREADS)
        sK[i] = i < m ? ((unsigned long long)draw(R.run_uid, seed32, (uint32_t)t, (uint32_t)i, TAG_CSO_PAIR, 0).x << 32) |
                            (uint32_t)i
                      : ~0ull;
    __syncthreads();
    for (int k = 2; k <= N; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int p = tid; p < N / 2; p += CSO_THREADS) {
                const int i = ((p & ~(j - 1)) << 1) | (p & (j - 1));   // i has bit j clear, partner i + j
                const unsigned long long a = sK[i], b = sK[i + j];
                if ((a > b) == ((i & k) == 0)) {
                    sK[i] = b;
                    sK[i + j] = a;
                }
            }
            __syncthreads();
        }
    for (int k = tid; k < h; k += CSO_THREADS) {
        const int a = (int)(uint32_t)sK[2 * k], b = (int)(uint32_t)sK[2 * k + 1];
        const float ka = err_key(sE[a]), kb = err_key(sE[b]);
        const bool a_wins = ka < kb || (ka == kb && a < b);
        R.W[k] = a_wins ? a : b;
        R.L[t & 1][k] = a_wins ? b : a;
    }
}

// Iteration t, one workgroup per (run, slice of CSO_SLICE dimensions): the
// swarm mean of each coordinate, then the losers' moves.
__global__ __launch_bounds__(CSO_THREADS) void k_cso_update(const CsoDev *__restrict__ runs, uint32_t seed32, int t)
{
    const CsoDev &R = runs[blockIdx.x];
    if (t > R.iters) return;
    const int tid = threadIdx.x, m = R.m, h = R.h, D = R.dim;
    const int j0 = blockIdx.y * CSO_SLICE;
    if (j0 >= D) return;
    const int nd = min(D - j0, CSO_SLICE);
    float *__restrict__ X = R.X + (int64_t)j0 * R.ldx;
    float *__restrict__ V = R.V + (int64_t)j0 * R.ldx;
    float *__restrict__ G = R.G[t & 1] + (int64_t)j0 * R.ldg;
    const int ldx = R.ldx, ldg = R.ldg;
    const float lb = R.lb, ub = R.ub, phi = R.phi;
    const uint32_t uid = R.run_uid;
    __shared__ int sW[CSO_MAX_M / 2], sL[CSO_MAX_M / 2];
    __shared__ float sXbar[CSO_SLICE];
    const int32_t *Lt = R.L[t & 1];
    for (int k = tid; k < h; k += CSO_THREADS) {
        sW[k] = R.W[k];
        sL[k] = Lt[k];
    }
    // means: wave w sums the coordinates w, w + 4, ... of the slice, all
    // loads first; a fixed lane-strided sum and butterfly per coordinate
    // (the same bits in every lane and for any slicing)
    const int lane = tid & 63, wave = tid >> 6;
    constexpr int PER_WAVE = CSO_SLICE / (CSO_THREADS / 64);
    float part[PER_WAVE];
#pragma unroll
    for (int c = 0; c < PER_WAVE; ++c) {
        part[c] = 0.f;
        const int jl = wave + c * (CSO_THREADS / 64);
        if (jl < nd)
            for (int i = lane; i < m; i += 64) part[c] += X[(int64_t)jl * ldx + i];
    }
#pragma unroll
    for (int c = 0; c < PER_WAVE; ++c) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) part[c] += __shfl_xor(part[c], o, 64);
        const int jl = wave + c * (CSO_THREADS / 64);
        if (lane == 0 && jl < nd) sXbar[jl] = part[c] / (float)m;
    }
    __syncthreads();
    // losers: work items (coordinate jl, pair k), item q = jl h + k, taken
    // CSO_THREADS apart in batches of UB per thread, loads of a batch before
    // its stores; (jl, k) advance without division
    constexpr int UB = 4;
    const int sj = CSO_THREADS / h, sk = CSO_THREADS % h;
    int jq = tid / h, kq = tid % h;
    while (jq < nd) {
        int jj[UB], kk[UB];
        float xl[UB], vl[UB], xw[UB];
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            jj[u] = jq;
            kk[u] = kq;
            kq += sk;
            jq += sj;
            if (kq >= h) {
                kq -= h;
                ++jq;
            }
            const int64_t row = (int64_t)min(jj[u], nd - 1) * ldx;
            xl[u] = X[row + sL[kk[u]]];
            vl[u] = V[row + sL[kk[u]]];
            xw[u] = X[row + sW[kk[u]]];
        }
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            if (jj[u] >= nd) break;
            const int l = sL[kk[u]];
            const u32x4 r = draw(uid, seed32, (uint32_t)t, (uint32_t)l, TAG_CSO_R, (uint32_t)(j0 + jj[u]));
            float v = u24f(r.x) * vl[u] + u24f(r.y) * (xw[u] - xl[u]) + phi * u24f(r.z) * (sXbar[jj[u]] - xl[u]);
            float x = xl[u] + v;
            if (x < lb) { x = lb; v = 0.f; }
            else if (x > ub) { x = ub; v = 0.f; }
            const int64_t row = (int64_t)jj[u] * ldx;
            X[row + l] = x;
            V[row + l] = v;
            G[(int64_t)jj[u] * ldg + kk[u]] = x;
        }
    }
}

// Double-precision error of a float point (the final check): rows of z by
// the workgroup, then the objective by thread 0 (valid there only).
template <int FUNC>
__device__ double error_f64(const CsoDev &R, const float *x, double *sZ, const Consts &K)
{
    const int D = R.dim;
    for (int r = threadIdx.x; r < D; r += CSO_THREADS) {
        double z = 0.0;
        for (int k = 0; k < D; ++k) z = fma(R.M64[(int64_t)r * D + k], (double)x[k] - R.o[k], z);
        sZ[r] = z;
    }
    __syncthreads();
    double e = 0.0;
    if (threadIdx.x == 0) {
        Acc<double> acc;
        acc.init();
        for (int r = 0; r < D; ++r) {
            double tab = 0.0;
            if constexpr (FUNC == ELLIPSOID) tab = pow(10.0, 6.0 * r / (D - 1));
            if constexpr (FUNC == GRIEWANK) tab = 1.0 / sqrt((double)(r + 1));
            add_term<FUNC>(acc, sZ[r], r + 1 < D ? sZ[r + 1] : 0.0, r + 1 < D, tab, K.kd);
        }
        e = finalize<FUNC>(acc, D);
    }
    return e;
}

// Results; the best point is re-evaluated in double once below 1e-6.
__global__ __launch_bounds__(CSO_THREADS) void k_cso_finish(const CsoDev *__restrict__ runs, Consts K)
{
    const CsoDev R = runs[blockIdx.x];   // by value: stores through its pointers cannot alias it
    __shared__ double sZ[MAX_DIM];
    const float be = R.best[1];
    double e64 = (double)be;
    if (be < 1e-6f) {
        switch (R.func) {
        case ELLIPSOID: e64 = error_f64<ELLIPSOID>(R, R.bestx, sZ, K); break;
        case ROSENBROCK: e64 = error_f64<ROSENBROCK>(R, R.bestx, sZ, K); break;
        case RASTRIGIN: e64 = error_f64<RASTRIGIN>(R, R.bestx, sZ, K); break;
        case SCHWEFEL: e64 = error_f64<SCHWEFEL>(R, R.bestx, sZ, K); break;
        case GRIEWANK: e64 = error_f64<GRIEWANK>(R, R.bestx, sZ, K); break;
        default: e64 = error_f64<ACKLEY>(R, R.bestx, sZ, K); break;
        }
    }
    if (threadIdx.x == 0) {
        sevo_run_result &o = R.res[R.out_index];
        o.best_e = e64;
        o.best_e32 = be;
        o.success = e64 <= 1e-8 ? 1 : 0;
        o.fes = (int64_t)R.m + (int64_t)R.iters * R.h;
        o.generations = R.iters;
        o.restarts = 0;
    }
    if (R.best_x_out)
        for (int j = threadIdx.x; j < R.dim; j += CSO_THREADS)
            R.best_x_out[(int64_t)R.out_index * R.max_dim + j] = (double)R.bestx[j];
}

int iterations_of(const sevo_run_desc &d)
{
    const int64_t h = d.np / 2;
    const int it = d.budget <= d.np ? 0 : (int)((d.budget - d.np + h - 1) / h);
    return d.max_generations > 0 ? std::min(it, d.max_generations) : it;
}

}  // namespace

hipError_t exec_cso_launch(const Launch &L, hipStream_t stream, uint32_t seed32, const Consts &k)
{
    const CsoDev *d = (const CsoDev *)L.d;
    switch (L.ks) {
    case CSO_INIT:
        hipLaunchKernelGGL(k_cso_init, dim3((unsigned)L.n, (unsigned)L.grid), dim3(CSO_THREADS), 0, stream, d, seed32);
        break;
    case CSO_BEGIN:
        hipLaunchKernelGGL(k_cso_begin, dim3((unsigned)L.n), dim3(CSO_THREADS), 0, stream, d);
        break;
    case CSO_PAIR:
        hipLaunchKernelGGL(k_cso_pair, dim3((unsigned)L.n), dim3(CSO_THREADS), 0, stream, d, seed32, L.total);
        break;
    case CSO_UPDATE:
        hipLaunchKernelGGL(k_cso_update, dim3((unsigned)L.n, (unsigned)L.grid), dim3(CSO_THREADS), 0, stream, d,
                           seed32, L.total);
        break;
    case CSO_FINISH:
        hipLaunchKernelGGL(k_cso_finish, dim3((unsigned)L.n), dim3(CSO_THREADS), 0, stream, d, k);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int cso_runs(sevo_ctx *ctx, const sevo_run_desc *runs, int n, int precision, sevo_run_result *results,
             float *trace, int64_t trace_len, double *best_x, int max_dim, hipStream_t stream)
{
    std::vector<int> idx;
    for (int r = 0; r < n; ++r)
        if (runs[r].algo == SEVO_ALGO_CSO) idx.push_back(r);
    if (idx.empty()) return SEVO_OK;
    const int nr = (int)idx.size();

    // state of every run in the workspace, 64-float aligned pieces
    auto up64 = [](size_t v) { return (v + 63) & ~(size_t)63; };
    std::vector<size_t> off(nr);
    size_t total = 0;
    for (int q = 0; q < nr; ++q) {
        const sevo_run_desc &d = runs[idx[q]];
        const size_t D = d.prob.dim, ldx = (d.np + 15) & ~15, ldg = (d.np / 2 + 15) & ~15;
        off[q] = total;
        total += up64(2 * D * ldx) + up64(2 * D * ldg) + up64(2 * ldx) + up64(4 * ldg) + up64(D) + 64;
    }
    float *ws = nullptr;
    int rc = ctx_ws(ctx).get(ctx, WS_CSO, total * sizeof(float), (void **)&ws);
    if (rc) return rc;

    std::vector<CsoDev> devs(nr);
    std::vector<EvalDesc> init_items, g_items[2];
    int max_slices = 1, t_max = 0;
    for (int q = 0; q < nr; ++q) {
        const sevo_run_desc &d = runs[idx[q]];
        InstanceView I;
        if ((rc = lookup_instance(ctx, &d.prob, d.instance, &I))) return rc;
        CsoDev &R = devs[q];
        R.func = d.prob.func;
        R.dim = d.prob.dim;
        R.m = d.np;
        R.h = d.np / 2;
        R.ldx = (d.np + 15) & ~15;
        R.ldg = (R.h + 15) & ~15;
        R.run_uid = d.run_uid;
        R.iters = iterations_of(d);
        R.budget = d.budget;
        R.lb = (float)d.prob.lb;
        R.ub = (float)d.prob.ub;
        R.phi = (float)d.c1;
        const size_t D = R.dim;
        float *b = ws + off[q];
        R.X = b;
        R.V = b + D * R.ldx;
        b += up64(2 * D * R.ldx);
        R.G[0] = b;
        R.G[1] = b + D * R.ldg;
        b += up64(2 * D * R.ldg);
        R.E[0] = b;
        R.E[1] = b + R.ldx;
        b += up64(2 * (size_t)R.ldx);
        R.EG = b;
        R.L[0] = reinterpret_cast<int32_t *>(b + R.ldg);
        R.L[1] = reinterpret_cast<int32_t *>(b + 2 * R.ldg);
        R.W = reinterpret_cast<int32_t *>(b + 3 * R.ldg);
        b += up64(4 * (size_t)R.ldg);
        R.bestx = b;
        b += up64(D);
        R.best = b;
        R.o = I.o;
        R.M64 = I.M64;
        R.res = results;
        R.trace = trace;
        R.trace_len = trace_len;
        R.best_x_out = best_x;
        R.max_dim = max_dim;
        R.out_index = idx[q];
        max_slices = std::max(max_slices, (R.dim + CSO_SLICE - 1) / CSO_SLICE);
        t_max = std::max(t_max, R.iters);
        EvalDesc e{};
        e.o = I.o;
        e.Mfrag = I.Mfrag;
        e.tab = I.tab;
        e.M64 = I.M64;
        e.Mbf = I.Mbf;
        e.func = R.func;
        e.dim = R.dim;
        EvalDesc ei = e;
        ei.x = R.X;
        ei.err = R.E[0];
        ei.ld = R.ldx;
        ei.n = R.m;
        init_items.push_back(ei);
        for (int p = 0; p < 2; ++p) {
            EvalDesc eg = e;
            eg.x = R.G[p];
            eg.err = R.EG;
            eg.ld = R.ldg;
            eg.n = R.h;
            g_items[p].push_back(eg);
        }
    }

    // evaluation launches, prepared once; one partial-sum buffer serves all
    const size_t pf = std::max(large_partial_floats(init_items, precision), large_partial_floats(g_items[0], precision));
    const size_t sb = std::max(large_operand_bytes(init_items, precision), large_operand_bytes(g_items[0], precision));
    float *part = nullptr;
    void *opnd = nullptr;
    if (pf && (rc = ctx_ws(ctx).get(ctx, WS_PARTIAL, pf * sizeof(float), (void **)&part))) return rc;
    if (sb && (rc = ctx_ws(ctx).get(ctx, WS_OPERANDS, sb, &opnd))) return rc;
    std::vector<PreparedLaunch> ev_init, ev_g[2];
    if ((rc = prepare_eval(ctx, init_items, precision, part, opnd, ev_init))) return rc;
    for (int p = 0; p < 2; ++p)
        if ((rc = prepare_eval(ctx, g_items[p], precision, part, opnd, ev_g[p]))) return rc;

    // one staged blob: the run table, then every evaluation table (256-byte aligned)
    std::vector<char> blob(devs.size() * sizeof(CsoDev));
    std::memcpy(blob.data(), devs.data(), blob.size());
    std::vector<size_t> toff;
    auto append = [&](std::vector<PreparedLaunch> &v) {
        for (auto &p : v) {
            blob.resize((blob.size() + 255) & ~(size_t)255);
            toff.push_back(blob.size());
            blob.insert(blob.end(), p.table.begin(), p.table.end());
        }
    };
    append(ev_init);
    append(ev_g[0]);
    append(ev_g[1]);
    const void *base = nullptr;
    int slot;
    if ((rc = stage_blob(ctx, blob, stream, &base, &slot))) return rc;
    size_t ti = 0;
    for (auto *v : {&ev_init, &ev_g[0], &ev_g[1]})
        for (auto &p : *v) p.L.d = static_cast<const char *>(base) + toff[ti++];
    const CsoDev *d_runs = static_cast<const CsoDev *>(base);

    auto cso = [&](int kind, int t, int grid) {
        return emit_launch(ctx, Launch{L_CSO, d_runs, nr, kind, t, grid, false, false, 0, 0, 0}, stream);
    };
    auto evals = [&](std::vector<PreparedLaunch> &v) {
        for (auto &p : v) {
            const int e = emit_launch(ctx, p.L, stream);
            if (e) return e;
        }
        return (int)SEVO_OK;
    };
    if ((rc = cso(CSO_INIT, 0, max_slices)) || (rc = evals(ev_init)) || (rc = cso(CSO_BEGIN, 0, 1))) return rc;
    for (int t = 1; t <= t_max + 1; ++t) {
        if ((rc = cso(CSO_PAIR, t, 1))) return rc;
        if (t > t_max) break;
        if ((rc = cso(CSO_UPDATE, t, max_slices)) || (rc = evals(ev_g[t & 1]))) return rc;
    }
    if ((rc = cso(CSO_FINISH, 0, 1))) return rc;
    return finish_slot(ctx, slot, stream);
}

}  // namespace sevo
