// run.hip -- whole runs in persistent fused generation kernels.
//
// One workgroup (4 waves) carries one run from initialisation to its budget
// without returning to the host: every generation is variation, the MFMA
// evaluation of the new points (rotation from LDS, objective straight from
// the accumulators), the best-so-far recorder and selection, separated by
// workgroup barriers.  The instance (rotation fragments, shift, per-row
// table) is staged in LDS once per run; the population lives in a
// library-owned workspace that stays in L2 / Infinity Cache.  Runs are
// grouped by dimension class (one kernel instantiation per class) and the
// classes run concurrently on internal streams.
//
// Precision FP64 runs the plain path instead: one run at a time, one launch
// per generation step, all arithmetic in double (the baseline the batched
// path is compared with).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "../../include/sevo.h"
#include "algo.h"
#include "tile.h"
#include "state.h"

namespace sevo {

constexpr int RUN_MAX_NP = 256;

struct RunDev {
    int32_t algo, func, dim, np, npp;
    uint32_t run_uid;
    int32_t H, pnum;
    int64_t budget;
    float F, w, c1, c2, vmax;
    uint32_t thr;
    float lb, ub;
    const double *o;
    const float *Mfrag;
    const float *tab;
    const double *M64;
    float *X, *U, *V, *P, *eX, *eU, *eP, *bestx;
    sevo_run_result *res;
    float *trace;
    int64_t trace_len;
    double *best_x_out;
    int32_t max_dim;
    int32_t out_index;
};

// (key, index) pairs are combined so that the earlier pair wins ties: over
// positions in index order this gives the minimum key and, among equal
// keys, the lowest index.
__device__ __forceinline__ void keep_earlier(float &v, int &idx, float ov, int oi)
{
    if (ov <= v) { v = ov; idx = oi; }
}

// Inclusive prefix minimum of (key, index) over the block, earlier index on
// ties; every thread's prefix is left in sPv / sPi (and returned).  Wave
// scans by shuffles, then one exchange of the four wave totals.
__device__ __forceinline__ void prefix_min(float v, int idx, float *sPv, int *sPi, float *sWv, int *sWi,
                                           float &pv, int &pi)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const float ov = __shfl_up(v, off, 64);
        const int oi = __shfl_up(idx, off, 64);
        if (lane >= off) keep_earlier(v, idx, ov, oi);
    }
    if (lane == 63) { sWv[wave] = v; sWi[wave] = idx; }
    __syncthreads();
    if (wave > 0) {
        float cv = sWv[0];
        int ci = sWi[0];
        for (int w = 1; w < wave; ++w) {
            // carry (earlier waves) against wave w's total: the carry is earlier
            float tv = sWv[w];
            int ti = sWi[w];
            keep_earlier(tv, ti, cv, ci);
            cv = tv;
            ci = ti;
        }
        keep_earlier(v, idx, cv, ci);
    }
    sPv[tid] = v;
    sPi[tid] = idx;
    __syncthreads();
    pv = v;
    pi = idx;
}

// Sums over the block of N doubles per thread (fixed order: lanes by a
// shuffle tree, then waves 0..3 in order).  Every thread gets the sums.
template <int N>
__device__ __forceinline__ void block_sums(double (&v)[N], double *sRed /* [4 * N] */)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < N; ++k) sRed[wave * N + k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = ((sRed[k] + sRed[N + k]) + sRed[2 * N + k]) + sRed[3 * N + k];
    __syncthreads();
}

template <int KS>
__device__ __forceinline__ void eval_pop(const RunDev &R, const float *Y, float *eY, const float *sA,
                                         const double *sO, const float *sT, const Consts &K)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kq = lane >> 4, pc = lane & 15;
    const int ntile = (R.np + 15) / 16;
    for (int ct = wave; ct < ntile; ct += 4) {
        const int p0 = ct * 16;
        float b[KS][1];
        load_b<KS, 1>(b, gin<float>(Y), R.npp, R.dim, R.np, p0, kq, pc, sO);
        SEVO_GLOBAL float *E = gout<float>(eY);
        switch (R.func) {
        case ELLIPSOID: tile_body<ELLIPSOID, KS, 1>(b, sA, sT, lane, R.dim, R.np, p0, K.kf, E); break;
        case ROSENBROCK: tile_body<ROSENBROCK, KS, 1>(b, sA, sT, lane, R.dim, R.np, p0, K.kf, E); break;
        case RASTRIGIN: tile_body<RASTRIGIN, KS, 1>(b, sA, sT, lane, R.dim, R.np, p0, K.kf, E); break;
        case SCHWEFEL: tile_body<SCHWEFEL, KS, 1>(b, sA, sT, lane, R.dim, R.np, p0, K.kf, E); break;
        case GRIEWANK: tile_body<GRIEWANK, KS, 1>(b, sA, sT, lane, R.dim, R.np, p0, K.kf, E); break;
        default: tile_body<ACKLEY, KS, 1>(b, sA, sT, lane, R.dim, R.np, p0, K.kf, E); break;
        }
    }
}

// Double-precision error of one float point (the final check): rows of z by
// all threads into LDS, then the objective by thread 0.  Every thread of the
// workgroup must call it.
template <int FUNC>
__device__ __forceinline__ double check_f64(const RunDev &R, const float *x, double *sZ, const Consts &K)
{
    const int D = R.dim;
    for (int r = threadIdx.x; r < D; r += 256) {
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

template <int KS>
__global__ __launch_bounds__(256) void k_run(const RunDev *__restrict__ runs, uint32_t seed32, Consts K)
{
    constexpr int RT = (KS + 3) / 4;
    __shared__ __attribute__((aligned(16))) float sA[RT * KS * 64];
    __shared__ double sO[KS * 4];
    __shared__ float sT[RT * 16];
    __shared__ unsigned long long sKey[256];
    __shared__ int sRank[256];
    __shared__ float sF[256], sCR[256];
    __shared__ float sPv[256];
    __shared__ int sPi[256];
    __shared__ float sWv[4];
    __shared__ int sWi[4];
    __shared__ double sRed[4 * 5];
    __shared__ double sZ[128];
    // per-individual choices of the generation, read by the element loops
    __shared__ int sDa[256], sDb[256], sDc[256], sJr[256], sFlag[256];
    __shared__ float sFi[256];
    __shared__ uint32_t sThr[256];
    __shared__ float sMF[16], sMCR[16];
    __shared__ int sPos, sG, sCopy;
    __shared__ float sBest, sBestB;

    const RunDev R = runs[blockIdx.x];
    const int tid = threadIdx.x;
    const int D = R.dim, np = R.np, npp = R.npp;
    const bool pso = R.algo == SEVO_ALGO_PSO, shade = R.algo == SEVO_ALGO_SHADE;

    stage_rotation<KS>(sA, R.Mfrag);
    for (int q = tid; q < KS * 4; q += 256) sO[q] = q < D ? R.o[q] : 0.0;
    for (int q = tid; q < RT * 16; q += 256) sT[q] = R.tab[q];
    if (tid < 16) { sMF[tid] = 0.5f; sMCR[tid] = 0.5f; }
    if (tid == 0) { sPos = 0; sG = 0; sBest = INFINITY; sBestB = INFINITY; sCopy = -1; }

    // Element loops: wave w takes coordinate blocks w, w + 4, ...; its lanes
    // take individuals, so every access to the [D][npp] state is coalesced
    // and the loads of one work item are independent of each other.
    const int lane = tid & 63, wave = tid >> 6;

    // generation 0: x uniform in the box (double, then rounded to float)
    for (int jb = wave; jb * 4 < D; jb += 4)
        for (int i = lane; i < np; i += 64) {
            const u32x4 w = draw(R.run_uid, seed32, 0, (uint32_t)i, TAG_INIT_X, (uint32_t)jb);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int j = jb * 4 + e;
                if (j < D) {
                    const float x = (float)((double)R.lb + ((double)R.ub - (double)R.lb) * u24d(word(w, e)));
                    R.X[j * npp + i] = x;
                    if (pso) { R.V[j * npp + i] = 0.f; R.P[j * npp + i] = x; }
                }
            }
        }
    __syncthreads();

    int64_t fe = 0;
    int gen = 0;
    // recorder for the np evaluations eY (in index order) made at fe0
    auto record = [&](const float *Y, const float *eY) {
        float pv;
        int pi;
        const float before = sBest;
        prefix_min(tid < np ? err_key(eY[tid]) : INFINITY, tid, sPv, sPi, sWv, sWi, pv, pi);
        if (tid < np && R.trace) {
            const int64_t c = fe + tid + 1;
            if (c % TRACE_EVERY == 0) {
                const int64_t k = c / TRACE_EVERY - 1;
                if (k < R.trace_len) R.trace[(int64_t)R.out_index * R.trace_len + k] = fminf(before, pv);
            }
        }
        if (tid == 0) {
            const int lim = (int)min<int64_t>((int64_t)np, R.budget - fe);
            sCopy = -1;
            if (lim > 0 && sPv[lim - 1] < sBestB) { sBestB = sPv[lim - 1]; sCopy = sPi[lim - 1]; }
            sBest = fminf(before, sPv[np - 1]);
        }
        __syncthreads();
        const int cp = sCopy;
        if (cp >= 0)
            for (int j = tid; j < D; j += 256) R.bestx[j] = Y[j * npp + cp];
        __syncthreads();
    };
    // gbest = argmin e(p), lowest index on ties
    auto global_best = [&]() {
        float pv;
        int pi;
        prefix_min(tid < np ? err_key(R.eP[tid]) : INFINITY, tid, sPv, sPi, sWv, sWi, pv, pi);
        if (tid == 0) sG = sPi[255];
        __syncthreads();
    };
    // dst[j][i] = src[j][i] for the individuals with sFlag[i] set
    auto copy_flagged = [&](float *dst, const float *src) {
        for (int j = wave; j < D; j += 4)
            for (int i = lane; i < np; i += 64)
                if (sFlag[i]) dst[j * npp + i] = src[j * npp + i];
        __syncthreads();
    };

    eval_pop<KS>(R, R.X, R.eX, sA, sO, sT, K);
    __syncthreads();
    record(R.X, R.eX);
    if (pso) {
        if (tid < np) R.eP[tid] = R.eX[tid];
        __syncthreads();
        global_best();
    }
    fe = np;

    while (fe < R.budget) {
        ++gen;
        const uint32_t t = (uint32_t)gen;
        if (pso) {
            // ---- PSO: update, evaluate, personal and global bests ----
            const int g = sG;
            for (int jb = wave; jb * 2 < D; jb += 4)
                for (int i = lane; i < np; i += 64) {
                    const u32x4 wd = draw(R.run_uid, seed32, t, (uint32_t)i, TAG_PSO_R, (uint32_t)jb);
                    float xj[2], vv[2], pj[2], pg[2];
#pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        const int row = min(jb * 2 + e, D - 1) * npp;
                        xj[e] = R.X[row + i];
                        vv[e] = R.V[row + i];
                        pj[e] = R.P[row + i];
                        pg[e] = R.P[row + g];
                    }
#pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        const int j = jb * 2 + e;
                        if (j < D) {
                            const int row = j * npp;
                            const float r1 = u24f(word(wd, 2 * e)), r2 = u24f(word(wd, 2 * e + 1));
                            float vj = R.w * vv[e] + R.c1 * r1 * (pj[e] - xj[e]) + R.c2 * r2 * (pg[e] - xj[e]);
                            vj = fminf(fmaxf(vj, -R.vmax), R.vmax);
                            float xn = xj[e] + vj;
                            if (xn < R.lb) { xn = R.lb; vj = 0.f; }
                            else if (xn > R.ub) { xn = R.ub; vj = 0.f; }
                            R.X[row + i] = xn;
                            R.V[row + i] = vj;
                        }
                    }
                }
            __syncthreads();
            eval_pop<KS>(R, R.X, R.eX, sA, sO, sT, K);
            __syncthreads();
            record(R.X, R.eX);
            if (tid < np) {
                const bool imp = err_key(R.eX[tid]) < err_key(R.eP[tid]);
                if (imp) R.eP[tid] = R.eX[tid];
                sFlag[tid] = imp ? 1 : 0;
            }
            __syncthreads();
            copy_flagged(R.P, R.X);
            global_best();
        } else {
            // ---- DE rand/1/bin or SHADE current-to-pbest/1 ----
            if (shade) {
                // ranking by (error, index): every key counts the keys below it
                if (tid < np) {
                    const uint32_t bits = __float_as_uint(err_key(R.eX[tid]));
                    const uint32_t ord = (bits & 0x80000000u) ? ~bits : (bits | 0x80000000u);
                    sKey[tid] = ((unsigned long long)ord << 32) | (uint32_t)tid;
                }
                __syncthreads();
                if (tid < np) {
                    const unsigned long long key = sKey[tid];
                    int rank = 0;
                    for (int q = 0; q < np; ++q) rank += sKey[q] < key ? 1 : 0;
                    sRank[rank] = tid;
                }
                __syncthreads();
            }
            if (tid < np) {
                const int i = tid;
                if (shade) {
                    const ShadeDraw d = shade_draw(R.run_uid, seed32, t, i, np, D, R.H, R.pnum, sMF, sMCR);
                    sF[i] = d.F;
                    sCR[i] = d.CR;
                    sFi[i] = d.F;
                    sThr[i] = cr_threshold((double)d.CR);
                    sDa[i] = d.r1;
                    sDb[i] = d.r2;
                    sDc[i] = sRank[d.pbest_rank];
                    sJr[i] = d.jrand;
                } else {
                    int ia, ib, ic, jrand;
                    de_donors(R.run_uid, seed32, t, i, np, D, ia, ib, ic, jrand);
                    sFi[i] = R.F;
                    sThr[i] = R.thr;
                    sDa[i] = ia;
                    sDb[i] = ib;
                    sDc[i] = ic;
                    sJr[i] = jrand;
                }
            }
            __syncthreads();
            for (int jb = wave; jb * 4 < D; jb += 4)
                for (int i = lane; i < np; i += 64) {
                    const u32x4 w = draw(R.run_uid, seed32, t, (uint32_t)i, TAG_CROSS, (uint32_t)jb);
                    const int ia = sDa[i], ib = sDb[i], ic = sDc[i], jrand = sJr[i];
                    const float Fi = sFi[i];
                    const uint32_t thr = sThr[i];
                    float xi[4], xa[4], xb[4], xc[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int row = min(jb * 4 + e, D - 1) * npp;
                        xi[e] = R.X[row + i];
                        xa[e] = R.X[row + ia];
                        xb[e] = R.X[row + ib];
                        xc[e] = R.X[row + ic];
                    }
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int j = jb * 4 + e;
                        if (j < D) {
                            // SHADE: ic is the pbest individual, v = x + F (x_pbest - x) + F (x_r1 - x_r2)
                            float v;
                            if (shade) v = xi[e] + Fi * (xc[e] - xi[e]) + Fi * (xa[e] - xb[e]);
                            else v = xa[e] + Fi * (xb[e] - xc[e]);
                            bool m;
                            R.U[j * npp + i] = cross_repair<float>(word(w, e), thr, j, jrand, v, xi[e], R.lb, R.ub, m);
                        }
                    }
                }
            __syncthreads();
            eval_pop<KS>(R, R.U, R.eU, sA, sO, sT, K);
            __syncthreads();
            record(R.U, R.eU);
            double st[5] = {0.0, 0.0, 0.0, 0.0, 0.0};   // sum dl, dl CR, dl F^2, dl F, successes
            if (tid < np) {
                const float ku = err_key(R.eU[tid]), kx = err_key(R.eX[tid]);
                if (shade && ku < kx) {
                    double dl = (double)kx - (double)ku;
                    if (!(dl <= 1e30)) dl = 1e30;
                    st[0] = dl;
                    st[1] = dl * sCR[tid];
                    st[2] = dl * sF[tid] * sF[tid];
                    st[3] = dl * sF[tid];
                    st[4] = 1.0;
                }
                const bool rep = ku <= kx;
                if (rep) R.eX[tid] = R.eU[tid];
                sFlag[tid] = rep ? 1 : 0;
            }
            __syncthreads();
            copy_flagged(R.X, R.U);
            if (shade) {
                block_sums<5>(st, sRed);
                if (tid == 0 && st[4] > 0.0) {
                    sMCR[sPos] = (float)(st[1] / st[0]);
                    sMF[sPos] = (float)(st[2] / st[3]);
                    sPos = (sPos + 1) % R.H;
                }
                __syncthreads();
            }
        }
        fe += np;
    }

    // results; the best point is re-evaluated in double once below 1e-6
    const float be = sBestB;
    double e64 = (double)be;
    if (be < 1e-6f) {
        switch (R.func) {
        case ELLIPSOID: e64 = check_f64<ELLIPSOID>(R, R.bestx, sZ, K); break;
        case ROSENBROCK: e64 = check_f64<ROSENBROCK>(R, R.bestx, sZ, K); break;
        case RASTRIGIN: e64 = check_f64<RASTRIGIN>(R, R.bestx, sZ, K); break;
        case SCHWEFEL: e64 = check_f64<SCHWEFEL>(R, R.bestx, sZ, K); break;
        case GRIEWANK: e64 = check_f64<GRIEWANK>(R, R.bestx, sZ, K); break;
        default: e64 = check_f64<ACKLEY>(R, R.bestx, sZ, K); break;
        }
    }
    if (tid == 0) {
        sevo_run_result &o = R.res[R.out_index];
        o.best_e = e64;
        o.best_e32 = be;
        o.success = e64 <= 1e-8 ? 1 : 0;
        o.fes = fe;
        o.generations = gen;
        o.reserved = 0;
    }
    if (R.best_x_out)
        for (int j = tid; j < D; j += 256) R.best_x_out[(int64_t)R.out_index * R.max_dim + j] = (double)R.bestx[j];
}

typedef void (*RunKernel)(const RunDev *, uint32_t, Consts);

template <int KS>
static RunKernel run_kernel() { return k_run<KS>; }

static RunKernel run_table(int ks)
{
    switch (ks) {
#define SEVO_KS_CASE(v) case v: return run_kernel<v>();
        SEVO_KS_CASE(1) SEVO_KS_CASE(2) SEVO_KS_CASE(3) SEVO_KS_CASE(4) SEVO_KS_CASE(5)
        SEVO_KS_CASE(6) SEVO_KS_CASE(7) SEVO_KS_CASE(8) SEVO_KS_CASE(9) SEVO_KS_CASE(10)
        SEVO_KS_CASE(11) SEVO_KS_CASE(12) SEVO_KS_CASE(13) SEVO_KS_CASE(14) SEVO_KS_CASE(15)
        SEVO_KS_CASE(16) SEVO_KS_CASE(17) SEVO_KS_CASE(18) SEVO_KS_CASE(19) SEVO_KS_CASE(20)
        SEVO_KS_CASE(21) SEVO_KS_CASE(22) SEVO_KS_CASE(23) SEVO_KS_CASE(24) SEVO_KS_CASE(25)
        SEVO_KS_CASE(26) SEVO_KS_CASE(27) SEVO_KS_CASE(28) SEVO_KS_CASE(29) SEVO_KS_CASE(30)
#undef SEVO_KS_CASE
    default: return nullptr;
    }
}

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

int validate_runs(sevo_ctx *ctx, const sevo_run_desc *runs, int n, int precision, int64_t trace_len,
                  const float *trace, const double *best_x, int max_dim)
{
    if (n < 1 || !runs) return set_error(ctx, SEVO_EINVAL, "no runs");
    if (precision != SEVO_FP32 && precision != SEVO_FP64)
        return set_error(ctx, SEVO_EINVAL, "runs take precision FP32 or FP64");
    if (trace_len < 0 || (trace_len > 0 && !trace)) return set_error(ctx, SEVO_EINVAL, "bad trace");
    for (int r = 0; r < n; ++r) {
        const sevo_run_desc &d = runs[r];
        const sevo_problem &p = d.prob;
        if (p.func < 0 || p.func >= NFUNC || p.dim < 2 || p.dim > MAX_DIM || !(p.lb < p.ub))
            return set_error(ctx, SEVO_EINVAL, "run has an invalid problem");
        if (d.algo != SEVO_ALGO_DE && d.algo != SEVO_ALGO_PSO && d.algo != SEVO_ALGO_SHADE)
            return set_error(ctx, SEVO_EINVAL, "unknown algorithm");
        const int min_np = d.algo == SEVO_ALGO_PSO ? 1 : 4;
        if (d.np < min_np || d.np > RUN_MAX_NP) return set_error(ctx, SEVO_EINVAL, "np outside [4 (1 for PSO), 256]");
        if (d.budget < 1) return set_error(ctx, SEVO_EINVAL, "budget < 1");
        if (d.algo == SEVO_ALGO_DE && (!std::isfinite(d.F) || !(d.CR >= 0 && d.CR <= 1)))
            return set_error(ctx, SEVO_EINVAL, "DE needs finite F and CR in [0, 1]");
        if (d.algo == SEVO_ALGO_PSO && !(d.vmax > 0))
            return set_error(ctx, SEVO_EINVAL, "PSO needs vmax > 0");
        if (d.algo == SEVO_ALGO_SHADE && (d.H < 1 || d.H > 16 || !(d.p > 0 && d.p <= 1)))
            return set_error(ctx, SEVO_EINVAL, "SHADE needs H in [1, 16] and p in (0, 1]");
        if (best_x && max_dim < p.dim) return set_error(ctx, SEVO_EINVAL, "max_dim < dim");
        if (precision == SEVO_FP32 && p.dim > SMALL_D_MAX)
            return set_error(ctx, SEVO_EUNSUPPORTED, "fused runs support D <= 120");
        if (precision == SEVO_FP64 && d.algo == SEVO_ALGO_SHADE)
            return set_error(ctx, SEVO_EUNSUPPORTED, "the double-precision run path has DE and PSO");
    }
    return SEVO_OK;
}

int run_fused(sevo_ctx *ctx, const sevo_run_desc *runs, int n, sevo_run_result *results, float *trace,
              int64_t trace_len, double *best_x, int max_dim, hipStream_t stream)
{
    // workspace
    size_t total = 0;
    std::vector<size_t> off(n);
    for (int r = 0; r < n; ++r) {
        const int npp = (runs[r].np + 15) & ~15;
        const size_t D = runs[r].prob.dim;
        off[r] = total;
        total += 4 * D * npp + 3 * (size_t)npp + D;
        total = (total + 63) & ~(size_t)63;
    }
    float *ws = nullptr;
    int rc = ctx_ws(ctx).get(ctx, WS_RUN, total * sizeof(float), (void **)&ws);
    if (rc) return rc;
    std::map<int, std::vector<RunDev>> groups;
    std::map<int, std::vector<double>> cost;
    for (int r = 0; r < n; ++r) {
        const sevo_run_desc &d = runs[r];
        InstanceView I;
        if ((rc = lookup_instance(ctx, &d.prob, d.instance, &I))) return rc;
        RunDev R{};
        R.algo = d.algo;
        R.func = d.prob.func;
        R.dim = d.prob.dim;
        R.np = d.np;
        R.npp = (d.np + 15) & ~15;
        R.run_uid = d.run_uid;
        R.H = d.H;
        R.pnum = d.algo == SEVO_ALGO_SHADE ? shade_pnum(d.p, d.np) : 0;
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
        const size_t DN = (size_t)R.dim * R.npp;
        R.X = b; R.U = b + DN; R.V = b + 2 * DN; R.P = b + 3 * DN;
        R.eX = b + 4 * DN; R.eU = R.eX + R.npp; R.eP = R.eU + R.npp; R.bestx = R.eP + R.npp;
        R.res = results;
        R.trace = trace;
        R.trace_len = trace_len;
        R.best_x_out = best_x;
        R.max_dim = max_dim;
        R.out_index = r;
        const int ks = ks_of(R.dim);
        groups[ks].push_back(R);
        cost[ks].push_back((double)d.budget * R.dim * R.dim);
    }
    const int ng = (int)groups.size();
    std::vector<hipStream_t> ss(ng);
    if ((rc = fork_streams(ctx, stream, ng, ss.data()))) return rc;
    int g = 0;
    for (auto &kv : groups) {
        std::vector<RunDev> &v = kv.second;
        // longest runs first, so the tail is short
        std::vector<int> order(v.size());
        for (size_t i = 0; i < v.size(); ++i) order[i] = (int)i;
        const std::vector<double> &c = cost[kv.first];
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return c[a] > c[b]; });
        std::vector<char> blob(v.size() * sizeof(RunDev));
        for (size_t i = 0; i < v.size(); ++i) std::memcpy(blob.data() + i * sizeof(RunDev), &v[order[i]], sizeof(RunDev));
        const void *d = nullptr;
        int slot;
        if ((rc = stage_blob(ctx, blob, ss[g], &d, &slot))) return rc;
        RunKernel k = run_table(kv.first);
        hipLaunchKernelGGL(k, dim3((unsigned)v.size()), dim3(256), 0, ss[g], (const RunDev *)d,
                           ctx_seed32(ctx), ctx_consts(ctx));
        if (hipGetLastError() != hipSuccess) return set_error(ctx, SEVO_EDEVICE, "run kernel launch failed");
        if ((rc = finish_slot(ctx, slot, ss[g]))) return rc;
        ++g;
    }
    return join_streams(ctx, stream, ng, ss.data());
}

}  // namespace

extern "C" int sevo_run(sevo_ctx *ctx, const sevo_run_desc *runs, int32_t n_runs, int32_t precision,
                        sevo_run_result *results, float *trace, int64_t trace_len, double *best_x,
                        int32_t max_dim, void *stream)
{
    if (!ctx) return set_error(nullptr, SEVO_EINVAL, "ctx is NULL");
    if (!results) return set_error(ctx, SEVO_EINVAL, "results is NULL");
    int rc = validate_runs(ctx, runs, n_runs, precision, trace_len, trace, best_x, max_dim);
    if (rc) return rc;
    DeviceScope dg(ctx);
    if (precision == SEVO_FP32)
        return run_fused(ctx, runs, n_runs, results, trace, trace_len, best_x, max_dim, (hipStream_t)stream);
    return run_plain_f64(ctx, runs, n_runs, results, trace, trace_len, best_x, max_dim, (hipStream_t)stream);
}
