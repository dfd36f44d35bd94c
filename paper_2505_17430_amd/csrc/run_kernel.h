// run_kernel.h -- whole runs in persistent fused generation kernels (the
// device code; instantiated per algorithm family in run_de.hip,
// run_shade.hip, run_lshade.hip, run_pso.hip and run_psode.hip, launched by
// run.hip).
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
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
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
    float *X, *U, *V, *P, *bestx;   // workspace (X .. P unused when on chip)
    // L-SHADE: pbest fraction and archive bound (double, as the schedule is
    // computed), final population size, archive [dim][acap] in the workspace
    double p, r_arc;
    int32_t np_min, acap;
    float *Arc;
    int32_t topology, velocity;     // PSO: 0/1 global best / ring; inertia / spherical
    sevo_run_result *res;
    float *trace;
    int64_t trace_len;
    double *best_x_out;
    int32_t max_dim;
    int32_t out_index;
    // parameter observer: rows (muF, muCR) after each generation, or null;
    // JADE's adaptation rate; DE's CR for the observer rows
    float *mu;
    int64_t mu_len;
    double c_adapt;
    float CR;
    // L-SHADE-Restart: restarts enabled, and the convergence threshold
    int32_t restart;
    double restart_tol;
    // generations after which the run stops (0: at the budget)
    int32_t gen_cap;
    // the run's state when it stops (null: not wanted), rows of st_np
    // points, st_dim rows per run, st_arc archive columns
    int32_t st_np, st_dim, st_arc;
    float *st_x, *st_e, *st_u, *st_eu, *st_v, *st_p, *st_ep, *st_mem, *st_arc_out;
    int32_t *st_cnt;
};

// A team carries one run: the whole workgroup (256 threads, phases separated
// by block barriers) or one wave (64 lanes, which run in lockstep: phases
// only need the team's memory operations ordered, no barrier).  The four
// wave teams of a workgroup run four runs of the same instance, which is
// staged in LDS once for all of them.
template <bool WAVE>
struct Team;

template <>
struct Team<false> {
    static constexpr int SIZE = 256, NW = 4;
    int tid, lane, wave, slot;
    __device__ Team() : tid(threadIdx.x), lane(threadIdx.x & 63), wave(threadIdx.x >> 6), slot(0) {}
    __device__ static void sync() { __syncthreads(); }
};

template <>
struct Team<true> {
    static constexpr int SIZE = 64, NW = 1;
    int tid, lane, wave, slot;
    // slot is wave-uniform; saying so keeps the run's descriptor in scalar registers
    __device__ Team()
        : tid(threadIdx.x & 63), lane(threadIdx.x & 63), wave(0),
          slot(__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6))) {}
    __device__ static void sync()
    {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
};

// (key, index) pairs are combined so that the earlier pair wins ties: over
// positions in index order this gives the minimum key and, among equal
// keys, the lowest index.
__device__ __forceinline__ void keep_earlier(float &v, int &idx, float ov, int oi)
{
    if (ov <= v) { v = ov; idx = oi; }
}

// Inclusive prefix minimum of (key, index) over the team, earlier index on
// ties; every member's prefix is left in sPv / sPi (the team's slices) and
// returned.  Wave scans by shuffles; a block team then exchanges the four
// wave totals.
template <bool WAVE>
__device__ __forceinline__ void prefix_min(const Team<WAVE> &t, float v, int idx, float *sPv, int *sPi,
                                           float *sWv, int *sWi, float &pv, int &pi)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const float ov = __shfl_up(v, off, 64);
        const int oi = __shfl_up(idx, off, 64);
        if (t.lane >= off) keep_earlier(v, idx, ov, oi);
    }
    if constexpr (!WAVE) {
        if (t.lane == 63) { sWv[t.wave] = v; sWi[t.wave] = idx; }
        __syncthreads();
        if (t.wave > 0) {
            float cv = sWv[0];
            int ci = sWi[0];
            for (int w = 1; w < t.wave; ++w) {
                // carry (earlier waves) against wave w's total: the carry is earlier
                float tv = sWv[w];
                int ti = sWi[w];
                keep_earlier(tv, ti, cv, ci);
                cv = tv;
                ci = ti;
            }
            keep_earlier(v, idx, cv, ci);
        }
    }
    sPv[t.tid] = v;
    sPi[t.tid] = idx;
    t.sync();
    pv = v;
    pi = idx;
}

// Nearest integer, halves away from zero, of a non-negative double (the
// C library's lround on the values used here).
__device__ __forceinline__ int round_half_up(double x)
{
    const double f = floor(x);
    return (int)(x - f >= 0.5 ? f + 1.0 : f);
}

// L-SHADE population size after fe of budget evaluations.
__device__ __forceinline__ int lshade_np(int np_init, int np_min, int64_t budget, int64_t fe)
{
    const double v = (double)(np_min - np_init) * (double)fe / (double)budget + (double)np_init;
    return min(max(round_half_up(v), np_min), np_init);
}

// Exclusive count of the set flags before this member, in member order;
// total receives the count over the team.
template <bool WAVE>
__device__ __forceinline__ int team_exclusive_count(const Team<WAVE> &t, bool flag, int *sWc, int &total)
{
    const unsigned long long m = __ballot(flag);
    int excl = __popcll(m & ((1ull << t.lane) - 1ull));
    total = __popcll(m);
    if constexpr (!WAVE) {
        if (t.lane == 0) sWc[t.wave] = total;
        __syncthreads();
        int before = 0, all = 0;
        for (int w = 0; w < 4; ++w) {
            if (w < t.wave) before += sWc[w];
            all += sWc[w];
        }
        __syncthreads();
        excl += before;
        total = all;
    }
    return excl;
}

// Sums over the team of N doubles per member, in a fixed order (lanes by a
// shuffle tree, then waves 0..3 in order); every member gets the sums.
template <int N, bool WAVE>
__device__ __forceinline__ void team_sums(const Team<WAVE> &t, double (&v)[N], double (&sRed)[4 * N])
{
#pragma unroll
    for (int k = 0; k < N; ++k)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    if constexpr (!WAVE) {
        if (t.lane == 0)
#pragma unroll
            for (int k = 0; k < N; ++k) sRed[t.wave * N + k] = v[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = ((sRed[k] + sRed[N + k]) + sRed[2 * N + k]) + sRed[3 * N + k];
        __syncthreads();
    }
}

// Errors of the np points Y ([dim][npp], in LDS when ONCHIP, else in the
// workspace) into eY (LDS): the team's waves take 16-point tiles in turn.
template <int KS, bool ONCHIP, bool WAVE>
__device__ __forceinline__ void eval_pop(const Team<WAVE> &t, const RunDev &R, int np, const float *Y, float *eY,
                                         const float *sA, const double *sO, const float *sT, const Consts &K)
{
    const int lane = t.lane;
    const int kq = lane >> 4, pc = lane & 15;
    const int ntile = (np + 15) / 16;
    constexpr int NW = Team<WAVE>::NW;
    // from the workspace, the next tile's loads are in flight while the
    // current one is computed (while the extra registers are affordable)
    constexpr bool PF = !ONCHIP && KS <= 13;
    auto load = [&](float (&dst)[KS][1], int p0) {
        if constexpr (ONCHIP) load_raw_lds<KS, 1>(dst, Y, R.npp, R.dim, np, p0, kq, pc);
        else load_raw<KS, 1>(dst, gin<float>(Y), R.npp, R.dim, np, p0, kq, pc);
    };
    float b[KS][1], bn[KS][1];
    if (t.wave < ntile) load(b, t.wave * 16);
    for (int ct = t.wave; ct < ntile; ct += NW) {
        const int p0 = ct * 16, nx = ct + NW;
        if constexpr (PF)
            if (nx < ntile) load(bn, nx * 16);
        shift_raw<KS, 1>(b, R.dim, np, p0, kq, pc, sO);
        switch (R.func) {
        case ELLIPSOID: tile_body<ELLIPSOID, KS, 1>(b, sA, sT, lane, R.dim, np, p0, K.kf, eY); break;
        case ROSENBROCK: tile_body<ROSENBROCK, KS, 1>(b, sA, sT, lane, R.dim, np, p0, K.kf, eY); break;
        case RASTRIGIN: tile_body<RASTRIGIN, KS, 1>(b, sA, sT, lane, R.dim, np, p0, K.kf, eY); break;
        case SCHWEFEL: tile_body<SCHWEFEL, KS, 1>(b, sA, sT, lane, R.dim, np, p0, K.kf, eY); break;
        case GRIEWANK: tile_body<GRIEWANK, KS, 1>(b, sA, sT, lane, R.dim, np, p0, K.kf, eY); break;
        default: tile_body<ACKLEY, KS, 1>(b, sA, sT, lane, R.dim, np, p0, K.kf, eY); break;
        }
        if (nx < ntile) {
            if constexpr (PF) {
#pragma unroll
                for (int k = 0; k < KS; ++k) b[k][0] = bn[k][0];
            } else {
                load(b, nx * 16);
            }
        }
    }
}

// Spherical PSO update (SPSO-2011) of the team's np particles, from the
// positions X to Y (the same array for an update in place).  li[i] is particle i's neighbourhood best (ring) or the
// global best g; sc and part are team scratch in LDS.  Pass 1 sums, per
// particle, |G - x|^2 and |z|^2 over each wave's coordinate blocks (waves in
// order); pass 2 moves to x' = G + r z / |z| with r = |G - x| u^(1/D).
template <bool WAVE>
__device__ __forceinline__ void spherical_update(const Team<WAVE> &t, const RunDev &R, uint32_t seed32,
                                                           uint32_t tg, int np, bool ring, int g, const float *X,
                                                           float *Y, float *V,
                                                           const float *P, const int *li_arr, float *sc,
                                                           float *part)
{
    constexpr int NW = Team<WAVE>::NW;
    const int D = R.dim, npp = R.npp, nb2 = (D + 1) / 2, lane = t.lane, wave = t.wave, tid = t.tid;
    const float c = R.c1;
    auto centre = [&](int i, int li, int row, float xj) {
        const float pp = xj + c * (P[row + i] - xj);
        if (li == i) return (xj + pp) * 0.5f;
        const float lp = xj + c * (P[row + li] - xj);
        return (xj + pp + lp) / 3.f;
    };
    auto normals = [&](int i, int jb, float &z0, float &z1) {
        const u32x4 w = draw(R.run_uid, seed32, tg, (uint32_t)i, TAG_PSO_S, (uint32_t)jb);
        const float rad = sqrtf(-2.f * logf(1.f - u24f(w.x)));
        float sn, cs;
        sincospif(2.f * u24f(w.y), &sn, &cs);
        z0 = rad * cs;
        z1 = rad * sn;
    };
    // Partial sums by coordinate block modulo 4, whatever the team: a block
    // team's wave w owns the blocks w, w + 4, ...; a wave team keeps all four
    // partials itself.  The same additions in the same order either way.
    for (int i = lane; i < np; i += 64) {
        const int li = ring ? li_arr[i] : g;
        float r2[4] = {0.f, 0.f, 0.f, 0.f}, q2[4] = {0.f, 0.f, 0.f, 0.f};
        for (int jb = wave; jb < nb2; jb += NW) {
            float z[2];
            normals(i, jb, z[0], z[1]);
            float rs = 0.f, qs = 0.f;
            for (int e = 0; e < 2; ++e) {
                const int j = jb * 2 + e;
                if (j < D) {
                    const int row = j * npp;
                    const float xj = X[row + i], d = centre(i, li, row, xj) - xj;
                    rs += d * d;
                    qs += z[e] * z[e];
                }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if ((jb & 3) == k) { r2[k] += rs; q2[k] += qs; }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (WAVE || k == wave) {
                part[k * 256 + i] = r2[k];
                part[1024 + k * 256 + i] = q2[k];
            }
    }
    t.sync();
    if (tid < np) {
        float r2 = part[tid], q2 = part[1024 + tid];
        for (int k = 1; k < 4; ++k) {
            r2 += part[k * 256 + tid];
            q2 += part[1024 + k * 256 + tid];
        }
        const float u = u24f(draw(R.run_uid, seed32, tg, (uint32_t)tid, TAG_PSO_SR, 0).x);
        const float r = sqrtf(r2) * exp2f(log2f(u) / (float)D);
        sc[tid] = q2 > 0.f ? r / sqrtf(q2) : 0.f;
    }
    t.sync();
    for (int jb = wave; jb < nb2; jb += NW)
        for (int i = lane; i < np; i += 64) {
            const int li = ring ? li_arr[i] : g;
            const float s = sc[i];
            float z[2];
            normals(i, jb, z[0], z[1]);
            for (int e = 0; e < 2; ++e) {
                const int j = jb * 2 + e;
                if (j < D) {
                    const int row = j * npp;
                    const float xj = X[row + i];
                    const float xs = centre(i, li, row, xj) + s * z[e];
                    float vj = R.w * V[row + i] + (xs - xj);
                    vj = fminf(fmaxf(vj, -R.vmax), R.vmax);
                    float xn = xj + vj;
                    if (xn < R.lb) { xn = R.lb; vj = 0.f; }
                    else if (xn > R.ub) { xn = R.ub; vj = 0.f; }
                    Y[row + i] = xn;
                    V[row + i] = vj;
                }
            }
        }
}

// Double-precision error of one float point (the final check): rows of z by
// the team into sZ, then the objective by the team's first member (the
// value is valid there only).  Every member of the team must call it.
template <int FUNC, bool WAVE>
__device__ __forceinline__ double check_f64(const Team<WAVE> &t, const RunDev &R, const float *x, double *sZ,
                                            const Consts &K)
{
    const int D = R.dim;
    for (int r = t.tid; r < D; r += Team<WAVE>::SIZE) {
        double z = 0.0;
        for (int k = 0; k < D; ++k) z = fma(R.M64[(int64_t)r * D + k], (double)x[k] - R.o[k], z);
        sZ[r] = z;
    }
    t.sync();
    double e = 0.0;
    if (t.tid == 0) {
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

// Whole runs.  WAVE: four runs per workgroup, one per wave, all of the same
// instance (the host groups them; a slot with np = 0 is empty); otherwise
// one run per workgroup.  ONCHIP: each run's population (X and U, or X, V
// and P for PSO) lives in dynamic LDS, dyn_stride floats per run; otherwise
// in the library workspace.
// Algorithm families, one kernel each, so that a kernel holds only its own
// algorithm's paths and registers.
enum { FAM_DE = 0, FAM_SHADE = 1, FAM_LSHADE = 2, FAM_PSO = 3, FAM_PSODE = 4, FAM_LSHADE_RS = 5, NFAM = 6 };
inline int family_of(int algo)
{
    return algo == SEVO_ALGO_PSO ? FAM_PSO
         : algo == SEVO_ALGO_SHADE ? FAM_SHADE
         : algo == SEVO_ALGO_LSHADE || algo == SEVO_ALGO_JADE ? FAM_LSHADE
         : algo == SEVO_ALGO_LSHADE_RS ? FAM_LSHADE_RS
         : algo == SEVO_ALGO_PSODE ? FAM_PSODE
                                    : FAM_DE;
}

template <int KS, bool ONCHIP, bool WAVE, int FAM>
__global__ __launch_bounds__(256, 2) void k_run(const RunDev *__restrict__ runs, uint32_t seed32, Consts K,
                                                int dyn_stride)
{
    extern __shared__ __attribute__((aligned(16))) float sDyn[];
    constexpr int RT = (KS + 3) / 4;
    constexpr int TS = Team<WAVE>::SIZE;
    __shared__ __attribute__((aligned(16))) float sA[RT * KS * 64];
    __shared__ double sO[KS * 4];
    __shared__ float sT[RT * 16];
    // per-individual arrays: 256 entries, one 64-entry slice per wave team
    __shared__ unsigned long long sKeyA[256];
    __shared__ int sRankA[256];
    __shared__ float sFA[256], sCRA[256];
    __shared__ float sPvA[256];
    __shared__ int sPiA[256];
    __shared__ int sDaA[256], sDbA[256], sDcA[256], sJrA[256], sFlagA[256];
    __shared__ float sFiA[256];
    __shared__ uint32_t sThrA[256];
    __shared__ float sEXA[256], sEUA[256], sEPA[256];   // errors of x, of trials / new positions, of pbests
    __shared__ float sWv[4];
    __shared__ int sWi[4], sWc[4];
    __shared__ int sOwnA[768];            // L-SHADE: archive slot owners (192 per wave team)
    __shared__ int sNaA[4], sCutA[4];     // L-SHADE: archive size, slot of a removal
    __shared__ float sPart[2 * 4 * 256];  // spherical PSO: per-wave partial |G - x|^2, |z|^2
    constexpr int NSUM = 7;               // sums of the DE-family memory update
    __shared__ double sRed[4 * NSUM];
    __shared__ double sZA[WAVE ? 4 : 1][128];
    // per-team scalars
    __shared__ float sMFA[4][16], sMCRA[4][16];
    __shared__ int sPosA[4], sGA[4], sCopyA[4];
    __shared__ float sBestA[4], sBestBA[4];

    const Team<WAVE> t;
    const int tid = t.tid, s = t.slot, base = WAVE ? s * 64 : 0;
    const int run_index = WAVE ? blockIdx.x * 4 + s : blockIdx.x;

    // the instance, shared by the workgroup's runs
    {
        const RunDev &R0 = runs[WAVE ? blockIdx.x * 4 : blockIdx.x];
        stage_rotation<KS>(sA, R0.Mfrag);
        const int D0 = R0.dim;
        for (int q = threadIdx.x; q < KS * 4; q += 256) sO[q] = q < D0 ? R0.o[q] : 0.0;
        for (int q = threadIdx.x; q < RT * 16; q += 256) sT[q] = R0.tab[q];
    }
    __syncthreads();

    // read in place (scalar loads where it is used), not copied: a copy held
    // the whole descriptor in registers and made the larger kernels spill
    const RunDev &R = runs[run_index];
    if (WAVE && R.np == 0) return;   // empty slot: no barrier follows for wave teams
    const int D = R.dim, npp = R.npp;
    int np = R.np;   // L-SHADE shrinks it
    // the host launches each family's runs apart
    constexpr bool pso = FAM == FAM_PSO;
    // L-SHADE-Restart is L-SHADE with the restart block, kept in a kernel of
    // its own so that the others do not carry its registers
    constexpr bool rs_fam = FAM == FAM_LSHADE_RS;
    constexpr bool lshade = FAM == FAM_LSHADE || rs_fam;
    // PSODE: a PSO move and a SHADE generation from the same population,
    // then the pairwise/3 selection
    constexpr bool psode = FAM == FAM_PSODE;
    constexpr bool shade = FAM == FAM_SHADE || lshade || psode;
    // JADE runs in the L-SHADE kernel: one parameter pair (H = 1), no
    // reduction (np_min = np), its own parameter update
    const bool jade = lshade && R.algo == SEVO_ALGO_JADE;
    constexpr bool moves = pso || psode;   // makes a PSO move each generation
    // X population; U DE trials; V velocities; P personal bests (PSODE: the
    // population itself); Y where the PSO move goes (PSO: in place)
    float *X, *U, *V, *P, *Y;
    if constexpr (ONCHIP) {
        X = sDyn + (WAVE ? s * dyn_stride : 0);
        U = X + D * npp;
        V = psode ? X + 2 * D * npp : U;   // PSO keeps its velocities in U's place
        P = psode ? X : X + 2 * D * npp;
        Y = psode ? X + 3 * D * npp : X;
    } else {
        X = R.X;
        U = R.U;
        V = R.V;
        P = psode ? X : R.P;
        Y = psode ? R.P : X;
    }
    unsigned long long *sKey = sKeyA + base;
    int *sRank = sRankA + base, *sPi = sPiA + base;
    int *sDa = sDaA + base, *sDb = sDbA + base, *sDc = sDcA + base, *sJr = sJrA + base, *sFlag = sFlagA + base;
    float *sF = sFA + base, *sCR = sCRA + base, *sPv = sPvA + base, *sFi = sFiA + base;
    uint32_t *sThr = sThrA + base;
    float *sEX = sEXA + base, *sEU = sEUA + base, *sEP = sEPA + base;
    float *sMF = sMFA[s], *sMCR = sMCRA[s];
    double *sZ = sZA[WAVE ? s : 0];
    if (tid < 16) { sMF[tid] = 0.5f; sMCR[tid] = 0.5f; }
    if (tid == 0) {
        sPosA[s] = 0; sGA[s] = 0; sBestA[s] = INFINITY; sBestBA[s] = INFINITY; sCopyA[s] = -1;
        sNaA[s] = 0;
    }
    int *sOwn = sOwnA + (WAVE ? s * 192 : 0);

    // Element loops: the team's wave w takes coordinate blocks w, w + NW, ...;
    // its lanes take individuals, so every access to the [D][npp] state is
    // coalesced and the loads of one work item are independent of each other.
    const int lane = t.lane, wave = t.wave;
    constexpr int NW = Team<WAVE>::NW;

    // population k: x uniform in the box (double, then rounded to float),
    // k = 0 at generation 0, k >= 1 at L-SHADE-Restart's restarts
    auto draw_population = [&](uint32_t k) {
        for (int jb = wave; jb * 4 < D; jb += NW)
            for (int i = lane; i < np; i += 64) {
                const u32x4 w = draw(R.run_uid, seed32, 0, (uint32_t)i, TAG_INIT_X, (uint32_t)jb, k);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int j = jb * 4 + e;
                    if (j < D) {
                        const float x = (float)((double)R.lb + ((double)R.ub - (double)R.lb) * u24d(word(w, e)));
                        X[j * npp + i] = x;
                        if (pso) { V[j * npp + i] = 0.f; P[j * npp + i] = x; }
                        if (psode) V[j * npp + i] = 0.f;
                    }
                }
            }
        t.sync();
    };
    draw_population(0);

    int64_t fe = 0;
    int64_t fe_r = 0;   // L-SHADE-Restart: evaluations before the latest restart
    int gen = 0, restarts = 0;
    // recorder for the np evaluations eY (in index order) made at fe0
    auto record = [&](const float *Y, const float *eY) {
        float pv;
        int pi;
        const float before = sBestA[s];
        prefix_min(t, tid < np ? err_key(eY[tid]) : INFINITY, tid, sPv, sPi, sWv, sWi, pv, pi);
        if (tid < np && R.trace) {
            const int64_t c = fe + tid + 1;
            if (c % TRACE_EVERY == 0) {
                const int64_t k = c / TRACE_EVERY - 1;
                if (k < R.trace_len) R.trace[(int64_t)R.out_index * R.trace_len + k] = fminf(before, pv);
            }
        }
        if (tid == 0) {
            const int lim = (int)min<int64_t>((int64_t)np, R.budget - fe);
            sCopyA[s] = -1;
            if (lim > 0 && sPv[lim - 1] < sBestBA[s]) { sBestBA[s] = sPv[lim - 1]; sCopyA[s] = sPi[lim - 1]; }
            sBestA[s] = fminf(before, sPv[np - 1]);
        }
        t.sync();
        const int cp = sCopyA[s];
        if (cp >= 0)
            for (int j = tid; j < D; j += TS) R.bestx[j] = Y[j * npp + cp];
        t.sync();
    };
    // gbest = argmin of the personal bests' errors e, lowest index on ties
    auto global_best = [&](const float *e) {
        float pv;
        int pi;
        prefix_min(t, tid < np ? err_key(e[tid]) : INFINITY, tid, sPv, sPi, sWv, sWi, pv, pi);
        if (tid == 0) sGA[s] = sPi[TS - 1];
        t.sync();
    };
    // dst[j][i] = src[j][i] for the individuals with sFlag[i] set
    // (chunks of 8 rows: loads before stores)
    auto copy_flagged = [&](float *dst, const float *src) {
        constexpr int CP_CH = ONCHIP ? 1 : 8;
        for (int j0 = wave * CP_CH; j0 < D; j0 += NW * CP_CH)
            for (int i = lane; i < np; i += 64) {
                const bool f = sFlag[i] != 0;
                float v[CP_CH];
#pragma unroll
                for (int c = 0; c < CP_CH; ++c) v[c] = src[min(j0 + c, D - 1) * npp + i];
#pragma unroll
                for (int c = 0; c < CP_CH; ++c)
                    if (f && j0 + c < D) dst[(j0 + c) * npp + i] = v[c];
            }
        t.sync();
    };

    // parameter observer row g: JADE's pair, the memory means of the
    // success-history family (a terminal CR slot counts as 0), DE's fixed
    // F and CR, NaN for PSO
    auto observe = [&](int g) {
        if (tid == 0 && R.mu && g < R.mu_len) {
            float mf = NAN, mcr = NAN;
            if (shade) {
                double f = 0.0, cr = 0.0;
                for (int k = 0; k < R.H; ++k) {
                    f += (double)sMF[k];
                    cr += sMCR[k] < 0.f ? 0.0 : (double)sMCR[k];
                }
                mf = (float)(f / R.H);
                mcr = (float)(cr / R.H);
            } else if (!moves) {
                mf = R.F;
                mcr = R.CR;
            }
            float *row = R.mu + ((int64_t)R.out_index * R.mu_len + g) * 2;
            row[0] = mf;
            row[1] = mcr;
        }
    };

    eval_pop<KS, ONCHIP>(t, R, np, X, sEX, sA, sO, sT, K);
    t.sync();
    record(X, sEX);
    observe(0);
    if (pso) {
        if (tid < np) sEP[tid] = sEX[tid];
        t.sync();
        global_best(sEP);
    }
    if (psode && R.topology == 0) global_best(sEX);
    fe = np;

    // state rows of this run in the caller's snapshot arrays
    const int64_t st_row = (int64_t)R.out_index * R.st_dim;
    // a population [D][npp] and its errors into snapshot rows of st_np
    auto put_state = [&](float *dst, float *dst_e, const float *Y, const float *eY) {
        for (int j = wave; j < D; j += NW)
            for (int i = lane; i < np; i += 64) dst[(st_row + j) * R.st_np + i] = Y[j * npp + i];
        if (dst_e)
            for (int i = tid; i < np; i += TS) dst_e[(int64_t)R.out_index * R.st_np + i] = eY[i];
    };

    while (fe < R.budget && (R.gen_cap <= 0 || gen < R.gen_cap)) {
        ++gen;
        const uint32_t tg = (uint32_t)gen;
        // the generation after which the run stops (PSODE makes 2 np evaluations)
        const bool last_gen = (R.gen_cap > 0 && gen >= R.gen_cap) || fe + (psode ? 2 : 1) * (int64_t)np >= R.budget;
        int np_next = np;   // L-SHADE: the size after this generation
        if constexpr (moves) {
            // ---- PSO: update, evaluate, personal and global bests ----
            // (PSODE: the move goes to Y, its errors to sEP; the personal
            // bests are the population)
            const float *eB = pso ? sEP : sEX;   // errors of the personal bests
            float *eY = pso ? sEX : sEP;         // errors of the moved particles
            const int g = sGA[s];
            const bool ring = R.topology == 1;
            if (ring) {
                // neighbourhood best among {i-1, i, i+1}: lowest error, then lowest index
                if (tid < np) {
                    const int c0 = (tid + np - 1) % np, c2 = (tid + 1) % np;
                    int best = c0;
                    float kb = err_key(eB[c0]);
                    const int cand[2] = {tid, c2};
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const float kc = err_key(eB[cand[q]]);
                        if (kc < kb || (kc == kb && cand[q] < best)) { best = cand[q]; kb = kc; }
                    }
                    sDa[tid] = best;
                }
                t.sync();
            }
            const int nb2 = (D + 1) / 2;
            if (R.velocity == 0) {
            // chunks of PSO_CH coordinate blocks: all loads of a chunk are
            // issued before its stores, so a chunk costs one memory round trip
            // (from LDS a round trip is short and one block at a time saves
            // registers)
            constexpr int PSO_CH = ONCHIP ? 1 : (KS <= 13 ? 4 : 2);
            for (int jb0 = wave * PSO_CH; jb0 < nb2; jb0 += NW * PSO_CH)
                for (int i = lane; i < np; i += 64) {
                    float xj[PSO_CH][2], vv[PSO_CH][2], pj[PSO_CH][2], pg[PSO_CH][2];
#pragma unroll
                    for (int c = 0; c < PSO_CH; ++c)
#pragma unroll
                        for (int e = 0; e < 2; ++e) {
                            const int row = min((jb0 + c) * 2 + e, D - 1) * npp;
                            xj[c][e] = X[row + i];
                            vv[c][e] = V[row + i];
                            pj[c][e] = P[row + i];
                            pg[c][e] = P[row + (ring ? sDa[i] : g)];
                        }
#pragma unroll
                    for (int c = 0; c < PSO_CH; ++c) {
                        const int jb = jb0 + c;
                        if (jb >= nb2) break;
                        const u32x4 wd = draw(R.run_uid, seed32, tg, (uint32_t)i, TAG_PSO_R, (uint32_t)jb);
#pragma unroll
                        for (int e = 0; e < 2; ++e) {
                            const int j = jb * 2 + e;
                            if (j < D) {
                                const int row = j * npp;
                                const float r1 = u24f(word(wd, 2 * e)), r2 = u24f(word(wd, 2 * e + 1));
                                float vj = R.w * vv[c][e] + R.c1 * r1 * (pj[c][e] - xj[c][e]) +
                                           R.c2 * r2 * (pg[c][e] - xj[c][e]);
                                vj = fminf(fmaxf(vj, -R.vmax), R.vmax);
                                float xn = xj[c][e] + vj;
                                if (xn < R.lb) { xn = R.lb; vj = 0.f; }
                                else if (xn > R.ub) { xn = R.ub; vj = 0.f; }
                                Y[row + i] = xn;
                                V[row + i] = vj;
                            }
                        }
                    }
                }
            } else {
                spherical_update<WAVE>(t, R, seed32, tg, np, ring, g, X, Y, V, P, sDa, sFi, sPart + WAVE * s * 64);
            }
            t.sync();
            eval_pop<KS, ONCHIP>(t, R, np, Y, eY, sA, sO, sT, K);
            t.sync();
            record(Y, eY);
            if constexpr (pso) {
                if (tid < np) {
                    const bool imp = err_key(sEX[tid]) < err_key(sEP[tid]);
                    if (imp) sEP[tid] = sEX[tid];
                    sFlag[tid] = imp ? 1 : 0;
                }
                t.sync();
                copy_flagged(P, X);
                global_best(sEP);
            } else {
                fe += np;   // the DE half's evaluations follow
            }
        }
        if constexpr (!pso) {
            // ---- DE rand/1/bin or SHADE current-to-pbest/1 ----
            if (shade) {
                // ranking by (error, index): every key counts the keys below it
                if (tid < np) {
                    const uint32_t bits = __float_as_uint(err_key(sEX[tid]));
                    const uint32_t ord = (bits & 0x80000000u) ? ~bits : (bits | 0x80000000u);
                    sKey[tid] = ((unsigned long long)ord << 32) | (uint32_t)tid;
                }
                t.sync();
                if (tid < np) {
                    const unsigned long long key = sKey[tid];
                    int rank = 0;
                    for (int q = 0; q < np; ++q) rank += sKey[q] < key ? 1 : 0;
                    sRank[rank] = tid;
                }
                t.sync();
            }
            if (tid < np) {
                const int i = tid;
                if (shade) {
                    const int pnum = lshade ? min(max(round_half_up(R.p * (double)np), 2), np) : R.pnum;
                    const int n2 = lshade ? np + sNaA[s] : np;
                    const ShadeDraw d = shade_draw(R.run_uid, seed32, tg, i, np, n2, D, R.H, pnum, sMF, sMCR);
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
                    de_donors(R.run_uid, seed32, tg, i, np, D, ia, ib, ic, jrand);
                    sFi[i] = R.F;
                    sThr[i] = R.thr;
                    sDa[i] = ia;
                    sDb[i] = ib;
                    sDc[i] = ic;
                    sJr[i] = jrand;
                }
            }
            t.sync();
            // chunks of DE_CH coordinate blocks, loads before stores (see PSO);
            // two blocks fit the registers of every workspace variant
            constexpr int DE_CH = ONCHIP ? 1 : 2;
            const int nb4 = (D + 3) / 4;
            for (int jb0 = wave * DE_CH; jb0 < nb4; jb0 += NW * DE_CH)
                for (int i = lane; i < np; i += 64) {
                    const int ia = sDa[i], ib = sDb[i], ic = sDc[i], jrand = sJr[i];
                    const float Fi = sFi[i];
                    const uint32_t thr = sThr[i];
                    float xi[DE_CH][4], xa[DE_CH][4], xb[DE_CH][4], xc[DE_CH][4];
#pragma unroll
                    for (int c = 0; c < DE_CH; ++c)
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int jj = min((jb0 + c) * 4 + e, D - 1), row = jj * npp;
                            xi[c][e] = X[row + i];
                            xa[c][e] = X[row + ia];
                            // L-SHADE's r2 may index the archive (values >= np)
                            const float *pb = ib < np ? X + row + ib : R.Arc + (size_t)jj * R.acap + (ib - np);
                            xb[c][e] = *pb;
                            xc[c][e] = X[row + ic];
                        }
#pragma unroll
                    for (int c = 0; c < DE_CH; ++c) {
                        const int jb = jb0 + c;
                        if (jb >= nb4) break;
                        const u32x4 w = draw(R.run_uid, seed32, tg, (uint32_t)i, TAG_CROSS, (uint32_t)jb);
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int j = jb * 4 + e;
                            if (j < D) {
                                // SHADE: ic is the pbest individual, v = x + F (x_pbest - x) + F (x_r1 - x_r2)
                                float v;
                                if (shade) v = xi[c][e] + Fi * (xc[c][e] - xi[c][e]) + Fi * (xa[c][e] - xb[c][e]);
                                else v = xa[c][e] + Fi * (xb[c][e] - xc[c][e]);
                                bool m;
                                U[j * npp + i] = cross_repair<float>(word(w, e), thr, j, jrand, v, xi[c][e], R.lb,
                                                                     R.ub, m);
                            }
                        }
                    }
                }
            t.sync();
            eval_pop<KS, ONCHIP>(t, R, np, U, sEU, sA, sO, sT, K);
            t.sync();
            if (last_gen && R.st_u) put_state(R.st_u, R.st_eu, U, sEU);
            record(U, sEU);
            // sums of dl, dl CR, dl CR^2, dl F^2, dl F, successes, successes with CR > 0
            double st[NSUM] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            bool succ = false;
            if (tid < np) {
                const float ku = err_key(sEU[tid]), kx = err_key(sEX[tid]);
                succ = ku < kx;
                if (shade && succ) {
                    // JADE: plain means (weight 1); the others weight by the improvement
                    double dl = jade ? 1.0 : (double)kx - (double)ku;
                    if (!(dl <= 1e30)) dl = 1e30;
                    const double cr = sCR[tid], f = sF[tid];
                    st[0] = dl;
                    st[1] = dl * cr;
                    st[2] = dl * cr * cr;
                    st[3] = dl * f * f;
                    st[4] = dl * f;
                    st[5] = 1.0;
                    st[6] = cr > 0.0 ? 1.0 : 0.0;
                }
            }
            if (lshade) {
                // improved parents into the archive, in index order: appended
                // below the bound, else over a random member; where several
                // land on one slot the highest index wins (it came last)
                const int amax = round_half_up(R.r_arc * (double)np), na = sNaA[s];
                int total;
                const int k = team_exclusive_count(t, succ, sWc, total);
                int at = -1;
                if (succ) {
                    if (na + k < amax) at = na + k;
                    else if (amax > 0)
                        at = (int)range_map(draw(R.run_uid, seed32, tg, (uint32_t)tid, TAG_LSHADE_A, 0).x,
                                            (uint32_t)amax);
                }
                for (int q = tid; q < amax; q += TS) sOwn[q] = -1;
                t.sync();
                if (at >= 0) atomicMax(&sOwn[at], tid);
                t.sync();
                if (tid < np) sDa[tid] = at >= 0 && sOwn[at] == tid ? at : -1;
                t.sync();
                for (int j = wave; j < D; j += NW)
                    for (int i = lane; i < np; i += 64) {
                        const int slot = sDa[i];
                        if (slot >= 0) R.Arc[(size_t)j * R.acap + slot] = X[j * npp + i];
                    }
                t.sync();
                if (tid == 0) sNaA[s] = min(amax, na + total);
            }
            if constexpr (psode) {
                // pairwise/3: the DE result X3 (the trial where not worse than
                // its parent), the velocity set to X3 - X, then the PSO move
                // where strictly better than X3
                if (tid < np) {
                    const float kx = err_key(sEX[tid]), ku = err_key(sEU[tid]), ky = err_key(sEP[tid]);
                    const bool rep = ku <= kx;
                    const bool pw = ky < (rep ? ku : kx);
                    sEX[tid] = pw ? sEP[tid] : (rep ? sEU[tid] : sEX[tid]);
                    sFlag[tid] = (rep ? 1 : 0) | (pw ? 2 : 0);
                }
                t.sync();
                constexpr int SEL_CH = ONCHIP ? 1 : 4;
                for (int j0 = wave * SEL_CH; j0 < D; j0 += NW * SEL_CH)
                    for (int i = lane; i < np; i += 64) {
                        const int f = sFlag[i];
                        float xv[SEL_CH], uv[SEL_CH], yv[SEL_CH];
#pragma unroll
                        for (int c = 0; c < SEL_CH; ++c) {
                            const int row = min(j0 + c, D - 1) * npp;
                            xv[c] = X[row + i];
                            uv[c] = U[row + i];
                            yv[c] = Y[row + i];
                        }
#pragma unroll
                        for (int c = 0; c < SEL_CH; ++c)
                            if (j0 + c < D) {
                                const int row = (j0 + c) * npp;
                                V[row + i] = (f & 1) ? uv[c] - xv[c] : 0.f;
                                if (f) X[row + i] = (f & 2) ? yv[c] : uv[c];
                            }
                    }
                t.sync();
            } else {
                if (tid < np) {
                    const bool rep = err_key(sEU[tid]) <= err_key(sEX[tid]);
                    if (rep) sEX[tid] = sEU[tid];
                    sFlag[tid] = rep ? 1 : 0;
                }
                t.sync();
                copy_flagged(X, U);
            }
            if (shade) {
                team_sums<NSUM>(t, st, sRed);
                if (tid == 0 && st[5] > 0.0 && jade) {
                    // muCR towards the mean of S_CR, muF towards the Lehmer mean of S_F
                    const double c = R.c_adapt;
                    sMCR[0] = (float)((1.0 - c) * (double)sMCR[0] + c * (st[1] / st[0]));
                    sMF[0] = (float)((1.0 - c) * (double)sMF[0] + c * (st[3] / st[4]));
                } else if (tid == 0 && st[5] > 0.0) {
                    const int pos = sPosA[s];
                    if (lshade)   // weighted Lehmer mean; terminal value kept or set
                        sMCR[pos] = (sMCR[pos] < 0.f || st[6] == 0.0) ? -1.f : (float)(st[2] / st[1]);
                    else          // SHADE: weighted arithmetic mean
                        sMCR[pos] = (float)(st[1] / st[0]);
                    sMF[pos] = (float)(st[3] / st[4]);
                    sPosA[s] = (pos + 1) % R.H;
                }
                t.sync();
            }
            observe(gen);
            if (psode && R.topology == 0) global_best(sEX);
            if (lshade) {
                // linear population size reduction (from the latest restart to the
                // budget): the best nn stay, in index order
                const int nn = min(lshade_np(R.np, R.np_min, R.budget - fe_r, fe - fe_r + np), np);
                if (nn < np) {
                    if (tid < np) {
                        const uint32_t bits = __float_as_uint(err_key(sEX[tid]));
                        const uint32_t ord = (bits & 0x80000000u) ? ~bits : (bits | 0x80000000u);
                        sKey[tid] = ((unsigned long long)ord << 32) | (uint32_t)tid;
                    }
                    t.sync();
                    bool keep = false;
                    if (tid < np) {
                        const unsigned long long key = sKey[tid];
                        int rank = 0;
                        for (int q = 0; q < np; ++q) rank += sKey[q] < key ? 1 : 0;
                        keep = rank < nn;
                    }
                    int kept;
                    const int to = team_exclusive_count(t, keep, sWc, kept);
                    if (tid < np) sDb[tid] = keep ? to : -1;
                    t.sync();
                    for (int j = wave; j < D; j += NW)
                        for (int i = lane; i < np; i += 64) {
                            const int d = sDb[i];
                            if (d >= 0) U[j * npp + d] = X[j * npp + i];
                        }
                    if (tid < np && keep) sEU[to] = sEX[tid];
                    t.sync();
                    float *tx = X; X = U; U = tx;
                    float *te = sEX; sEX = sEU; sEU = te;
                    // the archive down to its new bound by random removals,
                    // the last member moving into the freed slot
                    const int amax2 = round_half_up(R.r_arc * (double)nn);
                    int na = sNaA[s];
                    for (uint32_t k = 0; na > amax2; ++k) {
                        if (tid == 0)
                            sCutA[s] = (int)range_map(draw(R.run_uid, seed32, tg, k, TAG_LSHADE_S, 0).x,
                                                      (uint32_t)na);
                        t.sync();
                        const int cut = sCutA[s];
                        if (cut != na - 1)
                            for (int j = tid; j < D; j += TS)
                                R.Arc[(size_t)j * R.acap + cut] = R.Arc[(size_t)j * R.acap + na - 1];
                        t.sync();
                        --na;
                    }
                    if (tid == 0) sNaA[s] = na;
                    t.sync();
                    np_next = nn;
                }
            }
        }
        fe += np;
        np = np_next;
        if (rs_fam && R.restart && fe < R.budget) {
            // L-SHADE-Restart: restart once the population's errors span at
            // most restart_tol (NaN counts as +infinity: never converged)
            float pv;
            int pi;
            prefix_min(t, tid < np ? err_key(sEX[tid]) : INFINITY, tid, sPv, sPi, sWv, sWi, pv, pi);
            const float lo = sPv[TS - 1];
            t.sync();
            prefix_min(t, tid < np ? -err_key(sEX[tid]) : INFINITY, tid, sPv, sPi, sWv, sWi, pv, pi);
            const float hi = -sPv[TS - 1];
            t.sync();
            if ((double)(hi - lo) <= R.restart_tol) {
                // a fresh population, memories at 0.5, an empty archive, and
                // the size schedule started over
                ++restarts;
                fe_r = fe;
                np = R.np;
                draw_population((uint32_t)restarts);
                eval_pop<KS, ONCHIP>(t, R, np, X, sEX, sA, sO, sT, K);
                t.sync();
                record(X, sEX);
                fe += np;
                if (tid < 16) { sMF[tid] = 0.5f; sMCR[tid] = 0.5f; }
                if (tid == 0) { sPosA[s] = 0; sNaA[s] = 0; }
                t.sync();
            }
        }
    }

    // observer rows of generations not made (PSO: every row) are NaN
    if (R.mu)
        for (int64_t g = (pso ? 0 : gen + 1) + tid; g < R.mu_len; g += TS) {
            float *row = R.mu + ((int64_t)R.out_index * R.mu_len + g) * 2;
            row[0] = NAN;
            row[1] = NAN;
        }

    // the state the run stopped in
    if (R.st_x) {
        put_state(R.st_x, R.st_e, X, sEX);
        if (moves && R.st_v) put_state(R.st_v, nullptr, V, nullptr);
        if (pso && R.st_p) put_state(R.st_p, R.st_ep, P, sEP);
        if (shade && R.st_mem && tid < 16) {
            R.st_mem[(int64_t)R.out_index * 32 + tid] = sMF[tid];
            R.st_mem[(int64_t)R.out_index * 32 + 16 + tid] = sMCR[tid];
        }
        if (lshade && R.st_arc_out) {
            const int na = sNaA[s];
            for (int j = wave; j < D; j += NW)
                for (int a = lane; a < na; a += 64)
                    R.st_arc_out[(st_row + j) * R.st_arc + a] = R.Arc[(size_t)j * R.acap + a];
        }
        if (R.st_cnt && tid == 0) {
            int32_t *c = R.st_cnt + (int64_t)R.out_index * 4;
            c[0] = np;
            c[1] = lshade ? sNaA[s] : 0;
            c[2] = shade ? sPosA[s] : 0;
            c[3] = moves && R.topology == 0 ? sGA[s] : 0;
        }
    }

    // results; the best point is re-evaluated in double once below 1e-6
    const float be = sBestBA[s];
    double e64 = (double)be;
    if (be < 1e-6f) {
        switch (R.func) {
        case ELLIPSOID: e64 = check_f64<ELLIPSOID>(t, R, R.bestx, sZ, K); break;
        case ROSENBROCK: e64 = check_f64<ROSENBROCK>(t, R, R.bestx, sZ, K); break;
        case RASTRIGIN: e64 = check_f64<RASTRIGIN>(t, R, R.bestx, sZ, K); break;
        case SCHWEFEL: e64 = check_f64<SCHWEFEL>(t, R, R.bestx, sZ, K); break;
        case GRIEWANK: e64 = check_f64<GRIEWANK>(t, R, R.bestx, sZ, K); break;
        default: e64 = check_f64<ACKLEY>(t, R, R.bestx, sZ, K); break;
        }
    }
    if (tid == 0) {
        sevo_run_result &o = R.res[R.out_index];
        o.best_e = e64;
        o.best_e32 = be;
        o.success = e64 <= 1e-8 ? 1 : 0;
        o.fes = fe;
        o.generations = gen;
        o.restarts = restarts;
    }
    if (R.best_x_out)
        for (int j = tid; j < D; j += TS) R.best_x_out[(int64_t)R.out_index * R.max_dim + j] = (double)R.bestx[j];
}

typedef void (*RunKernel)(const RunDev *, uint32_t, Consts, int);

// The kernel of a (k-step class, placement, team) of family FAM; nullptr
// outside 1 .. 30 k-steps.  Each family instantiates it in its own source.
template <int FAM, int KS>
RunKernel kernel_of(bool onchip, bool wave)
{
    if (wave) return onchip ? k_run<KS, true, true, FAM> : k_run<KS, false, true, FAM>;
    return onchip ? k_run<KS, true, false, FAM> : k_run<KS, false, false, FAM>;
}

template <int FAM>
RunKernel family_table(int ks, bool onchip, bool wave)
{
    switch (ks) {
#define SEVO_KS_CASE(v) case v: return kernel_of<FAM, v>(onchip, wave);
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

RunKernel run_table_de(int ks, bool onchip, bool wave);
RunKernel run_table_shade(int ks, bool onchip, bool wave);
RunKernel run_table_lshade(int ks, bool onchip, bool wave);
RunKernel run_table_pso(int ks, bool onchip, bool wave);
RunKernel run_table_psode(int ks, bool onchip, bool wave);
RunKernel run_table_lshade_rs(int ks, bool onchip, bool wave);
inline RunKernel run_table(int fam, int ks, bool onchip, bool wave)
{
    switch (fam) {
    case FAM_DE: return run_table_de(ks, onchip, wave);
    case FAM_SHADE: return run_table_shade(ks, onchip, wave);
    case FAM_LSHADE: return run_table_lshade(ks, onchip, wave);
    case FAM_PSO: return run_table_pso(ks, onchip, wave);
    case FAM_PSODE: return run_table_psode(ks, onchip, wave);
    case FAM_LSHADE_RS: return run_table_lshade_rs(ks, onchip, wave);
    default: return nullptr;
    }
}

}  // namespace sevo
