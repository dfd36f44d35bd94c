// algo.h -- device pieces of the DE / PSO / SHADE generation steps shared by
// the one-step kernels (steps.hip) and the fused run kernels (run.hip):
// donor draws, binomial crossover with midpoint-target repair, the ordering
// of error values, and the SHADE parameter draws.
//
// Every random choice is a pure function of (run_uid, seed, generation t,
// individual i, tag, block), so results do not depend on how runs and
// individuals are mapped to workgroups and lanes.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "common.h"

namespace sevo {

// Ordering of error values: NaN counts as +infinity.
template <typename T>
__device__ __forceinline__ T err_key(T e)
{
    return isnan(e) ? T(INFINITY) : e;
}

// Index in [0, n) other than the m excluded indices ex[0..m) (any order):
// one draw over the n - m allowed values, then stepped past the excluded
// values in ascending order.
template <int m>
__device__ __forceinline__ int pick_excluding(uint32_t w, int n, const int (&ex)[m])
{
    int s[m];
#pragma unroll
    for (int a = 0; a < m; ++a) s[a] = ex[a];
#pragma unroll
    for (int a = 1; a < m; ++a)
#pragma unroll
        for (int b = m - 1; b >= a; --b)
            if (s[b - 1] > s[b]) { const int t = s[b]; s[b] = s[b - 1]; s[b - 1] = t; }
    int r = (int)range_map(w, (uint32_t)(n - m));
#pragma unroll
    for (int a = 0; a < m; ++a) r += (r >= s[a]) ? 1 : 0;
    return r;
}

// rand/1 donors r1, r2, r3 (distinct, != i) and jrand of individual i.
__device__ __forceinline__ void de_donors(uint32_t run_uid, uint32_t seed32, uint32_t t, int i,
                                          int np, int dim, int &r1, int &r2, int &r3, int &jrand)
{
    const u32x4 w = draw(run_uid, seed32, t, (uint32_t)i, TAG_DONORS, 0);
    const int e1[1] = {i};
    r1 = pick_excluding<1>(w.x, np, e1);
    const int e2[2] = {i, r1};
    r2 = pick_excluding<2>(w.y, np, e2);
    const int e3[3] = {i, r1, r2};
    r3 = pick_excluding<3>(w.z, np, e3);
    jrand = (int)range_map(w.w, (uint32_t)dim);
}

// Coordinate j of the trial: binomial crossover (donor where the 24-bit
// uniform is below CR, i.e. (w >> 8) < thr, or j = jrand), then the
// midpoint-target repair of a coordinate outside [lb, ub].
template <typename T>
__device__ __forceinline__ T cross_repair(uint32_t word, uint32_t thr, int j, int jrand, T v, T x,
                                          T lb, T ub, bool &mask)
{
    mask = ((word >> 8) < thr) || (j == jrand);
    T u = mask ? v : x;
    if (u < lb) u = T(0.5) * (lb + x);
    else if (u > ub) u = T(0.5) * (ub + x);
    return u;
}

// SHADE per-individual parameters: memory slot k, CR ~ N(M_CR[k], 0.1)
// clipped to [0, 1] (CR = 0 when the slot holds the terminal value, a
// negative number, which only L-SHADE sets), F ~ Cauchy(M_F[k], 0.1)
// redrawn while <= 0 (at most 64 draws, then F = M_F[k]) and capped at 1;
// pbest drawn from the top pnum of the ranking; r1 != i; r2 not in {i, r1}
// among n2 candidates (np for SHADE; np + archive size for L-SHADE, where
// values >= np index the archive); jrand.
struct ShadeDraw {
    int k, pbest_rank, r1, r2, jrand, retries;
    float F, CR;
};

__device__ __forceinline__ ShadeDraw shade_draw(uint32_t run_uid, uint32_t seed32, uint32_t t, int i,
                                                int np, int n2, int dim, int H, int pnum, const float *MF,
                                                const float *MCR)
{
    ShadeDraw d;
    const u32x4 wp = draw(run_uid, seed32, t, (uint32_t)i, TAG_SHADE_P, 0);
    d.k = (int)range_map(wp.x, (uint32_t)H);
    // Box-Muller on (1 - u1, u2): radius sqrt(-2 ln(1 - u1)), angle 2 pi u2
    const float u1 = u24f(wp.y), u2 = u24f(wp.z);
    const float nrm = sqrtf(-2.f * logf(1.f - u1)) * cospif(2.f * u2);
    float cr = MCR[d.k] + 0.1f * nrm;
    d.CR = MCR[d.k] < 0.f ? 0.f : fminf(fmaxf(cr, 0.f), 1.f);
    float F = -1.f;
    int retries = 0;
    for (; retries < 64; ++retries) {
        const u32x4 wc = draw(run_uid, seed32, t, (uint32_t)i, TAG_SHADE_C, 0, (uint32_t)retries);
        const float v = u24f(wc.x) - 0.5f;   // tan(pi v) = sin(pi v) / cos(pi v)
        const float Fc = MF[d.k] + 0.1f * (sinpif(v) / cospif(v));
        if (Fc > 0.f) { F = Fc; break; }
    }
    if (!(F > 0.f)) F = MF[d.k];
    d.F = fminf(F, 1.f);
    d.retries = retries;
    d.pbest_rank = (int)range_map(wp.w, (uint32_t)pnum);
    const u32x4 wd = draw(run_uid, seed32, t, (uint32_t)i, TAG_SHADE_D, 0);
    const int e1[1] = {i};
    d.r1 = pick_excluding<1>(wd.x, np, e1);
    const int e2[2] = {i, d.r1};
    d.r2 = pick_excluding<2>(wd.y, n2, e2);
    d.jrand = (int)range_map(wd.z, (uint32_t)dim);
    return d;
}

}  // namespace sevo
