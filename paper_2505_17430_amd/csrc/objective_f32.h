// objective_f32.h -- single-precision objective terms for the batched MFMA
// evaluation, written for VALU throughput.
//
// Same functions and cancellation-free forms as objective.h, with:
//  - sin and cos of pi*v from v = n + r, n = rint(v) (exact), |r| <= 1/2 and
//    the Taylor series of sin(pi r) to r^13 and cos(pi r) to r^12 (truncation
//    below 7e-10, float Horner error about 2e-7); sin^2 needs no sign;
//  - Griewank without logarithms: with y_i = 1 - cos a_i = 2 sin^2(a_i / 2),
//    Q = 1 - prod (1 - y_i) obeys Q <- Q + y (1 - Q), exact in real
//    arithmetic, free of cancellation near the optimum, and two partial Q
//    combine with the same rule; its additions are compensated;
//  - Schwefel branch-free: one sqrt of |u|, one reciprocal, one sincos, and
//    selects for the four regions of u = z + s;
//  - compensation per group of four rows: the four terms of a 16-row MFMA
//    tile that a lane holds are added plainly, then the group sum enters the
//    lane's running sum through an error-free TwoSum.  All terms of a sum
//    have the same sign, so the plain group adds cost at most 3 eps of the
//    result, independent of D.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"
#include "objective.h"

namespace sevo {

struct AccF {
    float s1, c1;   // main sum (compensated)
    float s2, c2;   // Ackley: sum sin^2(pi z); Griewank: Q = 1 - prod cos (compensated)
    __device__ __forceinline__ void init() { s1 = c1 = s2 = c2 = 0.f; }
};

// s + x = s' + err exactly (Knuth's TwoSum); err is added to the compensation.
__device__ __forceinline__ void two_sum_into(float &s, float &c, float x)
{
#pragma clang fp contract(off)
    const float t = s + x;
    const float bp = t - s;
    const float err = (s - (t - bp)) + (x - bp);
    s = t;
    c += err;
}

__device__ __forceinline__ float sin_pi_red(float r, float r2)
{
    float p = 4.6630280576761234e-4f;
    p = fmaf(p, r2, -7.370430945714348e-3f);
    p = fmaf(p, r2, 8.214588661112819e-2f);
    p = fmaf(p, r2, -5.992645293207919e-1f);
    p = fmaf(p, r2, 2.550164039877345f);
    p = fmaf(p, r2, -5.167712780049969f);
    p = fmaf(p, r2, 3.141592653589793f);
    return r * p;
}

__device__ __forceinline__ float cos_pi_red(float r2)
{
    float p = 1.929574309403922e-3f;
    p = fmaf(p, r2, -2.580689139001405e-2f);
    p = fmaf(p, r2, 2.3533063035889312e-1f);
    p = fmaf(p, r2, -1.3352627688545893f);
    p = fmaf(p, r2, 4.058712126416768f);
    p = fmaf(p, r2, -4.934802200544679f);
    return fmaf(p, r2, 1.f);
}

// sin^2(pi v)
__device__ __forceinline__ float sin2_pi(float v)
{
    const float r = v - rintf(v);
    const float s = sin_pi_red(r, r * r);
    return s * s;
}

// sin(pi v), cos(pi v)
__device__ __forceinline__ void sincos_pi(float v, float &s, float &c)
{
    const float n = rintf(v);
    const float r = v - n;
    const float r2 = r * r;
    const float sign = ((int)n & 1) ? -1.f : 1.f;
    s = sign * sin_pi_red(r, r2);
    c = sign * cos_pi_red(r2);
}

__device__ __forceinline__ float schwefel_g_f32(float z, const SchwefelConst<float> &K)
{
    constexpr float INV_PI = 0.318309886183790671538f;
    const float u = K.s + z;
    const float sq = __builtin_amdgcn_sqrtf(fabsf(u));   // hardware sqrt, about 1 ulp
    const bool pos = u > 0.f;
    // u > 0: t = z / (sqrt s + sqrt u), angle t/2; u <= 0: angle sqrt|u|.
    // The hardware reciprocal (about 1 ulp) replaces a correctly rounded
    // division, which the compiler would otherwise put behind a branch.
    const float th_pos = (0.5f * INV_PI) * (z * __builtin_amdgcn_rcpf(K.a + sq));
    const float th_neg = sq * INV_PI;
    const float theta = pos ? th_pos : th_neg;
    float sh, ch;
    sincos_pi(theta, sh, ch);
    const float sin_t = 2.f * sh * ch;
    const float cos_t = fmaf(-2.f * sh, sh, 1.f);
    const float cos_ah = K.ca * ch - K.sa * sh;
    const float sin_at = K.sa * cos_t + K.ca * sin_t;
    const float g_pos = (-2.f * K.s) * cos_ah * sh - z * sin_at;
    const float g_neg = K.c - u * sh;
    const float bh = z - K.zhi, bl = K.zlo - z;
    const float g_hi = fmaf(K.lambda * bh, bh, K.gp);
    const float g_lo = fmaf(K.lambda * bl, bl, K.gm);
    float g = pos ? g_pos : g_neg;
    g = (z > K.zhi) ? g_hi : g;
    g = (z < K.zlo) ? g_lo : g;
    return g;
}

// Terms of one lane's four consecutive rows (z[0..3], row r0 .. r0+3).
// valid = number of rows < dim (0..4); zn3 = z of row r0 + 4 (Rosenbrock);
// has_next3 = row r0 + 3 has a successor inside the point's dimension.
// tab = per-row table (ellipsoid weights; Griewank 1 / (2 pi sqrt(i))).
template <int FUNC>
__device__ __forceinline__ void add_group(AccF &a, const float z[4], float zn3, int valid,
                                          bool has_next3, const float tab[4],
                                          const SchwefelConst<float> &K)
{
    // Every term is computed for all four rows and then selected, so that the
    // fold is straight-line code (a conditional expression with a costly arm
    // would become a branch) and can be scheduled between matrix-core ops.
    float g1 = 0.f, g2 = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const bool ok = j < valid;
        const float zj = z[j];
        if constexpr (FUNC == ELLIPSOID) {
            const float t = tab[j] * zj * zj;
            g1 += ok ? t : 0.f;
        } else if constexpr (FUNC == ROSENBROCK) {
            const float zn = j < 3 ? z[j < 3 ? j + 1 : 0] : zn3;
            const bool nx = j < 3 ? (j + 1 < valid) : has_next3;
            const float q = fmaf(zj, zj, 2.f * zj) - zn;
            const float t = fmaf(100.f * q, q, zj * zj);
            g1 += (ok && nx) ? t : 0.f;
        } else if constexpr (FUNC == RASTRIGIN) {
            const float t = fmaf(20.f, sin2_pi(zj), zj * zj);
            g1 += ok ? t : 0.f;
        } else if constexpr (FUNC == SCHWEFEL) {
            const float t = schwefel_g_f32(zj, K);
            g1 += ok ? t : 0.f;
        } else if constexpr (FUNC == GRIEWANK) {
            const float t = zj * zj;
            const float yt = 2.f * sin2_pi(zj * tab[j]);
            g1 += ok ? t : 0.f;
            const float y = ok ? yt : 0.f;
            two_sum_into(a.s2, a.c2, y * (1.f - (a.s2 + a.c2)));
        } else {  // ACKLEY
            const float t = zj * zj;
            const float st = sin2_pi(zj);
            g1 += ok ? t : 0.f;
            g2 += ok ? st : 0.f;
        }
    }
    two_sum_into(a.s1, a.c1, g1);
    if constexpr (FUNC == ACKLEY) two_sum_into(a.s2, a.c2, g2);
}

// Merge accumulator b into a (b covers rows after a's or disjoint ones).
template <int FUNC>
__device__ __forceinline__ void merge_f(AccF &a, float s1, float c1, float s2, float c2)
{
    merge(a.s1, a.c1, s1, c1);
    if constexpr (FUNC == ACKLEY) {
        merge(a.s2, a.c2, s2, c2);
    } else if constexpr (FUNC == GRIEWANK) {
        // 1 - PaPb = Qa + Qb (1 - Qa)
        const float qa = a.s2 + a.c2, qb = s2 + c2;
        two_sum_into(a.s2, a.c2, qb * (1.f - qa));
    }
}

template <int FUNC>
__device__ __forceinline__ void merge_xor_f(AccF &a, int mask)
{
    const float s1 = __shfl_xor(a.s1, mask, 64);
    const float c1 = __shfl_xor(a.c1, mask, 64);
    float s2 = 0.f, c2 = 0.f;
    if constexpr (FUNC == ACKLEY || FUNC == GRIEWANK) {
        s2 = __shfl_xor(a.s2, mask, 64);
        c2 = __shfl_xor(a.c2, mask, 64);
    }
    merge_f<FUNC>(a, s1, c1, s2, c2);
}

template <int FUNC>
__device__ __forceinline__ float finalize_f(const AccF &a, float inv_dim)
{
    const float q = a.s1 + a.c1;
    if constexpr (FUNC == GRIEWANK) {
        return q * (1.f / 4000.f) + (a.s2 + a.c2);
    } else if constexpr (FUNC == ACKLEY) {
        const float ss = a.s2 + a.c2;
        return -20.f * expm1f(-0.2f * sqrtf(q * inv_dim)) - 2.718281828459045f * expm1f(-2.f * ss * inv_dim);
    } else {
        return q;
    }
}

}  // namespace sevo
