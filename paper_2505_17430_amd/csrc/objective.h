// objective.h -- per-coordinate terms and reductions of the six test
// functions, written for the GPU (float for the batched path, double for the
// plain path and the final check).
//
// Every function is evaluated in a form algebraically equal to its textbook
// definition but free of cancellation near the optimum z = 0, so that the
// error e = f - f* keeps its relative accuracy when it is tiny:
//   Rastrigin   z^2 - 10 cos(2 pi z) + 10        = z^2 + 20 sin^2(pi z)
//   Rosenbrock  100 (w_i^2 - w_{i+1})^2 + (w_i-1)^2, w = z + 1
//                                                = 100 (z_i^2 + 2 z_i - z_{i+1})^2 + z_i^2
//   Griewank    1 - prod cos(a_i) = -expm1(sum log1p(-2 sin^2(a_i / 2)))   (all cos > 0)
//               = 1 + exp(sum log|cos a_i|)       (odd number of negative cosines)
//   Ackley      20 - 20 exp(-0.2 r) + e - exp(mean cos 2 pi z)
//               = -20 expm1(-0.2 r) - e expm1(-(2/D) sum sin^2(pi z))
//   Schwefel    g(u) = c - u sin(sqrt u), u = s + z > 0: with a = sqrt s,
//               t = z / (a + sqrt(s + z)):
//               g = -2 s cos(a + t/2) sin(t/2) - z sin(a + t),
//               sin(a + t) and cos(a + t/2) expanded with sin a, cos a
//               precomputed in double.
// Sums are compensated (Neumaier per lane, error-free TwoSum merges across
// lanes).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "common.h"

namespace sevo {

template <typename T>
struct SchwefelConst {
    T s, a, sa, ca, c, zhi, zlo, gp, gm, lambda, nega_s;
};

// Compensated accumulator of two running sums plus the sign / zero flags of
// Griewank's cosine product.
template <typename T>
struct Acc {
    T s1, c1, s2, c2;
    int neg, zero;
    __device__ __forceinline__ void init() { s1 = c1 = s2 = c2 = T(0); neg = zero = 0; }
};

template <typename T>
__device__ __forceinline__ void neumaier(T &s, T &c, T x)
{
#pragma clang fp contract(off)
    const T t = s + x;
    c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
    s = t;
}

// (s, c) += (s2, c2) with the rounding error of the head addition kept.
template <typename T>
__device__ __forceinline__ void merge(T &s, T &c, T s2, T c2)
{
#pragma clang fp contract(off)
    const T t = s + s2;
    const T bp = t - s;
    const T err = (s - (t - bp)) + (s2 - bp);
    c = c + c2 + err;
    s = t;
}

__device__ __forceinline__ float sinpi_t(float x) { return sinpif(x); }
__device__ __forceinline__ double sinpi_t(double x) { return sinpi(x); }
__device__ __forceinline__ void sincos_t(float x, float *s, float *c) { sincosf(x, s, c); }
__device__ __forceinline__ void sincos_t(double x, double *s, double *c) { sincos(x, s, c); }

template <typename T>
__device__ __forceinline__ T schwefel_term(T z, const SchwefelConst<T> &K)
{
    if (z > K.zhi) {                       // u > 500
        const T b = z - K.zhi;
        return K.gp + K.lambda * b * b;
    }
    if (z < K.zlo) {                       // u < -500
        const T b = K.zlo - z;
        return K.gm + K.lambda * b * b;
    }
    if (z > K.nega_s) {                    // 0 < u <= 500: difference form
        const T t = z / (K.a + sqrt(K.s + z));
        const T h = T(0.5) * t;
        T sh, ch;
        sincos_t(h, &sh, &ch);
        const T sin_t = T(2) * sh * ch;
        const T cos_t = T(1) - T(2) * sh * sh;
        const T cos_ah = K.ca * ch - K.sa * sh;
        const T sin_at = K.sa * cos_t + K.ca * sin_t;
        return T(-2) * K.s * cos_ah * sh - z * sin_at;
    }
    const T u = -(z + K.s);                // u <= 0: c + |u| sin(sqrt|u|)
    return K.c + u * sin(sqrt(u));
}

// Add the term of coordinate r (value z, next coordinate zn, per-row table
// value tab = ellipsoid weight or 1/sqrt(r+1)) to the accumulator.
template <int FUNC, typename T>
__device__ __forceinline__ void add_term(Acc<T> &acc, T z, T zn, bool has_next, T tab,
                                         const SchwefelConst<T> &K)
{
    if constexpr (FUNC == ELLIPSOID) {
        neumaier(acc.s1, acc.c1, tab * z * z);
    } else if constexpr (FUNC == ROSENBROCK) {
        if (has_next) {
            const T q = z * z + T(2) * z - zn;
            neumaier(acc.s1, acc.c1, T(100) * q * q + z * z);
        }
    } else if constexpr (FUNC == RASTRIGIN) {
        const T sp = sinpi_t(z);
        neumaier(acc.s1, acc.c1, z * z + T(20) * sp * sp);
    } else if constexpr (FUNC == SCHWEFEL) {
        neumaier(acc.s1, acc.c1, schwefel_term(z, K));
    } else if constexpr (FUNC == GRIEWANK) {
        neumaier(acc.s1, acc.c1, z * z);
        const T h = sin(T(0.5) * z * tab);
        const T h2 = T(2) * h * h;
        const T cs = T(1) - h2;
        if (cs > T(0)) {
            neumaier(acc.s2, acc.c2, log1p(-h2));
        } else if (cs < T(0)) {
            neumaier(acc.s2, acc.c2, log(-cs));
            acc.neg ^= 1;
        } else {
            acc.zero = 1;
        }
    } else {  // ACKLEY
        neumaier(acc.s1, acc.c1, z * z);
        const T sp = sinpi_t(z);
        neumaier(acc.s2, acc.c2, sp * sp);
    }
}

template <int FUNC, typename T>
__device__ __forceinline__ T finalize(const Acc<T> &acc, int dim)
{
    if constexpr (FUNC == GRIEWANK) {
        const T L = acc.s2 + acc.c2;
        T one_minus_prod;
        if (acc.zero) one_minus_prod = T(1);
        else if (acc.neg) one_minus_prod = T(1) + exp(L);
        else one_minus_prod = -expm1(L);
        return (acc.s1 + acc.c1) / T(4000) + one_minus_prod;
    } else if constexpr (FUNC == ACKLEY) {
        const T D = T(dim);
        const T q = acc.s1 + acc.c1;
        const T ss = acc.s2 + acc.c2;
        return T(-20) * expm1(T(-0.2) * sqrt(q / D)) -
               T(2.718281828459045235360287) * expm1(T(-2) * ss / D);
    } else {
        return acc.s1 + acc.c1;
    }
}

// Merge the accumulators of lanes `lane ^ mask` into this lane.
template <typename T>
__device__ __forceinline__ void merge_xor(Acc<T> &acc, int mask)
{
    const T s1 = __shfl_xor(acc.s1, mask, 64);
    const T c1 = __shfl_xor(acc.c1, mask, 64);
    const T s2 = __shfl_xor(acc.s2, mask, 64);
    const T c2 = __shfl_xor(acc.c2, mask, 64);
    const int fl = __shfl_xor(acc.neg | (acc.zero << 1), mask, 64);
    merge(acc.s1, acc.c1, s1, c1);
    merge(acc.s2, acc.c2, s2, c2);
    acc.neg ^= fl & 1;
    acc.zero |= fl >> 1;
}

}  // namespace sevo
