// common.h -- definitions shared by the host runtime and the gfx950 kernels of
// the library: Philox4x32-10, the uniform / index maps of its words, the
// stream tags, function identifiers and the Schwefel constants.
//
// The stream map (who draws which counter) is the contract that makes every
// random draw reproducible and independent of how runs are mapped onto
// workgroups:
//   key     = (run_uid, lo32(seed) ^ hi32(seed))
//   counter = (t, i, tag << 24 | block, c3)
// with t the generation (0 = initialisation), i the individual, block the
// 4-coordinate (or 2-coordinate for PSO) group, c3 a retry index.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define SEVO_HD __host__ __device__ __forceinline__
#else
#define SEVO_HD inline
#endif

namespace sevo {

enum Func : int32_t { ELLIPSOID = 0, ROSENBROCK = 1, RASTRIGIN = 2, SCHWEFEL = 3,
                      GRIEWANK = 4, ACKLEY = 5, NFUNC = 6 };

enum Tag : uint32_t {
    TAG_INIT_X = 1,   // generation 0: one word per coordinate, block = j / 4
    TAG_DONORS = 2,   // DE rand/1: (r1, r2, r3, jrand)
    TAG_CROSS = 3,    // crossover uniforms, block = j / 4
    TAG_PSO_R = 4,    // PSO: (r1_j, r2_j, r1_{j+1}, r2_{j+1}), block = j / 2
    TAG_SHADE_P = 5,  // SHADE: (memory slot, normal u1, normal u2, pbest)
    TAG_SHADE_C = 6,  // SHADE: Cauchy uniform in word 0, c3 = retry
    TAG_SHADE_D = 7,  // SHADE: (r1, r2, jrand, unused)
    TAG_LSHADE_A = 8, // L-SHADE: archive slot of an improved parent when the archive is full
    TAG_LSHADE_S = 9, // L-SHADE: k-th archive removal after a reduction (individual = k)
    TAG_PSO_S = 10,   // spherical PSO: Box-Muller (u24(w0), u24(w1)) -> normals of dims 2b, 2b+1
    TAG_PSO_SR = 11,  // spherical PSO: radius uniform in word 0
    TAG_CSO_PAIR = 12, // CSO: pairing key of particle i in word 0
    TAG_CSO_R = 13,   // CSO: (r1, r2, r3) of loser l, block = coordinate j
    TAG_SHIFT_O = 16, // instance shift: two 53-bit uniforms per block
    TAG_ROT_N = 17,   // instance rotation: one Box-Muller pair per block
};

// Philox4x32 with ten rounds (Salmon, Moraes, Dror and Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11).  Round: multiply words 0 and 2 by the
// two round constants, swap the halves across and mix in the key; the key
// advances by the two Weyl increments between rounds.
struct u32x4 { uint32_t x, y, z, w; };

SEVO_HD u32x4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

SEVO_HD uint32_t fold_seed(uint64_t s) { return (uint32_t)s ^ (uint32_t)(s >> 32); }

SEVO_HD u32x4 draw(uint32_t run_uid, uint32_t seed32, uint32_t t, uint32_t i, uint32_t tag,
                   uint32_t block, uint32_t c3 = 0)
{
    return philox(t, i, (tag << 24) | (block & 0xFFFFFFu), c3, run_uid, seed32);
}

SEVO_HD uint32_t word(const u32x4 &w, int k)
{
    return k == 0 ? w.x : k == 1 ? w.y : k == 2 ? w.z : w.w;
}

// 24-bit uniform in [0, 1): exact in float and double.
SEVO_HD float u24f(uint32_t w) { return (float)(w >> 8) * 5.9604644775390625e-8f; }
SEVO_HD double u24d(uint32_t w) { return (double)(w >> 8) * 5.9604644775390625e-8; }

// 53-bit uniform in [0, 1) from two words (high 27 bits of a, high 26 of b).
SEVO_HD double u53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * 1.1102230246251565404e-16;
}

// Index in [0, n): high word of the 64-bit product w * n (multiply-shift).
SEVO_HD uint32_t range_map(uint32_t w, uint32_t n) { return (uint32_t)(((uint64_t)w * n) >> 32); }

// Integer crossover threshold T: coordinate j takes the donor when
// (w_j >> 8) < T, i.e. when its 24-bit uniform is below CR.
SEVO_HD uint32_t cr_threshold(double cr)
{
    if (!(cr > 0.0)) return 0u;
    if (cr >= 1.0) return 16777216u;
    double s = cr * 16777216.0;
    uint32_t f = (uint32_t)s;           // floor for s >= 0
    return ((double)f == s) ? f : f + 1u;
}

// Schwefel: s is the maximiser of u sin(sqrt u) near 421 (to double
// precision), c = s sin(sqrt s) makes the term vanish at u = s, lambda
// weights the quadratic continuation outside |u| <= 500.
constexpr double SCHWEFEL_S = 420.96874635998202731;
constexpr double SCHWEFEL_LAMBDA = 0.01;

constexpr int TRACE_EVERY = 200;

}  // namespace sevo
