// tile.h -- rotation and objective of one wave's 16*CT points on MFMA,
// shared by the batched evaluation kernels and the fused generation kernels.
//
// MFMA 16x16x4 f32 operand layout (lane l of 64):
//   A (16 x 4):  A[l % 16][l / 16]          one float per lane
//   B (4 x 16):  B[l / 16][l % 16]          one float per lane
//   D (16 x 16): D[4 (l / 16) + j][l % 16]  four floats per lane, j = 0..3
// so after the K loop lane l holds z rows 16 rt + 4 (l/16) + j of point l % 16.
#pragma once

#include "objective_f32.h"
#include "runtime.h"

namespace sevo {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// z rows 16 rt .. 16 rt + 15 of the wave's 16*CT points: the K loop on
// MFMA with A (the rotation fragments) from LDS and B (the shifted points)
// from registers.  With one column tile the even and odd k-steps go to two
// accumulators, so that two independent MFMA chains are in flight.
template <int KS, int CT>
__device__ __forceinline__ void rotate_rows(floatx4 (&z)[CT], const float (&b)[KS][CT], const float *sA,
                                            int rt, int lane)
{
    if constexpr (CT == 1) {
        floatx4 z0 = floatx4{0.f, 0.f, 0.f, 0.f}, z1 = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const float a = sA[(rt * KS + ks) * 64 + lane];
            if (ks & 1) z1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[ks][0], z1, 0, 0, 0);
            else z0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[ks][0], z0, 0, 0, 0);
        }
        z[0] = z0 + z1;
    } else {
#pragma unroll
        for (int c = 0; c < CT; ++c) z[c] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const float a = sA[(rt * KS + ks) * 64 + lane];
#pragma unroll
            for (int c = 0; c < CT; ++c) z[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[ks][c], z[c], 0, 0, 0);
        }
    }
}

// Fold row tile rt (zc) into the per-lane accumulators; zn is row tile
// rt + 1 (zeros after the last), which Rosenbrock's z_{r+1} needs for the
// last row of a lane group: row 4q+3 of lane group q takes row 4q+4 from
// lane l+16, and group 3 takes row 0 of the next tile (lane l-48).
template <int FUNC, int CT>
__device__ __forceinline__ void fold_rows(AccF (&acc)[CT], const floatx4 (&zc)[CT], const floatx4 (&zn)[CT],
                                          const float *sT, int rt, int lane, int dim,
                                          const SchwefelConst<float> &K)
{
    const int kq = lane >> 4;
    const int r0 = rt * 16 + kq * 4;
    const int valid = min(max(dim - r0, 0), 4);
    const float t4[4] = {sT[r0], sT[r0 + 1], sT[r0 + 2], sT[r0 + 3]};
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        const float z4[4] = {zc[c][0], zc[c][1], zc[c][2], zc[c][3]};
        float nx3 = 0.f;
        if constexpr (FUNC == ROSENBROCK) {
            const int src = (lane + 16) & 63;
            const float same = __shfl(zc[c][0], src, 64);
            const float next = __shfl(zn[c][0], src, 64);
            nx3 = kq < 3 ? same : next;
        }
        add_group<FUNC>(acc[c], z4, nx3, valid, r0 + 4 < dim, t4, K);
    }
}

// ---- split bf16 on the 16x16x32 bf16 MFMA ----
//
// Every float f of both operands is written as three bf16 terms,
// f = hi + mid + lo exactly: hi = bf16(f), mid = bf16(f - hi),
// lo = f - hi - mid (each difference exact, and lo fits 8 bits).  The six
// products down to order 2^-16, hi*hi, hi*mid + mid*hi, and
// hi*lo + mid*mid + lo*hi, are accumulated in float; the dropped ones are
// below 2^-24 of the product.  (Two terms and three products leave the
// 2^-17 representation error of each operand, which shows as up to 1.5e-5
// relative error of the Ellipsoid at D = 33: outside the tolerance.)
//
// MFMA 16x16x32 bf16 operand layout (lane l of 64):
//   A (16 x 32): A[l % 16][8 (l / 16) + e], e = 0..7 (eight bf16 per lane)
//   B (32 x 16): B[8 (l / 16) + e][l % 16]
//   D (16 x 16): as for the 16x16x4 f32 instruction.
// The contraction index of one MFMA may be ordered at will as long as A and
// B agree, so k-slot 8 (l / 16) + e of bf16 step s carries coordinate
// 4 (8 s + e) + l / 16: the coordinate that the float path's k-step 8 s + e
// gives lane group l / 16.  The shifted points load exactly as for the
// float path; the KS / 8 whole steps run on bf16 and the KS % 8 remaining
// float k-steps on the 16x16x4 f32 MFMA, so nothing is padded.  The
// rotation fragments are laid out to match on the host.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int KS>
struct Bf16Steps {
    static constexpr int SF = KS / 8;   // whole bf16 k-steps (32 coordinates each)
    static constexpr int RK = KS % 8;   // float k-steps after them
    static constexpr int RT = (KS + 3) / 4;
    // dynamic LDS: 3 terms x RT x SF x 64 vectors of eight bf16, then RT x RK x 64 floats
    static constexpr int NVEC = 3 * RT * SF * 64;
    static constexpr int LDS_BYTES = NVEC * 16 + RT * RK * 64 * 4;
};

template <int KS, int CT>
__device__ __forceinline__ void split3_b(bf16x8 (&bt)[3][Bf16Steps<KS>::SF][CT], const float (&b)[KS][CT])
{
    constexpr int SF = Bf16Steps<KS>::SF;
#pragma unroll
    for (int s = 0; s < SF; ++s)
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            bf16x8 h, m, l;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float f = b[8 * s + e][c];
                const __bf16 hv = (__bf16)f;
                const float r1 = f - (float)hv;
                const __bf16 mv = (__bf16)r1;
                h[e] = hv;
                m[e] = mv;
                l[e] = (__bf16)(r1 - (float)mv);
            }
            bt[0][s][c] = h;
            bt[1][s][c] = m;
            bt[2][s][c] = l;
        }
}

// z rows 16 rt .. 16 rt + 15 by the split: the product orders in three
// independent MFMA chains and the float remainder in a fourth, summed small
// terms first.
template <int KS, int CT>
__device__ __forceinline__ void rotate_rows_bf16(floatx4 (&z)[CT], const bf16x8 (&bt)[3][Bf16Steps<KS>::SF][CT],
                                                 const float (&b)[KS][CT], const bf16x8 *sAb, const float *sAr,
                                                 int rt, int lane)
{
    constexpr int SF = Bf16Steps<KS>::SF, RK = Bf16Steps<KS>::RK, RT = Bf16Steps<KS>::RT;
    floatx4 z0[CT], z1[CT], z2[CT], z3[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        z0[c] = floatx4{0.f, 0.f, 0.f, 0.f};
        z1[c] = z0[c];
        z2[c] = z0[c];
        z3[c] = z0[c];
    }
#pragma unroll
    for (int s = 0; s < SF; ++s) {
        const bf16x8 ah = sAb[((0 * RT + rt) * SF + s) * 64 + lane];
        const bf16x8 am = sAb[((1 * RT + rt) * SF + s) * 64 + lane];
        const bf16x8 al = sAb[((2 * RT + rt) * SF + s) * 64 + lane];
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            z0[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bt[0][s][c], z0[c], 0, 0, 0);
            z1[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bt[1][s][c], z1[c], 0, 0, 0);
            z2[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bt[2][s][c], z2[c], 0, 0, 0);
            z1[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bt[0][s][c], z1[c], 0, 0, 0);
            z2[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bt[1][s][c], z2[c], 0, 0, 0);
            z2[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bt[0][s][c], z2[c], 0, 0, 0);
        }
    }
#pragma unroll
    for (int r = 0; r < RK; ++r) {
        const float a = sAr[(rt * RK + r) * 64 + lane];
#pragma unroll
        for (int c = 0; c < CT; ++c) z3[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[8 * SF + r][c], z3[c], 0, 0, 0);
    }
#pragma unroll
    for (int c = 0; c < CT; ++c) z[c] = (z0[c] + z3[c]) + (z1[c] + z2[c]);
}

// Rotation and objective of one wave's 16*CT points, errors stored to E
// (global memory, or LDS in the fused run kernels); rot(z, rt) makes row
// tile rt of z.  The row tiles are software-pipelined: the MFMA chain of
// tile rt + 1 is issued before the objective of tile rt is folded, so
// matrix-core and vector work of one wave overlap, and z never leaves the
// registers.
template <int FUNC, int RT, int CT, typename Rot, typename EPtr>
__device__ __forceinline__ void tile_fold(Rot &&rot, const float *sT, int lane, int dim, int n, int p0,
                                          const SchwefelConst<float> &K, EPtr E)
{
    AccF acc[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[c].init();
    floatx4 zc[CT], zn[CT];
    rot(zc, 0);
#pragma nounroll
    for (int rt = 0; rt < RT - 1; ++rt) {
        rot(zn, rt + 1);
        fold_rows<FUNC, CT>(acc, zc, zn, sT, rt, lane, dim, K);
#pragma unroll
        for (int c = 0; c < CT; ++c) zc[c] = zn[c];
    }
#pragma unroll
    for (int c = 0; c < CT; ++c) zn[c] = floatx4{0.f, 0.f, 0.f, 0.f};
    fold_rows<FUNC, CT>(acc, zc, zn, sT, RT - 1, lane, dim, K);

    const int kq = lane >> 4, pc = lane & 15;
    const float inv_dim = 1.f / (float)dim;
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        merge_xor_f<FUNC>(acc[c], 16);
        merge_xor_f<FUNC>(acc[c], 32);
        const int p = p0 + c * 16 + pc;
        if (kq == 0 && p < n) E[p] = finalize_f<FUNC>(acc[c], inv_dim);
    }
}

// The float path: rotation fragments and points as floats on the 16x16x4
// f32 MFMA.
template <int FUNC, int KS, int CT, typename EPtr>
__device__ __forceinline__ void tile_body(const float (&b)[KS][CT], const float *sA, const float *sT,
                                          int lane, int dim, int n, int p0,
                                          const SchwefelConst<float> &K, EPtr E)
{
    tile_fold<FUNC, (KS + 3) / 4, CT>([&](floatx4(&z)[CT], int rt) { rotate_rows<KS, CT>(z, b, sA, rt, lane); },
                                      sT, lane, dim, n, p0, K, E);
}

// The split-bf16 path.
template <int FUNC, int KS, int CT, typename EPtr>
__device__ __forceinline__ void tile_body_bf16(const bf16x8 (&bt)[3][Bf16Steps<KS>::SF][CT],
                                               const float (&b)[KS][CT], const bf16x8 *sAb, const float *sAr,
                                               const float *sT, int lane, int dim, int n, int p0,
                                               const SchwefelConst<float> &K, EPtr E)
{
    tile_fold<FUNC, (KS + 3) / 4, CT>(
        [&](floatx4(&z)[CT], int rt) { rotate_rows_bf16<KS, CT>(z, bt, b, sAb, sAr, rt, lane); }, sT, lane, dim,
        n, p0, K, E);
}

// Coordinates of one wave's 16*CT points (p0 is the same for the whole
// wave), in two halves so a caller can keep the loads of the next tile in
// flight while it computes the current one.  load_raw only issues the
// loads: unconditional, from clamped and therefore always valid addresses
// (a load under a per-lane branch would be waited for before the next one
// is issued), each a wave-uniform row base plus a 32-bit per-lane byte
// offset (rows 4 ks .. 4 ks + 3 of lane group kq; points past n re-read
// point n - 1; rows past dim, which only the last k-step has, re-read row
// dim - 1).  Offsets stay below 2^32 for ld < 2^28, which the entry points
// check.  shift_raw then applies the shift in double, rounding d = x - o
// once to float, and zeroes rows past dim.
template <int KS, int CT>
__device__ __forceinline__ void load_raw(float (&raw)[KS][CT], const SEVO_GLOBAL float *__restrict__ X,
                                         int64_t ld, int dim, int n, int p0, int kq, int pc)
{
    const int pb = __builtin_amdgcn_readfirstlane(min(p0, n - 1));
    const SEVO_GLOBAL char *base = reinterpret_cast<const SEVO_GLOBAL char *>(X + pb);
    const int last = min(kq, dim - 1 - 4 * (KS - 1));
    uint32_t off[CT], offl[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        const uint32_t pl = (uint32_t)(min(p0 + c * 16 + pc, n - 1) - pb);
        off[c] = ((uint32_t)kq * (uint32_t)ld + pl) * 4u;
        offl[c] = ((uint32_t)last * (uint32_t)ld + pl) * 4u;
    }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const SEVO_GLOBAL char *row = base + (int64_t)(4 * ks) * ld * 4;
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const uint32_t o = ks == KS - 1 ? offl[c] : off[c];
            raw[ks][c] = *reinterpret_cast<const SEVO_GLOBAL float *>(row + o);
        }
    }
}

// The same loads from a population held in LDS (fused runs whose state
// fits on chip): clamped row and point indices, no address tricks needed.
template <int KS, int CT>
__device__ __forceinline__ void load_raw_lds(float (&raw)[KS][CT], const float *X, int ld, int dim, int n,
                                             int p0, int kq, int pc)
{
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int k = min(ks * 4 + kq, dim - 1);
#pragma unroll
        for (int c = 0; c < CT; ++c) raw[ks][c] = X[k * ld + min(p0 + c * 16 + pc, n - 1)];
    }
}

template <int KS, int CT>
__device__ __forceinline__ void shift_raw(float (&b)[KS][CT], int dim, int n, int p0, int kq, int pc,
                                          const double *sO)
{
    (void)n; (void)p0; (void)pc;   // lanes past n compute on a copy of point n - 1 and store nothing
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int k = ks * 4 + kq;
        const double ok = sO[k];
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const float d = (float)((double)b[ks][c] - ok);
            b[ks][c] = (ks < KS - 1 || k < dim) ? d : 0.f;
        }
    }
}

// Copy the rotation fragments (RT*KS*64 floats, a whole number of float4s,
// 16-byte aligned) from global memory to LDS: every thread first issues all
// of its float4 loads (unconditional, clamped index), then stores them.
template <int KS>
__device__ __forceinline__ void stage_rotation(float *sA, const float *Mfrag)
{
    constexpr int RT = (KS + 3) / 4;
    constexpr int NV = RT * KS * 16;
    constexpr int PER = (NV + 255) / 256;
    const SEVO_GLOBAL floatx4 *M4 = reinterpret_cast<const SEVO_GLOBAL floatx4 *>(gin<float>(Mfrag));
    floatx4 *s4 = reinterpret_cast<floatx4 *>(sA);
    floatx4 tmp[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) tmp[k] = M4[min((int)threadIdx.x + k * 256, NV - 1)];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int q = threadIdx.x + k * 256;
        if (q < NV) s4[q] = tmp[k];
    }
}

// The split-bf16 rotation fragments from global memory to LDS, as
// stage_rotation: the bf16 terms (Bf16Steps::NVEC vectors) from Mbf, then
// the float fragments of the remaining k-steps from Mfrag ([RT][KS][64]).
template <int KS>
__device__ __forceinline__ void stage_rotation_bf16(bf16x8 *sAb, float *sAr, const uint16_t *Mbf, const float *Mfrag)
{
    constexpr int NV = Bf16Steps<KS>::NVEC, RT = Bf16Steps<KS>::RT;
    constexpr int SF = Bf16Steps<KS>::SF, RK = Bf16Steps<KS>::RK;
    constexpr int PER = (NV + 255) / 256;
    const SEVO_GLOBAL floatx4 *M4 = reinterpret_cast<const SEVO_GLOBAL floatx4 *>(gin<uint16_t>(Mbf));
    floatx4 *s4 = reinterpret_cast<floatx4 *>(sAb);
    floatx4 tmp[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) tmp[k] = M4[min((int)threadIdx.x + k * 256, NV - 1)];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int q = threadIdx.x + k * 256;
        if (q < NV) s4[q] = tmp[k];
    }
    if constexpr (RK > 0) {
        const SEVO_GLOBAL float *Mf = gin<float>(Mfrag);
        for (int q = threadIdx.x; q < RT * RK * 64; q += 256) {
            const int rt = q / (RK * 64), r = (q / 64) % RK, l = q % 64;
            sAr[q] = Mf[(rt * KS + 8 * SF + r) * 64 + l];
        }
    }
}

}  // namespace sevo
