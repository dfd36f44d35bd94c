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

// Rotation and objective of one wave's 16*CT points, errors stored to E
// (global memory, or LDS in the fused run kernels).  The row tiles are
// software-pipelined: the MFMA chain of tile rt + 1 is issued before the
// objective of tile rt is folded, so matrix-core and vector work of one wave
// overlap, and z never leaves the registers.
template <int FUNC, int KS, int CT, typename EPtr>
__device__ __forceinline__ void tile_body(const float (&b)[KS][CT], const float *sA, const float *sT,
                                          int lane, int dim, int n, int p0,
                                          const SchwefelConst<float> &K, EPtr E)
{
    constexpr int RT = (KS + 3) / 4;
    AccF acc[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[c].init();
    floatx4 zc[CT], zn[CT];
    rotate_rows<KS, CT>(zc, b, sA, 0, lane);
#pragma nounroll
    for (int rt = 0; rt < RT - 1; ++rt) {
        rotate_rows<KS, CT>(zn, b, sA, rt + 1, lane);
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

template <int KS, int CT>
__device__ __forceinline__ void load_b(float (&b)[KS][CT], const SEVO_GLOBAL float *__restrict__ X,
                                       int64_t ld, int dim, int n, int p0, int kq, int pc,
                                       const double *sO)
{
    load_raw<KS, CT>(b, X, ld, dim, n, p0, kq, pc);
    shift_raw<KS, CT>(b, dim, n, p0, kq, pc, sO);
}

}  // namespace sevo
