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

// Rotation and objective of one wave's 16*CT points: for every 16-row tile
// of z the K loop runs on MFMA (A from LDS, B = the shifted points held in
// registers), then the tile's rows are folded into per-lane compensated
// accumulators straight from the accumulator registers.  Rosenbrock needs
// z_{r+1}: row 4q+3 of lane group q takes row 4q+4 from lane l+16, and the
// last row of a tile takes row 0 of the next tile (lane l-48), so its terms
// are added one tile late.
template <int FUNC, int KS, int CT>
__device__ __forceinline__ void tile_body(const float (&b)[KS][CT], const float *sA, const float *sT,
                                          int lane, int dim, int n, int p0,
                                          const SchwefelConst<float> &K, SEVO_GLOBAL float *__restrict__ E)
{
    constexpr int RT = (KS + 3) / 4;
    const int kq = lane >> 4;
    const int src = (lane + 16) & 63;
    AccF acc[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[c].init();
    floatx4 zp[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) zp[c] = floatx4{0.f, 0.f, 0.f, 0.f};

#pragma nounroll
    for (int rt = 0; rt < RT; ++rt) {
        floatx4 zc[CT];
#pragma unroll
        for (int c = 0; c < CT; ++c) zc[c] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const float a = sA[(rt * KS + ks) * 64 + lane];
#pragma unroll
            for (int c = 0; c < CT; ++c)
                zc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[ks][c], zc[c], 0, 0, 0);
        }
        if constexpr (FUNC == ROSENBROCK) {
            if (rt > 0) {
                const int r0 = (rt - 1) * 16 + kq * 4;
                const int valid = min(max(dim - r0, 0), 4);
#pragma unroll
                for (int c = 0; c < CT; ++c) {
                    const float nx_same = __shfl(zp[c][0], src, 64);
                    const float nx_next = __shfl(zc[c][0], src, 64);
                    const float z4[4] = {zp[c][0], zp[c][1], zp[c][2], zp[c][3]};
                    add_group<FUNC>(acc[c], z4, kq < 3 ? nx_same : nx_next, valid, r0 + 4 < dim, sT + r0, K);
                }
            }
#pragma unroll
            for (int c = 0; c < CT; ++c) zp[c] = zc[c];
        } else {
            const int r0 = rt * 16 + kq * 4;
            const int valid = min(max(dim - r0, 0), 4);
            const float t4[4] = {sT[r0], sT[r0 + 1], sT[r0 + 2], sT[r0 + 3]};
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                const float z4[4] = {zc[c][0], zc[c][1], zc[c][2], zc[c][3]};
                add_group<FUNC>(acc[c], z4, 0.f, valid, false, t4, K);
            }
        }
    }
    if constexpr (FUNC == ROSENBROCK) {
        const int r0 = (RT - 1) * 16 + kq * 4;
        const int valid = min(max(dim - r0, 0), 4);
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const float nb3 = __shfl(zp[c][0], src, 64);
            const float z4[4] = {zp[c][0], zp[c][1], zp[c][2], zp[c][3]};
            add_group<FUNC>(acc[c], z4, kq < 3 ? nb3 : 0.f, valid, kq < 3 && r0 + 4 < dim, sT + r0, K);
        }
    }
    const int pc = lane & 15;
    const float inv_dim = 1.f / (float)dim;
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        merge_xor_f<FUNC>(acc[c], 16);
        merge_xor_f<FUNC>(acc[c], 32);
        const int p = p0 + c * 16 + pc;
        if (kq == 0 && p < n) E[p] = finalize_f<FUNC>(acc[c], inv_dim);
    }
}

// Coordinates of one wave's 16*CT points, in two halves so a caller can
// keep the loads of the next tile in flight while it computes the current
// one: load_raw only issues the loads (unconditional, from a clamped and
// therefore always valid address -- a load under a per-lane branch would be
// waited for before the next one is issued); shift_raw then masks the
// padding and applies the shift in double, rounding d = x - o once to float.
template <int KS, int CT>
__device__ __forceinline__ void load_raw(float (&raw)[KS][CT], const SEVO_GLOBAL float *__restrict__ X,
                                         int64_t ld, int dim, int n, int p0, int kq, int pc)
{
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int k = min(ks * 4 + kq, dim - 1);
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int p = min(p0 + c * 16 + pc, n - 1);
            raw[ks][c] = X[(int64_t)k * ld + p];
        }
    }
}

template <int KS, int CT>
__device__ __forceinline__ void shift_raw(float (&b)[KS][CT], int dim, int n, int p0, int kq, int pc,
                                          const double *sO)
{
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int k = ks * 4 + kq;
        const double ok = sO[k];
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int p = p0 + c * 16 + pc;
            b[ks][c] = (k < dim && p < n) ? (float)((double)b[ks][c] - ok) : 0.f;
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
