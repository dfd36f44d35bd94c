// eval_large.hip -- evaluation of high-dimensional points (D > 120, up to
// 1024) as a tiled GEMM Z = M * (X - o 1^T) fused with the objective.
//
// A pre-pass (k_eval_operands) makes the shifted points once, in the
// precision's operand format (shift in double, one rounding to float).  A
// workgroup (4 waves) owns a 128-row x PT-point tile of Z (PT = 128 or
// 64).  The K loop stages 32 coordinates of its points in LDS, shared by the
// 4 waves, with the next chunk's loads issued before this chunk's MFMAs; each
// wave streams its own 32 rows of M (two 16-row MFMA tiles) from L2 and
// accumulates 2 x PT / 16 MFMA tiles.  Precision variants:
//   FP32        v_mfma_f32_16x16x4_f32 on float operands;
//   split bf16  every float is split into three bf16 terms, hi = bf16(f),
//               mid = bf16(f - hi), lo = bf16(f - hi - mid), whose sum is f
//               exactly; z += the six products of order 1 to 2^-16 (hi hi,
//               hi mid, mid hi, hi lo, lo hi, mid mid) on
//               v_mfma_f32_16x16x32_bf16, accumulated in float: the terms
//               left out are below float rounding, so the result is as
//               accurate as the FP32 path (two terms would leave each
//               operand a 2^-17 representation error, which the objective
//               can turn into more than 1e-5 e at a few hundred dimensions).
// After the K loop each wave folds its rows into compensated per-point
// partial sums; the workgroup writes one partial record per (row block,
// point), and a second pass merges the row blocks in a fixed order and adds
// Rosenbrock's terms that straddle two row blocks.
//
// MFMA 16x16x32 bf16 operand layout (lane l of 64):
//   A (16 x 32): A[l % 16][8 (l / 16) + e], e = 0..7 (eight bf16 per lane)
//   B (32 x 16): B[8 (l / 16) + e][l % 16]
//   D (16 x 16): as for the 16x16x4 f32 instruction.
#include "objective_f32.h"
#include "runtime.h"

namespace sevo {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t vu32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int xcd_remap_l(int b, int G)
{
    const int q = G >> 3, r = G & 7;
    const int x = b & 7, k = b >> 3;
    return x * q + (x < r ? x : r) + k;
}

__device__ __forceinline__ uint16_t to_bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

constexpr int KC = 32;                 // coordinates per K chunk

template <int FUNC, int CT>
__device__ __forceinline__ void fold_rows(const floatx4 (&z)[2][CT], int rt0, int w, int lane,
                                          int dim, const SEVO_GLOBAL float *__restrict__ tab,
                                          const float (*sZ0)[CT * 16], const SchwefelConst<float> &K,
                                          float (*sAcc)[CT * 16][4])
{
    const int kq = lane >> 4, pc = lane & 15;
    const int src = (lane + 16) & 63;
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        AccF a;
        a.init();
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
            const int r0 = (rt0 + rt) * 16 + kq * 4;
            const int valid = min(max(dim - r0, 0), 4);
            float nb3 = 0.f;
            if constexpr (FUNC == ROSENBROCK) {
                const float same = __shfl(z[rt][c][0], src, 64);
                if (rt == 0) {
                    const float nxt = __shfl(z[1][c][0], src, 64);
                    nb3 = kq < 3 ? same : nxt;
                } else {
                    nb3 = kq < 3 ? same : (w < 3 ? sZ0[w + 1][c * 16 + pc] : 0.f);
                }
            }
            // the last row of the workgroup pairs with the next row block:
            // that term is added by the combine pass
            const bool boundary = (rt == 1 && kq == 3 && w == 3);
            const float t4[4] = {valid > 0 ? tab[r0] : 0.f, valid > 1 ? tab[r0 + 1] : 0.f,
                                 valid > 2 ? tab[r0 + 2] : 0.f, valid > 3 ? tab[r0 + 3] : 0.f};
            const float z4[4] = {z[rt][c][0], z[rt][c][1], z[rt][c][2], z[rt][c][3]};
            add_group<FUNC>(a, z4, nb3, valid, (r0 + 4 < dim) && !boundary, t4, K);
        }
        merge_xor_f<FUNC>(a, 16);
        merge_xor_f<FUNC>(a, 32);
        if (kq == 0) {
            float *q = sAcc[w][c * 16 + pc];
            q[0] = a.s1;
            q[1] = a.c1;
            q[2] = a.s2;
            q[3] = a.c2;
        }
    }
}

template <int FUNC, int PT>
__device__ __forceinline__ void merge_waves(float rec[4], const float (*sAcc)[PT][4], int p)
{
    AccF a{rec[0], rec[1], rec[2], rec[3]};
    for (int q = 1; q < 4; ++q) merge_f<FUNC>(a, sAcc[q][p][0], sAcc[q][p][1], sAcc[q][p][2], sAcc[q][p][3]);
    rec[0] = a.s1;
    rec[1] = a.c1;
    rec[2] = a.s2;
    rec[3] = a.c2;
}

// GEMM operands, made once per point (the row-block workgroups of a point
// tile would otherwise each redo the shift and the split): d = x - o in
// double, rounded once to float, zero beyond n and dim.  Workgroup = 64
// points x 32 coordinates of one item; wave q takes coordinates 8q .. 8q + 7
// of every point (lanes = points, so the loads of one coordinate are
// contiguous).  Both layouts are tiled by (128-point tile, 32-coordinate
// chunk) in the order in which k_eval_large stages one chunk, so that its
// staging is a contiguous copy:
//   FP32        [tile][chunk][32 k][128 points] floats; lanes store one
//               coordinate row of 64 points, 256 contiguous bytes;
//   split bf16  hi, mid and lo arrays one after another, each
//               [tile][chunk][128 points][32 k]; the 8 coordinates of a lane
//               are packed into one 16-byte vector per array and go through
//               LDS so that the stores of a wave are 1 KB contiguous.
template <bool BF16>
__global__ __launch_bounds__(256) void k_eval_operands(const EvalDesc *__restrict__ items, int n_items,
                                                       int total_blocks)
{
    __shared__ vu32x4 sT[BF16 ? 3 : 1][BF16 ? 256 : 1];
    const int L = xcd_remap_l(blockIdx.x, total_blocks);
    const EvalDesc &it = items[reinterpret_cast<const int32_t *>(items + n_items)[L]];
    const int dim = it.dim, n = it.n;
    const int64_t ld = it.ld, np = large_npad(n), kp = large_kpad(dim);
    const int local = L - it.block0, pblocks = (int)(np / OPERAND_POINTS);
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int pb = local % pblocks, kc = local / pblocks;
    const int p = pb * OPERAND_POINTS + lane;
    const int k0 = kc * OPERAND_K + q * 8;
    const SEVO_GLOBAL float *__restrict__ X = gin<float>(it.x);
    const SEVO_GLOBAL double *og = gin<double>(it.o);
    const int64_t k32 = kp / OPERAND_K;
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int k = k0 + e;
        const float raw = X[(int64_t)min(k, dim - 1) * ld + min(p, n - 1)];
        v[e] = (k < dim && p < n) ? (float)((double)raw - og[min(k, dim - 1)]) : 0.f;
    }
    if constexpr (!BF16) {
        // chunk (tile pb / 2, kc) holds 4096 floats; this workgroup's points
        // are columns 64 (pb & 1) .. + 63 of its 32 rows
        SEVO_GLOBAL float *D = gout<float>(it.opnd) + ((int64_t)(pb >> 1) * k32 + kc) * 4096 + (pb & 1) * 64 + lane;
#pragma unroll
        for (int e = 0; e < 8; ++e) D[(q * 8 + e) * 128] = v[e];
    } else {
        // term t of each float (the remainder after the terms before it is
        // exact in float, so hi + mid + lo = v)
        uint16_t b[3][8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            float r = v[e];
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                b[t][e] = to_bf16_rne(r);
                r -= from_bf16(b[t][e]);
            }
        }
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            vu32x4 vt;
            vt.x = b[t][0] | ((uint32_t)b[t][1] << 16); vt.y = b[t][2] | ((uint32_t)b[t][3] << 16);
            vt.z = b[t][4] | ((uint32_t)b[t][5] << 16); vt.w = b[t][6] | ((uint32_t)b[t][7] << 16);
            sT[t][lane * 4 + q] = vt;
        }
        __syncthreads();
        // chunk (tile pb / 2, kc) holds 512 vectors; this workgroup's 64
        // points are its half (pb & 1)
        const int64_t base = ((int64_t)(pb >> 1) * k32 + kc) * 512 + (pb & 1) * 256;
#pragma unroll
        for (int t = 0; t < 3; ++t) gout<vu32x4>(it.opnd)[t * (np * kp / 8) + base + threadIdx.x] = sT[t][threadIdx.x];
    }
}

// PT points per workgroup: 128 (one operand tile) or 64 (half of one; twice
// the workgroups, half the accumulators, so more workgroups fit a CU and the
// last round of a grid that does not divide evenly is shorter)
template <bool BF16, int PT>
__global__ __launch_bounds__(256) void k_eval_large(const EvalDesc *__restrict__ items, int n_items,
                                                    int total_blocks, Consts K)
{
    constexpr int CT = PT / 16;        // column tiles per wave
    constexpr int SB = PT + 16;        // float staging row stride (bank offset 16)
    static_assert(PT == 64 || PT == 128, "a workgroup covers one operand tile or half of one");
    __shared__ __attribute__((aligned(16))) float sB[BF16 ? 4 : KC * SB];
    __shared__ __attribute__((aligned(16))) uint16_t sBt[BF16 ? 3 : 1][BF16 ? PT * KC : 8];
    __shared__ float sZ0[4][PT];
    __shared__ float sZL[PT];
    __shared__ float sAcc[4][PT][4];

    const int L = xcd_remap_l(blockIdx.x, total_blocks);
    const EvalDesc &it = items[reinterpret_cast<const int32_t *>(items + n_items)[L]];
    const int dim = it.dim, n = it.n, RB = it.rb;
    const int local = L - it.block0;
    const int rb = local % RB, pb = local / RB;
    const int p_base = pb * PT;
    // operand tile of these points and their first column in it
    const int64_t otile = p_base / LARGE_POINTS;
    const int ocol = p_base % LARGE_POINTS;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int kq = lane >> 4, pc = lane & 15;
    const int RT = (dim + 15) / 16, KS = (dim + 3) / 4, K32 = (dim + 31) / 32;
    const int rt0 = rb * 8 + w * 2;
    const SEVO_GLOBAL float *Mf = gin<float>(it.Mfrag);
    const SEVO_GLOBAL float *tab = gin<float>(it.tab);

    floatx4 z[2][CT];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int c = 0; c < CT; ++c) z[rt][c] = floatx4{0.f, 0.f, 0.f, 0.f};

    if constexpr (BF16) {
        // split operands from k_eval_operands: 128 points x 32 coordinates per
        // chunk and term array = 512 vectors of 8 bf16 (4 per point), of
        // which this workgroup's PT points take 4 PT contiguous ones, PT / 64
        // per thread and term; the next chunk's vectors and M fragments are
        // loaded before this chunk's MFMAs
        const int64_t kp = large_kpad(dim), np = large_npad(n);
        // global (not flat) loads: a flat load also counts against the LDS
        // counter, so the waits for this chunk's LDS reads would wait for the
        // next chunk's loads as well
        const SEVO_GLOBAL vu32x4 *Bt = gin<vu32x4>(it.opnd);
        const int64_t tstride = np * kp / 8;   // vectors per term array
        // tiled layout: chunk kk of the operand tile is 512 contiguous vectors,
        // point-major (vector 4 p + q = coordinates 8 q .. 8 q + 7 of point p).
        // In LDS the vectors are in the order the MFMA lanes read them:
        // slot 64 c + 16 q + i holds vector q of point 16 c + i, so a wave's
        // reads of one column tile, and its stores, are 1 KB contiguous (no
        // bank conflicts); its global loads still cover 1 KB contiguous.
        // Slot v + 256 holds the vector 256 past slot v's.
        constexpr int NV = PT / 64;
        const int t0 = threadIdx.x;
        const int64_t g0 = otile * K32 * 512 + ocol * 4 + ((t0 >> 6) * 16 + (t0 & 15)) * 4 + ((t0 >> 4) & 3);
        int sv[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) sv[j] = (t0 + 256 * j) * 8;
        const SEVO_GLOBAL uint16_t *Mh = gin<uint16_t>(it.Mbf);
        const int64_t mblock = (int64_t)RT * K32 * 512;   // bf16 per term block of M
        // a[r][t]: term t of row tile r's fragment of chunk kk, as raw words.
        // Row tiles past the matrix (in the last row block) load the last
        // real row tile again: their rows lie past dim, so the fold discards
        // them, and the MFMAs run unconditionally with nothing computed on
        // the fragments between their loads and their use (a select there
        // made the compiler wait for the next chunk's loads before this
        // chunk's MFMAs).
        const int rc0 = min(rt0, RT - 1), rc1 = min(rt0 + 1, RT - 1);
        auto load_a = [&](int kk, vu32x4 (&a)[2][3]) {
            const int64_t i0 = (((int64_t)rc0 * K32 + kk) * 64 + lane) * 8;
            const int64_t i1 = (((int64_t)rc1 * K32 + kk) * 64 + lane) * 8;
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                a[0][t] = *(const SEVO_GLOBAL vu32x4 *)(Mh + t * mblock + i0);
                a[1][t] = *(const SEVO_GLOBAL vu32x4 *)(Mh + t * mblock + i1);
            }
        };
        vu32x4 a[2][3];
        load_a(0, a);
        vu32x4 b[NV][3];
#pragma unroll
        for (int j = 0; j < NV; ++j)
#pragma unroll
            for (int t = 0; t < 3; ++t) b[j][t] = Bt[t * tstride + g0 + 256 * j];
#pragma unroll
        for (int j = 0; j < NV; ++j)
#pragma unroll
            for (int t = 0; t < 3; ++t) *reinterpret_cast<vu32x4 *>(sBt[t] + sv[j]) = b[j][t];
        __syncthreads();
        // every global load of the prologue is complete here; without this
        // wait the compiler's bookkeeping of the fragments loaded before the
        // loop makes each iteration wait for all loads in flight, the next
        // chunk's prefetch included (vmcnt 0; expcnt and lgkmcnt unconstrained)
        __builtin_amdgcn_s_waitcnt(0x0F70);
        for (int kk = 0; kk < K32; ++kk) {
            const bool more = kk + 1 < K32;
            vu32x4 na[2][3];
            if (more) {
                const int64_t d = (int64_t)(kk + 1) * 512;
#pragma unroll
                for (int j = 0; j < NV; ++j)
#pragma unroll
                    for (int t = 0; t < 3; ++t) b[j][t] = Bt[t * tstride + g0 + d + 256 * j];
                load_a(kk + 1, na);
            }
            // the three terms of column tile c + 1 are read from LDS while the
            // MFMAs of tile c run (double-buffered; the order is pinned below,
            // since the scheduler otherwise reads each tile into the same
            // registers just before its MFMAs and waits for every read)
            bf16x8 bb[2][3];
            auto read_b = [&](int c, bf16x8 (&d)[3]) {
                const int off = (c * 64 + lane) * 8;
#pragma unroll
                for (int t = 0; t < 3; ++t) d[t] = *reinterpret_cast<const bf16x8 *>(sBt[t] + off);
            };
            read_b(0, bb[0]);
            __builtin_amdgcn_sched_group_barrier(0x100, 3, 0);
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                if (c + 1 < CT) read_b(c + 1, bb[(c + 1) & 1]);
                const bf16x8 bh = bb[c & 1][0], bm = bb[c & 1][1], bl = bb[c & 1][2];
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const bf16x8 ah = __builtin_bit_cast(bf16x8, a[r][0]);
                    const bf16x8 am = __builtin_bit_cast(bf16x8, a[r][1]);
                    const bf16x8 al = __builtin_bit_cast(bf16x8, a[r][2]);
                    // smallest products first, so the float accumulation
                    // loses the least of them
                    z[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm, z[r][c], 0, 0, 0);
                    z[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, z[r][c], 0, 0, 0);
                    z[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, z[r][c], 0, 0, 0);
                    z[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh, z[r][c], 0, 0, 0);
                    z[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm, z[r][c], 0, 0, 0);
                    z[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, z[r][c], 0, 0, 0);
                }
                if (c + 1 < CT) __builtin_amdgcn_sched_group_barrier(0x100, 3, 0);   // LDS reads
                __builtin_amdgcn_sched_group_barrier(0x008, 12, 0);                 // MFMAs
            }
            __syncthreads();
            if (more) {
#pragma unroll
                for (int j = 0; j < NV; ++j)
#pragma unroll
                    for (int t = 0; t < 3; ++t) *reinterpret_cast<vu32x4 *>(sBt[t] + sv[j]) = b[j][t];
#pragma unroll
                for (int t = 0; t < 3; ++t) {
                    a[0][t] = na[0][t];
                    a[1][t] = na[1][t];
                }
            }
            __syncthreads();
        }
    } else {
        // float operands from k_eval_operands: 32 coordinates x 128 points
        // per chunk = 1024 vectors of 4 floats (32 per coordinate row), of
        // which this workgroup's PT points take PT / 4 of every row, PT / 32
        // per thread; the next chunk's vectors and M fragments are loaded
        // before this chunk's MFMAs (same structure as the split path)
        const SEVO_GLOBAL vu32x4 *Bf = gin<vu32x4>(it.opnd);
        constexpr int VPR = PT / 4, NV = PT / 32;
        // vector v of the workgroup = row v / VPR, 4 points at column v % VPR;
        // LDS row stride SB
        const int64_t g0 = otile * K32 * 1024 + (threadIdx.x / VPR) * 32 + ocol / 4 + threadIdx.x % VPR;
        int sv[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const int v = threadIdx.x + 256 * j;
            sv[j] = (v / VPR) * SB + (v % VPR) * 4;
        }
        constexpr int GSTEP = (256 / VPR) * 32;   // global vectors between a thread's rows
        const int64_t m0 = (int64_t)min(rt0, RT - 1) * KS * 64 + lane;
        const int64_t m1 = (int64_t)min(rt0 + 1, RT - 1) * KS * 64 + lane;
        // k-steps past the matrix read the last one (their operand rows are
        // zero, and the last chunk skips them); row tiles past the matrix
        // read the last real one, as in the split path (the fold discards
        // their rows)
        auto load_a = [&](int kk, float (&a0)[KC / 4], float (&a1)[KC / 4]) {
#pragma unroll
            for (int ks = 0; ks < KC / 4; ++ks) {
                const int64_t k = min(kk * (KC / 4) + ks, KS - 1);
                a0[ks] = Mf[m0 + k * 64];
                a1[ks] = Mf[m1 + k * 64];
            }
        };
        float a0[KC / 4], a1[KC / 4];
        load_a(0, a0, a1);
        vu32x4 b[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) b[j] = Bf[g0 + GSTEP * j];
#pragma unroll
        for (int j = 0; j < NV; ++j) *reinterpret_cast<vu32x4 *>(sB + sv[j]) = b[j];
        __syncthreads();
        // every global load of the prologue is complete here; without this
        // wait the compiler's bookkeeping of the fragments loaded before the
        // loop makes each iteration wait for all loads in flight, the next
        // chunk's prefetch included (vmcnt 0; expcnt and lgkmcnt unconstrained)
        __builtin_amdgcn_s_waitcnt(0x0F70);
        // every chunk but the last: all eight k-steps, the next chunk loaded
        // meanwhile
        for (int kk = 0; kk + 1 < K32; ++kk) {
            float n0[KC / 4], n1[KC / 4];
            const int64_t d = (int64_t)(kk + 1) * 1024;
#pragma unroll
            for (int j = 0; j < NV; ++j) b[j] = Bf[g0 + d + GSTEP * j];
            load_a(kk + 1, n0, n1);
            // the points of k-step ks + 1 are read from LDS while the MFMAs
            // of k-step ks run (double-buffered; the order is pinned, as in
            // the split path: CT / 2 paired reads, then 2 CT MFMAs)
            float bv[2][CT];
#pragma unroll
            for (int c = 0; c < CT; ++c) bv[0][c] = sB[kq * SB + c * 16 + pc];
            __builtin_amdgcn_sched_group_barrier(0x100, CT / 2, 0);
#pragma unroll
            for (int ks = 0; ks < KC / 4; ++ks) {
                if (ks + 1 < KC / 4) {
#pragma unroll
                    for (int c = 0; c < CT; ++c) bv[(ks + 1) & 1][c] = sB[((ks + 1) * 4 + kq) * SB + c * 16 + pc];
                }
#pragma unroll
                for (int c = 0; c < CT; ++c) {
                    z[0][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[ks], bv[ks & 1][c], z[0][c], 0, 0, 0);
                    z[1][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[ks], bv[ks & 1][c], z[1][c], 0, 0, 0);
                }
                if (ks + 1 < KC / 4) __builtin_amdgcn_sched_group_barrier(0x100, CT / 2, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 2 * CT, 0);
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < NV; ++j) *reinterpret_cast<vu32x4 *>(sB + sv[j]) = b[j];
#pragma unroll
            for (int ks = 0; ks < KC / 4; ++ks) {
                a0[ks] = n0[ks];
                a1[ks] = n1[ks];
            }
            __syncthreads();
        }
        // the last chunk (in LDS now): only its k-steps inside the matrix;
        // the operand rows past dim are zero, so the others add nothing
        const int nks = KS - (K32 - 1) * (KC / 4);
#pragma unroll
        for (int ks = 0; ks < KC / 4; ++ks) {
            if (ks < nks) {
#pragma unroll
                for (int c = 0; c < CT; ++c) {
                    const float bvc = sB[(ks * 4 + kq) * SB + c * 16 + pc];
                    z[0][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[ks], bvc, z[0][c], 0, 0, 0);
                    z[1][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[ks], bvc, z[1][c], 0, 0, 0);
                }
            }
        }
    }

    // first row of each wave (Rosenbrock neighbours across waves), last row
    // of the workgroup (neighbour in the next row block)
    if (kq == 0)
#pragma unroll
        for (int c = 0; c < CT; ++c) sZ0[w][c * 16 + pc] = z[0][c][0];
    if (w == 3 && kq == 3)
#pragma unroll
        for (int c = 0; c < CT; ++c) sZL[c * 16 + pc] = z[1][c][3];
    __syncthreads();
    switch (it.func) {
    case ELLIPSOID: fold_rows<ELLIPSOID, CT>(z, rt0, w, lane, dim, tab, sZ0, K.kf, sAcc); break;
    case ROSENBROCK: fold_rows<ROSENBROCK, CT>(z, rt0, w, lane, dim, tab, sZ0, K.kf, sAcc); break;
    case RASTRIGIN: fold_rows<RASTRIGIN, CT>(z, rt0, w, lane, dim, tab, sZ0, K.kf, sAcc); break;
    case SCHWEFEL: fold_rows<SCHWEFEL, CT>(z, rt0, w, lane, dim, tab, sZ0, K.kf, sAcc); break;
    case GRIEWANK: fold_rows<GRIEWANK, CT>(z, rt0, w, lane, dim, tab, sZ0, K.kf, sAcc); break;
    default: fold_rows<ACKLEY, CT>(z, rt0, w, lane, dim, tab, sZ0, K.kf, sAcc); break;
    }
    __syncthreads();
    if (threadIdx.x < PT) {
        const int p = threadIdx.x, pg = p_base + p;
        if (pg < n) {
            float rec[4] = {sAcc[0][p][0], sAcc[0][p][1], sAcc[0][p][2], sAcc[0][p][3]};
            switch (it.func) {
            case ACKLEY: merge_waves<ACKLEY, PT>(rec, sAcc, p); break;
            case GRIEWANK: merge_waves<GRIEWANK, PT>(rec, sAcc, p); break;
            default: merge_waves<ELLIPSOID, PT>(rec, sAcc, p); break;
            }
            SEVO_GLOBAL float *out = gout<float>(it.part) + ((int64_t)rb * n + pg) * 8;
            out[0] = rec[0];
            out[1] = rec[1];
            out[2] = rec[2];
            out[3] = rec[3];
            out[4] = 0.f;
            out[5] = sZ0[0][p];
            out[6] = sZL[p];
            out[7] = 0.f;
        }
    }
}

template <int FUNC>
__device__ __forceinline__ float combine_point(const SEVO_GLOBAL float *__restrict__ P, int n, int pg, int RB,
                                               int dim, const SchwefelConst<float> &K)
{
    AccF a;
    a.init();
    for (int rb = 0; rb < RB; ++rb) {
        const SEVO_GLOBAL float *q = P + ((int64_t)rb * n + pg) * 8;
        merge_f<FUNC>(a, q[0], q[1], q[2], q[3]);
        if constexpr (FUNC == ROSENBROCK) {
            if (rb + 1 < RB) {
                const float z4[4] = {q[6], P[((int64_t)(rb + 1) * n + pg) * 8 + 5], 0.f, 0.f};
                const float t4[4] = {0.f, 0.f, 0.f, 0.f};
                // one term: (last row of block rb, first row of block rb + 1)
                add_group<ROSENBROCK>(a, z4, 0.f, 2, false, t4, K);
            }
        }
    }
    return finalize_f<FUNC>(a, 1.f / (float)dim);
}

__global__ __launch_bounds__(256) void k_eval_large_combine(const EvalDesc *__restrict__ items,
                                                            int n_items, int total_blocks, Consts K)
{
    const int L = xcd_remap_l(blockIdx.x, total_blocks);
    const EvalDesc &it = items[reinterpret_cast<const int32_t *>(items + n_items)[L]];
    const int pg = (L - it.block0) * 256 + threadIdx.x;
    if (pg >= it.n) return;
    float e;
    switch (it.func) {
    case ELLIPSOID: e = combine_point<ELLIPSOID>(gin<float>(it.part), it.n, pg, it.rb, it.dim, K.kf); break;
    case ROSENBROCK: e = combine_point<ROSENBROCK>(gin<float>(it.part), it.n, pg, it.rb, it.dim, K.kf); break;
    case RASTRIGIN: e = combine_point<RASTRIGIN>(gin<float>(it.part), it.n, pg, it.rb, it.dim, K.kf); break;
    case SCHWEFEL: e = combine_point<SCHWEFEL>(gin<float>(it.part), it.n, pg, it.rb, it.dim, K.kf); break;
    case GRIEWANK: e = combine_point<GRIEWANK>(gin<float>(it.part), it.n, pg, it.rb, it.dim, K.kf); break;
    default: e = combine_point<ACKLEY>(gin<float>(it.part), it.n, pg, it.rb, it.dim, K.kf); break;
    }
    gout<float>(it.err)[pg] = e;
}

hipError_t launch_eval_large(const EvalDesc *d_items, int n_items, int total_blocks,
                             bool split_bf16, int points, const Consts &k, hipStream_t s)
{
    if (total_blocks <= 0) return hipSuccess;
    if (points != 64 && points != 128) return hipErrorInvalidValue;
    const auto kern = split_bf16 ? (points == 64 ? k_eval_large<true, 64> : k_eval_large<true, 128>)
                                 : (points == 64 ? k_eval_large<false, 64> : k_eval_large<false, 128>);
    hipLaunchKernelGGL(kern, dim3(total_blocks), dim3(256), 0, s, d_items, n_items, total_blocks, k);
    return hipGetLastError();
}

hipError_t launch_eval_operands(const EvalDesc *d_items, int n_items, int total_blocks, bool split_bf16,
                               hipStream_t s)
{
    if (total_blocks <= 0) return hipSuccess;
    if (split_bf16)
        hipLaunchKernelGGL(k_eval_operands<true>, dim3(total_blocks), dim3(256), 0, s, d_items, n_items,
                           total_blocks);
    else
        hipLaunchKernelGGL(k_eval_operands<false>, dim3(total_blocks), dim3(256), 0, s, d_items, n_items,
                           total_blocks);
    return hipGetLastError();
}

hipError_t launch_eval_large_combine(const EvalDesc *d_items, int n_items, int total_blocks,
                                     const Consts &k, hipStream_t s)
{
    if (total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_eval_large_combine, dim3(total_blocks), dim3(256), 0, s, d_items, n_items,
                       total_blocks, k);
    return hipGetLastError();
}

}  // namespace sevo
