// eval.hip -- batched evaluation kernels for gfx950.
//
// The transform z = M (x - o) of every point is the one dense contraction of
// the method: for a group of points that share an instance it is the GEMM
// Z = M * Dmat with Dmat = X - o 1^T (dimension x points).  The kernels keep
// the population's structure-of-arrays layout (point index fastest), do the
// shift in double and round d once to float, run the rotation on MFMA
// (v_mfma_f32_16x16x4_f32: z rows on the MFMA M axis, points on N, the
// dimension on K), and reduce the per-coordinate objective terms straight out
// of the accumulator registers with compensated sums and wave shuffles.
//
// MFMA 16x16x4 f32 operand layout (lane l of 64):
//   A (16 x 4):  A[l % 16][l / 16]          one float per lane
//   B (4 x 16):  B[l / 16][l % 16]          one float per lane
//   D (16 x 16): D[4 (l / 16) + j][l % 16]  four floats per lane, j = 0..3
// so after the K loop lane l holds z rows 16 rt + 4 (l/16) + j of point l % 16.
#include "runtime.h"

namespace sevo {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Workgroups are dispatched round-robin over the 8 XCDs.  Renumber them so
// that logical blocks [x q, (x + 1) q) all run on XCD x: consecutive logical
// blocks of one item then share that XCD's L2 copy of the item's rotation.
__device__ __forceinline__ int xcd_remap(int b, int G)
{
    const int q = G >> 3, r = G & 7;
    const int x = b & 7, k = b >> 3;
    return x * q + (x < r ? x : r) + k;
}

__device__ __forceinline__ int find_item(const EvalDesc *__restrict__ items, int n_items, int L)
{
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].block0 <= L) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

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
                                          const SchwefelConst<float> &K, float *__restrict__ E)
{
    constexpr int RT = (KS + 3) / 4;
    const int kq = lane >> 4;
    const int src = (lane + 16) & 63;
    Acc<float> acc[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[c].init();
    floatx4 zp[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) zp[c] = floatx4{0.f, 0.f, 0.f, 0.f};

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
                const int rbase = (rt - 1) * 16 + kq * 4;
#pragma unroll
                for (int c = 0; c < CT; ++c) {
                    const float nx_same = __shfl(zp[c][0], src, 64);
                    const float nx_next = __shfl(zc[c][0], src, 64);
                    const float nb3 = (kq < 3) ? nx_same : nx_next;
                    const float zn[4] = {zp[c][1], zp[c][2], zp[c][3], nb3};
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (rbase + j < dim) add_term<FUNC>(acc[c], zp[c][j], zn[j], rbase + j + 1 < dim, 0.f, K);
                }
            }
#pragma unroll
            for (int c = 0; c < CT; ++c) zp[c] = zc[c];
        } else {
            const int rbase = rt * 16 + kq * 4;
#pragma unroll
            for (int c = 0; c < CT; ++c)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (rbase + j < dim) add_term<FUNC>(acc[c], zc[c][j], 0.f, false, sT[rbase + j], K);
        }
    }
    if constexpr (FUNC == ROSENBROCK) {
        const int rbase = (RT - 1) * 16 + kq * 4;
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const float nb3 = __shfl(zp[c][0], src, 64);
            const float zn[4] = {zp[c][1], zp[c][2], zp[c][3], kq < 3 ? nb3 : 0.f};
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (rbase + j < dim) add_term<FUNC>(acc[c], zp[c][j], zn[j], rbase + j + 1 < dim, 0.f, K);
        }
    }
    const int pc = lane & 15;
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        merge_xor(acc[c], 16);
        merge_xor(acc[c], 32);
        const int p = p0 + c * 16 + pc;
        if (kq == 0 && p < n) E[p] = finalize<FUNC>(acc[c], dim);
    }
}

template <int KS>
__global__ __launch_bounds__(256) void k_eval_small(const EvalDesc *__restrict__ items, int n_items,
                                                    int total_blocks, int tpb, Consts K)
{
    constexpr int RT = (KS + 3) / 4;
    constexpr int CT = 2;
    __shared__ float sA[RT * KS * 64];
    __shared__ double sO[KS * 4];
    __shared__ float sT[RT * 16];

    const int L = xcd_remap(blockIdx.x, total_blocks);
    const EvalDesc &it = items[find_item(items, n_items, L)];
    const int dim = it.dim, n = it.n, func = it.func;
    const int64_t ld = it.ld;

    for (int q = threadIdx.x; q < RT * KS * 64; q += 256) sA[q] = it.Mfrag[q];
    for (int q = threadIdx.x; q < KS * 4; q += 256) sO[q] = q < dim ? it.o[q] : 0.0;
    for (int q = threadIdx.x; q < RT * 16; q += 256) sT[q] = it.tab[q];
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kq = lane >> 4, pc = lane & 15;
    const float *__restrict__ X = static_cast<const float *>(it.x);
    float *__restrict__ E = static_cast<float *>(it.err);
    const int ntiles = (n + SMALL_TILE_POINTS - 1) / SMALL_TILE_POINTS;
    const int t0 = (L - it.block0) * tpb;
    const int t1 = min(t0 + tpb, ntiles);

    for (int tile = t0; tile < t1; ++tile) {
        const int p0 = tile * SMALL_TILE_POINTS + wave * 16 * CT;
        float b[KS][CT];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int k = ks * 4 + kq;
            const double ok = sO[k];
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                const int p = p0 + c * 16 + pc;
                float v = 0.f;
                if (k < dim && p < n) v = (float)((double)X[(int64_t)k * ld + p] - ok);
                b[ks][c] = v;
            }
        }
        switch (func) {
        case ELLIPSOID: tile_body<ELLIPSOID, KS, CT>(b, sA, sT, lane, dim, n, p0, K.kf, E); break;
        case ROSENBROCK: tile_body<ROSENBROCK, KS, CT>(b, sA, sT, lane, dim, n, p0, K.kf, E); break;
        case RASTRIGIN: tile_body<RASTRIGIN, KS, CT>(b, sA, sT, lane, dim, n, p0, K.kf, E); break;
        case SCHWEFEL: tile_body<SCHWEFEL, KS, CT>(b, sA, sT, lane, dim, n, p0, K.kf, E); break;
        case GRIEWANK: tile_body<GRIEWANK, KS, CT>(b, sA, sT, lane, dim, n, p0, K.kf, E); break;
        default: tile_body<ACKLEY, KS, CT>(b, sA, sT, lane, dim, n, p0, K.kf, E); break;
        }
    }
}

int small_blocks_for(int n, int tiles_per_block)
{
    const int ntiles = (n + SMALL_TILE_POINTS - 1) / SMALL_TILE_POINTS;
    return (ntiles + tiles_per_block - 1) / tiles_per_block;
}

typedef void (*SmallKernel)(const EvalDesc *, int, int, int, Consts);

template <int KS>
static SmallKernel small_kernel() { return k_eval_small<KS>; }

static SmallKernel small_table(int ks)
{
    switch (ks) {
#define SEVO_KS_CASE(v) case v: return small_kernel<v>();
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

hipError_t launch_eval_small(const EvalDesc *d_items, int n_items, int ks, int total_blocks,
                             int tiles_per_block, const Consts &k, hipStream_t s)
{
    SmallKernel kern = small_table(ks);
    if (!kern) return hipErrorInvalidValue;
    if (total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(kern, dim3(total_blocks), dim3(256), 0, s, d_items, n_items, total_blocks,
                       tiles_per_block, k);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Double-precision path: one lane per point, z_r accumulated row by row with
// the rotation read through the scalar cache (uniform addresses) and x from
// the vector cache.  Terms are added one row late so Rosenbrock sees z_{r+1}.
template <int FUNC>
__device__ __forceinline__ double eval_point_f64(const double *__restrict__ X, int64_t ld, int p,
                                                 int dim, const double *__restrict__ o,
                                                 const double *__restrict__ M,
                                                 const SchwefelConst<double> &K)
{
    Acc<double> acc;
    acc.init();
    double zprev = 0.0;
    for (int r = 0; r < dim; ++r) {
        const double *Mr = M + (int64_t)r * dim;
        double zr = 0.0;
        for (int k = 0; k < dim; ++k) zr = fma(Mr[k], X[(int64_t)k * ld + p] - o[k], zr);
        if (r > 0) {
            const int q = r - 1;
            double tab = 0.0;
            if constexpr (FUNC == ELLIPSOID) tab = dim > 1 ? pow(10.0, 6.0 * q / (dim - 1)) : 1.0;
            if constexpr (FUNC == GRIEWANK) tab = 1.0 / sqrt((double)(q + 1));
            add_term<FUNC>(acc, zprev, zr, true, tab, K);
        }
        zprev = zr;
    }
    {
        const int q = dim - 1;
        double tab = 0.0;
        if constexpr (FUNC == ELLIPSOID) tab = dim > 1 ? pow(10.0, 6.0 * q / (dim - 1)) : 1.0;
        if constexpr (FUNC == GRIEWANK) tab = 1.0 / sqrt((double)(q + 1));
        add_term<FUNC>(acc, zprev, 0.0, false, tab, K);
    }
    return finalize<FUNC>(acc, dim);
}

__global__ __launch_bounds__(F64_POINTS) void k_eval_f64(const EvalDesc *__restrict__ items,
                                                         int n_items, int total_blocks, Consts K)
{
    const int L = xcd_remap(blockIdx.x, total_blocks);
    const EvalDesc &it = items[find_item(items, n_items, L)];
    const int p = (L - it.block0) * F64_POINTS + threadIdx.x;
    if (p >= it.n) return;
    const double *X = static_cast<const double *>(it.x);
    double *E = static_cast<double *>(it.err);
    double e;
    switch (it.func) {
    case ELLIPSOID: e = eval_point_f64<ELLIPSOID>(X, it.ld, p, it.dim, it.o, it.M64, K.kd); break;
    case ROSENBROCK: e = eval_point_f64<ROSENBROCK>(X, it.ld, p, it.dim, it.o, it.M64, K.kd); break;
    case RASTRIGIN: e = eval_point_f64<RASTRIGIN>(X, it.ld, p, it.dim, it.o, it.M64, K.kd); break;
    case SCHWEFEL: e = eval_point_f64<SCHWEFEL>(X, it.ld, p, it.dim, it.o, it.M64, K.kd); break;
    case GRIEWANK: e = eval_point_f64<GRIEWANK>(X, it.ld, p, it.dim, it.o, it.M64, K.kd); break;
    default: e = eval_point_f64<ACKLEY>(X, it.ld, p, it.dim, it.o, it.M64, K.kd); break;
    }
    E[p] = e;
}

hipError_t launch_eval_f64(const EvalDesc *d_items, int n_items, int total_blocks,
                           const Consts &k, hipStream_t s)
{
    if (total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_eval_f64, dim3(total_blocks), dim3(F64_POINTS), 0, s, d_items, n_items,
                       total_blocks, k);
    return hipGetLastError();
}

}  // namespace sevo
