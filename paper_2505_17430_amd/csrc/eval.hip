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
#include "tile.h"

namespace sevo {


// Workgroups are dispatched round-robin over the 8 XCDs.  Renumber them so
// that logical blocks [x q, (x + 1) q) all run on XCD x: consecutive logical
// blocks of one item then share that XCD's L2 copy of the item's rotation.
__device__ __forceinline__ int xcd_remap(int b, int G)
{
    const int q = G >> 3, r = G & 7;
    const int x = b & 7, k = b >> 3;
    return x * q + (x < r ? x : r) + k;
}

// Persistent grid: the tiles (64*CT points each) of all items of one call are
// numbered consecutively, item after item; workgroup L walks the contiguous
// range [L T / G, (L + 1) T / G).  The rotation of an item is staged in LDS
// when the walk enters the item, after the loads of the wave's first tile
// have been issued; each wave's loads of its next tile are in flight while
// the current one is shifted, rotated and reduced.  Logical
// workgroups are renumbered per XCD, so an XCD works through a contiguous
// stretch of items and their rotations stay in that XCD's L2.
template <int KS, int CT>
__global__ __launch_bounds__(256, CT == 1 ? 3 : 2) void k_eval_small(const EvalDesc *__restrict__ items, int n_items,
                                                    int total_tiles, int grid, Consts K)
{
    constexpr int RT = (KS + 3) / 4;
    constexpr int TILE = 64 * CT;
    __shared__ __attribute__((aligned(16))) float sA[RT * KS * 64];
    __shared__ double sO[KS * 4];
    __shared__ float sT[RT * 16];

    const int L = xcd_remap(blockIdx.x, grid);
    const int tb = (int)(((int64_t)L * total_tiles) / grid);
    const int te = (int)(((int64_t)(L + 1) * total_tiles) / grid);
    if (tb >= te) return;
    const int32_t *__restrict__ tile_item = reinterpret_cast<const int32_t *>(items + n_items);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kq = lane >> 4, pc = lane & 15;

    int cur = -1;
    const EvalDesc *it = nullptr;
    float b[KS][CT], bn[KS][CT];
    bool have_next = false;   // bn holds the raw coordinates of tile g
    for (int g = tb; g < te; ++g) {
        const int item = tile_item[g];
        const EvalDesc *ig = items + item;
        const int p0 = (g - ig->block0) * TILE + wave * 16 * CT;
        if (have_next) {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                for (int c = 0; c < CT; ++c) b[ks][c] = bn[ks][c];
        } else {
            // the tile's loads go out before the item's rotation is staged,
            // so that the two latencies overlap
            load_raw<KS, CT>(b, gin<float>(ig->x), ig->ld, ig->dim, ig->n, p0, kq, pc);
        }
        if (item != cur) {
            __syncthreads();   // every wave is done with the previous item's LDS
            cur = item;
            it = ig;
            const SEVO_GLOBAL double *og = gin<double>(it->o);
            const SEVO_GLOBAL float *tg = gin<float>(it->tab);
            stage_rotation<KS>(sA, it->Mfrag);
            for (int q = threadIdx.x; q < KS * 4; q += 256) sO[q] = q < it->dim ? og[q] : 0.0;
            for (int q = threadIdx.x; q < RT * 16; q += 256) sT[q] = tg[q];
            __syncthreads();
        }
        const int dim = it->dim, n = it->n;
        const int64_t ld = it->ld;
        const SEVO_GLOBAL float *__restrict__ X = gin<float>(it->x);
        SEVO_GLOBAL float *__restrict__ E = gout<float>(it->err);
        shift_raw<KS, CT>(b, dim, n, p0, kq, pc, sO);
        // the next tile's loads stay in flight while this tile is computed,
        // for the classes bound by memory (up to D = 32); above, the
        // registers serve the rotation better (D = 100: 152 against 160
        // VGPRs, 1 % faster) and the autotuner keeps one tile per workgroup
        have_next = KS <= 8 && g + 1 < te && tile_item[g + 1] == item;
        if (have_next) load_raw<KS, CT>(bn, X, ld, dim, n, p0 + TILE, kq, pc);
        switch (it->func) {
        case ELLIPSOID: tile_body<ELLIPSOID, KS, CT>(b, sA, sT, lane, dim, n, p0, K.kf, E); break;
        case ROSENBROCK: tile_body<ROSENBROCK, KS, CT>(b, sA, sT, lane, dim, n, p0, K.kf, E); break;
        case RASTRIGIN: tile_body<RASTRIGIN, KS, CT>(b, sA, sT, lane, dim, n, p0, K.kf, E); break;
        case SCHWEFEL: tile_body<SCHWEFEL, KS, CT>(b, sA, sT, lane, dim, n, p0, K.kf, E); break;
        case GRIEWANK: tile_body<GRIEWANK, KS, CT>(b, sA, sT, lane, dim, n, p0, K.kf, E); break;
        default: tile_body<ACKLEY, KS, CT>(b, sA, sT, lane, dim, n, p0, K.kf, E); break;
        }
    }
}

// The split-bf16 evaluation of D = 65 .. 112: the same persistent grid, loads
// and objective as k_eval_small, with the rotation's whole 32-coordinate
// steps as six bf16 products on v_mfma_f32_16x16x32_bf16 and the rest on the
// float MFMA.  The three bf16 terms of M and the remaining float fragments
// take up to 71 KB of dynamic LDS (Bf16Steps::LDS_BYTES), two workgroups
// per CU.
template <int KS, int CT>
__global__ __launch_bounds__(256, 2) void k_eval_small_bf16(const EvalDesc *__restrict__ items, int n_items,
                                                            int total_tiles, int grid, Consts K)
{
    constexpr int RT = Bf16Steps<KS>::RT, SF = Bf16Steps<KS>::SF;
    constexpr int TILE = 64 * CT;
    extern __shared__ __attribute__((aligned(16))) bf16x8 sAb[];
    float *sAr = reinterpret_cast<float *>(sAb + Bf16Steps<KS>::NVEC);
    __shared__ double sO[KS * 4];
    __shared__ float sT[RT * 16];

    const int L = xcd_remap(blockIdx.x, grid);
    const int tb = (int)(((int64_t)L * total_tiles) / grid);
    const int te = (int)(((int64_t)(L + 1) * total_tiles) / grid);
    if (tb >= te) return;
    const int32_t *__restrict__ tile_item = reinterpret_cast<const int32_t *>(items + n_items);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kq = lane >> 4, pc = lane & 15;

    int cur = -1;
    const EvalDesc *it = nullptr;
    float b[KS][CT], bn[KS][CT];
    bool have_next = false;   // bn holds the raw coordinates of tile g
    for (int g = tb; g < te; ++g) {
        const int item = tile_item[g];
        const EvalDesc *ig = items + item;
        const int p0 = (g - ig->block0) * TILE + wave * 16 * CT;
        if (have_next) {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                for (int c = 0; c < CT; ++c) b[ks][c] = bn[ks][c];
        } else {
            // the tile's loads go out before the item's rotation is staged
            load_raw<KS, CT>(b, gin<float>(ig->x), ig->ld, ig->dim, ig->n, p0, kq, pc);
        }
        if (item != cur) {
            __syncthreads();   // every wave is done with the previous item's LDS
            cur = item;
            it = ig;
            const SEVO_GLOBAL double *og = gin<double>(it->o);
            const SEVO_GLOBAL float *tg = gin<float>(it->tab);
            stage_rotation_bf16<KS>(sAb, sAr, it->Mbf, it->Mfrag);
            for (int q = threadIdx.x; q < KS * 4; q += 256) sO[q] = q < it->dim ? og[q] : 0.0;
            for (int q = threadIdx.x; q < RT * 16; q += 256) sT[q] = tg[q];
            __syncthreads();
        }
        const int dim = it->dim, n = it->n;
        const int64_t ld = it->ld;
        const SEVO_GLOBAL float *__restrict__ X = gin<float>(it->x);
        SEVO_GLOBAL float *__restrict__ E = gout<float>(it->err);
        if (!have_next) shift_raw<KS, CT>(b, dim, n, p0, kq, pc, sO);
        // the next tile's coordinates are loaded and shifted before this tile
        // is computed: holding them raw through the split and the MFMAs
        // would take more registers than this kernel has (measured: 9 spilled,
        // 117 against 108 us at D = 100)
        have_next = g + 1 < te && tile_item[g + 1] == item;
        if (have_next) {
            load_raw<KS, CT>(bn, X, ld, dim, n, p0 + TILE, kq, pc);
            shift_raw<KS, CT>(bn, dim, n, p0 + TILE, kq, pc, sO);
        }
        bf16x8 bt[3][SF][CT];
        split3_b<KS, CT>(bt, b);
        switch (it->func) {
        case ELLIPSOID: tile_body_bf16<ELLIPSOID, KS, CT>(bt, b, sAb, sAr, sT, lane, dim, n, p0, K.kf, E); break;
        case ROSENBROCK: tile_body_bf16<ROSENBROCK, KS, CT>(bt, b, sAb, sAr, sT, lane, dim, n, p0, K.kf, E); break;
        case RASTRIGIN: tile_body_bf16<RASTRIGIN, KS, CT>(bt, b, sAb, sAr, sT, lane, dim, n, p0, K.kf, E); break;
        case SCHWEFEL: tile_body_bf16<SCHWEFEL, KS, CT>(bt, b, sAb, sAr, sT, lane, dim, n, p0, K.kf, E); break;
        case GRIEWANK: tile_body_bf16<GRIEWANK, KS, CT>(bt, b, sAb, sAr, sT, lane, dim, n, p0, K.kf, E); break;
        default: tile_body_bf16<ACKLEY, KS, CT>(bt, b, sAb, sAr, sT, lane, dim, n, p0, K.kf, E); break;
        }
    }
}

// Points per wave: four 16-point column tiles up to D = 12, where the
// evaluation is bound by memory and more loads in flight per wave pay
// (measured at D = 10 over 16.7 M points: 236 us with four, 251 us with two,
// 246 us with eight), two up to D = 32, one for the larger dimensions.
#ifndef SEVO_CT_LARGE
#define SEVO_CT_LARGE 1
#endif
#ifndef SEVO_CT_TINY
#define SEVO_CT_TINY 4
#endif
constexpr int ct_for(int ks) { return ks <= 3 ? SEVO_CT_TINY : ks <= 8 ? 2 : SEVO_CT_LARGE; }

// Split bf16: column tiles per wave (two halve the LDS traffic of the
// fragments per MFMA).
#ifndef SEVO_CT_BF16
#define SEVO_CT_BF16 2
#endif
constexpr int ct_for_bf16(int ks) { return ks <= 8 ? 2 : SEVO_CT_BF16; }

int small_tile_points(int ks, bool bf16) { return 64 * (bf16 ? ct_for_bf16(ks) : ct_for(ks)); }

bool small_bf16_class(int ks) { return ks >= SMALL_BF16_KS_MIN && ks <= SMALL_BF16_KS_MAX; }

typedef void (*SmallKernel)(const EvalDesc *, int, int, int, Consts);

template <int KS>
static SmallKernel small_kernel(bool bf16)
{
    if constexpr (KS >= SMALL_BF16_KS_MIN && KS <= SMALL_BF16_KS_MAX)
        if (bf16) return k_eval_small_bf16<KS, ct_for_bf16(KS)>;
    return bf16 ? nullptr : k_eval_small<KS, ct_for(KS)>;
}

template <int KS>
static constexpr int small_dyn_lds_of() { return Bf16Steps<KS>::LDS_BYTES; }

// Dynamic LDS of a launch (the split-bf16 kernel's fragments; 0 for the
// float kernel).
static int small_dyn_lds(int ks, bool bf16)
{
    if (!bf16 || !small_bf16_class(ks)) return 0;
    switch (ks) {
#define SEVO_KS_CASE(v) case v: return small_dyn_lds_of<v>();
        SEVO_KS_CASE(9) SEVO_KS_CASE(10) SEVO_KS_CASE(11) SEVO_KS_CASE(12) SEVO_KS_CASE(13)
        SEVO_KS_CASE(14) SEVO_KS_CASE(15) SEVO_KS_CASE(16) SEVO_KS_CASE(17) SEVO_KS_CASE(18)
        SEVO_KS_CASE(19) SEVO_KS_CASE(20) SEVO_KS_CASE(21) SEVO_KS_CASE(22) SEVO_KS_CASE(23)
        SEVO_KS_CASE(24) SEVO_KS_CASE(25) SEVO_KS_CASE(26) SEVO_KS_CASE(27) SEVO_KS_CASE(28)
#undef SEVO_KS_CASE
    default: return 0;
    }
}

// The kernel of a launch, with its dynamic-LDS allowance raised once (above
// the default 64 KB where needed); nullptr if unavailable.
static SmallKernel small_ready(int ks, bool bf16);

static SmallKernel small_table(int ks, bool bf16)
{
    switch (ks) {
#define SEVO_KS_CASE(v) case v: return small_kernel<v>(bf16);
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

static SmallKernel small_ready(int ks, bool bf16)
{
    static int done[64] = {};   // split-bf16 kernels: 1 once the attribute is set, -1 if refused
    SmallKernel k = small_table(ks, bf16);
    if (!k || !bf16 || ks < 0 || ks >= 64) return k;
    if (!done[ks]) {
        done[ks] = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       small_dyn_lds(ks, true)) == hipSuccess ? 1 : -1;
        (void)hipGetLastError();
    }
    return done[ks] > 0 ? k : nullptr;
}

int small_resident_blocks(int ks, bool bf16)
{
    SmallKernel k = small_ready(ks, bf16);
    if (!k) return 1;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 256, small_dyn_lds(ks, bf16)) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return per_cu * cus;
}

hipError_t launch_eval_small(const EvalDesc *d_items, int n_items, int ks, int total_tiles, int grid,
                             bool bf16, const Consts &k, hipStream_t s)
{
    SmallKernel kern = small_ready(ks, bf16);
    if (!kern) return hipErrorInvalidValue;
    if (total_tiles <= 0 || grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), small_dyn_lds(ks, bf16), s, d_items, n_items, total_tiles,
                       grid, k);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Double-precision path: one lane per point, z_r accumulated row by row with
// the rotation read through the scalar cache (uniform addresses) and x from
// the vector cache.  Terms are added one row late so Rosenbrock sees z_{r+1}.
template <int FUNC>
__device__ __forceinline__ double eval_point_f64(const SEVO_GLOBAL double *__restrict__ X, int64_t ld,
                                                 int p, int dim, const SEVO_GLOBAL double *__restrict__ o,
                                                 const SEVO_GLOBAL double *__restrict__ M,
                                                 const SchwefelConst<double> &K)
{
    Acc<double> acc;
    acc.init();
    double zprev = 0.0;
    for (int r = 0; r < dim; ++r) {
        const SEVO_GLOBAL double *Mr = M + (int64_t)r * dim;
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
    const EvalDesc &it = items[reinterpret_cast<const int32_t *>(items + n_items)[L]];
    const int p = (L - it.block0) * F64_POINTS + threadIdx.x;
    if (p >= it.n) return;
    const SEVO_GLOBAL double *X = gin<double>(it.x);
    const SEVO_GLOBAL double *og = gin<double>(it.o);
    const SEVO_GLOBAL double *Mg = gin<double>(it.M64);
    SEVO_GLOBAL double *E = gout<double>(it.err);
    double e;
    switch (it.func) {
    case ELLIPSOID: e = eval_point_f64<ELLIPSOID>(X, it.ld, p, it.dim, og, Mg, K.kd); break;
    case ROSENBROCK: e = eval_point_f64<ROSENBROCK>(X, it.ld, p, it.dim, og, Mg, K.kd); break;
    case RASTRIGIN: e = eval_point_f64<RASTRIGIN>(X, it.ld, p, it.dim, og, Mg, K.kd); break;
    case SCHWEFEL: e = eval_point_f64<SCHWEFEL>(X, it.ld, p, it.dim, og, Mg, K.kd); break;
    case GRIEWANK: e = eval_point_f64<GRIEWANK>(X, it.ld, p, it.dim, og, Mg, K.kd); break;
    default: e = eval_point_f64<ACKLEY>(X, it.ld, p, it.dim, og, Mg, K.kd); break;
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
