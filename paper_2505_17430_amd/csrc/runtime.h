// runtime.h -- internal interface between the host runtime (runtime.hip) and
// the kernel launchers (eval.hip, steps.hip, run.hip).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"
#include "objective.h"

namespace sevo {

// Pointers read out of descriptors are generic; casting them to the global
// address space lets the compiler emit global (not flat) loads and stores,
// which do not tie up the LDS counter.
#define SEVO_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const SEVO_GLOBAL T *gin(const void *p)
{
    return (const SEVO_GLOBAL T *)p;
}
template <typename T>
__device__ __forceinline__ SEVO_GLOBAL T *gout(void *p)
{
    return (SEVO_GLOBAL T *)p;
}

// Largest dimension of the small-D evaluation path: its rotation (padded to
// 16-row tiles by 4-column steps) lives in LDS, <= 62 KB.
constexpr int SMALL_D_MAX = 120;
constexpr int MAX_DIM = 1024;
// Largest leading dimension of a population (32-bit per-lane load offsets).
constexpr int64_t MAX_LD = int64_t(1) << 28;

// One evaluation item as the kernels see it (a population of one
// (function, dimension, instance)).
struct EvalDesc {
    const void *x;          // [dim][ld], float or double
    void *err;              // [n], float or double
    const double *o;        // [dim]
    const float *Mfrag;     // [RT][KS][64] MFMA A-operand fragments of M (float)
    const float *tab;       // [RT * 16] per-row table (ellipsoid weight, 1/sqrt(i))
    const double *M64;      // [dim][dim] row-major
    const uint16_t *Mbf;    // bf16 term blocks hi, mid, lo: D > 120 [RT][KS32][64][8] in natural column
                            // order; D <= 120 [RT][KS / 8][64][8] in the small path's order
    float *part;            // large-D partial sums [RB][n][8] (workspace)
    void *opnd;             // large-D GEMM operands, large_operand_size npad kpad bytes (workspace; layout
                            // at k_eval_operands)
    int64_t ld;
    int32_t n;
    int32_t func;
    int32_t dim;
    int32_t block0;         // first logical block of this item
    int32_t nblocks;        // logical blocks of this item
    int32_t rb;             // large-D: row blocks
};

struct Consts {
    SchwefelConst<float> kf;
    SchwefelConst<double> kd;
};

Consts make_consts();

inline int ks_of(int dim) { return (dim + 3) / 4; }
inline int rt_of(int dim) { return (dim + 15) / 16; }
inline int ks32_of(int dim) { return (dim + 31) / 32; }

// eval.hip
// Split bf16 runs the small path's rotation on bf16 MFMA for these k-step
// classes (D = 65 .. 112).  Below, the float kernel serves both precisions:
// measured at D = 50 the split was slower (59-64 us against 56 us per
// 306,000 evaluations; the kernels are bound by vector work, which the
// split adds to) and at D <= 30 the work is bound by memory.  Above 112
// the fragments would leave room for one workgroup per CU only.
constexpr int SMALL_BF16_KS_MIN = 17;
constexpr int SMALL_BF16_KS_MAX = 28;
bool small_bf16_class(int ks);
int small_tile_points(int ks, bool bf16);            // points per workgroup tile
int small_resident_blocks(int ks, bool bf16);        // workgroups the whole GPU holds at once
// d_items: descriptors (block0 = first tile, nblocks = tiles of the item)
// followed by the tile -> item map.
hipError_t launch_eval_small(const EvalDesc *d_items, int n_items, int ks, int total_tiles, int grid,
                             bool bf16, const Consts &k, hipStream_t s);

constexpr int LARGE_ROWS = 128;          // rows of z per workgroup (4 waves x 32)
constexpr int LARGE_POINTS = 128;        // points per operand tile
// points: per workgroup, 128 (one operand tile) or 64 (half of one)
hipError_t launch_eval_large(const EvalDesc *d_items, int n_items, int total_blocks,
                             bool split_bf16, int points, const Consts &k, hipStream_t s);
hipError_t launch_eval_large_combine(const EvalDesc *d_items, int n_items, int total_blocks,
                                     const Consts &k, hipStream_t s);
// GEMM operands of the large-D points, made by a pre-pass: d = x - o
// (double, rounded once to float), zero beyond n and dim, tiled by
// (128-point tile, 32-coordinate chunk) in the order in which the
// evaluation stages one chunk:
//   FP32        [npad / 128][kpad / 32][32 k][128 points] floats;
//   split bf16  hi = bf16(d), mid = bf16(d - hi), lo = bf16(d - hi - mid):
//               the three arrays one after another, each
//               [npad / 128][kpad / 32][128 points][32 k].
// So 4 or 6 npad kpad bytes.  Workgroups of 64 points x 32 coordinates.
constexpr int OPERAND_POINTS = 64, OPERAND_K = 32;
__host__ __device__ inline int64_t large_npad(int n) { return ((int64_t)n + LARGE_POINTS - 1) / LARGE_POINTS * LARGE_POINTS; }
__host__ __device__ inline int64_t large_kpad(int dim) { return ((int64_t)dim + 31) / 32 * 32; }
// bytes of GEMM operand per padded (point, coordinate): one float, or three
// bf16 terms
__host__ __device__ inline int64_t large_operand_size(bool split_bf16) { return split_bf16 ? 6 : 4; }
hipError_t launch_eval_operands(const EvalDesc *d_items, int n_items, int total_blocks, bool split_bf16,
                               hipStream_t s);

constexpr int F64_POINTS = 64;           // points per workgroup of the double path
hipError_t launch_eval_f64(const EvalDesc *d_items, int n_items, int total_blocks,
                           const Consts &k, hipStream_t s);

}  // namespace sevo
