// steps.hip -- one generation at a time: DE rand/1/bin and gbest PSO steps
// as separate kernels (variation, batched evaluation, selection), for
// callers that drive their own loop, for parity tests, and as the plain
// one-run-per-launch double-precision path.
//
// Layout of every state buffer: run r, coordinate d, individual i at
// buf[r * run_stride + d * ld + i]; per-individual values at buf[r * ld + i].
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "../../include/sevo.h"
#include "algo.h"
#include "runtime.h"
#include "state.h"

namespace sevo {

struct StepGeom {
    int n_runs, np, dim;
    int64_t ld, rs;
    uint32_t run_uid0, seed32, t;
};

__device__ __forceinline__ bool thread_run_ind(const StepGeom &g, int &r, int &i)
{
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (int64_t)g.n_runs * g.np) return false;
    r = (int)(tid / g.np);
    i = (int)(tid % g.np);
    return true;
}

// LDS of the staged variation (k_de_variation_lds).  A population of at
// most VAR_LDS_WHOLE bytes is staged whole (rows = dim, nothing else in LDS).
// Otherwise the donors take 8 bytes per individual, followed by a slab of
// rows x np values: a slab of at least 4 rows within 32 KB when possible
// (four or more workgroups per CU), else within 64 KB.  0 rows: the
// population does not fit (or np is beyond the 16-bit indices) and the
// global gathers are used instead.
constexpr size_t VAR_LDS_WHOLE = 48 * 1024, VAR_LDS_SMALL = 32 * 1024, VAR_LDS_MAX = 64 * 1024;

__host__ __device__ inline size_t var_donor_bytes(int np) { return ((size_t)np * 8 + 15) & ~(size_t)15; }

inline int var_slab_rows(int dim, int np, size_t tsize)
{
    if ((size_t)dim * np * tsize <= VAR_LDS_WHOLE) return dim;
    if (np > 65535) return 0;
    for (size_t budget : {VAR_LDS_SMALL, VAR_LDS_MAX}) {
        const size_t d = var_donor_bytes(np);
        if (d >= budget) continue;
        const int rows = (int)((budget - d) / ((size_t)np * tsize)) / 4 * 4;
        if (rows >= 4) return rows < dim ? rows : dim;
    }
    return 0;
}

inline size_t var_lds_bytes(int dim, int np, int rows, size_t tsize)
{
    return (rows < dim ? var_donor_bytes(np) : 0) + (size_t)rows * np * tsize;
}

// Generation 0: x uniform in the box (computed in double, stored as T).
template <typename T>
__global__ void k_init_pop(StepGeom g, double lb, double ub, T *__restrict__ x, T *__restrict__ v,
                           T *__restrict__ p)
{
    int r, i;
    if (!thread_run_ind(g, r, i)) return;
    const uint32_t uid = g.run_uid0 + (uint32_t)r;
    for (int jb = 0; jb * 4 < g.dim; ++jb) {
        const u32x4 w = draw(uid, g.seed32, 0, (uint32_t)i, TAG_INIT_X, (uint32_t)jb);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = jb * 4 + e;
            if (j >= g.dim) break;
            const int64_t at = (int64_t)r * g.rs + (int64_t)j * g.ld + i;
            const T xv = (T)(lb + (ub - lb) * u24d(word(w, e)));
            x[at] = xv;
            if (v) v[at] = T(0);
            if (p) p[at] = xv;
        }
    }
}

// DE rand/1/bin variation: trial u of every individual of generation t.
template <typename T>
__global__ void k_de_variation(StepGeom g, T lb, T ub, T F, uint32_t thr, const T *__restrict__ x,
                               T *__restrict__ u, int32_t *__restrict__ donors)
{
    int r, i;
    if (!thread_run_ind(g, r, i)) return;
    const uint32_t uid = g.run_uid0 + (uint32_t)r;
    int r1, r2, r3, jrand;
    de_donors(uid, g.seed32, g.t, i, g.np, g.dim, r1, r2, r3, jrand);
    if (donors) {
        int32_t *dn = donors + (int64_t)r * 4 * g.ld + i;
        dn[0] = r1;
        dn[g.ld] = r2;
        dn[2 * g.ld] = r3;
        dn[3 * g.ld] = jrand;
    }
    const T *xr = x + (int64_t)r * g.rs;
    T *ur = u + (int64_t)r * g.rs;
    // chunks of VAR_CH coordinate blocks: all loads of a chunk (the parent
    // and three donor gathers per coordinate, rows past dim clamped to the
    // last) are issued before its stores, so a chunk costs one memory round
    // trip instead of one per coordinate
    constexpr int VAR_CH = 2;
    const int nb = (g.dim + 3) / 4;
    for (int jb0 = 0; jb0 < nb; jb0 += VAR_CH) {
        T xi[VAR_CH][4], xa[VAR_CH][4], xb[VAR_CH][4], xc[VAR_CH][4];
#pragma unroll
        for (int c = 0; c < VAR_CH; ++c)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t row = (int64_t)min((jb0 + c) * 4 + e, g.dim - 1) * g.ld;
                xi[c][e] = xr[row + i];
                xa[c][e] = xr[row + r1];
                xb[c][e] = xr[row + r2];
                xc[c][e] = xr[row + r3];
            }
#pragma unroll
        for (int c = 0; c < VAR_CH; ++c) {
            const int jb = jb0 + c;
            if (jb >= nb) break;
            const u32x4 w = draw(uid, g.seed32, g.t, (uint32_t)i, TAG_CROSS, (uint32_t)jb);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int j = jb * 4 + e;
                if (j >= g.dim) break;
                const T v = xa[c][e] + F * (xb[c][e] - xc[c][e]);
                bool m;
                ur[(int64_t)j * g.ld + i] = cross_repair<T>(word(w, e), thr, j, jrand, v, xi[c][e], lb, ub, m);
            }
        }
    }
}

// The same variation with the run's population staged in LDS, one workgroup
// per run, so that the donor gathers read LDS instead of one cache line per
// donor coordinate.  The population passes through LDS in slabs of `rows`
// coordinate rows (a multiple of 4, so that a crossover draw block never
// straddles two slabs; every row at once when it fits), each loaded with
// coalesced reads, and every individual's trial coordinates of the slab are
// made from it.  The donors of each individual are drawn with the first
// slab and, when there are more, kept in LDS as 16-bit indices.  Same draws,
// same arithmetic, same results as k_de_variation.
template <typename T, int STAGE_CH, bool FLAT>
__global__ __launch_bounds__(256) void k_de_variation_lds(StepGeom g, T lb, T ub, T F, uint32_t thr,
                                                          const T *__restrict__ x, T *__restrict__ u,
                                                          int32_t *__restrict__ donors, int rows)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char sRaw[];
    const bool slabs = rows < g.dim;   // the donors are kept for the later slabs
    uint16_t *sD = reinterpret_cast<uint16_t *>(sRaw);                                  // [np][4]
    T *sX = reinterpret_cast<T *>(sRaw + (slabs ? var_donor_bytes(g.np) : 0));         // [rows][np]
    const int r = blockIdx.x;
    const T *xr = x + (int64_t)r * g.rs;
    T *ur = u + (int64_t)r * g.rs;
    const uint32_t uid = g.run_uid0 + (uint32_t)r;
    // q / np for the staging indices (q < 2^16): the product with
    // ceil(2^32 / np), high word, is exact there
    const uint32_t inv_np = (uint32_t)(0xFFFFFFFFull / (uint32_t)g.np) + 1u;
    // the mutants and crossover of slab rows [j0, j0 + nr), from sX
    auto compute = [&](int j0, int nr) {
        for (int i = threadIdx.x; i < g.np; i += 256) {
            // donors drawn with the first slab, kept in LDS for the others
            int r1, r2, r3, jrand;
            if (j0 == 0) {
                de_donors(uid, g.seed32, g.t, i, g.np, g.dim, r1, r2, r3, jrand);
                if (slabs) {
                    sD[4 * i] = (uint16_t)r1;
                    sD[4 * i + 1] = (uint16_t)r2;
                    sD[4 * i + 2] = (uint16_t)r3;
                    sD[4 * i + 3] = (uint16_t)jrand;
                }
                if (donors) {
                    int32_t *dn = donors + (int64_t)r * 4 * g.ld + i;
                    dn[0] = r1;
                    dn[g.ld] = r2;
                    dn[2 * g.ld] = r3;
                    dn[3 * g.ld] = jrand;
                }
            } else {
                r1 = sD[4 * i];
                r2 = sD[4 * i + 1];
                r3 = sD[4 * i + 2];
                jrand = sD[4 * i + 3];
            }
            for (int jj = 0; jj < nr; jj += 4) {
                const u32x4 w = draw(uid, g.seed32, g.t, (uint32_t)i, TAG_CROSS, (uint32_t)((j0 + jj) >> 2));
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (jj + e >= nr) break;
                    const int j = j0 + jj + e;
                    const T *row = sX + (jj + e) * g.np;
                    const T v = row[r1] + F * (row[r2] - row[r3]);
                    bool m;
                    ur[(int64_t)j * g.ld + i] = cross_repair<T>(word(w, e), thr, j, jrand, v, row[i], lb, ub, m);
                }
            }
        }
    };
    // element q of the slab at row j0 (clamped, so always a valid address)
    auto slab_elem = [&](int j0, int n, int q) {
        q = min(q, n - 1);
        const int jj = (int)__umulhi((uint32_t)q, inv_np), i = q - jj * g.np;
        return xr[(int64_t)(j0 + jj) * g.ld + i];
    };
    if (!FLAT && slabs && rows * g.np <= 256 * STAGE_CH) {
        // a slab is one chunk per thread: the next slab's loads are issued
        // before this slab is computed and stored to LDS after it
        T v[STAGE_CH];
        int n = min(rows, g.dim) * g.np;
#pragma unroll
        for (int c = 0; c < STAGE_CH; ++c) v[c] = slab_elem(0, n, threadIdx.x + c * 256);
#pragma unroll
        for (int c = 0; c < STAGE_CH; ++c)
            if ((int)threadIdx.x + c * 256 < n) sX[threadIdx.x + c * 256] = v[c];
        for (int j0 = 0; j0 < g.dim; j0 += rows) {
            __syncthreads();   // slab j0 is in LDS
            const int nr = min(rows, g.dim - j0);
            const bool more = j0 + rows < g.dim;
            if (more) {
                n = min(rows, g.dim - j0 - rows) * g.np;
#pragma unroll
                for (int c = 0; c < STAGE_CH; ++c) v[c] = slab_elem(j0 + rows, n, threadIdx.x + c * 256);
            }
            compute(j0, nr);
            __syncthreads();   // slab j0 has been read and the donors written
            if (more) {
#pragma unroll
                for (int c = 0; c < STAGE_CH; ++c)
                    if ((int)threadIdx.x + c * 256 < n) sX[threadIdx.x + c * 256] = v[c];
            }
        }
        return;
    }
    for (int j0 = 0; j0 < g.dim; j0 += rows) {
        const int nr = min(rows, g.dim - j0);
        const int n = nr * g.np;
        __syncthreads();   // the previous slab has been read and the donors written
        if constexpr (FLAT) {
            // a whole population with ld = np and a 16-byte aligned start
            // (the host checks) is one contiguous array: 16-byte vectors, all
            // loads of a chunk of STAGE_CH per thread before their stores,
            // then the elements after the last whole vector
            typedef uint32_t u32x4v __attribute__((ext_vector_type(4)));
            constexpr int VW = 16 / sizeof(T);
            const int nv = n / VW;
            const u32x4v *xv = reinterpret_cast<const u32x4v *>(xr);
            u32x4v *sv = reinterpret_cast<u32x4v *>(sX);
            for (int q0 = threadIdx.x; q0 < nv; q0 += 256 * STAGE_CH) {
                u32x4v v[STAGE_CH];
#pragma unroll
                for (int c = 0; c < STAGE_CH; ++c) v[c] = xv[min(q0 + c * 256, nv - 1)];
#pragma unroll
                for (int c = 0; c < STAGE_CH; ++c)
                    if (q0 + c * 256 < nv) sv[q0 + c * 256] = v[c];
            }
            for (int q = nv * VW + (int)threadIdx.x; q < n; q += 256) sX[q] = xr[q];
        } else {
            // staging in chunks of STAGE_CH elements per thread, all loads of
            // a chunk issued before its stores
            for (int q0 = threadIdx.x; q0 < n; q0 += 256 * STAGE_CH) {
                T v[STAGE_CH];
#pragma unroll
                for (int c = 0; c < STAGE_CH; ++c) v[c] = slab_elem(j0, n, q0 + c * 256);
#pragma unroll
                for (int c = 0; c < STAGE_CH; ++c)
                    if (q0 + c * 256 < n) sX[q0 + c * 256] = v[c];
            }
        }
        __syncthreads();
        compute(j0, nr);
    }
}

// Greedy one-to-one selection: the trial replaces its parent when
// e(u) <= e(x), NaN counting as +infinity.
template <typename T>
__global__ void k_de_select(StepGeom g, T *__restrict__ x, T *__restrict__ ex, const T *__restrict__ u,
                            const T *__restrict__ eu, uint8_t *__restrict__ replaced)
{
    int r, i;
    if (!thread_run_ind(g, r, i)) return;
    const int64_t e_at = (int64_t)r * g.ld + i;
    const bool rep = err_key(eu[e_at]) <= err_key(ex[e_at]);
    if (replaced) replaced[e_at] = rep ? 1 : 0;
    if (!rep) return;
    ex[e_at] = eu[e_at];
    // chunks of 8 coordinates, loads before stores
    constexpr int SEL_CH = 8;
    const int64_t base = (int64_t)r * g.rs + i;
    for (int j0 = 0; j0 < g.dim; j0 += SEL_CH) {
        T v[SEL_CH];
#pragma unroll
        for (int c = 0; c < SEL_CH; ++c) v[c] = u[base + (int64_t)min(j0 + c, g.dim - 1) * g.ld];
#pragma unroll
        for (int c = 0; c < SEL_CH; ++c)
            if (j0 + c < g.dim) x[base + (int64_t)(j0 + c) * g.ld] = v[c];
    }
}

// PSO velocity and position update of iteration t (g fixed for the whole
// iteration): v = w v + c1 r1 (p - x) + c2 r2 (g - x), |v| <= vmax, x += v,
// a coordinate leaving the box is put on the bound with v = 0.
template <typename T>
__global__ void k_pso_update(StepGeom g, T lb, T ub, T w, T c1, T c2, T vmax, T *__restrict__ x,
                             T *__restrict__ v, const T *__restrict__ p, const int32_t *__restrict__ gbest)
{
    int r, i;
    if (!thread_run_ind(g, r, i)) return;
    const uint32_t uid = g.run_uid0 + (uint32_t)r;
    const int gi = min(max((int)gbest[r], 0), g.np - 1);   // a stale index must not leave the run
    const int64_t base = (int64_t)r * g.rs;
    // chunks of UPD_CH coordinate pairs: all loads of a chunk (rows past dim
    // clamped to the last) are issued before its stores
    constexpr int UPD_CH = 4;
    const int nb = (g.dim + 1) / 2;
    for (int jb0 = 0; jb0 < nb; jb0 += UPD_CH) {
        T xv[UPD_CH][2], vv[UPD_CH][2], pv[UPD_CH][2], gv[UPD_CH][2];
#pragma unroll
        for (int c = 0; c < UPD_CH; ++c)
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int64_t row = base + (int64_t)min((jb0 + c) * 2 + e, g.dim - 1) * g.ld;
                xv[c][e] = x[row + i];
                vv[c][e] = v[row + i];
                pv[c][e] = p[row + i];
                gv[c][e] = p[row + gi];
            }
#pragma unroll
        for (int c = 0; c < UPD_CH; ++c) {
            const int jb = jb0 + c;
            if (jb >= nb) break;
            const u32x4 wd = draw(uid, g.seed32, g.t, (uint32_t)i, TAG_PSO_R, (uint32_t)jb);
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int j = jb * 2 + e;
                if (j >= g.dim) break;
                const int64_t row = base + (int64_t)j * g.ld;
                const T r1 = (T)u24f(word(wd, 2 * e)), r2 = (T)u24f(word(wd, 2 * e + 1));
                const T xj = xv[c][e];
                T vj = w * vv[c][e] + c1 * r1 * (pv[c][e] - xj) + c2 * r2 * (gv[c][e] - xj);
                vj = vj > vmax ? vmax : (vj < -vmax ? -vmax : vj);
                T xn = xj + vj;
                if (xn < lb) { xn = lb; vj = T(0); }
                else if (xn > ub) { xn = ub; vj = T(0); }
                x[row + i] = xn;
                v[row + i] = vj;
            }
        }
    }
}

// Personal bests (strict improvement) and the global best (argmin of the
// personal-best errors, lowest index on ties); one workgroup per run.  At
// iteration 0 (init = 1) p = x was set by the init kernel and ep = ex.
template <typename T>
__global__ __launch_bounds__(256) void k_pso_best(StepGeom g, int init, const T *__restrict__ x,
                                                  const T *__restrict__ ex, T *__restrict__ p,
                                                  T *__restrict__ ep, int32_t *__restrict__ gbest)
{
    const int r = blockIdx.x;
    __shared__ T sv[256];
    __shared__ int si[256];
    T bv = T(INFINITY);
    int bi = 0x7fffffff;
    // passes of PB particles per thread: the errors of a pass are loaded
    // together, then the improved particles' coordinates are copied in chunks
    // of CP_CH coordinates, the loads of a chunk for all of them issued
    // before its stores
    constexpr int PB = 8, CP_CH = 8;
    for (int i0 = threadIdx.x; i0 < g.np; i0 += 256 * PB) {
        T kx[PB], kp[PB];
        bool imp[PB];
#pragma unroll
        for (int b = 0; b < PB; ++b) {
            const int i = min(i0 + b * 256, g.np - 1);
            const int64_t e_at = (int64_t)r * g.ld + i;
            kx[b] = ex[e_at];
            kp[b] = ep[e_at];
        }
#pragma unroll
        for (int b = 0; b < PB; ++b) {
            const int i = i0 + b * 256;
            imp[b] = i < g.np && (init || err_key(kx[b]) < err_key(kp[b]));
            if (imp[b]) {
                ep[(int64_t)r * g.ld + i] = kx[b];
                kp[b] = kx[b];
            }
            const T k = err_key(kp[b]);
            if (i < g.np && (k < bv || (k == bv && i < bi))) { bv = k; bi = i; }
        }
        if (!init) {
            const int64_t base = (int64_t)r * g.rs;
            for (int j0 = 0; j0 < g.dim; j0 += CP_CH) {
                T v[PB][CP_CH];
#pragma unroll
                for (int b = 0; b < PB; ++b)
#pragma unroll
                    for (int c = 0; c < CP_CH; ++c)
                        v[b][c] = imp[b] ? x[base + (int64_t)min(j0 + c, g.dim - 1) * g.ld + i0 + b * 256] : T(0);
#pragma unroll
                for (int b = 0; b < PB; ++b)
#pragma unroll
                    for (int c = 0; c < CP_CH; ++c)
                        if (imp[b] && j0 + c < g.dim) p[base + (int64_t)(j0 + c) * g.ld + i0 + b * 256] = v[b][c];
            }
        }
    }
    sv[threadIdx.x] = bv;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            const T ov = sv[threadIdx.x + off];
            const int oi = si[threadIdx.x + off];
            if (ov < sv[threadIdx.x] || (ov == sv[threadIdx.x] && oi < si[threadIdx.x])) {
                sv[threadIdx.x] = ov;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) gbest[r] = si[0] == 0x7fffffff ? 0 : si[0];
}

static int blocks_for(const StepGeom &g) { return (int)(((int64_t)g.n_runs * g.np + 255) / 256); }

// Recorder state of one plain run.
struct RecState {
    double best;        // best over all evaluations so far
    double best_b;      // best over the first `budget` evaluations
};

// Best-so-far recorder for the np evaluations eY (individual order) made
// after fe0 evaluations: trace entries at every multiple of 200, the best of
// the first `budget` evaluations and its point.  One workgroup, np <= 256.
__global__ __launch_bounds__(256) void k_record_f64(const double *__restrict__ Y, const double *__restrict__ eY,
                                                    int np, int dim, int64_t ld, int64_t fe0, int64_t budget,
                                                    RecState *rec, float *trace, int64_t trace_len,
                                                    double *bestx)
{
    __shared__ double sv[256];
    __shared__ int si[256];
    __shared__ int s_copy;
    const int tid = threadIdx.x;
    double v = tid < np ? err_key(eY[tid]) : INFINITY;
    int idx = tid;
    sv[tid] = v;
    si[tid] = idx;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        double ov = INFINITY;
        int oi = 0;
        if (tid >= off) { ov = sv[tid - off]; oi = si[tid - off]; }
        __syncthreads();
        if (tid >= off && ov <= v) { v = ov; idx = oi; }
        sv[tid] = v;
        si[tid] = idx;
        __syncthreads();
    }
    const double before = rec->best;
    __syncthreads();
    if (tid < np && trace) {
        const int64_t c = fe0 + tid + 1;
        if (c % TRACE_EVERY == 0 && c / TRACE_EVERY - 1 < trace_len)
            trace[c / TRACE_EVERY - 1] = (float)fmin(before, v);
    }
    if (tid == 0) {
        const int lim = (int)min<int64_t>((int64_t)np, budget - fe0);
        s_copy = -1;
        if (lim > 0 && sv[lim - 1] < rec->best_b) { rec->best_b = sv[lim - 1]; s_copy = si[lim - 1]; }
        rec->best = fmin(before, sv[np - 1]);
    }
    __syncthreads();
    if (s_copy >= 0)
        for (int j = tid; j < dim; j += 256) bestx[j] = Y[(int64_t)j * ld + s_copy];
}

__global__ void k_rec_init(RecState *rec, float *trace, int64_t trace_len)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) { rec->best = INFINITY; rec->best_b = INFINITY; }
    if (trace && i < trace_len) trace[i] = NAN;
}

__global__ void k_run_finish(const RecState *rec, sevo_run_result *out, int64_t fes, int gens,
                             const double *bestx, int dim, double *best_x_out)
{
    if (threadIdx.x == 0) {
        out->best_e = rec->best_b;
        out->best_e32 = (float)rec->best_b;
        out->success = rec->best_b <= 1e-8 ? 1 : 0;
        out->fes = fes;
        out->generations = gens;
        out->restarts = 0;
    }
    if (best_x_out)
        for (int j = threadIdx.x; j < dim; j += blockDim.x) best_x_out[j] = bestx[j];
}

}  // namespace sevo

using namespace sevo;

namespace {

int check_common(sevo_ctx *ctx, const sevo_problem *prob, int n_runs, int np, int64_t ld,
                 int64_t rs, int min_np, int precision)
{
    if (!prob) return set_error(ctx, SEVO_EINVAL, "problem is NULL");
    if (prob->func < 0 || prob->func >= NFUNC || prob->dim < 2 || prob->dim > MAX_DIM ||
        !(prob->lb < prob->ub))
        return set_error(ctx, SEVO_EINVAL, "invalid problem");
    if (precision != SEVO_FP32 && precision != SEVO_FP64 && precision != SEVO_SPLIT_BF16)
        return set_error(ctx, SEVO_EINVAL, "unknown precision");
    if (n_runs < 1) return set_error(ctx, SEVO_EINVAL, "n_runs < 1");
    if (np < min_np) return set_error(ctx, SEVO_EINVAL, "population too small");
    if (ld < np) return set_error(ctx, SEVO_EINVAL, "ld < np");
    if (ld > MAX_LD) return set_error(ctx, SEVO_EINVAL, "ld > 2^28");
    if (rs < (int64_t)prob->dim * ld) return set_error(ctx, SEVO_EINVAL, "run_stride < dim * ld");
    return SEVO_OK;
}

// Evaluate n_runs populations pop[r] (stride rs) into err[r] (stride ld).
int eval_runs(sevo_ctx *ctx, const sevo_problem *prob, uint32_t inst, int n_runs, int np,
              int64_t ld, int64_t rs, const void *pop, void *err, int precision, hipStream_t s)
{
    InstanceView I;
    int rc = lookup_instance(ctx, prob, inst, &I);
    if (rc) return rc;
    const size_t es = precision == SEVO_FP64 ? sizeof(double) : sizeof(float);
    std::vector<std::pair<EvalDesc, int>> items;
    items.reserve(n_runs);
    for (int r = 0; r < n_runs; ++r) {
        EvalDesc d{};
        d.x = (const char *)pop + (size_t)r * rs * es;
        d.err = (char *)err + (size_t)r * ld * es;
        d.o = I.o;
        d.Mfrag = I.Mfrag;
        d.tab = I.tab;
        d.M64 = I.M64;
        d.Mbf = I.Mbf;
        d.ld = ld;
        d.n = np;
        d.func = prob->func;
        d.dim = prob->dim;
        items.emplace_back(d, r);
    }
    return eval_items(ctx, items, precision, s);
}

template <typename T>
int de_step_t(sevo_ctx *ctx, const sevo_problem *prob, uint32_t inst, const sevo_de_state *st,
              const sevo_de_params *par, int precision, hipStream_t s)
{
    StepGeom g{st->n_runs, st->np, prob->dim, st->ld, st->run_stride, st->run_uid0,
               ctx_seed32(ctx), st->generation};
    const int nb = blocks_for(g);
    if (st->generation == 0) {
        hipLaunchKernelGGL(k_init_pop<T>, dim3(nb), dim3(256), 0, s, g, prob->lb, prob->ub,
                           (T *)st->x, (T *)nullptr, (T *)nullptr);
        if (hipGetLastError() != hipSuccess) return set_error(ctx, SEVO_EDEVICE, "init launch failed");
        return eval_runs(ctx, prob, inst, st->n_runs, st->np, st->ld, st->run_stride, st->x, st->ex,
                         precision, s);
    }
    const int rows = var_slab_rows(prob->dim, st->np, sizeof(T));
    // a whole population takes little LDS, so many workgroups share a CU and
    // short staging chunks (few registers) keep them resident; slabs of a
    // large population stage in one memory round trip each (measured at D =
    // 30: 2048 individuals 245 -> 206 us with 32-element chunks, 200
    // individuals 144 -> 150 us)
    const size_t lds = var_lds_bytes(prob->dim, st->np, rows, sizeof(T));
    // a whole dense population (ld = np) whose runs start on 16-byte
    // boundaries stages as one contiguous array of 16-byte vectors
    const bool flat = rows >= prob->dim && st->ld == st->np && (st->run_stride * sizeof(T)) % 16 == 0 &&
                      ((uintptr_t)st->x) % 16 == 0;
    if (flat)
        hipLaunchKernelGGL((k_de_variation_lds<T, 8, true>), dim3(st->n_runs), dim3(256), lds, s, g,
                           (T)prob->lb, (T)prob->ub, (T)par->F, cr_threshold(par->CR), (const T *)st->x,
                           (T *)st->u, st->donors, rows);
    else if (rows >= prob->dim)
        hipLaunchKernelGGL((k_de_variation_lds<T, 8, false>), dim3(st->n_runs), dim3(256), lds, s, g,
                           (T)prob->lb, (T)prob->ub, (T)par->F, cr_threshold(par->CR), (const T *)st->x,
                           (T *)st->u, st->donors, rows);
    else if (rows > 0)
        hipLaunchKernelGGL((k_de_variation_lds<T, 128 / sizeof(T), false>), dim3(st->n_runs), dim3(256), lds, s, g,
                           (T)prob->lb, (T)prob->ub, (T)par->F, cr_threshold(par->CR), (const T *)st->x,
                           (T *)st->u, st->donors, rows);
    else
        hipLaunchKernelGGL(k_de_variation<T>, dim3(nb), dim3(256), 0, s, g, (T)prob->lb, (T)prob->ub,
                           (T)par->F, cr_threshold(par->CR), (const T *)st->x, (T *)st->u, st->donors);
    if (hipGetLastError() != hipSuccess) return set_error(ctx, SEVO_EDEVICE, "variation launch failed");
    int rc = eval_runs(ctx, prob, inst, st->n_runs, st->np, st->ld, st->run_stride, st->u, st->eu,
                       precision, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_de_select<T>, dim3(nb), dim3(256), 0, s, g, (T *)st->x, (T *)st->ex,
                       (const T *)st->u, (const T *)st->eu, st->replaced);
    if (hipGetLastError() != hipSuccess) return set_error(ctx, SEVO_EDEVICE, "selection launch failed");
    return SEVO_OK;
}

template <typename T>
int pso_step_t(sevo_ctx *ctx, const sevo_problem *prob, uint32_t inst, const sevo_pso_state *st,
               const sevo_pso_params *par, int precision, hipStream_t s)
{
    StepGeom g{st->n_runs, st->np, prob->dim, st->ld, st->run_stride, st->run_uid0,
               ctx_seed32(ctx), st->iteration};
    const int nb = blocks_for(g);
    const int init = st->iteration == 0;
    if (init) {
        hipLaunchKernelGGL(k_init_pop<T>, dim3(nb), dim3(256), 0, s, g, prob->lb, prob->ub,
                           (T *)st->x, (T *)st->v, (T *)st->p);
    } else {
        hipLaunchKernelGGL(k_pso_update<T>, dim3(nb), dim3(256), 0, s, g, (T)prob->lb, (T)prob->ub,
                           (T)par->w, (T)par->c1, (T)par->c2, (T)par->vmax, (T *)st->x, (T *)st->v,
                           (const T *)st->p, (const int32_t *)st->gbest);
    }
    if (hipGetLastError() != hipSuccess) return set_error(ctx, SEVO_EDEVICE, "update launch failed");
    int rc = eval_runs(ctx, prob, inst, st->n_runs, st->np, st->ld, st->run_stride, st->x, st->ex,
                       precision, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_pso_best<T>, dim3(st->n_runs), dim3(256), 0, s, g, init, (const T *)st->x,
                       (const T *)st->ex, (T *)st->p, (T *)st->ep, st->gbest);
    if (hipGetLastError() != hipSuccess) return set_error(ctx, SEVO_EDEVICE, "best launch failed");
    return SEVO_OK;
}

}  // namespace

extern "C" {

int sevo_de_step(sevo_ctx *ctx, const sevo_problem *prob, uint32_t instance, const sevo_de_state *st,
                 const sevo_de_params *par, int32_t precision, void *stream)
{
    if (!ctx) return set_error(nullptr, SEVO_EINVAL, "ctx is NULL");
    if (!st || !par) return set_error(ctx, SEVO_EINVAL, "state or params is NULL");
    int rc = check_common(ctx, prob, st->n_runs, st->np, st->ld, st->run_stride, 4, precision);
    if (rc) return rc;
    if (!st->x || !st->ex) return set_error(ctx, SEVO_EINVAL, "x and ex are required");
    if (st->generation > 0 && (!st->u || !st->eu))
        return set_error(ctx, SEVO_EINVAL, "u and eu are required for generation >= 1");
    if (!std::isfinite(par->F) || !(par->CR >= 0.0 && par->CR <= 1.0))
        return set_error(ctx, SEVO_EINVAL, "F must be finite and CR in [0, 1]");
    DeviceScope dg(ctx);
    if (precision == SEVO_FP64) return de_step_t<double>(ctx, prob, instance, st, par, precision, (hipStream_t)stream);
    return de_step_t<float>(ctx, prob, instance, st, par, precision, (hipStream_t)stream);
}

int sevo_pso_step(sevo_ctx *ctx, const sevo_problem *prob, uint32_t instance, const sevo_pso_state *st,
                  const sevo_pso_params *par, int32_t precision, void *stream)
{
    if (!ctx) return set_error(nullptr, SEVO_EINVAL, "ctx is NULL");
    if (!st || !par) return set_error(ctx, SEVO_EINVAL, "state or params is NULL");
    int rc = check_common(ctx, prob, st->n_runs, st->np, st->ld, st->run_stride, 1, precision);
    if (rc) return rc;
    if (!st->x || !st->v || !st->p || !st->ex || !st->ep || !st->gbest)
        return set_error(ctx, SEVO_EINVAL, "x, v, p, ex, ep and gbest are required");
    if (!std::isfinite(par->w) || !std::isfinite(par->c1) || !std::isfinite(par->c2) || !(par->vmax > 0.0))
        return set_error(ctx, SEVO_EINVAL, "w, c1, c2 must be finite and vmax > 0");
    DeviceScope dg(ctx);
    if (precision == SEVO_FP64) return pso_step_t<double>(ctx, prob, instance, st, par, precision, (hipStream_t)stream);
    return pso_step_t<float>(ctx, prob, instance, st, par, precision, (hipStream_t)stream);
}

}  // extern "C"

// Plain double-precision runs: one run after another, one launch per step.
int sevo::run_plain_f64(sevo_ctx *ctx, const sevo_run_desc *runs, int n, sevo_run_result *results,
                        float *trace, int64_t trace_len, double *best_x, int max_dim, hipStream_t s)
{
    for (int r = 0; r < n; ++r) {
        const sevo_run_desc &d = runs[r];
        const int D = d.prob.dim, np = d.np;
        const int64_t ld = np, rs = (int64_t)D * np;
        const size_t need = sizeof(double) * (size_t)(4 * rs + 3 * ld + D) + sizeof(RecState) + 64 * 4;
        char *ws = nullptr;
        int rc = ctx_ws(ctx).get(ctx, WS_STEP, need, (void **)&ws);
        if (rc) return rc;
        double *X = (double *)ws, *U = X + rs, *V = U + rs, *P = V + rs;
        double *eX = P + rs, *eU = eX + ld, *eP = eU + ld, *bx = eP + ld;
        RecState *rec = (RecState *)(bx + D + 1);
        int32_t *gb = (int32_t *)(rec + 1);
        float *tr = trace ? trace + (int64_t)r * trace_len : nullptr;
        hipLaunchKernelGGL(k_rec_init, dim3((unsigned)((std::max<int64_t>(trace_len, 1) + 255) / 256)), dim3(256), 0, s,
                           rec, tr, trace_len);
        int64_t fe = 0;
        int gens = 0;
        if (d.algo == SEVO_ALGO_DE) {
            sevo_de_state st{1, np, ld, rs, d.run_uid, 0, X, eX, U, eU, nullptr, nullptr};
            sevo_de_params par{d.F, d.CR};
            if ((rc = sevo_de_step(ctx, &d.prob, d.instance, &st, &par, SEVO_FP64, s))) return rc;
            hipLaunchKernelGGL(k_record_f64, dim3(1), dim3(256), 0, s, X, eX, np, D, ld, fe, d.budget, rec, tr,
                               trace_len, bx);
            fe = np;
            while (fe < d.budget && (d.max_generations <= 0 || gens < d.max_generations)) {
                st.generation = (uint32_t)++gens;
                if ((rc = sevo_de_step(ctx, &d.prob, d.instance, &st, &par, SEVO_FP64, s))) return rc;
                // the trials are the generation's evaluations
                hipLaunchKernelGGL(k_record_f64, dim3(1), dim3(256), 0, s, U, eU, np, D, ld, fe, d.budget, rec,
                                   tr, trace_len, bx);
                fe += np;
            }
        } else {
            sevo_pso_state st{1, np, ld, rs, d.run_uid, 0, X, V, P, eX, eP, gb};
            sevo_pso_params par{d.w, d.c1, d.c2, d.vmax};
            for (;;) {
                if ((rc = sevo_pso_step(ctx, &d.prob, d.instance, &st, &par, SEVO_FP64, s))) return rc;
                hipLaunchKernelGGL(k_record_f64, dim3(1), dim3(256), 0, s, X, eX, np, D, ld, fe, d.budget, rec, tr,
                                   trace_len, bx);
                fe += np;
                if (fe >= d.budget || (d.max_generations > 0 && gens >= d.max_generations)) break;
                st.iteration = (uint32_t)++gens;
            }
        }
        hipLaunchKernelGGL(k_run_finish, dim3(1), dim3(64), 0, s, (const RecState *)rec, results + r, fe, gens,
                           (const double *)bx, D, best_x ? best_x + (int64_t)r * max_dim : nullptr);
        if (hipGetLastError() != hipSuccess) return set_error(ctx, SEVO_EDEVICE, "plain run launch failed");
    }
    return SEVO_OK;
}
