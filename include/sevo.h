/*
 * sevo.h -- C ABI of the MI355X (gfx950) batched shifted-rotated evaluation
 * and DE / PSO / SHADE generation library.
 *
 * What the calls compute is the method of "SEvoBench: A C++ Framework For
 * Evolutionary Single-Objective Optimization Benchmarking" (arXiv 2505.17430):
 *   - sevo_evaluate / sevo_evaluate_batch: the fitness evaluation that the
 *     Problem module provides to every algorithm (Sec. 2.3), here for
 *     randomly shifted and rotated instances of six continuous test
 *     functions, many problems / instances / populations per call (the
 *     multiple random instances per problem of Sec. 1 and Sec. 2.3; the
 *     transformed solution vector of Sec. 3.2);
 *   - sevo_de_step: one generation of the DE module (Sec. 2.2, Listing 1's
 *     binomial crossover and midpoint-target repair) with rand/1 mutation and
 *     greedy one-to-one selection;
 *   - sevo_pso_step: one iteration of the PSO module (Sec. 2.2) with the
 *     inertia-weight update and global-best topology;
 *   - sevo_run: the Experiment module's independent runs (Sec. 2.4, Listing
 *     3's evo_bench) for DE, PSO and SHADE (Listing 1) at once, each with a
 *     function-evaluation budget (Listing 4's loop) and the best-so-far
 *     record every 200 evaluations (Sec. 2.4, Sec. 3.2); also L-SHADE, the
 *     SHADE variant with an external archive and population size reduction
 *     that the DE module's archive and reduction mechanisms make (Sec. 2.2,
 *     and the L-SHADE family of Sec. 4), with restarts (L-SHADE-Restart);
 *   - sevo_run_observed: sevo_run with the suite observer that follows the
 *     adaptive parameters muF and muCR through each run (Sec. 4, second case
 *     study, Fig. 9), for JADE and the success-history family.
 *
 * Conventions shared by every call
 *   - Status: every call returns SEVO_OK (0) or a negative SEVO_E* code and
 *     never throws or aborts; sevo_last_error(ctx) returns the message of the
 *     last failure on that context.
 *   - Pointers: "device" pointers are HIP device memory on the context's GPU
 *     (for example torch tensors' data_ptr), "host" pointers are CPU memory.
 *     The caller owns every buffer it passes and keeps it alive until the
 *     work on `stream` has finished.  Descriptor structs are read during the
 *     call only.
 *   - Streams: `stream` is a hipStream_t (NULL = the default stream).  Calls
 *     are asynchronous on that stream unless stated otherwise; device faults
 *     surface as SEVO_EDEVICE from a later call or from sevo_sync.
 *   - Layout: populations are structure-of-arrays.  Coordinate d of point i
 *     is at x[d * ld + i] (the point index is the fast one, so a wavefront
 *     reads consecutive points of one coordinate).  Batched runs add a run
 *     stride: x[r * run_stride + d * ld + i].
 *   - Values: device fitness is the error e = f(x) - f*, never f itself, so
 *     single precision keeps its resolution near the optimum.
 *   - Threads: a context is not thread-safe; use one per host thread.
 */
#ifndef SEVO_H
#define SEVO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define SEVO_OK            0
#define SEVO_EINVAL       -1   /* bad argument: null pointer, size, enum, bounds   */
#define SEVO_ENOMEM       -2   /* host or device allocation failed                 */
#define SEVO_EDEVICE      -3   /* HIP runtime error (message carries its string)   */
#define SEVO_EUNSUPPORTED -4   /* valid request this build does not implement      */
#define SEVO_ESTATE       -5   /* call out of order (e.g. step before init)        */

/* ---- test functions: e(x) = f(x) - f*, z = M (x - o), indices 1..D ----
 * ELLIPSOID   sum 10^(6(i-1)/(D-1)) z_i^2                       (condition 1e6)
 * ROSENBROCK  sum_{i<D} 100 (w_i^2 - w_{i+1})^2 + (w_i - 1)^2,  w = z + 1
 * RASTRIGIN   sum z_i^2 - 10 cos(2 pi z_i) + 10
 * SCHWEFEL    sum g(z_i + s), g(u) = c - u sin(sqrt|u|) for |u| <= 500,
 *             g(u) = g(+-500) + 0.01 (|u| - 500)^2 beyond; s = 420.968746...,
 *             c = s sin(sqrt s) = 418.98288727... so that g(s) = 0
 * GRIEWANK    1 + sum z_i^2 / 4000 - prod cos(z_i / sqrt(i))
 * ACKLEY      -20 exp(-0.2 sqrt(sum z^2 / D)) - exp(sum cos(2 pi z) / D) + 20 + e
 */
enum { SEVO_ELLIPSOID = 0, SEVO_ROSENBROCK = 1, SEVO_RASTRIGIN = 2, SEVO_SCHWEFEL = 3,
       SEVO_GRIEWANK = 4, SEVO_ACKLEY = 5 };

/* Arithmetic of the evaluation.  FP32: FP64 shift, FP32 rotation on matrix
 * cores, compensated FP32 reduction; state and errors are float.
 * SPLIT_BF16: as FP32 but the rotation runs on the bf16 matrix cores with
 * FP32 accumulation: for D > 120 each float is split into two bf16 terms
 * and three products are kept (hi*hi + hi*lo + lo*hi); for 65 <= D <= 112
 * into three terms with the six products down to order 2^-16, the
 * coordinates past the last multiple of 32 on the FP32 matrix cores; other
 * D as FP32.  Both meet the evaluation tolerance.  FP64: everything in
 * double; state and errors are double. */
enum { SEVO_FP64 = 0, SEVO_FP32 = 1, SEVO_SPLIT_BF16 = 2 };

enum { SEVO_ALGO_DE = 0, SEVO_ALGO_PSO = 1, SEVO_ALGO_SHADE = 2, SEVO_ALGO_LSHADE = 3, SEVO_ALGO_PSODE = 4,
       SEVO_ALGO_CSO = 5, SEVO_ALGO_JADE = 6, SEVO_ALGO_LSHADE_RS = 7 };

typedef struct sevo_ctx sevo_ctx;   /* opaque, library-owned */

/* A problem: function, dimension, box [lb, ub]^D and optimum value f*.
 * (problem, instance) determines (o, M) deterministically from the
 * context's instance seed. */
typedef struct {
    int32_t func;
    int32_t dim;       /* 2 .. 1024 */
    double lb, ub;     /* lb < ub; populations live in [lb, ub]^dim */
    double f_star;     /* added only on output in double; 100 in the workloads */
} sevo_problem;

/* ---- context ---- */

/* Create a context on HIP device `hip_device`.  `base_seed` keys every
 * algorithm draw (Philox key word 1, low and high 32 bits xor-folded);
 * `instance_seed` keys the instance generator.  *out receives the context. */
int sevo_create(sevo_ctx **out, int32_t hip_device, uint64_t base_seed, uint64_t instance_seed);

/* Destroy the context and free everything it owns (instance cache, internal
 * workspaces).  Waits for the context's outstanding work. */
int sevo_destroy(sevo_ctx *ctx);

/* Message of the last failed call on ctx ("" if none).  Valid until the next
 * call on ctx.  Accepts NULL (then describes the last sevo_create failure). */
const char *sevo_last_error(const sevo_ctx *ctx);

/* Block until all work queued by this library on `stream` has finished and
 * report any asynchronous device error as SEVO_EDEVICE. */
int sevo_sync(sevo_ctx *ctx, void *stream);

/* ---- instances ---- */

/* Copy the instance (o, M) of (problem, instance) to host buffers
 * o_host[dim] and M_host[dim*dim] (row-major; z = M (x - o)).  Either may
 * be NULL.  The instance is generated on first use: o_j = -80 + 160 u,
 * u a 53-bit Philox uniform; M = Q of the Householder QR of a Philox /
 * Box-Muller N(0,1) matrix with diag(R) > 0.  Synchronous. */
int sevo_instance(sevo_ctx *ctx, const sevo_problem *prob, uint32_t instance,
                  double *o_host, double *M_host);

/* The same instance computed on the host only, without a context or a GPU
 * (for callers that evaluate elsewhere).  Synchronous; o_host[dim],
 * M_host[dim*dim] are required. */
int sevo_generate_instance(int32_t func, int32_t dim, uint32_t instance, uint64_t instance_seed,
                           double *o_host, double *M_host);

/* Register a user-defined instance for (problem, instance), replacing the
 * generated one (a user-defined problem, Sec. 2.3): o_host[dim] and
 * M_host[dim*dim] are copied; M need not be orthogonal.  Synchronous. */
int sevo_set_instance(sevo_ctx *ctx, const sevo_problem *prob, uint32_t instance,
                      const double *o_host, const double *M_host);

/* ---- evaluation ---- */

/* Errors of n points of one (problem, instance).
 *   x       device, [dim][ld] structure-of-arrays, float (FP32, SPLIT_BF16)
 *           or double (FP64); n <= ld <= 2^28.
 *   err_out device, [n], float or double like x: e = f(x) - f*.
 * n = 0 is a no-op.  Asynchronous on `stream`. */
int sevo_evaluate(sevo_ctx *ctx, const sevo_problem *prob, uint32_t instance,
                  const void *x, int64_t ld, int32_t n, void *err_out,
                  int32_t precision, void *stream);

/* Many (problem, instance, population) items in one launch sequence.  Items
 * may mix functions, dimensions and instances; each item is evaluated as by
 * sevo_evaluate.  `items` is a host array read during the call. */
typedef struct {
    sevo_problem prob;
    uint32_t instance;
    int32_t n;
    int64_t ld;           /* n <= ld <= 2^28 */
    const void *x;        /* device */
    void *err_out;        /* device */
} sevo_eval_item;

int sevo_evaluate_batch(sevo_ctx *ctx, const sevo_eval_item *items, int32_t n_items,
                        int32_t precision, void *stream);

/* sevo_evaluate_batch for callers that cannot allocate device memory (code
 * under stream capture, serving loops, harnesses that forbid hipMalloc): the
 * call allocates nothing.  Its descriptor tables go to a fixed device array
 * of the library, 1 MiB per GPU (about 16,000 items of 64 B plus 4 B per
 * tile of 64 to 128 points), held by every GPU the library runs on until the
 * process ends and shared by every call on that GPU: calls that overlap on
 * one GPU (other streams, other contexts) race on it; calls on one stream
 * are ordered.  Results are those of sevo_evaluate_batch, bit for bit.
 * Limits, each a clear error and nothing enqueued:
 *   - every item's instance must already be resident on the context (made by
 *     sevo_instance, sevo_set_instance or an earlier evaluation or run):
 *     otherwise SEVO_ESTATE;
 *   - precision FP32 or SPLIT_BF16 takes D <= 120 only (larger D needs the
 *     GEMM workspace): otherwise SEVO_EUNSUPPORTED; FP64 takes any D;
 *   - tables beyond the array's 1 MiB: SEVO_EINVAL.
 * The host tables are copied with hipMemcpyAsync on `stream`.  Asynchronous. */
int sevo_evaluate_batch_noalloc(sevo_ctx *ctx, const sevo_eval_item *items, int32_t n_items,
                                int32_t precision, void *stream);

/* Autotuning of the batched evaluation (optional).  For every dimension
 * class (k-steps ceil(D/4), D <= 120) present in `items`, times the launch
 * shapes that cannot change any result -- 1, 2, 3, 4, 6 or 8 tiles of
 * 64-256 points per workgroup, and the resident persistent grid -- on these
 * items (their err_out buffers are written, with the values
 * sevo_evaluate_batch gives), and keeps in the context for later calls the
 * first shape in that order whose time is within 2 % of the fastest (fewer
 * tiles per workgroup move fewer bytes).
 *   chosen  optional host [64]: per class, the tiles per workgroup chosen
 *           (0 = resident grid), -1 for classes not present.
 * Synchronises `stream`.  FP64 has nothing to tune (returns 0). */
int sevo_tune_evaluate(sevo_ctx *ctx, const sevo_eval_item *items, int32_t n_items, int32_t precision,
                       void *stream, int32_t *chosen);

/* ---- one generation at a time ---- */

/* State of `n_runs` runs of one (problem, instance): run r uses Philox key
 * run_uid0 + r.  All buffers are device memory of the precision's type
 * (float for FP32 / SPLIT_BF16, double for FP64), laid out as
 * buf[r * run_stride + d * ld + i] for populations and buf[r * ld + i] for
 * per-individual values.  `generation` is the counter t of the step being
 * made: 0 initialises (x uniform in the box, evaluated), t >= 1 makes
 * generation t from generation t - 1. */
typedef struct {
    int32_t n_runs;
    int32_t np;            /* population size, >= 4 */
    int64_t ld;            /* np <= ld <= 2^28 */
    int64_t run_stride;    /* >= dim * ld */
    uint32_t run_uid0;
    uint32_t generation;
    void *x;               /* in/out population                              */
    void *ex;              /* in/out errors of x                             */
    void *u;               /* out: trial vectors of this generation          */
    void *eu;              /* out: errors of the trials                      */
    int32_t *donors;       /* optional out, [r][4][ld]: r1, r2, r3, jrand     */
    uint8_t *replaced;     /* optional out, [r][ld]: 1 where the trial won    */
} sevo_de_state;

typedef struct {
    double F;              /* scale factor */
    double CR;             /* crossover rate; mask bit j is u_j < CR or j = jrand */
} sevo_de_params;

/* One DE rand/1/bin generation (t >= 1): donors r1, r2, r3 distinct and
 * != i, v = x_r1 + F (x_r2 - x_r3), binomial crossover with a forced jrand
 * coordinate, out-of-box coordinates repaired to the midpoint between the
 * bound and the parent coordinate, trials evaluated, then every trial
 * replaces its parent when e(u) <= e(x) (NaN counts as +infinity).
 * generation = 0 initialises x and ex instead.  Asynchronous. */
int sevo_de_step(sevo_ctx *ctx, const sevo_problem *prob, uint32_t instance,
                 const sevo_de_state *st, const sevo_de_params *par,
                 int32_t precision, void *stream);

typedef struct {
    int32_t n_runs;
    int32_t np;            /* swarm size, >= 1 */
    int64_t ld;            /* np <= ld <= 2^28 */
    int64_t run_stride;
    uint32_t run_uid0;
    uint32_t iteration;    /* 0 initialises; t >= 1 makes iteration t */
    void *x, *v, *p;       /* in/out positions, velocities, personal bests   */
    void *ex, *ep;         /* out errors of x; in/out errors of p             */
    int32_t *gbest;        /* in/out, device [n_runs]: index of the best p    */
} sevo_pso_state;

typedef struct {
    double w, c1, c2;      /* inertia, cognitive and social weights */
    double vmax;           /* |v_j| <= vmax */
} sevo_pso_params;

/* One synchronous PSO iteration (t >= 1): per coordinate
 * v = w v + c1 r1 (p - x) + c2 r2 (g - x) with r1, r2 uniform draws,
 * |v| clamped to vmax, x += v, a coordinate leaving the box is put on the
 * bound with its velocity zeroed; x evaluated; p replaced where
 * e(x) < e(p); gbest = argmin e(p), lowest index on ties.  iteration = 0
 * initialises x uniform, v = 0, p = x.  Asynchronous. */
int sevo_pso_step(sevo_ctx *ctx, const sevo_problem *prob, uint32_t instance,
                  const sevo_pso_state *st, const sevo_pso_params *par,
                  int32_t precision, void *stream);

/* ---- whole runs ---- */

typedef struct {
    sevo_problem prob;
    uint32_t instance;
    uint32_t run_uid;      /* Philox key word 0 of the run */
    int32_t algo;          /* SEVO_ALGO_* */
    int32_t np;            /* population / swarm size (CSO: even, 2 .. 1024) */
    int64_t budget;        /* function evaluations; whole generations are run */
    double F, CR;          /* DE */
    double w, c1, c2, vmax;/* PSO, PSODE; CSO: c1 = phi, the pull towards the swarm mean */
    double p;              /* SHADE, L-SHADE, PSODE, JADE: pbest fraction (top max(2, round(p NP))) */
    int32_t H;             /* SHADE, L-SHADE, PSODE: memory size (1 .. 16) */
    double r_arc;          /* L-SHADE, JADE: archive bound round(r_arc NP), 0 .. 2.9 (2.6 in L-SHADE,
                              1 in JADE) */
    int32_t np_min;        /* L-SHADE: population size at the budget, 4 .. np */
    int32_t topology;      /* PSO, PSODE: 0 global best, 1 ring {i-1, i, i+1} (FP32 runs) */
    int32_t velocity;      /* PSO, PSODE: 0 inertia weight, 1 spherical (SPSO-2011; FP32 runs) */
    int32_t max_generations; /* stop after this many generations (0: run to the budget); the budget
                              still sets L-SHADE's size schedule, so a run stopped early is the same
                              run up to that generation */
    double c;              /* JADE: adaptation rate of muF and muCR, 0 .. 1 (0.1 in JADE) */
    double restart_tol;    /* L-SHADE-Restart: restart once max e - min e over the population <= this */
} sevo_run_desc;

typedef struct {
    double best_e;         /* error of the best of the first `budget` evaluations;
                              recomputed in double on the GPU once below 1e-6 */
    float best_e32;        /* the same best as the single-precision path saw it */
    int32_t success;       /* best_e <= 1e-8 */
    int64_t fes;           /* evaluations made (the last generation may overshoot) */
    int32_t generations;   /* generations after initialisation */
    int32_t restarts;      /* L-SHADE-Restart: restarts made (0 for the others) */
} sevo_run_result;

/* Run n_runs independent runs to their budgets in persistent fused kernels
 * (precision FP32: single-precision state, double-precision shift and final
 * check; FP64: everything double, DE and global-best inertia PSO only;
 * SPLIT_BF16: CSO runs only, their evaluation with split-bf16 rotation).
 *   PSO variants (the PSO module's topology and velocity update, Listing 1):
 *   ring topology takes each particle's best personal best among
 *   {i-1, i, i+1} (mod np; lowest index on ties) in place of the global best;
 *   the spherical update (SPSO-2011) moves to a point drawn uniformly in the
 *   ball centred at G = (x + p' + l') / 3 (or (x + p') / 2 when the particle
 *   is its own neighbourhood best), p' = x + c1 (p - x), l' = x + c1 (l - x),
 *   of radius |G - x|: v = w v + x' - x; vmax and the box as for the inertia
 *   update.
 *   L-SHADE (Tanabe and Fukunaga, CEC 2014): SHADE's draws (a terminal CR
 *   memory gives CR = 0) with r2 from the population and the archive; every
 *   strictly improved parent enters the archive in index order (appended
 *   below round(r_arc NP), else written over a random member); both memories
 *   take the weighted Lehmer mean, the CR memory becoming terminal when all
 *   successful CR are 0; after each generation the population shrinks to
 *   round((np_min - np) FE / budget + np) by dropping the worst (the rest keep
 *   their order) and the archive to its new bound by random removals.
 *   PSODE (the PSO/DE hybrid with pairwise/3 selection, Sec. 4, Listing 4;
 *   FP32 runs, np >= 4): each generation moves a copy of the population by
 *   the PSO update above (topology, velocity; the population serves as the
 *   personal bests) and evaluates it, runs one SHADE generation on the
 *   population, sets the velocities to the DE displacement (trial minus
 *   parent where the trial won, else 0) and keeps per individual the PSO
 *   move where strictly better than the DE result.  2 np evaluations per
 *   generation, recorded as the PSO moves, then the DE trials; velocities
 *   start at 0.
 *   L-SHADE-Restart (SEVO_ALGO_LSHADE_RS; the state-triggered restart of
 *   the case study's L-SHADE family, Sec. 4): L-SHADE that, after a
 *   generation leaving budget, restarts once its population has converged
 *   (max e - min e over it <= restart_tol; NaN counts as +infinity, so it
 *   never converges): restart k = 1, 2, ... draws a fresh population of np
 *   (the initial draws with the last Philox counter word k), evaluates and
 *   records it, resets the memories to 0.5 and empties the archive, and the
 *   size schedule starts over from np at that point to np_min at the
 *   budget.  The best-so-far record spans all restarts.
 *   JADE (Zhang and Sanderson 2009; the algorithm of the parameter
 *   observer case study, Sec. 4; FP32 runs, np >= 4): L-SHADE's generation
 *   with one parameter pair (muF, muCR) in place of the memory (H is
 *   ignored), no population reduction (np_min is ignored) and the archive
 *   bound round(r_arc np); after each generation muCR <- (1 - c) muCR +
 *   c mean(S_CR) and muF <- (1 - c) muF + c sum(S_F^2) / sum(S_F), plain
 *   means over the strictly improved individuals (no change when none).
 *   CSO (the competitive swarm optimizer of the large-scale study, Sec. 3.3;
 *   precision FP32 or SPLIT_BF16, any D up to 1024): per iteration the
 *   swarm is paired at random (ascending Philox key), the lower error of a
 *   pair wins (ties: lower index), the winner stays and the loser moves by
 *   v = r1 v + r2 (x_w - x_l) + phi r3 (xbar - x_l), x_l += v (xbar the swarm
 *   mean, the box as for PSO); the np/2 losers are evaluated (recorded in
 *   pair order).  Each iteration is an update launch and the batched
 *   evaluation of all CSO runs' losers; velocities start at 0.
 *   results  device, [n_runs] sevo_run_result.
 *   trace    optional device [n_runs][trace_len] float: best error after
 *            200 (k+1) evaluations, NaN where the run made fewer.
 *   best_x   optional device [n_runs][max_dim] double: best point.
 * Asynchronous on `stream`. */
int sevo_run(sevo_ctx *ctx, const sevo_run_desc *runs, int32_t n_runs, int32_t precision,
             sevo_run_result *results, float *trace, int64_t trace_len,
             double *best_x, int32_t max_dim, void *stream);

/* sevo_run with the parameter observer of the second case study (Sec. 4,
 * Fig. 9: the adaptive muF and muCR of JADE followed through a run).
 *   mu       optional device [n_runs][mu_len][2] float: (muF, muCR) after g
 *            generations in row g (row 0: the initial values), NaN for
 *            generations the run did not make.  JADE: its parameter pair;
 *            SHADE, L-SHADE, PSODE: the means of the H memory slots (a
 *            terminal CR slot counts as 0, the CR it gives); DE: its fixed
 *            F and CR; PSO: NaN.
 *   mu_len   rows per run, >= 0 (0: no observer, as sevo_run).
 * Precision FP32 only (the fused kernels), and no CSO runs: otherwise
 * SEVO_EUNSUPPORTED.  Everything else as sevo_run.  Asynchronous. */
int sevo_run_observed(sevo_ctx *ctx, const sevo_run_desc *runs, int32_t n_runs, int32_t precision,
                      sevo_run_result *results, float *trace, int64_t trace_len, double *best_x,
                      int32_t max_dim, float *mu, int64_t mu_len, void *stream);

/* The state of each run when it stops (its budget or max_generations
 * reached): the population, its errors and the adaptive state the next
 * generation would start from.  Arrays are device memory owned by the
 * caller, indexed by the run's position in `runs`; rows are max_np long
 * and only a run's first np entries of a row are written (the rest keep
 * their contents).  Populations are structure-of-arrays like every
 * population of this library: coordinate d of individual i of run r is at
 * [(r * max_dim + d) * max_np + i].
 *   x, e     required: the population (PSO: the positions) and its errors.
 *   u, eu    optional: the trials of the last generation and their errors
 *            (DE, SHADE, L-SHADE, JADE, L-SHADE-Restart; PSODE: the DE
 *            half's); not written for PSO or for a run that made no
 *            generation.
 *   v        optional: velocities (PSO, PSODE).
 *   p, ep    optional: personal bests and their errors (PSO).
 *   memory   optional [n_runs][32]: M_F[0..H-1] at 0..15 and M_CR[0..H-1]
 *            at 16..31 (SHADE, L-SHADE, L-SHADE-Restart, PSODE; JADE: muF,
 *            muCR in slot 0; a terminal CR slot holds -1).
 *   archive  optional [n_runs][max_dim][max_arc]: the archive members
 *            (L-SHADE, JADE, L-SHADE-Restart), member a of coordinate d at
 *            [(r * max_dim + d) * max_arc + a].
 *   counts   optional [n_runs][4]: the population size when the run stopped
 *            (L-SHADE shrinks it), the archive size, the next memory slot
 *            to be written, and the global best index (PSO and PSODE with
 *            the global-best topology; 0 otherwise). */
typedef struct {
    int32_t max_np;        /* >= every run's np */
    int32_t max_dim;       /* >= every run's dim */
    int32_t max_arc;       /* >= round(r_arc np) of every archive run when `archive` is set */
    int32_t reserved;      /* 0 */
    float *x, *e;
    float *u, *eu;
    float *v;
    float *p, *ep;
    float *memory;
    float *archive;
    int32_t *counts;
} sevo_run_state;

/* sevo_run that also writes each run's final state to `state` (to continue
 * or inspect runs, and to compare them generation by generation with another
 * implementation).  Precision FP32, fused runs only (no CSO runs): otherwise
 * SEVO_EUNSUPPORTED.  Everything else as sevo_run.  Asynchronous. */
int sevo_run_snapshot(sevo_ctx *ctx, const sevo_run_desc *runs, int32_t n_runs, int32_t precision,
                      sevo_run_result *results, float *trace, int64_t trace_len, double *best_x,
                      int32_t max_dim, const sevo_run_state *state, void *stream);

/* ---- plans: work prepared once, then enqueued with launches only ----
 *
 * A plan holds everything a call needs on the device -- instances,
 * descriptor tables, workspace and launch shapes -- so that enqueueing it
 * allocates nothing, copies nothing and never waits on the host.  That makes
 * sevo_plan_launch safe to capture into a HIP graph (stream capture) and to
 * replay the graph, and cheap to call in a loop.  The buffers named when the
 * plan was made (points, errors, results, traces) are read and written by
 * every launch and must stay allocated while the plan is used; their
 * contents may change between launches.  Launches of one plan must not
 * overlap in time (they share the plan's workspace); different plans may.
 * A plan belongs to its context and must be destroyed before it. */
typedef struct sevo_plan sevo_plan;   /* opaque, library-owned */

/* The evaluation of `items`, as sevo_evaluate_batch (launch shapes: the
 * context's autotuned ones, else the defaults).  Synchronous. */
int sevo_plan_evaluate(sevo_ctx *ctx, const sevo_eval_item *items, int32_t n_items, int32_t precision,
                       sevo_plan **out);

/* Whole runs, as sevo_run with precision SEVO_FP32 (the persistent fused
 * kernels; the double-precision path is a host loop of launches and has no
 * plan: SEVO_EUNSUPPORTED).  Every launch restarts the runs from generation
 * 0 and rewrites results, trace and best_x.  Synchronous. */
int sevo_plan_run(sevo_ctx *ctx, const sevo_run_desc *runs, int32_t n_runs, int32_t precision,
                  sevo_run_result *results, float *trace, int64_t trace_len, double *best_x,
                  int32_t max_dim, sevo_plan **out);

/* Enqueue the plan's kernels on `stream` (the context's internal streams
 * join through events when a plan has concurrent launches).  Asynchronous. */
int sevo_plan_launch(sevo_plan *plan, void *stream);

/* Free the plan's device memory (waits for the device first).  NULL is a
 * no-op. */
int sevo_plan_destroy(sevo_plan *plan);

#ifdef __cplusplus
}
#endif
#endif /* SEVO_H */
