/*
 * oracle.h -- plain, slow FP64 CPU oracle for the batched shifted-rotated
 * evaluation and the DE / PSO / SHADE generation steps.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this code; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the GPU path: the
 * Philox generator, the instance generator, the six objective functions and
 * the algorithm steps are written here a second time, from their published
 * definitions, in double precision, with no blocking or fusion.
 *
 * Layout: populations are individual-major, x[i*dim + j] (the obvious CPU
 * layout).  Matrices are row-major.  All floating point is double; the
 * library is compiled with -O2 -ffp-contract=off and no fast-math.
 *
 * Parity pins (see tests/test_oracle_*.py): Philox known-answer vectors;
 * orthogonality, det and LAPACK-QR uniqueness of the rotation; f(o) = f*
 * exactly; textbook closed forms at M = I, o = 0; high-precision textbook
 * definitions at random points; D = 2 brute-force grid minima; exhaustive
 * donor enumeration; DE/PSO/SHADE invariants; resume bit-identity.
 */
#ifndef SEVO_ORACLE_H
#define SEVO_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Function identifiers (same numbering as the product ABI, by definition). */
enum { ORC_ELLIPSOID = 0, ORC_ROSENBROCK = 1, ORC_RASTRIGIN = 2,
       ORC_SCHWEFEL = 3, ORC_GRIEWANK = 4, ORC_ACKLEY = 5, ORC_NFUNC = 6 };
enum { ORC_ALGO_DE = 0, ORC_ALGO_PSO = 1, ORC_ALGO_SHADE = 2, ORC_ALGO_LSHADE = 3, ORC_ALGO_PSODE = 4,
       ORC_ALGO_CSO = 5, ORC_ALGO_JADE = 6, ORC_ALGO_LSHADE_RS = 7 };

/* Philox stream tags (third counter word, bits 24..31). */
enum { ORC_TAG_INIT_X = 1, ORC_TAG_DONORS = 2, ORC_TAG_CROSS = 3,
       ORC_TAG_PSO_R = 4, ORC_TAG_SHADE_P = 5, ORC_TAG_SHADE_C = 6,
       ORC_TAG_SHADE_D = 7, ORC_TAG_LSHADE_A = 8, ORC_TAG_LSHADE_S = 9,
       ORC_TAG_PSO_S = 10, ORC_TAG_PSO_SR = 11, ORC_TAG_CSO_PAIR = 12, ORC_TAG_CSO_R = 13,
       ORC_TAG_SHIFT_O = 16, ORC_TAG_ROT_N = 17 };

typedef struct {
    int32_t func;
    int32_t dim;
    double lb, ub;
} orc_problem;

/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Uniform and integer maps of 32-bit words. */
double   orc_u24(uint32_t w);                 /* (w >> 8) * 2^-24, in [0, 1)      */
double   orc_u53(uint32_t a, uint32_t b);     /* 53-bit uniform in [0, 1)         */
uint32_t orc_range(uint32_t w, uint32_t n);   /* floor(w * n / 2^32), in [0, n)   */
uint32_t orc_cr_threshold(double cr);         /* ceil(cr * 2^24), clamped to [0, 2^24] */

/* Instance (o, M) of (func, dim, instance); G (optional) receives the
 * Gaussian matrix before orthogonalisation.  Returns 0 or -1. */
int orc_instance(int32_t func, int32_t dim, uint32_t instance, uint64_t inst_seed,
                 double *o, double *M, double *G);

/* Householder QR of the n x n row-major matrix A; Q gets the orthogonal
 * factor with every diagonal entry of R made positive. */
int orc_householder_q(int32_t n, const double *A, double *Q);

/* Error e = f(x) - f* for one point, and for n points stored as
 * single-precision structure-of-arrays X[j*ld + i] (the GPU state type),
 * widened exactly. */
double orc_error(int32_t func, int32_t dim, const double *o, const double *M, const double *x);
void   orc_error_soa_f32(int32_t func, int32_t dim, const double *o, const double *M,
                         const float *X, int64_t ld, int32_t n, double *e);
void   orc_error_aos(int32_t func, int32_t dim, const double *o, const double *M,
                     const double *X, int32_t n, double *e);
/* Error as a function of the rotated vector z (M and o already applied). */
double orc_error_z(int32_t func, int32_t dim, const double *z);

/* ---- Differential evolution, rand/1/bin with midpoint-target repair ---- */
/* Population of restart k: as orc_init_population with the last counter
 * word k (k = 0 is the initial population). */
void orc_restart_population(const orc_problem *pb, int32_t np, uint32_t run_uid, uint64_t seed, uint32_t k,
                            double *X);
/* 1 when max e - min e over e[0..n) <= tol (NaN counts as +infinity). */
int orc_converged(const double *e, int32_t n, double tol);
/* Population initialisation (generation 0): X[i*dim + j] = lb + (ub-lb) u24. */
void orc_init_population(const orc_problem *pb, int32_t np, uint32_t run_uid,
                         uint64_t seed, double *X);

/* Donor indices (r1, r2, r3) and jrand from four raw words: r1 uniform over
 * the NP-1 indices other than i, r2 over the NP-2 others left, r3 over the
 * NP-3 left, each drawn once and stepped past the excluded indices. */
void orc_donors_from_words(int32_t np, int32_t dim, int32_t i, const uint32_t w[4],
                           int32_t out[4]);
/* Donor indices and jrand for individual i of generation t (rand/1). */
void orc_de_donors(int32_t np, int32_t dim, int32_t i, uint32_t run_uid, uint64_t seed,
                   uint32_t t, int32_t out[4]);

/* One synchronous generation.  Inputs X, eX; outputs trial U, eU and the
 * next population Xn, eXn (Xn may alias nothing).  Optional outputs
 * (NULL to skip): donors[i*4 + k], mask[i*dim + j], replaced[i]. */
int orc_de_generation(const orc_problem *pb, const double *o, const double *M,
                      int32_t np, double F, double CR, uint32_t run_uid, uint64_t seed,
                      uint32_t t, const double *X, const double *eX,
                      double *U, double *eU, double *Xn, double *eXn,
                      int32_t *donors, uint8_t *mask, uint8_t *replaced);

/* ---- PSO, inertia weight, global-best topology ---- */
int orc_pso_init(const orc_problem *pb, const double *o, const double *M, int32_t np,
                 uint32_t run_uid, uint64_t seed, double *X, double *V, double *P,
                 double *eX, double *eP, int32_t *g);
int orc_pso_iteration(const orc_problem *pb, const double *o, const double *M, int32_t np,
                      double w, double c1, double c2, double vmax,
                      uint32_t run_uid, uint64_t seed, uint32_t t,
                      double *X, double *V, double *P, double *eX, double *eP, int32_t *g);

/* ---- PSO variants of the PSO module (Listing 1's spherical velocity update
 * with ring topology) ----
 * topology 0: global best; 1: ring, the neighbourhood of i being
 * {i-1, i, i+1} (mod np) and l_i its best personal best (lowest index among
 * equal errors).  velocity 0: inertia weight, v = w v + c1 r1 (p - x) +
 * c2 r2 (p_l - x); velocity 1: spherical (SPSO-2011, Clerc): with
 * p' = x + c1 (p - x), l' = x + c1 (p_l - x), the centre G = (x + p' + l') / 3,
 * or (x + p') / 2 when l_i = i; x' uniform in the ball of centre G and
 * radius |G - x| (Gaussian direction, radius |G - x| u^(1/D)); v = w v + x' - x.
 * Both: |v_j| <= vmax, x += v, a coordinate leaving the box is put on the
 * bound with its velocity zeroed; pbest on strict improvement.
 * Draws: inertia as orc_pso_iteration (tag PSO_R); spherical: tag PSO_S
 * block b gives the normals of dimensions 2b, 2b+1 by Box-Muller on
 * (u24(w0), u24(w1)), tag PSO_SR word 0 the radius uniform. */
int orc_pso_variant_iteration(const orc_problem *pb, const double *o, const double *M, int32_t np,
                              int32_t topology, int32_t velocity, double w, double c1, double c2,
                              double vmax, uint32_t run_uid, uint64_t seed, uint32_t t,
                              double *X, double *V, double *P, double *eX, double *eP, int32_t *lbest);

/* ---- SHADE (success-history adaptation, current-to-pbest/1, no archive) ---- */
/* Per-individual draws: idx[i*6 + k] = (memory slot, pbest index, r1, r2,
 * jrand, Cauchy retries); F[i], CR[i]; sorted[] = ranking used for pbest;
 * margin[i*2 + 0] = smallest |F candidate| seen (distance of the F > 0
 * decisions from their threshold), margin[i*2 + 1] = smallest distance, in
 * units of 2^-24, between a crossover uniform and CR (jrand excluded).  All
 * optional outputs may be NULL. */
int orc_shade_generation(const orc_problem *pb, const double *o, const double *M,
                         int32_t np, double p, int32_t H, double *MF, double *MCR,
                         int32_t *pos, uint32_t run_uid, uint64_t seed, uint32_t t,
                         const double *X, const double *eX,
                         double *U, double *eU, double *Xn, double *eXn,
                         int32_t *idx, double *F, double *CR, double *margin,
                         uint8_t *mask, uint8_t *replaced, int32_t *sorted);
/* Memory update from the successful set (F, CR, improvement delta). */
void orc_shade_memory_update(int32_t H, double *MF, double *MCR, int32_t *pos,
                             int32_t n_s, const double *SF, const double *SCR,
                             const double *dS);
int32_t orc_shade_pnum(double p, int32_t np);

/* ---- L-SHADE (Tanabe & Fukunaga, CEC 2014): SHADE with an external
 * archive of replaced parents, linear population size reduction and the
 * weighted Lehmer mean for both memories (a terminal CR memory, stored as a
 * negative value, gives CR = 0) ----
 *
 * State of one run.  X / eX hold the current np individuals (individual-
 * major, rows beyond np unused); A the na archived parents (capacity acap).
 * One generation: ranking by (error, index); per individual the SHADE draws
 * (memory slot, CR, F with Cauchy retries, pbest among the top
 * max(2, round(p np)), r1 in P \ {i}, r2 in P u A \ {i, r1} -- values at or
 * above np index the archive -- and jrand); current-to-pbest/1, binomial
 * crossover, midpoint repair; evaluation; selection (e(u) <= e(x)); every
 * strictly improved parent enters the archive, in index order: appended
 * while the archive holds fewer than round(r_arc np) members, else written
 * over the member at range(w, that bound), w from tag LSHADE_A; memory
 * update; then reduction to np_next individuals (the best by (error,
 * index), kept in index order) and the archive cut to round(r_arc np_next)
 * by removing random members (k-th removal: position range(w, na) with w
 * from tag LSHADE_S and counter (t, k), the last member moved into it).
 * U / eU receive the np trials and their errors. */
typedef struct {
    int32_t np, na, acap, H, pos;
    double *X, *eX, *A;
    double MF[64], MCR[64];
} orc_lshade_state;

/* Population size after `fe` of `budget` evaluations:
 * round((np_min - np_init) fe / budget + np_init), within [np_min, np_init]. */
int32_t orc_lshade_np(int32_t np_init, int32_t np_min, int64_t budget, int64_t fe);
/* Archive bound round(r_arc np). */
int32_t orc_lshade_archive_max(double r_arc, int32_t np);
int orc_lshade_generation(const orc_problem *pb, const double *o, const double *M, orc_lshade_state *s,
                          double p, double r_arc, int32_t np_next, uint32_t run_uid, uint64_t seed,
                          uint32_t t, double *U, double *eU, int32_t *n_success);
/* Memory update of L-SHADE from the successful set. */
void orc_lshade_memory_update(int32_t H, double *MF, double *MCR, int32_t *pos, int32_t n_s,
                              const double *SF, const double *SCR, const double *dS);

/* ---- JADE (Zhang and Sanderson 2009), the algorithm whose adaptive
 * parameters muF and muCR the paper's second case study observes (Sec. 4,
 * Fig. 9) ----
 * The state is an orc_lshade_state with H = 1: MF[0] = muF, MCR[0] = muCR.
 * One generation is L-SHADE's (ranking, draws from slot 0 -- CR ~ N(muCR,
 * 0.1) clipped to [0, 1], F ~ Cauchy(muF, 0.1) redrawn while <= 0 and capped
 * at 1 --, current-to-pbest/1 with r2 from the population and the archive,
 * crossover, repair, selection, the archive of improved parents bounded by
 * round(r_arc np)) with no population reduction and JADE's parameter
 * update in place of the memory:
 *   muCR <- (1 - c) muCR + c mean(S_CR),
 *   muF  <- (1 - c) muF  + c sum(S_F^2) / sum(S_F),
 * plain (unweighted) means over the strictly improved individuals; nothing
 * changes when none improved. */
void orc_jade_update(double c, double *muF, double *muCR, int32_t n_s, const double *SF, const double *SCR);
int orc_jade_generation(const orc_problem *pb, const double *o, const double *M, orc_lshade_state *s,
                        double p, double r_arc, double c, uint32_t run_uid, uint64_t seed, uint32_t t,
                        double *U, double *eU, int32_t *n_success);

/* ---- PSODE: the PSO/DE hybrid with pairwise/3 selection of the case study
 * (Sec. 4, Listing 4) ----
 * One generation from the population X / eX and the velocities V:
 *  1. PSO half: a copy Y of X moves by the PSO module's update
 *     (orc_pso_variant_iteration with the given topology and velocity
 *     update; the personal bests are the population itself, since X_i is
 *     the best point evaluated at index i so far) and is evaluated (eY);
 *  2. DE half: one SHADE generation from X (orc_shade_generation) gives the
 *     trials U / eU and the population after its greedy selection, X3 / e3;
 *  3. V = X3 - X (zero where the trial lost);
 *  4. X_i = Y_i where e(Y_i) < e3_i (strictly; NaN counts as +infinity),
 *     else X3_i: the best of parent, DE trial and PSO move.
 * The two halves draw from disjoint streams (PSO and SHADE tags, counter t).
 * choice[i] (optional): 0 parent kept, 1 DE trial, 2 PSO move. */
int orc_psode_generation(const orc_problem *pb, const double *o, const double *M, int32_t np,
                         int32_t topology, int32_t velocity, double w, double c1, double c2,
                         double vmax, double p, int32_t H, double *MF, double *MCR, int32_t *pos,
                         uint32_t run_uid, uint64_t seed, uint32_t t, double *X, double *eX, double *V,
                         double *Y, double *eY, double *U, double *eU, uint8_t *choice);

/* ---- CSO: the competitive swarm optimizer (Cheng and Jin), the optimiser
 * of the large-scale study (Sec. 3.3: swarm of 300, D = 1000) ----
 * One iteration on the swarm X / V / e of m particles (m even):
 *  - pairing: the particles in ascending order of (w_i, i), w_i word 0 of
 *    the draw (tag CSO_PAIR, counter (t, i)), taken two at a time: pair k is
 *    (perm[2k], perm[2k+1]);
 *  - in each pair the particle of lower error wins (NaN counts as +inf; equal
 *    errors: the lower index wins);
 *  - the winner passes unchanged; the loser l learns from the winner w:
 *    v_j = r1 v_j + r2 (x_w,j - x_l,j) + phi r3 (xbar_j - x_l,j), x_l,j += v_j,
 *    xbar the mean position of the whole swarm before the iteration and
 *    (r1, r2, r3) the u24 of words 0, 1, 2 of the draw (tag CSO_R, counter
 *    (t, l), block j); a coordinate leaving the box is put on the bound with
 *    its velocity zeroed;
 *  - the losers are evaluated.
 * G / eG receive the m/2 new loser positions and their errors in pair order;
 * winner / loser (optional) the pairs. */
int orc_cso_iteration(const orc_problem *pb, const double *o, const double *M, int32_t m, double phi,
                      uint32_t run_uid, uint64_t seed, uint32_t t, double *X, double *V, double *e,
                      double *G, double *eG, int32_t *winner, int32_t *loser);

/* ---- Whole-run driver with FE accounting and the 200-FE recorder ---- */
typedef struct {
    int32_t algo;
    int32_t func, dim;
    double lb, ub;
    uint32_t instance;
    uint32_t run_uid;
    int32_t np;
    int64_t budget;        /* function evaluations */
    double F, CR;          /* DE */
    double w, c1, c2, vmax;/* PSO */
    double p;              /* SHADE / L-SHADE: pbest fraction */
    int32_t H;             /* SHADE / L-SHADE: memory size */
    double r_arc;          /* L-SHADE: archive bound per individual */
    int32_t np_min;        /* L-SHADE: final population size */
    int32_t topology;      /* PSO: 0 global best, 1 ring */
    int32_t velocity;      /* PSO: 0 inertia weight, 1 spherical */
    double c;              /* JADE: adaptation rate of muF and muCR */
    double restart_tol;    /* L-SHADE with restarts: convergence threshold */
} orc_run_desc;
/* L-SHADE-Restart runs (ORC_ALGO_LSHADE_RS; the state-triggered restart
 * that the paper's modular design makes, Sec. 4) are L-SHADE runs that,
 * after a generation leaving budget, restart once the population has
 * converged -- max e - min e over it <= restart_tol (orc_converged) --:
 * restart k (1, 2, ...) draws a fresh population of np individuals
 * (orc_restart_population with that k), evaluates and records it, resets
 * the memories to 0.5 (pos = 0) and empties the archive, and the size
 * schedule starts over: orc_lshade_np(np, np_min, budget - fe_r,
 * fe - fe_r + np_current), fe_r the evaluations made before the restart.
 * The generation counter keeps counting, and the best-so-far record spans
 * all restarts.
 * JADE runs take p, r_arc (the archive bound per individual: 1 in JADE) and
 * c; H and np_min are ignored (one parameter pair, no reduction).
 * CSO runs take np = m (even) and phi in c1; V starts at zero; an iteration
 * makes m/2 evaluations, recorded in pair order.
 * PSODE runs take the PSO fields (w, c1, c2, vmax, topology, velocity) and
 * SHADE's (p, H); V starts at zero; a generation makes 2 np evaluations,
 * recorded as the PSO moves in index order, then the DE trials. */

typedef struct {
    double best_e;         /* best error over the first `budget` evaluations */
    int64_t fes;           /* evaluations performed (whole generations) */
    int32_t generations;   /* generations after initialisation */
    int32_t success;       /* best_e <= 1e-8 */
    int32_t restarts;      /* L-SHADE-Restart: restarts made */
} orc_run_result;

#define ORC_TRACE_EVERY 200
int orc_run(const orc_run_desc *d, uint64_t seed, uint64_t inst_seed,
            orc_run_result *res, double *trace, int64_t trace_len, double *best_x);

/* orc_run with the parameter observer of the second case study (Sec. 4,
 * Fig. 9): mu[2g], mu[2g+1] (g < mu_len) receive (muF, muCR) after g
 * generations (g = 0: the initial state), NaN for generations not made.
 *   JADE: its muF and muCR;
 *   SHADE, L-SHADE, PSODE: the means of the H memory slots (a terminal CR
 *   slot counts as 0, the CR it gives);
 *   DE: its fixed F and CR;
 *   PSO, CSO: NaN (no such parameters). */
int orc_run_observed(const orc_run_desc *d, uint64_t seed, uint64_t inst_seed, orc_run_result *res,
                     double *trace, int64_t trace_len, double *best_x, double *mu, int64_t mu_len);

/* Constants of the Schwefel form (the argmax s and c = s sin sqrt s). */
double orc_schwefel_s(void);
double orc_schwefel_c(void);
double orc_schwefel_lambda(void);

#ifdef __cplusplus
}
#endif
#endif
