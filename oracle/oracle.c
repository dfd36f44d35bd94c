/*
 * oracle.c -- plain FP64 CPU oracle (test infrastructure only; see oracle.h).
 *
 * What it follows:
 *  - The paper's method: modular DE with binomial crossover and the
 *    midpoint-target bound repair, SHADE parameter adaptation with the
 *    current-to-pbest/1 mutation and no external archive (Sec. 2.2,
 *    Listing 1); gbest PSO and the ring / spherical variants (Sec. 2.2,
 *    Listing 1); L-SHADE (Sec. 2.2, Sec. 4); the PSODE hybrid with
 *    pairwise/3 selection (Sec. 4, Listing 4); the competitive swarm
 *    optimizer of the large-scale study (Sec. 3.3; Cheng and Jin 2015,
 *    global-mean variant); whole-generation iteration with
 *    function-evaluation accounting (Listing 4's loop structure); the
 *    best-so-far recorder every 200 evaluations (Sec. 2.4, Sec. 3.2);
 *    multiple random instances per problem (Sec. 1, Sec. 2.3).
 *  - The named textbook algorithms for what the paper leaves implicit:
 *    Storn & Price (1997) DE rand/1/bin; Shi & Eberhart (1998) inertia-weight
 *    PSO; Tanabe & Fukunaga (2013) SHADE; Salmon et al. (SC'11) Philox4x32-10;
 *    Box-Muller normals; Householder QR with the positive-diagonal convention
 *    (Mezzadri 2007) for the random rotation.
 *
 * Every value is double; x is widened exactly from the caller's floats.
 * Compile with -O2 -ffp-contract=off, never -ffast-math.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------- */
/* Philox4x32-10.  One round maps (c0,c1,c2,c3) with key (k0,k1) to
 *   (hi(B*c2) ^ c1 ^ k0, lo(B*c2), hi(A*c0) ^ c3 ^ k1, lo(A*c0))
 * with A = 0xD2511F53 and B = 0xCD9E8D57; the key is advanced by the Weyl
 * constants (0x9E3779B9, 0xBB67AE85) between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t pa = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t pb = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hia = (uint32_t)(pa >> 32), loa = (uint32_t)pa;
        uint32_t hib = (uint32_t)(pb >> 32), lob = (uint32_t)pb;
        uint32_t n0 = hib ^ c1 ^ k0;
        uint32_t n1 = lob;
        uint32_t n2 = hia ^ c3 ^ k1;
        uint32_t n3 = loa;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static uint32_t fold_seed(uint64_t seed)
{
    return (uint32_t)seed ^ (uint32_t)(seed >> 32);
}

/* Draw the 4 words of counter (c0, c1, tag<<24 | block, c3) under key (k0, seed). */
static void draw(uint32_t k0, uint64_t seed, uint32_t c0, uint32_t c1, uint32_t tag,
                 uint32_t block, uint32_t c3, uint32_t out[4])
{
    uint32_t ctr[4] = { c0, c1, (tag << 24) | (block & 0xFFFFFFu), c3 };
    uint32_t key[2] = { k0, fold_seed(seed) };
    orc_philox4x32_10(ctr, key, out);
}

double orc_u24(uint32_t w)
{
    return (double)(w >> 8) * (1.0 / 16777216.0);
}

double orc_u53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

uint32_t orc_range(uint32_t w, uint32_t n)
{
    return (uint32_t)(((uint64_t)w * (uint64_t)n) >> 32);
}

uint32_t orc_cr_threshold(double cr)
{
    if (!(cr > 0.0)) return 0;            /* also catches NaN */
    if (cr >= 1.0) return 16777216u;
    return (uint32_t)ceil(cr * 16777216.0);
}

/* Ordering key of an error value: NaN counts as +infinity. */
static double key_of(double e)
{
    return isnan(e) ? INFINITY : e;
}

/* ------------------------------------------------------------------------- */
/* Instances. */

int orc_householder_q(int32_t n, const double *A, double *Q)
{
    if (n < 1) return -1;
    double *R = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *V = (double *)malloc(sizeof(double) * (size_t)n * n); /* reflector k in row k */
    double *tmp = (double *)malloc(sizeof(double) * (size_t)n);
    if (!R || !V || !tmp) { free(R); free(V); free(tmp); return -1; }
    memcpy(R, A, sizeof(double) * (size_t)n * n);
    memset(V, 0, sizeof(double) * (size_t)n * n);

    /* R <- H_{n-2} ... H_0 A, with H_k = I - 2 v v^T acting on rows k..n-1. */
    for (int k = 0; k + 1 < n; ++k) {
        double norm2 = 0.0;
        for (int r = k; r < n; ++r) norm2 += R[(size_t)r * n + k] * R[(size_t)r * n + k];
        double norm = sqrt(norm2);
        if (norm == 0.0) continue;
        double x0 = R[(size_t)k * n + k];
        double alpha = (x0 >= 0.0) ? -norm : norm;
        double *v = V + (size_t)k * n;
        for (int r = k; r < n; ++r) v[r] = R[(size_t)r * n + k];
        v[k] -= alpha;
        double vn2 = 0.0;
        for (int r = k; r < n; ++r) vn2 += v[r] * v[r];
        double vn = sqrt(vn2);
        if (vn == 0.0) continue;
        for (int r = k; r < n; ++r) v[r] /= vn;
        /* R[k:, k:] -= 2 v (v^T R[k:, k:]) */
        for (int c = k; c < n; ++c) {
            double s = 0.0;
            for (int r = k; r < n; ++r) s += v[r] * R[(size_t)r * n + c];
            tmp[c] = s;
        }
        for (int r = k; r < n; ++r)
            for (int c = k; c < n; ++c)
                R[(size_t)r * n + c] -= 2.0 * v[r] * tmp[c];
    }

    /* Q = H_0 H_1 ... H_{n-2}: start from I and apply reflectors from the right. */
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c)
            Q[(size_t)r * n + c] = (r == c) ? 1.0 : 0.0;
    for (int k = 0; k + 1 < n; ++k) {
        const double *v = V + (size_t)k * n;
        /* Q[:, k:] -= 2 (Q[:, k:] v) v^T */
        for (int r = 0; r < n; ++r) {
            double s = 0.0;
            for (int c = k; c < n; ++c) s += Q[(size_t)r * n + c] * v[c];
            tmp[r] = s;
        }
        for (int r = 0; r < n; ++r)
            for (int c = k; c < n; ++c)
                Q[(size_t)r * n + c] -= 2.0 * tmp[r] * v[c];
    }
    /* Make diag(R) positive: flip column j of Q where R[j][j] < 0. */
    for (int j = 0; j < n; ++j) {
        if (R[(size_t)j * n + j] < 0.0)
            for (int r = 0; r < n; ++r) Q[(size_t)r * n + j] = -Q[(size_t)r * n + j];
    }
    free(R); free(V); free(tmp);
    return 0;
}

int orc_instance(int32_t func, int32_t dim, uint32_t instance, uint64_t inst_seed,
                 double *o, double *M, double *G)
{
    if (dim < 1 || func < 0 || func >= ORC_NFUNC) return -1;
    uint32_t w[4];
    /* Shift: o_j = -80 + 160 u53, two values per counter block. */
    for (int j = 0; j < dim; j += 2) {
        draw(instance, inst_seed, (uint32_t)func, (uint32_t)dim, ORC_TAG_SHIFT_O,
             (uint32_t)(j / 2), 0, w);
        o[j] = -80.0 + 160.0 * orc_u53(w[0], w[1]);
        if (j + 1 < dim) o[j + 1] = -80.0 + 160.0 * orc_u53(w[2], w[3]);
    }
    /* Gaussian matrix, row-major, one Box-Muller pair per counter block. */
    size_t n2 = (size_t)dim * dim;
    double *Gm = G ? G : (double *)malloc(sizeof(double) * n2);
    if (!Gm) return -1;
    for (size_t e = 0; e < n2; e += 2) {
        draw(instance, inst_seed, (uint32_t)func, (uint32_t)dim, ORC_TAG_ROT_N,
             (uint32_t)(e / 2), 0, w);
        double u1 = orc_u53(w[0], w[1]);
        double u2 = orc_u53(w[2], w[3]);
        double r = sqrt(-2.0 * log(1.0 - u1));
        Gm[e] = r * cos(2.0 * M_PI * u2);
        if (e + 1 < n2) Gm[e + 1] = r * sin(2.0 * M_PI * u2);
    }
    int rc = orc_householder_q(dim, Gm, M);
    if (!G) free(Gm);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Objective functions, e = f - f* with f* = 100, in forms algebraically equal
 * to the textbook definitions but free of cancellation near z = 0. */

/* Schwefel: g(u) = c - u sin(sqrt|u|) with u = z + s, s the argmax of
 * u sin(sqrt u) near 421 and c = s sin(sqrt s) so that g(s) = 0. */
static const double SCHWEFEL_S = 420.96874635998202731;
static const double SCHWEFEL_LAMBDA = 0.01;

double orc_schwefel_s(void) { return SCHWEFEL_S; }
double orc_schwefel_c(void) { return SCHWEFEL_S * sin(sqrt(SCHWEFEL_S)); }
double orc_schwefel_lambda(void) { return SCHWEFEL_LAMBDA; }

static double schwefel_plain(double u)
{
    return orc_schwefel_c() - u * sin(sqrt(fabs(u)));
}

static double schwefel_term(double z)
{
    double s = SCHWEFEL_S;
    double u = z + s;
    if (u > 500.0) {
        double b = u - 500.0;
        return schwefel_plain(500.0) + SCHWEFEL_LAMBDA * b * b;
    }
    if (u < -500.0) {
        double b = -500.0 - u;
        return schwefel_plain(-500.0) + SCHWEFEL_LAMBDA * b * b;
    }
    if (u > 0.0) {
        /* With a = sqrt(s), t = sqrt(s + z) - a = z / (a + sqrt(s + z)):
         * g = s (sin a - sin(a + t)) - z sin(a + t)
         *   = -2 s cos(a + t/2) sin(t/2) - z sin(a + t). */
        double a = sqrt(s);
        double t = z / (a + sqrt(u));
        return -2.0 * s * cos(a + 0.5 * t) * sin(0.5 * t) - z * sin(a + t);
    }
    return schwefel_plain(u);
}

double orc_error_z(int32_t func, int32_t dim, const double *z)
{
    double sum = 0.0;
    switch (func) {
    case ORC_ELLIPSOID:
        for (int i = 0; i < dim; ++i) {
            double w = (dim > 1) ? pow(10.0, 6.0 * (double)i / (double)(dim - 1)) : 1.0;
            sum += w * z[i] * z[i];
        }
        return sum;
    case ORC_ROSENBROCK:
        /* With w = z + 1: 100 (w_i^2 - w_{i+1})^2 + (w_i - 1)^2
         *              = 100 (z_i^2 + 2 z_i - z_{i+1})^2 + z_i^2. */
        for (int i = 0; i + 1 < dim; ++i) {
            double a = z[i] * z[i] + 2.0 * z[i] - z[i + 1];
            sum += 100.0 * a * a + z[i] * z[i];
        }
        return sum;
    case ORC_RASTRIGIN:
        /* z^2 - 10 cos(2 pi z) + 10 = z^2 + 20 sin^2(pi z). */
        for (int i = 0; i < dim; ++i) {
            double s = sin(M_PI * z[i]);
            sum += z[i] * z[i] + 20.0 * s * s;
        }
        return sum;
    case ORC_SCHWEFEL:
        for (int i = 0; i < dim; ++i) sum += schwefel_term(z[i]);
        return sum;
    case ORC_GRIEWANK: {
        /* 1 + sum z^2/4000 - prod cos(z_i / sqrt(i)), i = 1..D.
         * cos a = 1 - 2 sin^2(a/2); the product is sign * exp(sum log|cos a|),
         * and 1 - prod = -expm1(L) for a positive product, 1 + exp(L) otherwise. */
        double q = 0.0, L = 0.0;
        int negative = 0, zero = 0;
        for (int i = 0; i < dim; ++i) {
            q += z[i] * z[i];
            double a = z[i] / sqrt((double)(i + 1));
            double h = sin(0.5 * a);
            double c = 1.0 - 2.0 * h * h;
            if (c > 0.0) {
                L += log1p(-2.0 * h * h);
            } else if (c < 0.0) {
                L += log(-c);
                negative ^= 1;
            } else {
                zero = 1;
            }
        }
        double one_minus_prod;
        if (zero) one_minus_prod = 1.0;
        else if (!negative) one_minus_prod = -expm1(L);
        else one_minus_prod = 1.0 + exp(L);
        return q / 4000.0 + one_minus_prod;
    }
    case ORC_ACKLEY: {
        /* -20 exp(-0.2 sqrt(S2/D)) - exp(S1/D) + 20 + e with
         * S1 = sum cos(2 pi z) = D - 2 sum sin^2(pi z):
         * = -20 expm1(-0.2 sqrt(S2/D)) - e expm1(-(2/D) sum sin^2(pi z)). */
        double s2 = 0.0, ss = 0.0;
        for (int i = 0; i < dim; ++i) {
            s2 += z[i] * z[i];
            double s = sin(M_PI * z[i]);
            ss += s * s;
        }
        double D = (double)dim;
        return -20.0 * expm1(-0.2 * sqrt(s2 / D)) - exp(1.0) * expm1(-2.0 * ss / D);
    }
    default:
        return NAN;
    }
}

double orc_error(int32_t func, int32_t dim, const double *o, const double *M, const double *x)
{
    if (dim < 1) return NAN;
    double d[dim], z[dim];
    for (int j = 0; j < dim; ++j) d[j] = x[j] - o[j];
    for (int r = 0; r < dim; ++r) {
        double s = 0.0;
        for (int k = 0; k < dim; ++k) s += M[(size_t)r * dim + k] * d[k];
        z[r] = s;
    }
    return orc_error_z(func, dim, z);
}

void orc_error_soa_f32(int32_t func, int32_t dim, const double *o, const double *M,
                       const float *X, int64_t ld, int32_t n, double *e)
{
    double *x = (double *)malloc(sizeof(double) * (size_t)dim);
    if (!x) return;
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < dim; ++j) x[j] = (double)X[(size_t)j * ld + i];
        e[i] = orc_error(func, dim, o, M, x);
    }
    free(x);
}

void orc_error_aos(int32_t func, int32_t dim, const double *o, const double *M,
                   const double *X, int32_t n, double *e)
{
    for (int i = 0; i < n; ++i) e[i] = orc_error(func, dim, o, M, X + (size_t)i * dim);
}

/* ------------------------------------------------------------------------- */
/* Population initialisation: generation 0, tag INIT_X, one word per coordinate. */
void orc_restart_population(const orc_problem *pb, int32_t np, uint32_t run_uid, uint64_t seed, uint32_t k,
                            double *X)
{
    int D = pb->dim;
    uint32_t w[4];
    for (int i = 0; i < np; ++i)
        for (int j = 0; j < D; ++j) {
            if (j % 4 == 0) draw(run_uid, seed, 0, (uint32_t)i, ORC_TAG_INIT_X, (uint32_t)(j / 4), k, w);
            X[(size_t)i * D + j] = pb->lb + (pb->ub - pb->lb) * orc_u24(w[j % 4]);
        }
}

void orc_init_population(const orc_problem *pb, int32_t np, uint32_t run_uid,
                         uint64_t seed, double *X)
{
    orc_restart_population(pb, np, run_uid, seed, 0, X);
}

/* Index in [0, n) with the members of `excl` (distinct, any order) skipped:
 * draw r in [0, n - m) and step it past the excluded values in ascending order. */
static int32_t draw_excluding(uint32_t word, int32_t n, const int32_t *excl, int m)
{
    int32_t sorted[8];
    for (int a = 0; a < m; ++a) sorted[a] = excl[a];
    for (int a = 1; a < m; ++a)            /* insertion sort, m <= 3 */
        for (int b = a; b > 0 && sorted[b - 1] > sorted[b]; --b) {
            int32_t t = sorted[b]; sorted[b] = sorted[b - 1]; sorted[b - 1] = t;
        }
    int32_t r = (int32_t)orc_range(word, (uint32_t)(n - m));
    for (int a = 0; a < m; ++a)
        if (r >= sorted[a]) ++r;
    return r;
}

void orc_de_donors(int32_t np, int32_t dim, int32_t i, uint32_t run_uid, uint64_t seed,
                   uint32_t t, int32_t out[4])
{
    uint32_t w[4];
    draw(run_uid, seed, t, (uint32_t)i, ORC_TAG_DONORS, 0, 0, w);
    orc_donors_from_words(np, dim, i, w, out);
}

void orc_donors_from_words(int32_t np, int32_t dim, int32_t i, const uint32_t w[4],
                           int32_t out[4])
{
    int32_t ex[3];
    ex[0] = i;
    int32_t r1 = draw_excluding(w[0], np, ex, 1);
    ex[1] = r1;
    int32_t r2 = draw_excluding(w[1], np, ex, 2);
    ex[2] = r2;
    int32_t r3 = draw_excluding(w[2], np, ex, 3);
    out[0] = r1; out[1] = r2; out[2] = r3;
    out[3] = (int32_t)orc_range(w[3], (uint32_t)dim);
}

/* Binomial crossover of donor v with target x (mask from tag CROSS words),
 * then the midpoint-target repair of out-of-bounds coordinates. */
static void crossover_repair(const orc_problem *pb, int32_t i, uint32_t run_uid, uint64_t seed,
                             uint32_t t, uint32_t thr, int32_t jrand, const double *v,
                             const double *x, double *u, uint8_t *mask, double *margin)
{
    int D = pb->dim;
    uint32_t w[4];
    double mm = INFINITY;
    for (int j = 0; j < D; ++j) {
        if (j % 4 == 0) draw(run_uid, seed, t, (uint32_t)i, ORC_TAG_CROSS, (uint32_t)(j / 4), 0, w);
        uint32_t r24 = w[j % 4] >> 8;
        int m = (r24 < thr) || (j == jrand);
        if (j != jrand) {
            double gap = fabs((double)r24 + 0.5 - (double)thr);
            if (gap < mm) mm = gap;
        }
        double uj = m ? v[j] : x[j];
        if (uj < pb->lb) uj = 0.5 * (pb->lb + x[j]);
        else if (uj > pb->ub) uj = 0.5 * (pb->ub + x[j]);
        u[j] = uj;
        if (mask) mask[j] = (uint8_t)m;
    }
    if (margin) *margin = mm;
}

int orc_de_generation(const orc_problem *pb, const double *o, const double *M,
                      int32_t np, double F, double CR, uint32_t run_uid, uint64_t seed,
                      uint32_t t, const double *X, const double *eX,
                      double *U, double *eU, double *Xn, double *eXn,
                      int32_t *donors, uint8_t *mask, uint8_t *replaced)
{
    int D = pb->dim;
    if (np < 4 || D < 1) return -1;
    uint32_t thr = orc_cr_threshold(CR);
    double *v = (double *)malloc(sizeof(double) * (size_t)D);
    if (!v) return -1;
    for (int i = 0; i < np; ++i) {
        int32_t dn[4];
        orc_de_donors(np, D, i, run_uid, seed, t, dn);
        if (donors) memcpy(donors + (size_t)i * 4, dn, sizeof dn);
        const double *x1 = X + (size_t)dn[0] * D;
        const double *x2 = X + (size_t)dn[1] * D;
        const double *x3 = X + (size_t)dn[2] * D;
        for (int j = 0; j < D; ++j) v[j] = x1[j] + F * (x2[j] - x3[j]);
        crossover_repair(pb, i, run_uid, seed, t, thr, dn[3], v, X + (size_t)i * D,
                         U + (size_t)i * D, mask ? mask + (size_t)i * D : NULL, NULL);
    }
    free(v);
    orc_error_aos(pb->func, D, o, M, U, np, eU);
    /* Greedy one-to-one selection after all trials: ties go to the trial. */
    for (int i = 0; i < np; ++i) {
        int rep = key_of(eU[i]) <= key_of(eX[i]);
        if (replaced) replaced[i] = (uint8_t)rep;
        memcpy(Xn + (size_t)i * D, (rep ? U : X) + (size_t)i * D, sizeof(double) * (size_t)D);
        eXn[i] = rep ? eU[i] : eX[i];
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* PSO. */

static int32_t argmin_lowest(const double *e, int32_t n)
{
    int32_t best = 0;
    for (int i = 1; i < n; ++i)
        if (key_of(e[i]) < key_of(e[best])) best = i;
    return best;
}

int orc_pso_init(const orc_problem *pb, const double *o, const double *M, int32_t np,
                 uint32_t run_uid, uint64_t seed, double *X, double *V, double *P,
                 double *eX, double *eP, int32_t *g)
{
    int D = pb->dim;
    if (np < 1) return -1;
    orc_init_population(pb, np, run_uid, seed, X);
    memset(V, 0, sizeof(double) * (size_t)np * D);
    orc_error_aos(pb->func, D, o, M, X, np, eX);
    memcpy(P, X, sizeof(double) * (size_t)np * D);
    memcpy(eP, eX, sizeof(double) * (size_t)np);
    *g = argmin_lowest(eP, np);
    return 0;
}

int orc_pso_iteration(const orc_problem *pb, const double *o, const double *M, int32_t np,
                      double w, double c1, double c2, double vmax,
                      uint32_t run_uid, uint64_t seed, uint32_t t,
                      double *X, double *V, double *P, double *eX, double *eP, int32_t *g)
{
    int D = pb->dim;
    if (np < 1) return -1;
    const double *pg = P + (size_t)(*g) * D;
    double *gcopy = (double *)malloc(sizeof(double) * (size_t)D);
    if (!gcopy) return -1;
    memcpy(gcopy, pg, sizeof(double) * (size_t)D);
    uint32_t wd[4];
    for (int i = 0; i < np; ++i) {
        double *x = X + (size_t)i * D, *v = V + (size_t)i * D;
        const double *p = P + (size_t)i * D;
        for (int j = 0; j < D; ++j) {
            if (j % 2 == 0) draw(run_uid, seed, t, (uint32_t)i, ORC_TAG_PSO_R, (uint32_t)(j / 2), 0, wd);
            double r1 = orc_u24(wd[2 * (j % 2)]);
            double r2 = orc_u24(wd[2 * (j % 2) + 1]);
            double vj = w * v[j] + c1 * r1 * (p[j] - x[j]) + c2 * r2 * (gcopy[j] - x[j]);
            if (vj > vmax) vj = vmax;
            if (vj < -vmax) vj = -vmax;
            double xj = x[j] + vj;
            if (xj < pb->lb) { xj = pb->lb; vj = 0.0; }
            else if (xj > pb->ub) { xj = pb->ub; vj = 0.0; }
            x[j] = xj;
            v[j] = vj;
        }
    }
    free(gcopy);
    orc_error_aos(pb->func, D, o, M, X, np, eX);
    for (int i = 0; i < np; ++i)
        if (key_of(eX[i]) < key_of(eP[i])) {
            memcpy(P + (size_t)i * D, X + (size_t)i * D, sizeof(double) * (size_t)D);
            eP[i] = eX[i];
        }
    *g = argmin_lowest(eP, np);
    return 0;
}

/* Best personal best of i's neighbourhood: i itself for the global-best
 * topology is replaced by the global best; ring: {i-1, i, i+1} mod np. */
static int32_t neighbourhood_best(const double *eP, int32_t np, int32_t i, int32_t topology, int32_t g)
{
    if (topology == 0) return g;
    int32_t cand[3] = { (i + np - 1) % np, i, (i + 1) % np };
    int32_t best = cand[0];
    for (int k = 1; k < 3; ++k) {
        const int32_t c = cand[k];
        if (key_of(eP[c]) < key_of(eP[best]) || (key_of(eP[c]) == key_of(eP[best]) && c < best)) best = c;
    }
    return best;
}

int orc_pso_variant_iteration(const orc_problem *pb, const double *o, const double *M, int32_t np,
                              int32_t topology, int32_t velocity, double w, double c1, double c2,
                              double vmax, uint32_t run_uid, uint64_t seed, uint32_t t,
                              double *X, double *V, double *P, double *eX, double *eP, int32_t *lbest)
{
    const int D = pb->dim;
    if (np < 1 || topology < 0 || topology > 1 || velocity < 0 || velocity > 1) return -1;
    const size_t uD = (size_t)D;
    /* neighbourhood bests from the personal bests before this iteration */
    int32_t *l = (int32_t *)malloc(sizeof(int32_t) * (size_t)np);
    double *Pold = (double *)malloc(sizeof(double) * (size_t)np * uD);
    double *G = (double *)malloc(sizeof(double) * uD * 2);
    if (!l || !Pold || !G) { free(l); free(Pold); free(G); return -1; }
    const int32_t g = argmin_lowest(eP, np);
    for (int i = 0; i < np; ++i) l[i] = neighbourhood_best(eP, np, i, topology, g);
    if (lbest) memcpy(lbest, l, sizeof(int32_t) * (size_t)np);
    memcpy(Pold, P, sizeof(double) * (size_t)np * uD);
    double *z = G + uD;
    uint32_t wd[4];
    for (int i = 0; i < np; ++i) {
        double *x = X + (size_t)i * uD, *v = V + (size_t)i * uD;
        const double *p = Pold + (size_t)i * uD, *pl = Pold + (size_t)l[i] * uD;
        if (velocity == 0) {
            for (int j = 0; j < D; ++j) {
                if (j % 2 == 0) draw(run_uid, seed, t, (uint32_t)i, ORC_TAG_PSO_R, (uint32_t)(j / 2), 0, wd);
                const double r1 = orc_u24(wd[2 * (j % 2)]), r2 = orc_u24(wd[2 * (j % 2) + 1]);
                v[j] = w * v[j] + c1 * r1 * (p[j] - x[j]) + c2 * r2 * (pl[j] - x[j]);
            }
        } else {
            /* centre of gravity of x, p' and l' (or of x and p' when the
               particle is its own neighbourhood best) */
            double R2 = 0.0, z2 = 0.0;
            for (int j = 0; j < D; ++j) {
                const double pp = x[j] + c1 * (p[j] - x[j]);
                if (l[i] == i) {
                    G[j] = (x[j] + pp) / 2.0;
                } else {
                    const double lp = x[j] + c1 * (pl[j] - x[j]);
                    G[j] = (x[j] + pp + lp) / 3.0;
                }
                R2 += (G[j] - x[j]) * (G[j] - x[j]);
                if (j % 2 == 0) draw(run_uid, seed, t, (uint32_t)i, ORC_TAG_PSO_S, (uint32_t)(j / 2), 0, wd);
                const double rad = sqrt(-2.0 * log(1.0 - orc_u24(wd[0])));
                const double ang = 2.0 * M_PI * orc_u24(wd[1]);
                z[j] = j % 2 == 0 ? rad * cos(ang) : rad * sin(ang);
                z2 += z[j] * z[j];
            }
            uint32_t wr[4];
            draw(run_uid, seed, t, (uint32_t)i, ORC_TAG_PSO_SR, 0, 0, wr);
            const double r = sqrt(R2) * pow(orc_u24(wr[0]), 1.0 / (double)D);
            const double sc = z2 > 0.0 ? r / sqrt(z2) : 0.0;
            for (int j = 0; j < D; ++j) v[j] = w * v[j] + (G[j] + sc * z[j]) - x[j];
        }
        for (int j = 0; j < D; ++j) {
            double vj = v[j];
            if (vj > vmax) vj = vmax;
            if (vj < -vmax) vj = -vmax;
            double xj = x[j] + vj;
            if (xj < pb->lb) { xj = pb->lb; vj = 0.0; }
            else if (xj > pb->ub) { xj = pb->ub; vj = 0.0; }
            x[j] = xj;
            v[j] = vj;
        }
    }
    free(l); free(Pold); free(G);
    orc_error_aos(pb->func, D, o, M, X, np, eX);
    for (int i = 0; i < np; ++i)
        if (key_of(eX[i]) < key_of(eP[i])) {
            memcpy(P + (size_t)i * uD, X + (size_t)i * uD, sizeof(double) * uD);
            eP[i] = eX[i];
        }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* SHADE. */

int32_t orc_shade_pnum(double p, int32_t np)
{
    long k = lround(p * (double)np);
    if (k < 2) k = 2;
    if (k > np) k = np;
    return (int32_t)k;
}

void orc_shade_memory_update(int32_t H, double *MF, double *MCR, int32_t *pos,
                             int32_t n_s, const double *SF, const double *SCR,
                             const double *dS)
{
    (void)H;
    if (n_s <= 0) return;
    double total = 0.0;
    for (int k = 0; k < n_s; ++k) total += dS[k];
    double mcr = 0.0, num = 0.0, den = 0.0;
    for (int k = 0; k < n_s; ++k) {
        double wk = dS[k] / total;
        mcr += wk * SCR[k];
        num += wk * SF[k] * SF[k];
        den += wk * SF[k];
    }
    MCR[*pos] = mcr;
    MF[*pos] = num / den;
    *pos = (*pos + 1) % H;
}

static const double *g_sort_keys;
static int cmp_rank(const void *a, const void *b)
{
    int32_t ia = *(const int32_t *)a, ib = *(const int32_t *)b;
    double ka = key_of(g_sort_keys[ia]), kb = key_of(g_sort_keys[ib]);
    if (ka < kb) return -1;
    if (ka > kb) return 1;
    return (ia > ib) - (ia < ib);
}

#define SHADE_MAX_RETRIES 64
#define SHADE_DELTA_CAP 1e30

int orc_shade_generation(const orc_problem *pb, const double *o, const double *M,
                         int32_t np, double p, int32_t H, double *MF, double *MCR,
                         int32_t *pos, uint32_t run_uid, uint64_t seed, uint32_t t,
                         const double *X, const double *eX,
                         double *U, double *eU, double *Xn, double *eXn,
                         int32_t *idx, double *Fo, double *CRo, double *margin,
                         uint8_t *mask, uint8_t *replaced, int32_t *sorted_out)
{
    int D = pb->dim;
    if (np < 4 || D < 1 || H < 1) return -1;
    int32_t *rank = (int32_t *)malloc(sizeof(int32_t) * (size_t)np);
    double *v = (double *)malloc(sizeof(double) * (size_t)D);
    double *Fi = (double *)malloc(sizeof(double) * (size_t)np);
    double *CRi = (double *)malloc(sizeof(double) * (size_t)np);
    if (!rank || !v || !Fi || !CRi) { free(rank); free(v); free(Fi); free(CRi); return -1; }
    for (int i = 0; i < np; ++i) rank[i] = i;
    /* Single-threaded sort: the comparator reads a file-scope pointer. */
    g_sort_keys = eX;
    qsort(rank, (size_t)np, sizeof(int32_t), cmp_rank);
    if (sorted_out) memcpy(sorted_out, rank, sizeof(int32_t) * (size_t)np);
    int32_t pnum = orc_shade_pnum(p, np);

    for (int i = 0; i < np; ++i) {
        uint32_t wp[4], wc[4], wd[4];
        draw(run_uid, seed, t, (uint32_t)i, ORC_TAG_SHADE_P, 0, 0, wp);
        int32_t k = (int32_t)orc_range(wp[0], (uint32_t)H);
        /* CR ~ N(M_CR[k], 0.1) by Box-Muller, clamped to [0, 1]. */
        double nrm = sqrt(-2.0 * log(1.0 - orc_u24(wp[1]))) * cos(2.0 * M_PI * orc_u24(wp[2]));
        double cr = MCR[k] + 0.1 * nrm;
        if (cr < 0.0) cr = 0.0;
        if (cr > 1.0) cr = 1.0;
        /* F ~ Cauchy(M_F[k], 0.1), redrawn while F <= 0, truncated at 1. */
        int retries = 0;
        double F = -1.0, fmargin = INFINITY, cmargin = INFINITY;
        while (retries < SHADE_MAX_RETRIES) {
            draw(run_uid, seed, t, (uint32_t)i, ORC_TAG_SHADE_C, 0, (uint32_t)retries, wc);
            double Fc = MF[k] + 0.1 * tan(M_PI * (orc_u24(wc[0]) - 0.5));
            if (fabs(Fc) < fmargin) fmargin = fabs(Fc);
            if (Fc > 0.0) { F = Fc; break; }
            ++retries;
        }
        if (!(F > 0.0)) F = MF[k];
        if (F > 1.0) F = 1.0;
        int32_t pb_idx = rank[orc_range(wp[3], (uint32_t)pnum)];
        draw(run_uid, seed, t, (uint32_t)i, ORC_TAG_SHADE_D, 0, 0, wd);
        int32_t ex[2] = { i, 0 };
        int32_t r1 = draw_excluding(wd[0], np, ex, 1);
        ex[1] = r1;
        int32_t r2 = draw_excluding(wd[1], np, ex, 2);
        int32_t jrand = (int32_t)orc_range(wd[2], (uint32_t)D);
        const double *xi = X + (size_t)i * D;
        const double *xp = X + (size_t)pb_idx * D;
        const double *x1 = X + (size_t)r1 * D;
        const double *x2 = X + (size_t)r2 * D;
        for (int j = 0; j < D; ++j)
            v[j] = xi[j] + F * (xp[j] - xi[j]) + F * (x1[j] - x2[j]);
        crossover_repair(pb, i, run_uid, seed, t, orc_cr_threshold(cr), jrand, v, xi,
                         U + (size_t)i * D, mask ? mask + (size_t)i * D : NULL, &cmargin);
        if (margin) { margin[2 * (size_t)i] = fmargin; margin[2 * (size_t)i + 1] = cmargin; }
        Fi[i] = F;
        CRi[i] = cr;
        if (idx) {
            int32_t *q = idx + (size_t)i * 6;
            q[0] = k; q[1] = pb_idx; q[2] = r1; q[3] = r2; q[4] = jrand; q[5] = retries;
        }
        if (Fo) Fo[i] = F;
        if (CRo) CRo[i] = cr;
    }
    orc_error_aos(pb->func, D, o, M, U, np, eU);

    int32_t n_s = 0;
    double *SF = (double *)malloc(sizeof(double) * (size_t)np * 3);
    if (!SF) { free(rank); free(v); free(Fi); free(CRi); return -1; }
    double *SCR = SF + np, *dS = SF + 2 * (size_t)np;
    for (int i = 0; i < np; ++i) {
        double ku = key_of(eU[i]), kx = key_of(eX[i]);
        int rep = ku <= kx;
        if (ku < kx) {
            double d = kx - ku;
            if (!(d <= SHADE_DELTA_CAP)) d = SHADE_DELTA_CAP;
            SF[n_s] = Fi[i]; SCR[n_s] = CRi[i]; dS[n_s] = d; ++n_s;
        }
        if (replaced) replaced[i] = (uint8_t)rep;
        memcpy(Xn + (size_t)i * D, (rep ? U : X) + (size_t)i * D, sizeof(double) * (size_t)D);
        eXn[i] = rep ? eU[i] : eX[i];
    }
    orc_shade_memory_update(H, MF, MCR, pos, n_s, SF, SCR, dS);
    free(SF); free(rank); free(v); free(Fi); free(CRi);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* L-SHADE (Tanabe & Fukunaga, CEC 2014). */

int32_t orc_lshade_np(int32_t np_init, int32_t np_min, int64_t budget, int64_t fe)
{
    double v = (double)(np_min - np_init) * (double)fe / (double)budget + (double)np_init;
    long k = lround(v);
    if (k < np_min) k = np_min;
    if (k > np_init) k = np_init;
    return (int32_t)k;
}

int32_t orc_lshade_archive_max(double r_arc, int32_t np)
{
    long k = lround(r_arc * (double)np);
    return k < 0 ? 0 : (int32_t)k;
}

void orc_lshade_memory_update(int32_t H, double *MF, double *MCR, int32_t *pos, int32_t n_s,
                              const double *SF, const double *SCR, const double *dS)
{
    if (n_s <= 0) return;
    double total = 0.0, cr_max = 0.0;
    for (int k = 0; k < n_s; ++k) {
        total += dS[k];
        if (SCR[k] > cr_max) cr_max = SCR[k];
    }
    double nf = 0.0, df = 0.0, nc = 0.0, dc = 0.0;
    for (int k = 0; k < n_s; ++k) {
        double wk = dS[k] / total;
        nf += wk * SF[k] * SF[k];
        df += wk * SF[k];
        nc += wk * SCR[k] * SCR[k];
        dc += wk * SCR[k];
    }
    /* the terminal CR value is kept once reached, or set when every
       successful CR was zero */
    if (MCR[*pos] < 0.0 || cr_max == 0.0) MCR[*pos] = -1.0;
    else MCR[*pos] = nc / dc;
    MF[*pos] = nf / df;
    *pos = (*pos + 1) % H;
}

void orc_jade_update(double c, double *muF, double *muCR, int32_t n_s, const double *SF, const double *SCR)
{
    if (n_s <= 0) return;
    double scr = 0.0, sf = 0.0, sf2 = 0.0;
    for (int k = 0; k < n_s; ++k) {
        scr += SCR[k];
        sf += SF[k];
        sf2 += SF[k] * SF[k];
    }
    *muCR = (1.0 - c) * *muCR + c * (scr / (double)n_s);   /* arithmetic mean */
    *muF = (1.0 - c) * *muF + c * (sf2 / sf);               /* Lehmer mean */
}

/* One generation of L-SHADE (jade = 0) or JADE (jade = 1, adaptation rate
 * c): the two differ only in the parameter update after the selection. */
static int archive_generation(const orc_problem *pb, const double *o, const double *M, orc_lshade_state *s,
                              double p, double r_arc, int32_t np_next, int jade, double c, uint32_t run_uid,
                              uint64_t seed, uint32_t t, double *U, double *eU, int32_t *n_success)
{
    const int D = pb->dim, np = s->np;
    if (np < 4 || D < 1 || s->H < 1 || np_next < 4 || np_next > np) return -1;
    const size_t uD = (size_t)D;
    int32_t *rank = (int32_t *)malloc(sizeof(int32_t) * (size_t)np);
    double *v = (double *)malloc(sizeof(double) * uD);
    double *Fi = (double *)malloc(sizeof(double) * (size_t)np * 5);
    double *tmp = (double *)malloc(sizeof(double) * (size_t)np * (uD + 1));
    if (!rank || !v || !Fi || !tmp) { free(rank); free(v); free(Fi); free(tmp); return -1; }
    double *CRi = Fi + np, *SF = Fi + 2 * (size_t)np, *SCR = Fi + 3 * (size_t)np, *dS = Fi + 4 * (size_t)np;
    for (int i = 0; i < np; ++i) rank[i] = i;
    g_sort_keys = s->eX;
    qsort(rank, (size_t)np, sizeof(int32_t), cmp_rank);
    const int32_t pnum = orc_shade_pnum(p, np);
    const int32_t H = s->H;

    /* variation */
    for (int i = 0; i < np; ++i) {
        uint32_t wp[4], wc[4], wd[4];
        draw(run_uid, seed, t, (uint32_t)i, ORC_TAG_SHADE_P, 0, 0, wp);
        const int32_t k = (int32_t)orc_range(wp[0], (uint32_t)H);
        double cr = 0.0;
        if (s->MCR[k] >= 0.0) {
            double nrm = sqrt(-2.0 * log(1.0 - orc_u24(wp[1]))) * cos(2.0 * M_PI * orc_u24(wp[2]));
            cr = s->MCR[k] + 0.1 * nrm;
            if (cr < 0.0) cr = 0.0;
            if (cr > 1.0) cr = 1.0;
        }
        int retries = 0;
        double F = -1.0, cm = INFINITY;
        while (retries < SHADE_MAX_RETRIES) {
            draw(run_uid, seed, t, (uint32_t)i, ORC_TAG_SHADE_C, 0, (uint32_t)retries, wc);
            double Fc = s->MF[k] + 0.1 * tan(M_PI * (orc_u24(wc[0]) - 0.5));
            if (Fc > 0.0) { F = Fc; break; }
            ++retries;
        }
        if (!(F > 0.0)) F = s->MF[k];
        if (F > 1.0) F = 1.0;
        const int32_t pbi = rank[orc_range(wp[3], (uint32_t)pnum)];
        draw(run_uid, seed, t, (uint32_t)i, ORC_TAG_SHADE_D, 0, 0, wd);
        int32_t ex[2] = { i, 0 };
        const int32_t r1 = draw_excluding(wd[0], np, ex, 1);
        ex[1] = r1;
        const int32_t r2 = draw_excluding(wd[1], np + s->na, ex, 2);   /* >= np: archive */
        const int32_t jrand = (int32_t)orc_range(wd[2], (uint32_t)D);
        const double *xi = s->X + (size_t)i * uD, *xp = s->X + (size_t)pbi * uD;
        const double *x1 = s->X + (size_t)r1 * uD;
        const double *x2 = r2 < np ? s->X + (size_t)r2 * uD : s->A + (size_t)(r2 - np) * uD;
        for (int j = 0; j < D; ++j) v[j] = xi[j] + F * (xp[j] - xi[j]) + F * (x1[j] - x2[j]);
        crossover_repair(pb, i, run_uid, seed, t, orc_cr_threshold(cr), jrand, v, xi, U + (size_t)i * uD, NULL,
                         &cm);
        Fi[i] = F;
        CRi[i] = cr;
    }
    orc_error_aos(pb->func, D, o, M, U, np, eU);

    /* selection; improved parents enter the archive in index order */
    const int32_t amax = orc_lshade_archive_max(r_arc, np);
    int32_t n_s = 0;
    for (int i = 0; i < np; ++i) {
        const double ku = key_of(eU[i]), kx = key_of(s->eX[i]);
        if (ku < kx) {
            double d = kx - ku;
            if (!(d <= SHADE_DELTA_CAP)) d = SHADE_DELTA_CAP;
            SF[n_s] = Fi[i]; SCR[n_s] = CRi[i]; dS[n_s] = d; ++n_s;
            int32_t at = -1;
            if (s->na < amax) {
                at = s->na++;
            } else if (amax > 0) {
                uint32_t wa[4];
                draw(run_uid, seed, t, (uint32_t)i, ORC_TAG_LSHADE_A, 0, 0, wa);
                at = (int32_t)orc_range(wa[0], (uint32_t)amax);
            }
            if (at >= 0) memcpy(s->A + (size_t)at * uD, s->X + (size_t)i * uD, sizeof(double) * uD);
        }
        if (ku <= kx) {
            memcpy(s->X + (size_t)i * uD, U + (size_t)i * uD, sizeof(double) * uD);
            s->eX[i] = eU[i];
        }
    }
    if (jade) orc_jade_update(c, &s->MF[0], &s->MCR[0], n_s, SF, SCR);
    else orc_lshade_memory_update(H, s->MF, s->MCR, &s->pos, n_s, SF, SCR, dS);
    if (n_success) *n_success = n_s;

    /* population size reduction: keep the best np_next, in index order */
    if (np_next < np) {
        for (int i = 0; i < np; ++i) rank[i] = i;
        g_sort_keys = s->eX;
        qsort(rank, (size_t)np, sizeof(int32_t), cmp_rank);
        uint8_t *keep = (uint8_t *)calloc((size_t)np, 1);
        if (!keep) { free(rank); free(v); free(Fi); free(tmp); return -1; }
        for (int r = 0; r < np_next; ++r) keep[rank[r]] = 1;
        int32_t m = 0;
        for (int i = 0; i < np; ++i) {
            if (!keep[i]) continue;
            memcpy(tmp + (size_t)m * uD, s->X + (size_t)i * uD, sizeof(double) * uD);
            tmp[(size_t)np * uD + m] = s->eX[i];
            ++m;
        }
        for (int i = 0; i < np_next; ++i) {
            memcpy(s->X + (size_t)i * uD, tmp + (size_t)i * uD, sizeof(double) * uD);
            s->eX[i] = tmp[(size_t)np * uD + i];
        }
        free(keep);
        s->np = np_next;
        /* archive cut to its new bound by random removals */
        const int32_t amax2 = orc_lshade_archive_max(r_arc, np_next);
        for (uint32_t k = 0; s->na > amax2; ++k) {
            uint32_t wr[4];
            draw(run_uid, seed, t, k, ORC_TAG_LSHADE_S, 0, 0, wr);
            const int32_t at = (int32_t)orc_range(wr[0], (uint32_t)s->na);
            if (at != s->na - 1)
                memcpy(s->A + (size_t)at * uD, s->A + (size_t)(s->na - 1) * uD, sizeof(double) * uD);
            --s->na;
        }
    }
    free(rank); free(v); free(Fi); free(tmp);
    return 0;
}

int orc_lshade_generation(const orc_problem *pb, const double *o, const double *M, orc_lshade_state *s,
                          double p, double r_arc, int32_t np_next, uint32_t run_uid, uint64_t seed,
                          uint32_t t, double *U, double *eU, int32_t *n_success)
{
    return archive_generation(pb, o, M, s, p, r_arc, np_next, 0, 0.0, run_uid, seed, t, U, eU, n_success);
}

int orc_jade_generation(const orc_problem *pb, const double *o, const double *M, orc_lshade_state *s,
                        double p, double r_arc, double c, uint32_t run_uid, uint64_t seed, uint32_t t,
                        double *U, double *eU, int32_t *n_success)
{
    if (s->H != 1) return -1;
    return archive_generation(pb, o, M, s, p, r_arc, s->np, 1, c, run_uid, seed, t, U, eU, n_success);
}

/* ------------------------------------------------------------------------- */
/* PSODE (pairwise/3 selection). */

int orc_psode_generation(const orc_problem *pb, const double *o, const double *M, int32_t np,
                         int32_t topology, int32_t velocity, double w, double c1, double c2,
                         double vmax, double p, int32_t H, double *MF, double *MCR, int32_t *pos,
                         uint32_t run_uid, uint64_t seed, uint32_t t, double *X, double *eX, double *V,
                         double *Y, double *eY, double *U, double *eU, uint8_t *choice)
{
    const int D = pb->dim;
    if (np < 4) return -1;
    const size_t n = (size_t)np * (size_t)D;
    double *P = (double *)malloc(sizeof(double) * n);
    double *X3 = (double *)malloc(sizeof(double) * n);
    double *eP = (double *)malloc(sizeof(double) * (size_t)np);
    double *e3 = (double *)malloc(sizeof(double) * (size_t)np);
    uint8_t *rep = (uint8_t *)malloc((size_t)np);
    int rc = -1;
    if (!P || !X3 || !eP || !e3 || !rep) goto done;
    /* 1. the PSO half moves a copy; the personal bests are the population */
    memcpy(Y, X, sizeof(double) * n);
    memcpy(P, X, sizeof(double) * n);
    memcpy(eP, eX, sizeof(double) * (size_t)np);
    if (orc_pso_variant_iteration(pb, o, M, np, topology, velocity, w, c1, c2, vmax, run_uid, seed, t,
                                  Y, V, P, eY, eP, NULL) != 0)
        goto done;
    /* 2. the DE half: one SHADE generation with its own greedy selection */
    if (orc_shade_generation(pb, o, M, np, p, H, MF, MCR, pos, run_uid, seed, t, X, eX, U, eU, X3, e3,
                             NULL, NULL, NULL, NULL, NULL, rep, NULL) != 0)
        goto done;
    for (int i = 0; i < np; ++i) {
        double *x = X + (size_t)i * D, *v = V + (size_t)i * D;
        const double *x3 = X3 + (size_t)i * D, *y = Y + (size_t)i * D;
        /* 3. the velocity becomes the DE displacement */
        for (int j = 0; j < D; ++j) v[j] = x3[j] - x[j];
        /* 4. pairwise selection between the PSO move and the DE result */
        const int pso_wins = key_of(eY[i]) < key_of(e3[i]);
        memcpy(x, pso_wins ? y : x3, sizeof(double) * (size_t)D);
        eX[i] = pso_wins ? eY[i] : e3[i];
        if (choice) choice[i] = (uint8_t)(pso_wins ? 2 : (rep[i] ? 1 : 0));
    }
    rc = 0;
done:
    free(P); free(X3); free(eP); free(e3); free(rep);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* CSO. */

static const uint32_t *g_pair_keys;
static int cmp_pair(const void *a, const void *b)
{
    const int32_t ia = *(const int32_t *)a, ib = *(const int32_t *)b;
    const uint32_t ka = g_pair_keys[ia], kb = g_pair_keys[ib];
    if (ka != kb) return ka < kb ? -1 : 1;
    return ia < ib ? -1 : (ia > ib ? 1 : 0);
}

int orc_cso_iteration(const orc_problem *pb, const double *o, const double *M, int32_t m, double phi,
                      uint32_t run_uid, uint64_t seed, uint32_t t, double *X, double *V, double *e,
                      double *G, double *eG, int32_t *winner, int32_t *loser)
{
    const int D = pb->dim;
    if (m < 2 || m % 2 != 0) return -1;
    const int h = m / 2;
    uint32_t *keys = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)m);
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
    int32_t *lo = (int32_t *)malloc(sizeof(int32_t) * (size_t)h);
    double *xbar = (double *)calloc((size_t)D, sizeof(double));
    if (!keys || !perm || !lo || !xbar) { free(keys); free(perm); free(lo); free(xbar); return -1; }
    uint32_t w[4];
    /* random pairing: sort by the drawn key, then by index */
    for (int i = 0; i < m; ++i) {
        draw(run_uid, seed, t, (uint32_t)i, ORC_TAG_CSO_PAIR, 0, 0, w);
        keys[i] = w[0];
        perm[i] = i;
    }
    g_pair_keys = keys;
    qsort(perm, (size_t)m, sizeof(int32_t), cmp_pair);
    /* mean position of the swarm before the iteration */
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < D; ++j) xbar[j] += X[(size_t)i * D + j];
    for (int j = 0; j < D; ++j) xbar[j] /= (double)m;
    for (int k = 0; k < h; ++k) {
        const int32_t a = perm[2 * k], b = perm[2 * k + 1];
        const double ka = key_of(e[a]), kb = key_of(e[b]);
        const int a_wins = ka < kb || (ka == kb && a < b);
        const int32_t wi = a_wins ? a : b, li = a_wins ? b : a;
        if (winner) winner[k] = wi;
        if (loser) loser[k] = li;
        lo[k] = li;
        const double *xw = X + (size_t)wi * D;
        double *xl = X + (size_t)li * D, *vl = V + (size_t)li * D;
        for (int j = 0; j < D; ++j) {
            draw(run_uid, seed, t, (uint32_t)li, ORC_TAG_CSO_R, (uint32_t)j, 0, w);
            const double r1 = orc_u24(w[0]), r2 = orc_u24(w[1]), r3 = orc_u24(w[2]);
            double v = r1 * vl[j] + r2 * (xw[j] - xl[j]) + phi * r3 * (xbar[j] - xl[j]);
            double x = xl[j] + v;
            if (x < pb->lb) { x = pb->lb; v = 0.0; }
            else if (x > pb->ub) { x = pb->ub; v = 0.0; }
            xl[j] = x;
            vl[j] = v;
        }
        memcpy(G + (size_t)k * D, xl, sizeof(double) * (size_t)D);
    }
    orc_error_aos(pb->func, D, o, M, G, h, eG);
    for (int k = 0; k < h; ++k) e[lo[k]] = eG[k];
    free(keys); free(perm); free(lo); free(xbar);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Run driver. */

typedef struct {
    int64_t fe;
    int64_t budget;
    double best;          /* best over all evaluations so far */
    double best_budget;   /* best over the first `budget` evaluations */
    double *trace;
    int64_t trace_len;
    double *best_x;
    int dim;
} recorder;

static void record(recorder *r, double e, const double *x)
{
    r->fe += 1;
    if (key_of(e) < r->best) r->best = e;
    if (r->fe <= r->budget && key_of(e) < r->best_budget) {
        r->best_budget = e;
        if (r->best_x) memcpy(r->best_x, x, sizeof(double) * (size_t)r->dim);
    }
    if (r->trace && r->fe % ORC_TRACE_EVERY == 0) {
        int64_t k = r->fe / ORC_TRACE_EVERY - 1;
        if (k < r->trace_len) r->trace[k] = r->best;
    }
}

int orc_converged(const double *e, int32_t n, double tol)
{
    double lo = INFINITY, hi = -INFINITY;
    for (int i = 0; i < n; ++i) {
        const double k = key_of(e[i]);
        if (k < lo) lo = k;
        if (k > hi) hi = k;
    }
    return hi - lo <= tol;   /* false when an error is NaN or infinite */
}

/* Observer row g: (muF, muCR). */
static void observe(double *mu, int64_t mu_len, int64_t g, double muF, double muCR)
{
    if (mu && g < mu_len) {
        mu[2 * g] = muF;
        mu[2 * g + 1] = muCR;
    }
}

/* Observer row g of a success-history memory: the means of its H slots, a
 * terminal CR slot (negative) counted as the CR of 0 it gives. */
static void observe_memory(double *mu, int64_t mu_len, int64_t g, int H, const double *MF, const double *MCR)
{
    double f = 0.0, cr = 0.0;
    for (int k = 0; k < H; ++k) {
        f += MF[k];
        cr += MCR[k] < 0.0 ? 0.0 : MCR[k];
    }
    observe(mu, mu_len, g, f / H, cr / H);
}

int orc_run(const orc_run_desc *d, uint64_t seed, uint64_t inst_seed,
            orc_run_result *res, double *trace, int64_t trace_len, double *best_x)
{
    return orc_run_observed(d, seed, inst_seed, res, trace, trace_len, best_x, NULL, 0);
}

int orc_run_observed(const orc_run_desc *d, uint64_t seed, uint64_t inst_seed, orc_run_result *res,
                     double *trace, int64_t trace_len, double *best_x, double *mu, int64_t mu_len)
{
    int D = d->dim, np = d->np;
    if (D < 1 || np < 1) return -1;
    if ((d->algo == ORC_ALGO_DE || d->algo == ORC_ALGO_SHADE || d->algo == ORC_ALGO_LSHADE ||
         d->algo == ORC_ALGO_PSODE || d->algo == ORC_ALGO_JADE || d->algo == ORC_ALGO_LSHADE_RS) && np < 4)
        return -1;
    for (int64_t k = 0; mu && k < 2 * mu_len; ++k) mu[k] = NAN;
    orc_problem pb = { d->func, D, d->lb, d->ub };
    size_t pop = (size_t)np * D;
    double *o = (double *)malloc(sizeof(double) * (size_t)D);
    double *M = (double *)malloc(sizeof(double) * (size_t)D * D);
    double *buf = (double *)malloc(sizeof(double) * (pop * 4 + (size_t)np * 4));
    if (!o || !M || !buf) { free(o); free(M); free(buf); return -1; }
    if (orc_instance(d->func, D, d->instance, inst_seed, o, M, NULL) != 0) {
        free(o); free(M); free(buf); return -1;
    }
    double *X = buf, *A = buf + pop, *B = buf + 2 * pop, *C = buf + 3 * pop;
    double *eX = buf + 4 * pop, *eA = eX + np, *eB = eA + np, *eC = eB + np;
    for (int64_t k = 0; trace && k < trace_len; ++k) trace[k] = NAN;

    recorder rec = { 0, d->budget, INFINITY, INFINITY, trace, trace_len, best_x, D };
    int gens = 0, restarts = 0;
    int rc = 0;
    if (d->algo == ORC_ALGO_PSO) {
        double *V = A, *P = B, *eP = eA;
        int32_t g = 0;
        orc_pso_init(&pb, o, M, np, d->run_uid, seed, X, V, P, eX, eP, &g);
        for (int i = 0; i < np; ++i) record(&rec, eX[i], X + (size_t)i * D);
        while (rec.fe < d->budget) {
            ++gens;
            if (d->topology == 0 && d->velocity == 0)
                orc_pso_iteration(&pb, o, M, np, d->w, d->c1, d->c2, d->vmax, d->run_uid, seed,
                                  (uint32_t)gens, X, V, P, eX, eP, &g);
            else if (orc_pso_variant_iteration(&pb, o, M, np, d->topology, d->velocity, d->w, d->c1, d->c2,
                                               d->vmax, d->run_uid, seed, (uint32_t)gens, X, V, P, eX, eP,
                                               NULL) != 0) {
                rc = -1;
                break;
            }
            for (int i = 0; i < np; ++i) record(&rec, eX[i], X + (size_t)i * D);
        }
    } else if (d->algo == ORC_ALGO_DE || d->algo == ORC_ALGO_SHADE) {
        double *U = A, *Xn = B, *eU = eA, *eXn = eB;
        (void)C; (void)eC;
        double MF[64], MCR[64];
        int32_t pos = 0;
        int H = d->H > 0 ? d->H : 1;
        if (H > 64) H = 64;
        for (int k = 0; k < H; ++k) { MF[k] = 0.5; MCR[k] = 0.5; }
        orc_init_population(&pb, np, d->run_uid, seed, X);
        orc_error_aos(d->func, D, o, M, X, np, eX);
        for (int i = 0; i < np; ++i) record(&rec, eX[i], X + (size_t)i * D);
        if (d->algo == ORC_ALGO_DE) observe(mu, mu_len, 0, d->F, d->CR);
        else observe_memory(mu, mu_len, 0, H, MF, MCR);
        while (rec.fe < d->budget) {
            ++gens;
            if (d->algo == ORC_ALGO_DE)
                rc = orc_de_generation(&pb, o, M, np, d->F, d->CR, d->run_uid, seed,
                                       (uint32_t)gens, X, eX, U, eU, Xn, eXn, NULL, NULL, NULL);
            else
                rc = orc_shade_generation(&pb, o, M, np, d->p, H, MF, MCR, &pos, d->run_uid,
                                          seed, (uint32_t)gens, X, eX, U, eU, Xn, eXn,
                                          NULL, NULL, NULL, NULL, NULL, NULL, NULL);
            if (rc != 0) break;
            for (int i = 0; i < np; ++i) record(&rec, eU[i], U + (size_t)i * D);
            memcpy(X, Xn, sizeof(double) * pop);
            memcpy(eX, eXn, sizeof(double) * (size_t)np);
            if (d->algo == ORC_ALGO_DE) observe(mu, mu_len, gens, d->F, d->CR);
            else observe_memory(mu, mu_len, gens, H, MF, MCR);
        }
    } else if (d->algo == ORC_ALGO_LSHADE || d->algo == ORC_ALGO_JADE || d->algo == ORC_ALGO_LSHADE_RS) {
        const int jade = d->algo == ORC_ALGO_JADE;
        const int restart = d->algo == ORC_ALGO_LSHADE_RS;
        int64_t fe_r = 0;   /* evaluations before the current restart */
        const int32_t np_min = jade ? np : d->np_min;
        if (np_min < 4 || np_min > np) { free(o); free(M); free(buf); return -1; }
        orc_lshade_state st;
        memset(&st, 0, sizeof(st));
        st.np = np;
        st.H = jade ? 1 : d->H > 0 ? (d->H > 64 ? 64 : d->H) : 1;
        st.acap = orc_lshade_archive_max(d->r_arc, np) + 1;
        st.X = X;
        st.eX = eX;
        st.A = (double *)malloc(sizeof(double) * (size_t)st.acap * D);
        if (!st.A) { free(o); free(M); free(buf); return -1; }
        for (int k = 0; k < st.H; ++k) { st.MF[k] = 0.5; st.MCR[k] = 0.5; }
        double *U = A, *eU = eA;
        orc_init_population(&pb, np, d->run_uid, seed, X);
        orc_error_aos(d->func, D, o, M, X, np, eX);
        for (int i = 0; i < np; ++i) record(&rec, eX[i], X + (size_t)i * D);
        observe_memory(mu, mu_len, 0, st.H, st.MF, st.MCR);
        while (rec.fe < d->budget) {
            ++gens;
            const int32_t np_old = st.np;
            if (jade) {
                rc = orc_jade_generation(&pb, o, M, &st, d->p, d->r_arc, d->c, d->run_uid, seed,
                                         (uint32_t)gens, U, eU, NULL);
            } else {
                /* the size schedule runs from the latest restart to the budget */
                const int32_t np_next = orc_lshade_np(np, np_min, d->budget - fe_r, rec.fe - fe_r + np_old);
                rc = orc_lshade_generation(&pb, o, M, &st, d->p, d->r_arc,
                                           np_next < np_old ? np_next : np_old, d->run_uid, seed,
                                           (uint32_t)gens, U, eU, NULL);
            }
            if (rc != 0) break;
            for (int i = 0; i < np_old; ++i) record(&rec, eU[i], U + (size_t)i * D);
            observe_memory(mu, mu_len, gens, st.H, st.MF, st.MCR);
            if (restart && rec.fe < d->budget && orc_converged(st.eX, st.np, d->restart_tol)) {
                /* a fresh population of np_init, memories at 0.5, an empty
                   archive and the size schedule started over */
                ++restarts;
                fe_r = rec.fe;
                st.np = np;
                orc_restart_population(&pb, np, d->run_uid, seed, (uint32_t)restarts, X);
                orc_error_aos(d->func, D, o, M, X, np, eX);
                for (int i = 0; i < np; ++i) record(&rec, eX[i], X + (size_t)i * D);
                for (int k = 0; k < st.H; ++k) { st.MF[k] = 0.5; st.MCR[k] = 0.5; }
                st.pos = 0;
                st.na = 0;
            }
        }
        free(st.A);
    } else if (d->algo == ORC_ALGO_PSODE) {
        double *V = A, *Y = B, *U = C, *eY = eB, *eU = eC;
        double MF[64], MCR[64];
        int32_t pos = 0;
        int H = d->H > 0 ? (d->H > 64 ? 64 : d->H) : 1;
        for (int k = 0; k < H; ++k) { MF[k] = 0.5; MCR[k] = 0.5; }
        orc_init_population(&pb, np, d->run_uid, seed, X);
        orc_error_aos(d->func, D, o, M, X, np, eX);
        memset(V, 0, sizeof(double) * pop);
        for (int i = 0; i < np; ++i) record(&rec, eX[i], X + (size_t)i * D);
        observe_memory(mu, mu_len, 0, H, MF, MCR);
        while (rec.fe < d->budget) {
            ++gens;
            rc = orc_psode_generation(&pb, o, M, np, d->topology, d->velocity, d->w, d->c1, d->c2, d->vmax,
                                      d->p, H, MF, MCR, &pos, d->run_uid, seed, (uint32_t)gens, X, eX, V,
                                      Y, eY, U, eU, NULL);
            if (rc != 0) break;
            for (int i = 0; i < np; ++i) record(&rec, eY[i], Y + (size_t)i * D);
            for (int i = 0; i < np; ++i) record(&rec, eU[i], U + (size_t)i * D);
            observe_memory(mu, mu_len, gens, H, MF, MCR);
        }
    } else if (d->algo == ORC_ALGO_CSO) {
        double *V = A, *G = B, *eG = eA;
        if (np < 2 || np % 2 != 0) { free(o); free(M); free(buf); return -1; }
        orc_init_population(&pb, np, d->run_uid, seed, X);
        orc_error_aos(d->func, D, o, M, X, np, eX);
        memset(V, 0, sizeof(double) * pop);
        for (int i = 0; i < np; ++i) record(&rec, eX[i], X + (size_t)i * D);
        while (rec.fe < d->budget) {
            ++gens;
            rc = orc_cso_iteration(&pb, o, M, np, d->c1, d->run_uid, seed, (uint32_t)gens, X, V, eX, G, eG,
                                   NULL, NULL);
            if (rc != 0) break;
            for (int k = 0; k < np / 2; ++k) record(&rec, eG[k], G + (size_t)k * D);
        }
    } else {
        rc = -1;
    }
    if (res) {
        res->best_e = rec.best_budget;
        res->fes = rec.fe;
        res->generations = gens;
        res->success = rec.best_budget <= 1e-8;
        res->restarts = restarts;
    }
    free(o); free(M); free(buf);
    return rc;
}
