/*
 * sap_oracle.c -- plain, slow, obviously-correct FP64 CPU oracle for the
 * Secant-Avoidance Projection (SAP) method of Kvinge, Farnell, Kirby and
 * Peterson, "A GPU-Oriented Algorithm Design for Secant-Based Dimensionality
 * Reduction" (2018).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header, table or helper with
 * the HIP library; both consume the same seeded input bytes and nothing else.
 *
 * Conventions (all arrays row-major, all arithmetic FP64):
 *   X : N x n points.  FP32 inputs are promoted to FP64 by the caller; the
 *       promotion is exact, and so is the FP64 difference of two FP32 values.
 *   P : n x k, P[l*k + c] = component l of basis vector p_c.
 *   Pairs are unordered, i < j, with pair index
 *       q(i, j) = i*N - i*(i+1)/2 + (j - i - 1).
 *
 * What is computed, and where the paper defines it:
 *   - unit secants s = (x_i - x_j)/||x_i - x_j|| for all distinct pairs
 *     (Sec. 2 and Sec. 4, the displayed definition of s);
 *   - the projected norm r_ij = ||P^T s_ij|| and its minimum and argmin over
 *     the secant set (Sec. 4, the objective argmax_P min_s ||P^T s||, and
 *     Algorithm 1, the argmin step);
 *   - the update: pick the basis vector most aligned with the worst secant,
 *     modified Gram-Schmidt on {P P^T s, the other basis vectors}, then replace
 *     the first vector by the unit vector along (1-a) P P^T s + a (s - P P^T s)
 *     (Sec. 4 prose and Algorithm 1, the argmax / MGS / shift steps);
 *   - the length threshold: secants shorter than min_len are discarded before
 *     normalisation (Sec. 7);
 *   - the soft-min loss L = -tau log sum exp(-r_ij/tau) and its gradient in P,
 *     which the paper does not contain: it is the differentiable surrogate of
 *     the same min, defined here from first principles (d r / d P = s c^T / r).
 *
 * Readings where the paper is silent or ambiguous:
 *   - duplicate points (d = 0) have no unit secant and are dropped; so is any
 *     secant with d < min_len (min_len = 0 still drops d = 0);
 *   - argmin ties go to the lexicographically smallest (r, i, j);
 *   - argmax ties (choice of p_t) go to the smallest index;
 *   - if every <p_c, s> is exactly zero the paper says to take p_1; then
 *     P P^T s = 0 cannot be normalised, and the only consistent reading is
 *     u = unit(a s) = s, giving P' = [s, p_2, ..., p_k] (s is orthogonal to
 *     span(P), so P' is orthonormal);
 *   - the shift combines the *unnormalised* P P^T s and s - P P^T s (literal
 *     reading, rule 0).  Rule 1 combines their unit vectors instead.
 *   - the loop runs `iters` updates; the trace holds iters+1 evaluations,
 *     the last one for the returned P.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_EARG 1
#define ORACLE_ENOPAIRS 2
#define ORACLE_EDEGENERATE 3
#define ORACLE_ENOMEM 4

typedef struct {
    double r_min;      /* min over kept pairs of ||P^T s_ij||            */
    int64_t i, j;      /* its pair, lexicographically smallest (r, i, j) */
    double r_second;   /* second entry of the sorted (r, i, j) list      */
    int64_t i2, j2;
    double r_max;      /* max over kept pairs (projection bound check)   */
    int64_t n_pairs;   /* number of kept pairs                           */
    int64_t n_dropped; /* duplicates and secants shorter than min_len    */
} oracle_min_t;

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

int64_t oracle_pair_index(int64_t N, int64_t i, int64_t j) {
    return i * N - i * (i + 1) / 2 + (j - i - 1);
}

/* Unit secant of pair (i, j): s = (x_i - x_j) / ||x_i - x_j||.
 * Returns the length d (0 for a duplicate, in which case s is untouched). */
static double unit_secant(const double *X, int32_t n, int64_t i, int64_t j,
                          double *s) {
    const double *xi = X + (size_t)i * n, *xj = X + (size_t)j * n;
    double d2 = 0.0;
    for (int32_t l = 0; l < n; ++l) {
        double t = xi[l] - xj[l];
        s[l] = t;
        d2 += t * t;
    }
    double d = sqrt(d2);
    if (d > 0.0)
        for (int32_t l = 0; l < n; ++l) s[l] = s[l] / d;
    return d;
}

/* Exported form of unit_secant for callers that need s itself. */
double oracle_unit_secant(const double *X, int64_t N, int32_t n, int64_t i,
                          int64_t j, double *s) {
    if (!X || !s || i < 0 || j < 0 || i >= N || j >= N || i == j) return -1.0;
    return unit_secant(X, n, i < j ? i : j, i < j ? j : i, s);
}

/* c = P^T s (k values) and returns ||c||. */
static double project_norm(const double *P, int32_t n, int32_t k,
                           const double *s, double *c) {
    for (int32_t q = 0; q < k; ++q) c[q] = 0.0;
    for (int32_t l = 0; l < n; ++l)
        for (int32_t q = 0; q < k; ++q) c[q] += P[(size_t)l * k + q] * s[l];
    double r2 = 0.0;
    for (int32_t q = 0; q < k; ++q) r2 += c[q] * c[q];
    return sqrt(r2);
}

/* lexicographic (r, i, j) order */
static int lex_less(double r, int64_t i, int64_t j, double r2, int64_t i2,
                    int64_t j2) {
    if (r != r2) return r < r2;
    if (i != i2) return i < i2;
    return j < j2;
}

typedef struct {
    double r[2];
    int64_t i[2], j[2];
    double rmax;
    int64_t kept, dropped;
} top2_t;

static void top2_init(top2_t *t) {
    t->r[0] = t->r[1] = INFINITY;
    t->i[0] = t->i[1] = t->j[0] = t->j[1] = INT64_MAX;
    t->rmax = -INFINITY;
    t->kept = t->dropped = 0;
}

static void top2_push(top2_t *t, double r, int64_t i, int64_t j) {
    if (lex_less(r, i, j, t->r[0], t->i[0], t->j[0])) {
        t->r[1] = t->r[0]; t->i[1] = t->i[0]; t->j[1] = t->j[0];
        t->r[0] = r; t->i[0] = i; t->j[0] = j;
    } else if (lex_less(r, i, j, t->r[1], t->i[1], t->j[1])) {
        t->r[1] = r; t->i[1] = i; t->j[1] = j;
    }
}

/* Minimum projected unit-secant norm over the kept secant set. */
int oracle_min_secant(const double *X, int64_t N, int32_t n, const double *P,
                      int32_t k, double min_len, oracle_min_t *out) {
    if (!X || !P || !out || N < 2 || n < 1 || k < 1 || k > n || min_len < 0)
        return ORACLE_EARG;
    top2_t best;
    top2_init(&best);
    int fail = 0;
#pragma omp parallel
    {
        top2_t loc;
        top2_init(&loc);
        double *s = (double *)malloc(sizeof(double) * (size_t)n);
        double *c = (double *)malloc(sizeof(double) * (size_t)k);
        const int ok = s && c;
        if (!ok) {
#pragma omp atomic write
            fail = 1;
        }
        {
#pragma omp for schedule(dynamic, 4)
            for (int64_t i = 0; i < N - 1; ++i) {
                if (!ok) continue;
                for (int64_t j = i + 1; j < N; ++j) {
                    double d = unit_secant(X, n, i, j, s);
                    if (d == 0.0 || d < min_len) { loc.dropped++; continue; }
                    double r = project_norm(P, n, k, s, c);
                    loc.kept++;
                    if (r > loc.rmax) loc.rmax = r;
                    top2_push(&loc, r, i, j);
                }
            }
        }
#pragma omp critical
        {
            for (int m = 0; m < 2; ++m)
                if (loc.r[m] < INFINITY) top2_push(&best, loc.r[m], loc.i[m], loc.j[m]);
            if (loc.rmax > best.rmax) best.rmax = loc.rmax;
            best.kept += loc.kept;
            best.dropped += loc.dropped;
        }
        free(s);
        free(c);
    }
    if (fail) return ORACLE_ENOMEM;
    out->n_pairs = best.kept;
    out->n_dropped = best.dropped;
    if (best.kept == 0) return ORACLE_ENOPAIRS;
    out->r_min = best.r[0]; out->i = best.i[0]; out->j = best.j[0];
    out->r_second = best.r[1]; out->i2 = best.i[1]; out->j2 = best.j[1];
    out->r_max = best.rmax;
    return ORACLE_OK;
}

/* r and d of one pair (any order of i, j; i != j). */
int oracle_pair_r(const double *X, int64_t N, int32_t n, const double *P,
                  int32_t k, int64_t i, int64_t j, double *r, double *d) {
    if (!X || !P || !r || !d || i < 0 || j < 0 || i >= N || j >= N || i == j)
        return ORACLE_EARG;
    double *s = (double *)malloc(sizeof(double) * (size_t)n);
    double *c = (double *)malloc(sizeof(double) * (size_t)k);
    if (!s || !c) { free(s); free(c); return ORACLE_ENOMEM; }
    int64_t a = i < j ? i : j, b = i < j ? j : i;
    *d = unit_secant(X, n, a, b, s);
    *r = (*d > 0.0) ? project_norm(P, n, k, s, c) : NAN;
    free(s);
    free(c);
    return ORACLE_OK;
}

/* r of a list of pairs ij[2e], ij[2e+1] (NaN for a duplicate). */
int oracle_pairs_r(const double *X, int64_t N, int32_t n, const double *P,
                   int32_t k, const int64_t *ij, int64_t count, double *r_out) {
    if (!X || !P || !ij || !r_out || count < 0) return ORACLE_EARG;
    for (int64_t e = 0; e < count; ++e) {
        int64_t i = ij[2 * e], j = ij[2 * e + 1];
        if (i < 0 || j < 0 || i >= N || j >= N || i == j) return ORACLE_EARG;
    }
    int fail = 0;
#pragma omp parallel
    {
        double *s = (double *)malloc(sizeof(double) * (size_t)n);
        double *c = (double *)malloc(sizeof(double) * (size_t)k);
        const int ok = s && c;
        if (!ok) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(static)
        for (int64_t e = 0; e < count; ++e) {
            if (!ok) continue;
            int64_t i = ij[2 * e], j = ij[2 * e + 1];
            int64_t a = i < j ? i : j, b = i < j ? j : i;
            double d = unit_secant(X, n, a, b, s);
            r_out[e] = d > 0.0 ? project_norm(P, n, k, s, c) : NAN;
        }
        free(s);
        free(c);
    }
    return fail ? ORACLE_ENOMEM : ORACLE_OK;
}

/* Every pair's r (NaN for a dropped pair) and d, in pair-index order. */
int oracle_all_r(const double *X, int64_t N, int32_t n, const double *P,
                 int32_t k, double min_len, double *r_out, double *d_out) {
    if (!X || !P || !r_out || N < 2 || k < 1 || k > n) return ORACLE_EARG;
    int fail = 0;
#pragma omp parallel
    {
        double *s = (double *)malloc(sizeof(double) * (size_t)n);
        double *c = (double *)malloc(sizeof(double) * (size_t)k);
        const int ok = s && c;
        if (!ok) {
#pragma omp atomic write
            fail = 1;
        }
        {
#pragma omp for schedule(dynamic, 4)
            for (int64_t i = 0; i < N - 1; ++i) {
                if (!ok) continue;
                for (int64_t j = i + 1; j < N; ++j) {
                    int64_t q = oracle_pair_index(N, i, j);
                    double d = unit_secant(X, n, i, j, s);
                    if (d_out) d_out[q] = d;
                    r_out[q] = (d == 0.0 || d < min_len) ? NAN
                                                         : project_norm(P, n, k, s, c);
                }
            }
        }
        free(s);
        free(c);
    }
    return fail ? ORACLE_ENOMEM : ORACLE_OK;
}

/* One SAP update (Sec. 4; Algorithm 1, the argmax, MGS and shift steps).
 * s is the worst unit secant; P_out receives P' (n x k).  t_out receives the
 * chosen column p_t (0-based).  rule 0 = literal shift, 1 = unit-vector shift. */
int oracle_step(const double *P, int32_t n, int32_t k, const double *s,
                double alpha, int32_t rule, double *P_out, int32_t *t_out) {
    if (!P || !s || !P_out || n < 1 || k < 1 || k > n || !(alpha >= 0.0) ||
        !(alpha <= 1.0) || (rule != 0 && rule != 1))
        return ORACLE_EARG;
    double *c = (double *)malloc(sizeof(double) * (size_t)k);
    double *A = (double *)malloc(sizeof(double) * (size_t)n * k); /* vectors, one per row */
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
    double *u = (double *)malloc(sizeof(double) * (size_t)n);
    int st = ORACLE_OK;
    if (!c || !A || !v || !u) { st = ORACLE_ENOMEM; goto done; }

    /* c = P^T s: the inner products <p_c, s> */
    for (int32_t q = 0; q < k; ++q) {
        double acc = 0.0;
        for (int32_t l = 0; l < n; ++l) acc += P[(size_t)l * k + q] * s[l];
        c[q] = acc;
    }
    /* p_t = argmax |<p_c, s>|, first index on ties */
    int32_t t = 0;
    double cmax = fabs(c[0]);
    for (int32_t q = 1; q < k; ++q)
        if (fabs(c[q]) > cmax) { cmax = fabs(c[q]); t = q; }
    if (t_out) *t_out = t;

    if (cmax == 0.0) {
        /* every <p_c, s> is zero: p_t = p_1, and the new first vector is s */
        for (int32_t l = 0; l < n; ++l) {
            P_out[(size_t)l * k] = s[l];
            for (int32_t q = 1; q < k; ++q)
                P_out[(size_t)l * k + q] = P[(size_t)l * k + q];
        }
        goto done;
    }

    /* v = P P^T s = P c */
    for (int32_t l = 0; l < n; ++l) {
        double acc = 0.0;
        for (int32_t q = 0; q < k; ++q) acc += P[(size_t)l * k + q] * c[q];
        v[l] = acc;
    }
    /* ordered input of MGS: v, then p_1..p_k without p_t */
    for (int32_t l = 0; l < n; ++l) A[l] = v[l];
    for (int32_t q = 0, m = 1; q < k; ++q) {
        if (q == t) continue;
        for (int32_t l = 0; l < n; ++l) A[(size_t)m * n + l] = P[(size_t)l * k + q];
        ++m;
    }
    /* modified Gram-Schmidt: each vector loses its component along every
     * earlier result vector, one at a time, then is normalised */
    for (int32_t m = 0; m < k; ++m) {
        double *a = A + (size_t)m * n;
        for (int32_t p = 0; p < m; ++p) {
            const double *qv = A + (size_t)p * n;
            double dot = 0.0;
            for (int32_t l = 0; l < n; ++l) dot += qv[l] * a[l];
            for (int32_t l = 0; l < n; ++l) a[l] -= dot * qv[l];
        }
        double nrm = 0.0;
        for (int32_t l = 0; l < n; ++l) nrm += a[l] * a[l];
        nrm = sqrt(nrm);
        if (!(nrm > 0.0)) { st = ORACLE_EDEGENERATE; goto done; }
        for (int32_t l = 0; l < n; ++l) a[l] /= nrm;
    }
    /* the shift: u along (1-a) v + a (s - v) */
    if (rule == 0) {
        for (int32_t l = 0; l < n; ++l)
            u[l] = (1.0 - alpha) * v[l] + alpha * (s[l] - v[l]);
    } else {
        double nv = 0.0, nw = 0.0;
        for (int32_t l = 0; l < n; ++l) {
            nv += v[l] * v[l];
            nw += (s[l] - v[l]) * (s[l] - v[l]);
        }
        nv = sqrt(nv);
        nw = sqrt(nw);
        for (int32_t l = 0; l < n; ++l)
            u[l] = (1.0 - alpha) * v[l] / nv + (nw > 0.0 ? alpha * (s[l] - v[l]) / nw : 0.0);
    }
    double nu = 0.0;
    for (int32_t l = 0; l < n; ++l) nu += u[l] * u[l];
    nu = sqrt(nu);
    if (!(nu > 0.0)) { st = ORACLE_EDEGENERATE; goto done; }
    for (int32_t l = 0; l < n; ++l) {
        P_out[(size_t)l * k] = u[l] / nu;
        for (int32_t q = 1; q < k; ++q) P_out[(size_t)l * k + q] = A[(size_t)q * n + l];
    }
done:
    free(c); free(A); free(v); free(u);
    return st;
}

/* max_{a,b} |(P^T P - I)_{ab}| */
double oracle_orth_error(const double *P, int32_t n, int32_t k) {
    double e = 0.0;
    for (int32_t a = 0; a < k; ++a)
        for (int32_t b = 0; b < k; ++b) {
            double acc = 0.0;
            for (int32_t l = 0; l < n; ++l)
                acc += P[(size_t)l * k + a] * P[(size_t)l * k + b];
            double d = fabs(acc - (a == b ? 1.0 : 0.0));
            if (d > e) e = d;
        }
    return e;
}

/* Algorithm 1 from a given start P0: `iters` updates, iters+1 evaluations.
 * Traces (each iters+1 long, any may be NULL): min, (i, j) pairs interleaved,
 * runner-up value, orthonormality error of the evaluated P. */
int oracle_run(const double *X, int64_t N, int32_t n, const double *P0,
               int32_t k, double alpha, double min_len, int32_t rule,
               int32_t iters, double *P_out, double *tr_min, int64_t *tr_ij,
               double *tr_second, double *tr_orth) {
    if (!X || !P0 || !P_out || iters < 0) return ORACLE_EARG;
    size_t nk = (size_t)n * k;
    double *P = (double *)malloc(sizeof(double) * nk);
    double *Pn = (double *)malloc(sizeof(double) * nk);
    double *s = (double *)malloc(sizeof(double) * (size_t)n);
    int st = ORACLE_OK;
    if (!P || !Pn || !s) { st = ORACLE_ENOMEM; goto done; }
    memcpy(P, P0, sizeof(double) * nk);
    for (int32_t it = 0; it <= iters; ++it) {
        oracle_min_t m;
        st = oracle_min_secant(X, N, n, P, k, min_len, &m);
        if (st) goto done;
        if (tr_min) tr_min[it] = m.r_min;
        if (tr_ij) { tr_ij[2 * it] = m.i; tr_ij[2 * it + 1] = m.j; }
        if (tr_second) tr_second[it] = m.r_second;
        if (tr_orth) tr_orth[it] = oracle_orth_error(P, n, k);
        if (it == iters) break;
        (void)unit_secant(X, n, m.i, m.j, s);
        st = oracle_step(P, n, k, s, alpha, rule, Pn, NULL);
        if (st) goto done;
        memcpy(P, Pn, sizeof(double) * nk);
    }
    memcpy(P_out, P, sizeof(double) * nk);
done:
    free(P); free(Pn); free(s);
    return st;
}

/* The secant matrix S of Sec. 4: every kept unit secant as a column (pairs
 * in pair-index order; dropped pairs -- duplicates, d < min_len -- are left
 * out).  S is n x cap, column-major (column q at S + q*n).  Returns the
 * number of columns written, or -1 if cap is too small or an argument is
 * bad. */
int64_t oracle_secant_matrix(const double *X, int64_t N, int32_t n, double min_len,
                             double *S, int64_t cap) {
    if (!X || !S || N < 2 || n < 1 || min_len < 0) return -1;
    int64_t q = 0;
    for (int64_t i = 0; i < N - 1; ++i)
        for (int64_t j = i + 1; j < N; ++j) {
            if (q >= cap) return -1;
            double d = unit_secant(X, n, i, j, S + (size_t)q * n);
            if (d == 0.0 || d < min_len) continue;   /* the column is overwritten next */
            ++q;
        }
    return q;
}

/* Kahan-compensated running sum */
typedef struct { double s, c; } ksum_t;
static void kadd(ksum_t *k, double x) {
    double y = x - k->c;
    double t = k->s + y;
    k->c = (t - k->s) - y;
    k->s = t;
}

/* Soft-min of the projected unit-secant norms and its gradient in P.
 *   L = -tau log sum_ij exp(-r_ij / tau)
 *     = r_min - tau log sum_ij exp(-(r_ij - r_min)/tau)
 *   dL/dP = sum_ij w_ij s_ij c_ij^T / r_ij,  c = P^T s,
 *   w_ij  = exp(-(r_ij - L)/tau)  (so that sum w = 1).
 * A pair with r_ij = 0 has no gradient; it adds 0 and is counted in n_zero.
 * Sums run row by row (Kahan within a row) and rows are added in order, so
 * the result does not depend on the thread count.  G may be NULL. */
int oracle_softmin(const double *X, int64_t N, int32_t n, const double *P,
                   int32_t k, double tau, double min_len, double *L_out,
                   double *G, double *wsum_out, int64_t *n_pairs,
                   int64_t *n_zero) {
    if (!X || !P || !L_out || N < 2 || k < 1 || k > n || !(tau > 0.0) ||
        min_len < 0)
        return ORACLE_EARG;
    oracle_min_t m;
    int st = oracle_min_secant(X, N, n, P, k, min_len, &m);
    if (st) return st;
    const double rmin = m.r_min;
    const int64_t BR = 64; /* rows per gradient block */
    const int64_t nblk = (N + BR - 1) / BR;
    double *rowsum = (double *)calloc((size_t)N, sizeof(double));
    double *Gb = G ? (double *)calloc((size_t)nblk * n * k, sizeof(double)) : NULL;
    int64_t *zb = (int64_t *)calloc((size_t)nblk, sizeof(int64_t));
    if (!rowsum || (G && !Gb) || !zb) {
        free(rowsum); free(Gb); free(zb);
        return ORACLE_ENOMEM;
    }
    /* pass 1: the partition sum */
    int fail = 0;
#pragma omp parallel
    {
        double *s = (double *)malloc(sizeof(double) * (size_t)n);
        double *c = (double *)malloc(sizeof(double) * (size_t)k);
        const int ok = s && c;
        if (!ok) {
#pragma omp atomic write
            fail = 1;
        }
        {
#pragma omp for schedule(dynamic, 4)
            for (int64_t i = 0; i < N - 1; ++i) {
                if (!ok) continue;
                ksum_t acc = {0.0, 0.0};
                for (int64_t j = i + 1; j < N; ++j) {
                    double d = unit_secant(X, n, i, j, s);
                    if (d == 0.0 || d < min_len) continue;
                    double r = project_norm(P, n, k, s, c);
                    kadd(&acc, exp(-(r - rmin) / tau));
                }
                rowsum[i] = acc.s;
            }
        }
        free(s); free(c);
    }
    if (fail) { free(rowsum); free(Gb); free(zb); return ORACLE_ENOMEM; }
    ksum_t tot = {0.0, 0.0};
    for (int64_t i = 0; i < N; ++i) kadd(&tot, rowsum[i]);
    const double L = rmin - tau * log(tot.s);
    *L_out = L;
    if (n_pairs) *n_pairs = m.n_pairs;

    /* pass 2: weights and gradient, blocked by rows */
    ksum_t wtot = {0.0, 0.0};
#pragma omp parallel
    {
        double *s = (double *)malloc(sizeof(double) * (size_t)n);
        double *c = (double *)malloc(sizeof(double) * (size_t)k);
        const int ok = s && c;
        if (!ok) {
#pragma omp atomic write
            fail = 1;
        }
        {
#pragma omp for schedule(dynamic, 1)
            for (int64_t b = 0; b < nblk; ++b) {
                if (!ok) continue;
                double *g = Gb ? Gb + (size_t)b * n * k : NULL;
                int64_t i1 = (b + 1) * BR < N ? (b + 1) * BR : N;
                for (int64_t i = b * BR; i < i1; ++i) {
                    ksum_t acc = {0.0, 0.0};
                    for (int64_t j = i + 1; j < N; ++j) {
                        double d = unit_secant(X, n, i, j, s);
                        if (d == 0.0 || d < min_len) continue;
                        double r = project_norm(P, n, k, s, c);
                        double w = exp(-(r - L) / tau);
                        kadd(&acc, w);
                        if (r == 0.0) { zb[b]++; continue; }
                        if (g) {
                            double f = w / r;
                            for (int32_t l = 0; l < n; ++l)
                                for (int32_t q = 0; q < k; ++q)
                                    g[(size_t)l * k + q] += f * s[l] * c[q];
                        }
                    }
                    rowsum[i] = acc.s;
                }
            }
        }
        free(s); free(c);
    }
    if (fail) { free(rowsum); free(Gb); free(zb); return ORACLE_ENOMEM; }
    for (int64_t i = 0; i < N; ++i) kadd(&wtot, rowsum[i]);
    if (wsum_out) *wsum_out = wtot.s;
    int64_t nz = 0;
    for (int64_t b = 0; b < nblk; ++b) nz += zb[b];
    if (n_zero) *n_zero = nz;
    if (G) {
        memset(G, 0, sizeof(double) * (size_t)n * k);
        for (int64_t b = 0; b < nblk; ++b)
            for (size_t e = 0; e < (size_t)n * k; ++e) G[e] += Gb[(size_t)b * n * k + e];
    }
    free(rowsum); free(Gb); free(zb);
    return ORACLE_OK;
}
