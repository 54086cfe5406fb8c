/*
 * cm_oracle.c -- plain FP64 CPU oracle of the learned cost model and of beam
 * selection, from Anderson et al., "Efficient Automatic Scheduling of Imaging
 * and Vision Pipelines for the GPU" (OOPSLA 2021).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * definition that the GPU path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never calls it and shares no code, header or table with it.
 *
 * Everything is computed in double precision from float32 inputs widened
 * exactly, with scalar loops in the order the paper states the model
 * (Sec. 5.2): log transform of the features, two fully connected embeddings,
 * the embeddings stacked, a fully connected layer, a second one giving
 * non-negative coefficients, the coefficients applied to the hand-derived
 * per-stage cost terms (App. B: every cost component is linear in the learned
 * coefficients), and the per-stage predictions summed over all stages.
 * Build: gcc -O2 -ffp-contract=off -fopenmp (no fast-math).
 *
 * Readings where the paper is silent (each listed in the design notes):
 *  - both feature groups are log-transformed with log1p (operation counts can
 *    be zero);
 *  - there is no activation after the embeddings;
 *  - "positive weights" are produced by a ReLU, so exact zeros are allowed;
 *    the ReLU lets a NaN through (as the usual ML-framework ReLU does), so an
 *    invalid feature gives a NaN cost instead of a silently finite one;
 *  - every layer has a bias;
 *  - the algorithm-specific features are one vector per (query, stage),
 *    shared by all candidates of the query;
 *  - the best candidate is the one with the lowest predicted runtime; ties go
 *    to the lower candidate index; -0 equals +0; NaN ranks after +inf.
 *
 * The FP8 form (cmo_eval_fp8) is the same model evaluated with the
 * quantization points of the 8-bit precision form (the paper fixes no
 * precision; this form is a reading): e4m3 codes of log1p(x) * s_in as
 * inputs, the schedule embedding folded into the first layer, per-layer
 * power-of-two weight scales, hidden activations quantized with a given
 * scale; everything between the quantization points in FP64.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "cm_oracle.h"

/* Parameter blob layout: W_p[24][56] b_p[24] W_s[24][40] b_s[24]
 * W_1[32][48] b_1[32] W_2[8][32] b_2[8]; matrices are [out][in]. */
#define FP 56
#define FS 40
#define E 24
#define H 32
#define C 8

typedef struct {
    const float *Wp, *bp, *Ws, *bs, *W1, *b1, *W2, *b2;
} cmo_params;

static cmo_params split_params(const float *blob)
{
    cmo_params p;
    const float *q = blob;
    p.Wp = q; q += E * FP;
    p.bp = q; q += E;
    p.Ws = q; q += E * FS;
    p.bs = q; q += E;
    p.W1 = q; q += H * 2 * E;
    p.b1 = q; q += H;
    p.W2 = q; q += C * H;
    p.b2 = q; q += C;
    return p;
}

int32_t cmo_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int32_t cmo_n_params(void) { return E * FP + E + E * FS + E + H * 2 * E + H + C * H + C; }

/* One (candidate, stage) evaluation, Sec. 5.2: coefficients c[8] and the
 * stage's predicted cost sum_j c_j * t_j. */
static double stage_eval(const cmo_params *P, const float *pipe_s,
                         const float *sched_si, const float *terms_si,
                         double *coef_out)
{
    double p[FP], x[FS], z[2 * E], h[H], c[C];
    /* log transform of both feature groups */
    for (int f = 0; f < FP; ++f) p[f] = log1p((double)pipe_s[f]);
    for (int f = 0; f < FS; ++f) x[f] = log1p((double)sched_si[f]);
    /* two embeddings, stacked: algorithm embedding first */
    for (int e = 0; e < E; ++e) {
        double a = (double)P->bp[e];
        for (int f = 0; f < FP; ++f) a += (double)P->Wp[e * FP + f] * p[f];
        z[e] = a;
    }
    for (int e = 0; e < E; ++e) {
        double a = (double)P->bs[e];
        for (int f = 0; f < FS; ++f) a += (double)P->Ws[e * FS + f] * x[f];
        z[E + e] = a;
    }
    /* fully connected layer with ReLU */
    for (int j = 0; j < H; ++j) {
        double a = (double)P->b1[j];
        for (int k = 0; k < 2 * E; ++k) a += (double)P->W1[j * 2 * E + k] * z[k];
        h[j] = a < 0.0 ? 0.0 : a; /* ReLU; a NaN passes through */
    }
    /* output layer with ReLU: the non-negative coefficients */
    for (int m = 0; m < C; ++m) {
        double a = (double)P->b2[m];
        for (int j = 0; j < H; ++j) a += (double)P->W2[m * H + j] * h[j];
        c[m] = a < 0.0 ? 0.0 : a;
    }
    /* coefficients weight the hand-derived cost terms (App. B) */
    double v = 0.0;
    for (int m = 0; m < C; ++m) v += c[m] * (double)terms_si[m];
    if (coef_out)
        for (int m = 0; m < C; ++m) coef_out[m] = c[m];
    return v;
}

void cmo_eval(const float *params, int32_t S, int32_t N, const float *pipe,
              const float *sched, const float *terms, double *cost_out,
              double *stage_cost_out, double *coef_out, int32_t nthreads)
{
    cmo_params P = split_params(params);
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
#endif
    for (int64_t i = 0; i < (int64_t)N; ++i) {
        /* per-stage predictions summed over all stages, ascending stage order */
        double total = 0.0;
        for (int64_t s = 0; s < (int64_t)S; ++s) {
            const int64_t row = s * (int64_t)N + i;
            double *co = coef_out ? coef_out + row * C : NULL;
            double v = stage_eval(&P, pipe + s * FP, sched + row * FS,
                                  terms + row * C, co);
            if (stage_cost_out) stage_cost_out[row] = v;
            total += v;
        }
        cost_out[i] = total;
    }
    (void)nthreads;
}

/* ---- FP8 (e4m3) form ---- */

/* OCP 8-bit floating point E4M3: sign, 4 exponent bits (bias 7), 3 mantissa
 * bits; exponent 0 holds subnormals m * 2^-9; no infinities; exponent 15 with
 * mantissa 7 is NaN, so the largest finite magnitude is 1.75 * 2^8 = 448. */
double cmo_e4m3_decode(uint8_t code)
{
    const int sign = code >> 7, e = (code >> 3) & 15, m = code & 7;
    if (e == 15 && m == 7) return NAN;
    const double v = e == 0 ? ldexp((double)m, -9) : ldexp(1.0 + m / 8.0, e - 7);
    return sign ? -v : v;
}

/* Nearest e4m3 value, ties to the even code (the code's last bit is the
 * mantissa's last bit), magnitudes at or above 448 saturate to 448, NaN maps
 * to the positive NaN code.  Found by comparing against every finite code;
 * val[c] holds the value of code c for c < 0x7F. */
static uint8_t nearest_code(const double *val, double v)
{
    if (isnan(v)) return 0x7F;
    const uint8_t sign = signbit(v) ? 0x80 : 0x00;
    const double a = fabs(v);
    if (a >= 448.0) return sign | 0x7E;
    int best = 0;
    double bd = INFINITY;
    for (int c = 0; c <= 0x7E; ++c) {
        const double d = fabs(val[c] - a);
        if (d < bd || (d == bd && (c & 1) == 0)) {
            bd = d;
            best = c;
        }
    }
    return (uint8_t)(sign | best);
}

static void code_values(double *val)
{
    for (int c = 0; c <= 0x7E; ++c) val[c] = cmo_e4m3_decode((uint8_t)c);
}

uint8_t cmo_e4m3_encode(double v)
{
    double val[0x7F];
    code_values(val);
    return nearest_code(val, v);
}

/* The largest power of two not above 448 / amax (1 when amax is 0). */
double cmo_fp8_scale(double amax)
{
    if (!(amax > 0.0)) return 1.0;
    int e;
    frexp(448.0 / amax, &e);
    return ldexp(1.0, e - 1);
}

static double q8(double v) { return cmo_e4m3_decode(cmo_e4m3_encode(v)); }

void cmo_fp8_codes(const float *x, int64_t n, double in_scale, uint8_t *out)
{
    double val[0x7F];
    code_values(val);
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int64_t i = 0; i < n; ++i) out[i] = nearest_code(val, log1p((double)x[i]) * in_scale);
}

/* How far the e4m3 value of x >= 0 may move when x is only known to within
 * +-e: rounding is monotone, so any value x' in [x - e, x + e] rounds to a
 * value between those of x - e and x + e, and so does x itself. */
static double rounding_swing(double x, double e)
{
    return q8(x + e) - q8(x - e < 0.0 ? 0.0 : x - e);
}

void cmo_eval_fp8(const float *params, double in_scale, double act_scale, int32_t S,
                  int32_t N, const float *pipe, const uint8_t *codes, const float *terms,
                  double *cost_out, double acc_tol, double *bound_out, int32_t nthreads,
                  double *stage_cost_out, double *stage_bound_out)
{
    const int want_bound = bound_out != NULL || stage_bound_out != NULL;
    cmo_params P = split_params(params);
    /* folded first layer over the schedule features and its bias share */
    double Wf[H][FS], beta[H], Wq1[H][FS], Wq2[C][H];
    double amax1 = 0.0, amax2 = 0.0;
    for (int h = 0; h < H; ++h) {
        double b = 0.0;
        for (int e = 0; e < E; ++e) b += (double)P.W1[h * 2 * E + E + e] * (double)P.bs[e];
        beta[h] = b;
        for (int f = 0; f < FS; ++f) {
            double a = 0.0;
            for (int e = 0; e < E; ++e)
                a += (double)P.W1[h * 2 * E + E + e] * (double)P.Ws[e * FS + f];
            Wf[h][f] = a;
            if (fabs(a) > amax1) amax1 = fabs(a);
        }
    }
    for (int c = 0; c < C; ++c)
        for (int h = 0; h < H; ++h)
            if (fabs((double)P.W2[c * H + h]) > amax2) amax2 = fabs((double)P.W2[c * H + h]);
    const double sw1 = cmo_fp8_scale(amax1), sw2 = cmo_fp8_scale(amax2);
    for (int h = 0; h < H; ++h)
        for (int f = 0; f < FS; ++f) Wq1[h][f] = q8(Wf[h][f] * sw1);
    for (int c = 0; c < C; ++c)
        for (int h = 0; h < H; ++h) Wq2[c][h] = q8((double)P.W2[c * H + h] * sw2);

    /* per stage: the algorithm embedding's share of the first layer, and the
     * sum of the magnitudes of its terms (for the error bound) */
    const size_t nu = (size_t)(S > 0 ? S : 1) * H;
    double *u = (double *)malloc(sizeof(double) * nu);
    double *uabs = (double *)malloc(sizeof(double) * nu);
    if (!u || !uabs) {
        free(u);
        free(uabs);
        return;
    }
    for (int s = 0; s < S; ++s) {
        double p[FP], ep[E], epabs[E];
        for (int f = 0; f < FP; ++f) p[f] = log1p((double)pipe[s * FP + f]);
        for (int e = 0; e < E; ++e) {
            double a = (double)P.bp[e], m = fabs((double)P.bp[e]);
            for (int f = 0; f < FP; ++f) {
                a += (double)P.Wp[e * FP + f] * p[f];
                m += fabs((double)P.Wp[e * FP + f] * p[f]);
            }
            ep[e] = a;
            epabs[e] = m;
        }
        for (int h = 0; h < H; ++h) {
            double a = (double)P.b1[h], m = fabs((double)P.b1[h]) + fabs(beta[h]);
            for (int e = 0; e < E; ++e) {
                a += (double)P.W1[h * 2 * E + e] * ep[e];
                m += fabs((double)P.W1[h * 2 * E + e]) * epabs[e];
            }
            u[s * H + h] = a + beta[h];
            uabs[s * H + h] = m;
        }
    }
    const double s1 = sw1 * in_scale, s2 = sw2 * act_scale;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
#endif
    for (int64_t i = 0; i < (int64_t)N; ++i) {
        double stage_sum = 0.0, bound = 0.0;
        for (int64_t s = 0; s < (int64_t)S; ++s) {
            const int64_t row = s * (int64_t)N + i;
            const uint8_t *q = codes + row * FS;
            double hq[H], swing[H];
            for (int h = 0; h < H; ++h) {
                double a = s1 * u[s * H + h], pmax = 0.0;
                for (int f = 0; f < FS; ++f) {
                    const double prod = Wq1[h][f] * cmo_e4m3_decode(q[f]);
                    a += prod;
                    if (fabs(prod) > pmax) pmax = fabs(prod);
                }
                const double pre = a / s1;
                const double x = (pre < 0.0 ? 0.0 : pre) * act_scale; /* ReLU, scale */
                hq[h] = q8(x);
                if (want_bound) {
                    /* a product sum off by acc_tol of its largest term, the
                     * hoisted row off by 1e-5 of its terms' magnitudes */
                    const double e =
                        (acc_tol * pmax / s1 + 1e-5 * uabs[s * H + h]) * act_scale;
                    swing[h] = isnan(x) ? 0.0 : rounding_swing(x, e);
                }
            }
            double v = 0.0, sbound = 0.0;
            for (int c = 0; c < C; ++c) {
                double a = 0.0, pmax = 0.0, flips = 0.0;
                for (int h = 0; h < H; ++h) {
                    a += Wq2[c][h] * hq[h];
                    if (fabs(Wq2[c][h] * hq[h]) > pmax) pmax = fabs(Wq2[c][h] * hq[h]);
                    if (want_bound) flips += fabs(Wq2[c][h]) * swing[h];
                }
                a = a / s2 + (double)P.b2[c];
                v += (a < 0.0 ? 0.0 : a) * (double)terms[row * C + c];
                /* ReLU moves its output by at most its input's change */
                if (want_bound)
                    sbound += (flips + acc_tol * pmax) / s2 * fabs((double)terms[row * C + c]);
            }
            /* the stage's predicted cost (Sec. 5.2) and its share of the bound */
            if (stage_cost_out != NULL) stage_cost_out[row] = v;
            if (stage_bound_out != NULL) stage_bound_out[row] = sbound;
            bound += sbound;
            stage_sum += v;
        }
        cost_out[i] = stage_sum;
        if (bound_out) bound_out[i] = bound;
    }
    free(u);
    free(uabs);
    (void)nthreads;
}

/* ---- beam selection: the k best states of a priority queue (Sec. 4) ---- */

typedef struct {
    double key;
    int32_t idx;
    int32_t nan;
} cmo_item;

/* Total order: lower predicted cost first, NaN after every number, -0 == +0
 * (numeric comparison), equal costs by ascending candidate index.  With the
 * index as the last key this is exactly the order a stable sort produces. */
static int item_cmp(const void *a, const void *b)
{
    const cmo_item *A = (const cmo_item *)a, *B = (const cmo_item *)b;
    if (A->nan != B->nan) return A->nan - B->nan;
    if (!A->nan) {
        if (A->key < B->key) return -1;
        if (A->key > B->key) return 1;
    }
    return (A->idx > B->idx) - (A->idx < B->idx);
}

int32_t cmo_select(const double *cost, int32_t N, int32_t k, int32_t *idx_out,
                   double *val_out)
{
    if (N < 0 || k < 0) return -1;
    cmo_item *it = (cmo_item *)malloc(sizeof(cmo_item) * (size_t)(N > 0 ? N : 1));
    if (!it) return -2;
    for (int32_t i = 0; i < N; ++i) {
        it[i].key = cost[i];
        it[i].idx = i;
        it[i].nan = isnan(cost[i]) ? 1 : 0;
    }
    qsort(it, (size_t)N, sizeof(cmo_item), item_cmp);
    for (int32_t j = 0; j < k; ++j) {
        if (j < N) {
            idx_out[j] = it[j].idx;
            val_out[j] = it[j].key;
        } else { /* fewer candidates than beam slots: padding */
            idx_out[j] = -1;
            val_out[j] = INFINITY;
        }
    }
    free(it);
    return 0;
}

/* ---- freezing of the lowest-cost stages (Sec. 3.2) ---- */

/* The stages of the kept schedule are ordered by their predicted cost, in the
 * same total order as the beam (ascending, -0 == +0, NaN last, ties by lower
 * stage index), and all but ceil(log2 S) of them, the cheapest, are frozen. */
int32_t cmo_freeze(const double *stage_cost, int32_t S, uint8_t *frozen_out)
{
    if (S < 1) return -1;
    cmo_item *it = (cmo_item *)malloc(sizeof(cmo_item) * (size_t)S);
    if (!it) return -2;
    for (int32_t s = 0; s < S; ++s) {
        it[s].key = stage_cost[s];
        it[s].idx = s;
        it[s].nan = isnan(stage_cost[s]) ? 1 : 0;
    }
    qsort(it, (size_t)S, sizeof(cmo_item), item_cmp);
    int32_t unfrozen = 0; /* ceil(log2 S) */
    while (((int64_t)1 << unfrozen) < (int64_t)S) ++unfrozen;
    for (int32_t j = 0; j < S; ++j) frozen_out[it[j].idx] = j < S - unfrozen ? 1 : 0;
    free(it);
    return 0;
}

/* ---- known-bad-state penalty (Sec. 4.5) ---- */

/* A candidate whose hash is in the set of hashes already judged unpromising
 * gets the penalty added to its cost.  The addition is float32 (the cost is
 * the float32 value the beam ranks); the set is searched linearly. */
void cmo_penalize_f32(float *cost, const uint64_t *hashes, int64_t N, const uint64_t *bad,
                      int64_t n_bad, float penalty)
{
    for (int64_t i = 0; i < N; ++i) {
        int seen = 0;
        for (int64_t j = 0; j < n_bad && !seen; ++j) seen = hashes[i] == bad[j];
        if (seen) cost[i] = cost[i] + penalty;
    }
}

/* ---- hierarchical sampling (Sec. 3.1, Sec. 4.4) ---- */

/* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014; the public-domain
 * reference generator): the state advances by the golden-ratio increment and
 * each output is the state passed through a xorshift-multiply mix.  Output
 * number i (from 0) of the stream started at `seed` depends only on
 * (seed, i), which makes it a counter-based generator. */
uint64_t cmo_splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

typedef struct {
    uint64_t hash;
    uint32_t key;  /* the random draw: high 32 bits of the generator's output */
    int32_t idx;
} cmo_opt;

static int opt_cmp(const void *a, const void *b)
{
    const cmo_opt *A = (const cmo_opt *)a, *B = (const cmo_opt *)b;
    if (A->hash != B->hash) return A->hash < B->hash ? -1 : 1;
    if (A->key != B->key) return A->key < B->key ? -1 : 1;
    return A->idx < B->idx ? -1 : (A->idx > B->idx ? 1 : 0);
}

/* Options with equal structural hashes form a bucket; from a bucket of B
 * options, max(1, ceil(log2 B)) representatives are drawn at random without
 * replacement: the ones with the smallest random keys (ties by lower index),
 * key i being drawn from output i of the generator seeded with `seed`.
 * Writes the representatives' indices ascending to out_idx and returns how
 * many there are (<0 on bad sizes / no memory). */
int64_t cmo_sample(const uint64_t *hashes, int64_t n, uint64_t seed, int32_t *out_idx)
{
    if (n < 0) return -1;
    if (n == 0) return 0;
    cmo_opt *o = (cmo_opt *)malloc(sizeof(cmo_opt) * (size_t)n);
    uint8_t *keep = (uint8_t *)calloc((size_t)n, 1);
    if (!o || !keep) {
        free(o);
        free(keep);
        return -2;
    }
    for (int64_t i = 0; i < n; ++i) {
        o[i].hash = hashes[i];
        o[i].key = (uint32_t)(cmo_splitmix64(seed, (uint64_t)i) >> 32);
        o[i].idx = (int32_t)i;
    }
    qsort(o, (size_t)n, sizeof(cmo_opt), opt_cmp);
    for (int64_t b = 0; b < n;) {
        int64_t e = b;
        while (e < n && o[e].hash == o[b].hash) ++e;
        const int64_t B = e - b;
        int64_t reps = 0; /* ceil(log2 B), at least 1 */
        while (((int64_t)1 << reps) < B) ++reps;
        if (reps < 1) reps = 1;
        for (int64_t j = b; j < b + reps && j < e; ++j) keep[o[j].idx] = 1;
        b = e;
    }
    int64_t count = 0;
    for (int64_t i = 0; i < n; ++i)
        if (keep[i]) out_idx[count++] = (int32_t)i;
    free(o);
    free(keep);
    return count;
}
