/*
 * cm_oracle.h -- FP64 CPU oracle of the learned cost model (Anderson et al.,
 * OOPSLA 2021, Sec. 5.2 and App. B) and of beam selection (Sec. 4).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark.  Independent of the GPU library.
 */
#ifndef CM_ORACLE_H
#define CM_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* Threads an nthreads <= 0 call uses (OpenMP's maximum). */
int32_t cmo_max_threads(void);

/* Length of the float32 parameter blob (4184). */
int32_t cmo_n_params(void);

/* Predicted runtime of each of the N candidates of one query with S stages.
 * pipe[S][56], sched[S][N][40], terms[S][N][8] are float32 (host).
 * cost_out[N] (required), stage_cost_out[S][N] and coef_out[S][N][8]
 * (optional, may be NULL) receive FP64 results.  nthreads <= 0: all cores. */
void cmo_eval(const float *params, int32_t S, int32_t N, const float *pipe,
              const float *sched, const float *terms, double *cost_out,
              double *stage_cost_out, double *coef_out, int32_t nthreads);

/* OCP e4m3 codec: decode a code; encode with round-to-nearest (ties to even),
 * saturation at +-448 and NaN -> 0x7F. */
double cmo_e4m3_decode(uint8_t code);
uint8_t cmo_e4m3_encode(double v);
/* Per-layer scale of the FP8 form: the largest power of two <= 448 / amax. */
double cmo_fp8_scale(double amax);

/* Input codes of the FP8 form: out[i] = e4m3(log1p(x[i]) * in_scale), FP64. */
void cmo_fp8_codes(const float *x, int64_t n, double in_scale, uint8_t *out);

/* FP8 form of cmo_eval: codes[S][N][40] are e4m3 codes of log1p(x) * in_scale;
 * weights quantized per layer (first layer folded: W_1[:, 24:] W_s), hidden
 * activations quantized as e4m3(ReLU(h) * act_scale); FP64 in between.
 * bound_out[N] (optional, may be NULL): per candidate, how far its cost may
 * move when every sum of e4m3 products (first layer, coefficient layer) is off
 * by acc_tol times its largest product and every hoisted row by 1e-5 of the
 * magnitudes of its terms: the hidden values whose rounding may then change
 * contribute their possible e4m3 swing through |W_2|, and each coefficient
 * its own error, times |terms|.
 * stage_cost_out[S][N] and stage_bound_out[S][N] (optional, may be NULL):
 * every stage's predicted cost (the terms Sec. 5.2 sums over stages) and that
 * stage's share of the bound (the shares add up to bound_out). */
void cmo_eval_fp8(const float *params, double in_scale, double act_scale, int32_t S,
                  int32_t N, const float *pipe, const uint8_t *codes, const float *terms,
                  double *cost_out, double acc_tol, double *bound_out, int32_t nthreads,
                  double *stage_cost_out, double *stage_bound_out);

/* The k best candidates: ascending cost, ties by lower index, -0 == +0, NaN
 * last; k > N pads with (-1, +inf).  Returns 0, or <0 on bad sizes / no memory. */
int32_t cmo_select(const double *cost, int32_t N, int32_t k, int32_t *idx_out,
                   double *val_out);

/* Freezing (Sec. 3.2): frozen_out[s] = 1 for the S - ceil(log2 S) lowest-cost
 * stages of one candidate (order as cmo_select, by stage index on ties), else
 * 0.  Returns 0, or <0 on S < 1 / no memory. */
int32_t cmo_freeze(const double *stage_cost, int32_t S, uint8_t *frozen_out);

/* Known-bad-state penalty (Sec. 4.5): cost[i] += penalty (float32) where
 * hashes[i] is one of bad[0, n_bad) (any order). */
void cmo_penalize_f32(float *cost, const uint64_t *hashes, int64_t N, const uint64_t *bad,
                      int64_t n_bad, float penalty);

/* Hierarchical sampling (Sec. 3.1): SplitMix64 output i of the stream seeded
 * with seed; and the representatives of the buckets of equal hashes,
 * max(1, ceil(log2 B)) per bucket of B options with the smallest keys
 * (high 32 bits of output i for option i, ties by index), written ascending
 * to out_idx (capacity n).  Returns their count, or <0. */
uint64_t cmo_splitmix64(uint64_t seed, uint64_t i);
int64_t cmo_sample(const uint64_t *hashes, int64_t n, uint64_t seed, int32_t *out_idx);

#ifdef __cplusplus
}
#endif
#endif
