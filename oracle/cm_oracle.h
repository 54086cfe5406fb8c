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

/* The k best candidates: ascending cost, ties by lower index, -0 == +0, NaN
 * last; k > N pads with (-1, +inf).  Returns 0, or <0 on bad sizes / no memory. */
int32_t cmo_select(const double *cost, int32_t N, int32_t k, int32_t *idx_out,
                   double *val_out);

#ifdef __cplusplus
}
#endif
#endif
