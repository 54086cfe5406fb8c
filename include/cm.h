/*
 * cm.h -- C ABI of the batched learned-cost-model evaluator with beam top-k,
 * for AMD Instinct MI355X (gfx950).
 *
 * The method is the cost model and beam selection of Anderson et al.,
 * "Efficient Automatic Scheduling of Imaging and Vision Pipelines for the
 * GPU" (OOPSLA 2021):
 *   - Sec. 5.2: per stage, the algorithm-specific features and the
 *     log-transformed schedule features each pass through a fully connected
 *     embedding; the two embeddings are stacked and a fully connected network
 *     produces a vector of non-negative coefficients;
 *   - Sec. 5.2 and App. B: the coefficients weight hand-derived per-stage cost
 *     terms (every cost component is linear in the coefficients); the
 *     per-stage predictions are summed over all stages;
 *   - Sec. 4 and Sec. 4.4: the search keeps a priority queue of the k best
 *     candidate states; evaluated candidates are added to that beam.
 *
 * Conventions
 *   - Every function returns a cm_status; CM_OK is 0 and errors are negative.
 *     Arguments are validated on the host before any device work; a failed
 *     call leaves outputs untouched.  cm_last_error() gives a thread-local
 *     message for the last failure.  No C++ exception crosses this boundary.
 *   - "device pointer" = memory allocated on the GPU the call runs on;
 *     "host pointer" = ordinary CPU memory.  The caller owns every feature,
 *     term, cost and result buffer; the library owns models, workspaces and
 *     servers and never frees caller memory.
 *   - Streams are passed as cm_stream (a hipStream_t; NULL = legacy default
 *     stream).  Device calls are asynchronous on that stream.
 *   - Model dimensions are fixed: 56 algorithm features, 40 schedule
 *     features, two 24-wide embeddings, 32 hidden units, 8 coefficients and
 *     8 cost terms per (stage, candidate).
 */
#ifndef CM_H
#define CM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CM_VERSION_MAJOR 0
#define CM_VERSION_MINOR 1

#define CM_N_PIPE_FEATURES 56
#define CM_N_SCHED_FEATURES 40
#define CM_EMBED 24
#define CM_HIDDEN 32
#define CM_N_COEFS 8
#define CM_N_PARAMS 4184     /* float32 parameters, layout in cm_model_create */
#define CM_MAX_K 256         /* largest beam width of cm_topk_per_query */
#define CM_STAGE_CHUNK 32    /* sets the stage split of CM_BF16 (see cm_eval_batch) */
#define CM_STEP_MAX_QUERIES 256 /* queries per cm_step_run */
#define CM_STATIC_MAX_STAGES 32768 /* stages per cm_eval_batch_static call */

typedef int32_t cm_status;
enum {
    CM_OK = 0,
    CM_EINVAL = -1,       /* bad argument, size, layout or alignment */
    CM_ENOMEM = -2,       /* device or pinned host allocation failed */
    CM_EDEVICE = -3,      /* a HIP call failed (launch, copy, sync) */
    CM_EAGAIN = -4,       /* not ready yet / queue full: try again */
    CM_E2BIG = -5,        /* request exceeds a capacity fixed at creation */
    CM_ENOTFOUND = -6,    /* unknown ticket or session */
    CM_ECANCELED = -7,    /* work dropped because its session or server closed */
    CM_EUNSUPPORTED = -8  /* precision or feature not available */
};

/* Arithmetic of an evaluation.
 *   CM_FP32: schedule features stored as float32 raw values; every step in
 *            float32 on the vector ALUs.
 *   CM_BF16: schedule features stored as bfloat16 raw values (2 bytes);
 *            the two dense layers run on bf16 matrix cores with float32
 *            accumulation, each product split into high and low bf16 parts
 *            (three bf16 products) so that the arithmetic error stays near
 *            float32; cost terms stay float32.
 *   CM_FP8:  schedule features stored as OCP e4m3 codes of
 *            log1p(x) * s_in (1 byte each; cm_fp8_encode writes them), so the
 *            log transform is done once at encoding; both dense layers run on
 *            fp8 matrix cores with e4m3 weights, the hidden activations are
 *            re-quantized to e4m3, accumulation and cost terms are float32.
 *            The model must first be given its FP8 form with
 *            cm_model_prepare_fp8 (the scales s_in and s_h). */
typedef int32_t cm_precision;
enum { CM_FP32 = 0, CM_BF16 = 1, CM_FP8 = 2 };

typedef void *cm_stream; /* hipStream_t */

typedef struct cm_model cm_model;
typedef struct cm_workspace cm_workspace;

/* Model shape.  Every field must equal the CM_* constant above. */
typedef struct {
    int32_t n_pipe_features;  /* 56 */
    int32_t n_sched_features; /* 40 */
    int32_t embed;            /* 24 */
    int32_t hidden;           /* 32 */
    int32_t n_coefs;          /* 8 */
} cm_model_desc;

/* Create a model from a host float32 parameter blob of CM_N_PARAMS values,
 * in this order, matrices row-major [out][in]:
 *   W_p[24][56] b_p[24]   algorithm-feature embedding   (Sec. 5.2)
 *   W_s[24][40] b_s[24]   schedule-feature embedding    (Sec. 5.2)
 *   W_1[32][48] b_1[32]   layer over the stacked [e_p; e_s] (e_p first), ReLU
 *   W_2[8][32]  b_2[8]    coefficient layer, ReLU -> non-negative coefficients
 * The library copies the blob to the current HIP device and derives the
 * packed forms its kernels read, among them a table of the bf16 evaluator's
 * log transform, which a small kernel on the null stream fills (the call
 * waits for it).  params_host is not retained.  A model is immutable and may
 * be shared by concurrent calls.
 * Errors: CM_EINVAL (NULL pointer, wrong dimensions, non-finite parameter),
 * CM_ENOMEM, CM_EDEVICE. */
cm_status cm_model_create(const cm_model_desc *desc, const float *params_host,
                          cm_model **out);
cm_status cm_model_destroy(cm_model *model);

/* Capacities of a workspace, per call. */
typedef struct {
    int32_t max_queries;  /* queries per call (>= 1) */
    int64_t max_stages;   /* sum over queries of n_stages */
    int64_t max_cands;    /* sum over queries of n_cands */
    int64_t max_rows;     /* sum over queries of n_stages * n_cands */
    int32_t max_k;        /* largest k passed to cm_topk_per_query (<= CM_MAX_K) */
} cm_workspace_desc;

/* Device scratch for cm_eval_batch / cm_topk_per_query: per-stage hoisted
 * vectors, partial stage sums, per-tile beam lists and arrival counters,
 * allocated once on the current device.  A workspace serves one stream at a
 * time: two calls in flight on different streams with the same workspace
 * race.  Errors: CM_EINVAL, CM_ENOMEM, CM_EDEVICE. */
cm_status cm_workspace_create(const cm_workspace_desc *desc, cm_workspace **out);
cm_status cm_workspace_destroy(cm_workspace *ws);

/* One query = one beam step of one search session: n_cands candidate
 * schedules over the same n_stages stages.  Offsets are element offsets into
 * the batch's base pointers:
 *   pipe  + pipe_off  : float32 [n_stages][56]          algorithm features
 *   sched + sched_off : [n_stages][n_cands][40]         schedule features,
 *                       float32 (CM_FP32), bfloat16 bits (CM_BF16) or
 *                       e4m3 codes (CM_FP8, see cm_fp8_encode);
 *                       sched_off must be a multiple of 8 elements
 *   terms + terms_off : float32 [n_stages][n_cands][8]  cost terms;
 *                       terms_off must be a multiple of 4
 *   cost  + cost_off  : float32 [n_cands]               predicted runtimes
 * Raw feature values are taken as-is (the log transform is applied inside). */
typedef struct {
    int32_t n_stages;   /* >= 1 */
    int32_t n_cands;    /* >= 0 */
    int64_t pipe_off;
    int64_t sched_off;
    int64_t terms_off;
    int64_t cost_off;
} cm_query;

typedef struct {
    int32_t n_queries;        /* >= 0 */
    const cm_query *queries;  /* host array of n_queries descriptors */
    const float *pipe;        /* device */
    const void *sched;        /* device */
    const float *terms;       /* device */
} cm_batch;

/* Predicted runtime of every candidate of every query (Sec. 5.2):
 *   cost[i] = sum over stages s of  sum_j c_j(s, i) * terms[s][i][j],
 *   c(s, i) = ReLU(W_2 ReLU(W_1 [W_p log1p(pipe[s]) + b_p ;
 *                                W_s log1p(sched[s][i]) + b_s] + b_1) + b_2).
 * The stage sum is Kahan-compensated float32 in ascending stage order.  In
 * CM_BF16 the stages are first split into P contiguous near-equal parts
 * (P = 1 for n_stages <= CM_STAGE_CHUNK/2, 2 for <= CM_STAGE_CHUNK, 4 for
 * <= 2*CM_STAGE_CHUNK, else 8),
 * each summed with compensation, and the parts' (sum, compensation) pairs are
 * combined in ascending order.  Every candidate's result depends only on its
 * own query's data: the same query gives bit-identical costs alone or inside
 * any batch.
 * cost_out is a device pointer; results land at cost_out[cost_off + i].
 * Asynchronous on `stream`; allocates nothing.
 * CM_FP8 evaluates the FP8 form described below (cm_model_prepare_fp8).
 * Size limit of CM_BF16 and CM_FP8: their kernels address one query's
 * features and terms with 32-bit byte offsets, so each query's
 * n_stages * n_cands * 80 (CM_BF16) or * 40 (CM_FP8) feature bytes and
 * n_stages * n_cands * 32 term bytes must stay at or below 2^32 - 2^16;
 * CM_FP32 has no such limit.  The descriptors are checked before the model
 * or workspace is read.
 * Errors: CM_EINVAL (bad descriptor, misaligned offset, NULL pointer, CM_FP8
 * on a model without an FP8 form), CM_E2BIG (batch exceeds the workspace, or
 * a query exceeds the size limit), CM_EUNSUPPORTED (precision), CM_EDEVICE
 * (launch failure). */
cm_status cm_eval_batch(const cm_model *model, cm_precision precision,
                        const cm_batch *batch, cm_workspace *ws, float *cost_out,
                        cm_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * cm_eval_batch without a workspace.  Same validation, kernels and results,
 * bit for bit, as cm_eval_batch.  The per-stage hoisted rows (32 floats per
 * stage) go to a scratch array that the library holds in device memory,
 * one copy per device (4 MiB, kept until the process ends); its address is
 * looked up when the first model is created on the device.  The call makes
 * no allocation of any kind.
 * Limit: the batch's n_stages summed over its queries must be at most
 * CM_STATIC_MAX_STAGES (else CM_E2BIG, before any device work).
 * Every call on one device uses that device's one scratch array, which keeps
 * the last call's contents: calls that overlap on one device (different
 * streams or threads) race and give wrong costs; serialise them.
 * Errors: as cm_eval_batch (no workspace errors), CM_E2BIG above the limit,
 * CM_EUNSUPPORTED for a device ordinal of 64 or more. */
cm_status cm_eval_batch_static(const cm_model *model, cm_precision precision,
                               const cm_batch *batch, float *cost_out, cm_stream stream);

/* cm_eval_batch that also writes every stage's predicted cost (the v_s that
 * Sec. 5.2 sums over stages, as added to the stage sum):
 *   stage_cost_out[terms_off / 8 + s * n_cands + i] = v_s(i),
 * i.e. a [n_stages][n_cands] float32 array per query at one eighth of its terms
 * offset (device pointer; terms_off must be a multiple of 8).  Costs and
 * their bits are those of cm_eval_batch.  Errors as cm_eval_batch. */
cm_status cm_eval_stages(const cm_model *model, cm_precision precision,
                         const cm_batch *batch, cm_workspace *ws, float *cost_out,
                         float *stage_cost_out, cm_stream stream);

/* Hierarchical sampling (Sec. 3.1, Sec. 4.4): before featurization and
 * evaluation, the enumerated options of a query are grouped into buckets by
 * their structural hash, and only a few random representatives of every
 * bucket go on to the cost model: max(1, ceil(log2 B)) of a bucket of B
 * options (log2 B rounded up, at least one), drawn without replacement.
 * The draw is reproducible: option i gets the random key
 *   key(i) = (SplitMix64 output i of the stream seeded with seeds[q]) >> 32
 * (SplitMix64 of Steele, Lea and Flood, OOPSLA 2014: the state advances by
 * 0x9E3779B97F4A7C15, outputs pass a xorshift-multiply mix), and a bucket's
 * representatives are its members with the smallest keys, equal keys by
 * lower index.
 *
 * A sampler owns the device scratch for up to max_queries queries and
 * max_options options per call (about 60 bytes per option).  For query q of
 * `batch` (only n_cands = its option count and cost_off are read),
 * hashes[cost_off + i] (device uint64) is option i's structural hash; the
 * representatives' indices are written ascending to sel_idx[cost_off + j]
 * (device int32, room for n_cands) and their number to sel_count[q]
 * (device).  seeds is a host array of n_queries seeds.  Asynchronous on
 * `stream` (the descriptors are staged through pinned memory); allocates
 * nothing.  One sampler serves one stream at a time.
 * Errors: CM_EINVAL (NULL pointer, bad descriptor, wrong device), CM_E2BIG
 * (more queries or options than the sampler holds), CM_ENOMEM (create),
 * CM_EDEVICE. */
typedef struct cm_sampler cm_sampler;
cm_status cm_sampler_create(int32_t max_queries, int64_t max_options, cm_sampler **out);
cm_status cm_sampler_destroy(cm_sampler *sampler);
cm_status cm_sample_buckets(cm_sampler *sampler, const cm_batch *batch, const uint64_t *hashes,
                            const uint64_t *seeds, int32_t *sel_idx, int32_t *sel_count,
                            cm_stream stream);

/* Memoized feature rows (Sec. 3.3): featurizations are memoized and reused
 * across the schedules that share a kernel, so many (stage, candidate) rows
 * repeat.  cm_eval_batch over a row table: batch->sched points at a table of
 * table_rows schedule-feature rows (40 values each, in the precision's
 * storage: bfloat16 bits for CM_BF16, e4m3 codes for CM_FP8), and each
 * query's sched_off is an offset into row_idx (device int32), which holds
 * its [n_stages][n_cands] row numbers; row (s, i) is table row
 * row_idx[sched_off + s * n_cands + i].  Cost terms stay per (stage,
 * candidate) as in cm_eval_batch (they hold the featurization's components
 * that are always recomputed).  Results are bit-identical to cm_eval_batch
 * on the materialized rows.  A row number outside [0, table_rows) gives that
 * candidate a NaN cost (the table is never read outside its bounds).
 * table_rows * row bytes must stay below 4 GiB; the size limit of
 * cm_eval_batch applies to the terms only.  CM_FP32 is not supported.
 * Errors: as cm_eval_batch, CM_EINVAL (table_rows, row_idx),
 * CM_EUNSUPPORTED (CM_FP32). */
cm_status cm_eval_indexed(const cm_model *model, cm_precision precision,
                          const cm_batch *batch, const int32_t *row_idx, int64_t table_rows,
                          cm_workspace *ws, float *cost_out, cm_stream stream);

/* Known-bad-state penalty of the multi-pass search (Sec. 4.5): before
 * selection, a candidate whose structural hash (at the depth of the current
 * pass, computed by the caller) is among the hashes already judged
 * unpromising gets `penalty` added to its predicted cost, which moves it back
 * in the beam.  For every query, candidate i with hashes[cost_off + i] in
 * bad_sorted[0, n_bad) gets cost[cost_off + i] += penalty (float32 addition,
 * in place).  hashes (uint64), bad_sorted (uint64, ascending, duplicates
 * allowed) and cost are device pointers.  The paper gives no magnitude for
 * the penalty; any non-NaN float is accepted (+inf pushes such candidates
 * behind every finite cost).  Only n_cands and cost_off of each descriptor
 * are read.  Run cm_topk_per_query afterwards.  Asynchronous on `stream`;
 * allocates nothing.  Errors: CM_EINVAL (bad descriptor, NULL pointer,
 * n_bad < 0, NaN penalty), CM_EDEVICE. */
cm_status cm_penalize_known_bad(const cm_batch *batch, const uint64_t *hashes,
                                const uint64_t *bad_sorted, int64_t n_bad, float penalty,
                                float *cost, cm_stream stream);

/* Freezing of low-cost stages (Sec. 3.2): after a pre-pass, the schedule
 * options of the lowest-cost stages of the kept schedule are frozen, all but
 * ceil(log2 S) of them (S = the query's n_stages; a non-integer log2 is
 * rounded up, so at least one stage is frozen and, for S >= 2, at least one
 * stays free).  For query q the kept candidate is c = cand[q * cand_stride]
 * (device int32; e.g. idx_out of cm_topk_per_query with stride k for each
 * beam's best); its stage costs are read from stage_cost as cm_eval_stages
 * writes them.  Stages are ranked by ascending cost, equal costs by lower
 * stage index, -0 equal to +0, NaN after every number; the first
 * S - ceil(log2 S) are frozen.  Writes frozen_out[row] = 1 (frozen) or 0, one
 * uint8 per stage, rows in batch order (query q's stage s at the sum of
 * n_stages of queries 0..q-1, plus s; device).  A c outside [0, n_cands)
 * freezes nothing.  Only n_stages, n_cands and terms_off of each descriptor
 * are read.  Asynchronous on `stream`; allocates nothing.
 * Errors: CM_EINVAL (bad descriptor, terms_off not a multiple of 8, NULL
 * pointer, cand_stride < 1), CM_EDEVICE. */
cm_status cm_freeze_stages(const float *stage_cost, const cm_batch *batch,
                           const int32_t *cand, int64_t cand_stride, uint8_t *frozen_out,
                           cm_stream stream);

/* Per-stage hoist (Sec. 5.2): the algorithm features of a stage are shared by
 * every candidate of its query, so their share of the first layer is
 * computed once per stage:
 *   U[row][j] = b_1[j] + sum_e W_1[j][e] (W_p log1p(pipe[s]) + b_p)[e]
 * (for CM_BF16 and CM_FP8 also + sum_e W_1[j][24 + e] b_s[e], since those
 * forms fold the schedule embedding into the first layer; for CM_FP8 the row
 * is then multiplied by s_h, that form's hidden scale, as set by the model's
 * last cm_model_prepare_fp8).  Rows are written in batch order:
 * query q's stage s goes to row (n_stages of queries 0..q-1) + s, 32 floats
 * per row, into U_out (device, 16-byte aligned, at least sum(n_stages) * 32
 * floats).  Only n_stages, pipe_off and pipe are read.  Asynchronous on
 * `stream`; allocates nothing.  Errors: CM_EINVAL, CM_EUNSUPPORTED,
 * CM_EDEVICE. */
cm_status cm_hoist_stages(const cm_model *model, cm_precision precision,
                          const cm_batch *batch, float *U_out, cm_stream stream);

/* cm_eval_batch without the hoist: reads the per-stage rows U (device, laid
 * out as cm_hoist_stages writes them for the same precision and batch order)
 * instead of computing them; one kernel launch per 32 queries.  Same results,
 * errors and asynchrony as cm_eval_batch. */
cm_status cm_eval_hoisted(const cm_model *model, cm_precision precision,
                          const cm_batch *batch, const float *U, cm_workspace *ws,
                          float *cost_out, cm_stream stream);

/* Beam selection (Sec. 4): for every query q, the k candidates with the
 * lowest predicted runtime, ascending; equal costs are ranked by the lower
 * candidate index, -0 equals +0 and NaN ranks after +inf.  Reads
 * cost[cost_off + i] for i < n_cands of each query (a device pointer).
 * Writes idx_out[q*k + j] (query-local candidate index) and
 * val_out[q*k + j] (that candidate's cost, bit for bit); when n_cands < k the
 * tail is padded with (-1, +inf).  1 <= k <= min(CM_MAX_K, ws max_k).
 * Asynchronous on `stream`; allocates nothing.
 * Errors: CM_EINVAL, CM_E2BIG, CM_EDEVICE. */
cm_status cm_topk_per_query(const float *cost, const cm_batch *batch, int32_t k,
                            cm_workspace *ws, int32_t *idx_out, float *val_out,
                            cm_stream stream);

/* ------------------------------------------------------------------------
 * FP8 form (CM_FP8).  An 8-bit reading of the model of Sec. 5.2: every
 * quantization point is an OCP e4m3 value (sign, 4 exponent bits with bias
 * 7, 3 mantissa bits, subnormals, largest finite 448, no infinities, NaN
 * codes 0x7F and 0xFF), rounded to nearest with ties to the even code and
 * saturated at +-448; each scale is a power of two, so scaling and unscaling
 * are exact.  Per stage s and candidate i:
 *   code[f] = e4m3(log1p(sched[s][i][f]) * s_in)                (input)
 *   a[j]    = sum_f e4m3(Wf[j][f] s_w1) dec(code[f])            (fp8 matrix core)
 *   h[j]    = e4m3(ReLU(a[j] / (s_w1 s_in) + U[s][j]) * s_h)    (hidden)
 *   c[m]    = ReLU(sum_j e4m3(W_2[m][j] s_w2) h[j] / (s_w2 s_h) + b_2[m])
 *   cost[i] = sum_s sum_m c[m] terms[s][i][m]   (Kahan float32, stage parts
 *                                                 as for CM_BF16)
 * with Wf = W_1[:, 24:] W_s (the schedule embedding folded into the first
 * layer), U[s] the hoisted row of cm_hoist_stages before its FP8 scale, and
 * s_w1, s_w2 the largest powers of two with s |W| <= 448 over Wf and W_2.
 * The matrix instruction sums its e4m3 products with less than float32
 * precision (measured on gfx950: within about 6e-4 of the largest product),
 * so a hidden value that lands that close to an e4m3 rounding midpoint may
 * round to the neighbouring code; the hoisted row is added afterwards in
 * float32.  A NaN code gives a NaN cost.
 * ------------------------------------------------------------------------ */

/* Derive the FP8 form of `model` for input scale s_in = in_scale and hidden
 * scale s_h = act_scale (both positive powers of two; every derived scale
 * must stay within [2^-60, 2^60]).  Host work plus one small synchronous
 * copy to the model's device.  Replaces an earlier FP8 form; must not run
 * while any call that uses this model with CM_FP8 is in flight, and rows
 * hoisted for CM_FP8 before it are stale after it.
 * Errors: CM_EINVAL (NULL model, scale not a power of two or out of range),
 * CM_ENOMEM, CM_EDEVICE. */
cm_status cm_model_prepare_fp8(cm_model *model, float in_scale, float act_scale);

/* Suggested scales for the FP8 form from a host sample of n_rows (stage,
 * candidate) rows: pipe_rows[n_rows][56] and sched_rows[n_rows][40], raw
 * float32 features as for CM_FP32.  *in_scale_out is the largest power of
 * two s with s * 2 * max|log1p(x)| <= 448 over the schedule features;
 * *act_scale_out the same over the float64 model's hidden activations
 * ReLU(h) (a factor 2 of headroom for rows outside the sample; 1 when the
 * maximum is 0).  Rows with a non-finite value are skipped.  Host only.
 * Errors: CM_EINVAL (NULL pointer, n_rows < 1). */
cm_status cm_fp8_calibrate(const cm_model *model, int64_t n_rows, const float *pipe_rows,
                           const float *sched_rows, float *in_scale_out,
                           float *act_scale_out);

/* codes[i] = e4m3(log1p(x[i]) * in_scale) for i < n, on the device, with
 * log1p taken in float32 (within a few ulps; a value within that distance of
 * an e4m3 midpoint may take the neighbouring code): x is
 * float32 (device, 16-byte aligned), codes uint8 (device, 16-byte aligned,
 * may not overlap x).  Round to nearest even, saturation at +-448, NaN (e.g.
 * x < -1) -> 0x7F.  in_scale: a positive power of two.  Asynchronous on
 * `stream`; allocates nothing.  Errors: CM_EINVAL, CM_EDEVICE. */
cm_status cm_fp8_encode(const float *x, int64_t n, float in_scale, uint8_t *codes,
                        cm_stream stream);

/* ------------------------------------------------------------------------
 * Persistent beam step: hoist + evaluate + select for a ragged batch in one
 * persistent launch that is replayed as a HIP graph.
 *
 * A step object owns device descriptors, control words and selection lists
 * for `slots` steps that may be in flight at once.  cm_step_run writes the
 * batch's descriptors into pinned host memory; the step then runs as
 *   copy of the descriptors to the device -> hoist (only when U is NULL) ->
 *   one persistent CM_BF16 or CM_FP8 evaluation kernel whose workgroups take tasks
 *   from a device-wide queue, with each query's top-k selection run by the
 *   workgroup that finishes the query's last task,
 * either as one graph launch (captured once per slot and configuration) or
 * as plain launches.  The launch shape depends only on the configuration,
 * never on the batch.  Results are bit-identical to cm_eval_batch /
 * cm_eval_hoisted (same precision) followed by cm_topk_per_query, for every
 * configuration.
 * ------------------------------------------------------------------------ */
typedef struct cm_step cm_step;

typedef struct {
    int32_t max_queries;  /* 1 .. CM_STEP_MAX_QUERIES */
    int64_t max_stages;   /* sum over queries of n_stages */
    int64_t max_cands;    /* sum over queries of n_cands */
    int32_t max_k;        /* 1 .. CM_MAX_K */
    int32_t slots;        /* 1 .. 8: steps in flight at once (descriptor sets) */
} cm_step_desc;

/* Launch configuration; none of it changes the results. */
typedef struct {
    int32_t grid;         /* persistent workgroups (8 waves each); 0 = two per
                             compute unit */
    int32_t group_tiles;  /* row-tile groups per task: 1, 2, 4 or 8 (a group is
                             8 / P tiles of 32 candidates) */
    int32_t use_graph;    /* 1: replay a captured graph; 0: plain launches */
} cm_step_config;

/* Create a step on the current device for `model`, which must outlive it.
 * CM_BF16 and CM_FP8 are supported (CM_EUNSUPPORTED otherwise); CM_FP8 needs
 * the model's FP8 form (CM_EINVAL otherwise), whose hidden scale the step's
 * own hoist reads at run time.  Allocates device
 * memory for the descriptors, control words, hoisted rows and selection
 * lists of every slot, and pinned host memory for the descriptors.
 * Errors: CM_EINVAL, CM_EUNSUPPORTED, CM_ENOMEM, CM_EDEVICE. */
cm_status cm_step_create(const cm_model *model, cm_precision precision,
                         const cm_step_desc *desc, cm_step **out);
/* Waits for the step's work in flight, then frees everything it owns. */
cm_status cm_step_destroy(cm_step *step);

/* One beam step of every query of `batch` (layouts as for cm_eval_batch
 * with the step's precision; the batch's base pointers and every output pointer are
 * device pointers):
 *   - U: hoisted rows as cm_hoist_stages writes them for this batch, or
 *     NULL to hoist inside the step (then pipe must be given);
 *   - cost_out[cost_off + i]: every candidate's predicted runtime;
 *   - idx_out[q*k + j], val_out[q*k + j]: query q's beam, as
 *     cm_topk_per_query writes it.
 * Asynchronous on `stream`.  The call waits on the host only when the slot
 * it reuses is still in flight (more than `slots` steps queued).  Calls on
 * one step are serialised; steps in flight on different streams use
 * different slots.  Errors: CM_EINVAL, CM_E2BIG (capacity, or a query above
 * cm_eval_batch's size limit), CM_EDEVICE. */
cm_status cm_step_run(cm_step *step, const cm_batch *batch, const float *U, int32_t k,
                      float *cost_out, int32_t *idx_out, float *val_out, cm_stream stream);

cm_status cm_step_set_config(cm_step *step, const cm_step_config *cfg);
cm_status cm_step_get_config(const cm_step *step, cm_step_config *cfg);

/* Autotuner: times every configuration of a built-in candidate set on this
 * batch (grid 1, 2 and 4 workgroups per compute unit x group_tiles 1, 2, 4,
 * 8 x graph replay or plain launches; `reps` timed runs each after one
 * untimed run, median of HIP event times on `stream`), keeps the fastest as
 * the step's configuration and returns it in *best (and its median time in
 * microseconds in *best_us, if not NULL).  The pick is also stored in the
 * library's tuning cache under (the device's architecture name, the step's
 * precision, ceil(log2 queries), ceil(log2 rows)) of this batch; when the
 * environment variable CM_TUNE_CACHE names a file, the cache is read from it
 * on first use and written back after every autotune.  Synchronous.  The
 * runs write the outputs like cm_step_run.  Errors: as cm_step_run. */
cm_status cm_step_autotune(cm_step *step, const cm_batch *batch, const float *U, int32_t k,
                           float *cost_out, int32_t *idx_out, float *val_out, cm_stream stream,
                           int32_t reps, cm_step_config *best, float *best_us);

/* The tuning cache's configuration for batches of n_queries queries and
 * `rows` rows on this step's device and precision: the entry of the nearest
 * bucket (closest query bucket, then closest row bucket; rows <= 0: the
 * largest row bucket).  Does not change the step.  cm_server_create applies
 * the entry for its max_batch_queries to its steps.  Errors: CM_EINVAL,
 * CM_ENOTFOUND (no entry for this architecture and precision). */
cm_status cm_step_tuned_config(const cm_step *step, int32_t n_queries, int64_t rows,
                               cm_step_config *out);

/* Kernel-only GPU time, in microseconds, of the step's most recent run (the
 * persistent evaluation-and-selection kernel alone, without the descriptor
 * copy or the hoist): from the first of its workgroups to start to the last
 * to finish, read from the GPU's constant-rate real-time counter (100 MHz)
 * by the kernel itself.  Waits for that run to finish.  Errors: CM_EINVAL,
 * CM_ENOTFOUND (the step has not run), CM_EDEVICE. */
cm_status cm_step_kernel_time(cm_step *step, float *us);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of beam-step queries from many concurrent
 * search sessions (each session runs the beam search of Sec. 4 over one
 * pipeline and submits one query per beam step).
 *
 * A server owns a worker thread, `max_slots` HIP streams each with a
 * persistent step (above), and device pools for its sessions.  Requests are
 * queued by cm_serve_submit and admitted by the worker in submission order
 * as slots and memory free up (at an idle server, with no micro-batch on the
 * device, the submitting call admits and launches them itself when its
 * thread's current device is the server's): a request is admitted when a slot is free,
 * the device bytes of the admitted, unfinished requests plus its own stay
 * within `arena_bytes`, and its session has no other request in flight (a
 * beam step depends on the previous one; later requests of such a session
 * wait without blocking other sessions).  Each admission round launches the
 * admitted requests as one micro-batch on a free slot's stream, so
 * micro-batches on different slots overlap on the device.  Session state
 * stays on the device: the hoisted rows of its stages (computed once, at
 * open) and its latest beam.  Every result is the same as the request
 * evaluated alone (cm_eval_batch in the server's precision +
 * cm_topk_per_query), bit for bit.
 * ------------------------------------------------------------------------ */
typedef struct cm_server cm_server;

typedef struct {
    cm_precision precision;     /* CM_BF16, or CM_FP8 (model with its FP8 form) */
    int32_t k;                  /* largest beam width of a request, 1 .. CM_MAX_K */
    int64_t arena_bytes;        /* admission limit, see cm_serve_submit */
    int32_t max_slots;          /* micro-batches in flight, 1 .. 8 */
    int32_t max_pending;        /* queued, not yet admitted requests */
    int32_t max_sessions;       /* open sessions */
    int32_t max_stages;         /* stages of a session's pipeline */
    int32_t max_batch_queries;  /* requests per micro-batch, 1 .. CM_STEP_MAX_QUERIES */
    int64_t max_batch_cands;    /* candidates per micro-batch (and per request) */
} cm_server_cfg;

/* One beam step of a session: n_cands candidates over the session's stages.
 * sched and terms are device pointers owned by the caller, laid out as for
 * cm_eval_batch (bf16 bits or e4m3 codes [S][n_cands][40], as the server's
 * precision, and float32 [S][n_cands][8], 16-byte aligned), and must stay valid and unchanged until the request's
 * result has been polled or the request canceled. */
typedef struct {
    int32_t n_cands;      /* 0 .. max_batch_cands */
    int32_t k;            /* 1 .. cfg k */
    const void *sched;
    const float *terms;
} cm_request;

/* A completed request.  idx and val are host arrays of capacity `k` (set by
 * the caller, at least the request's k); the beam is written there as
 * cm_topk_per_query writes it.  Times are microseconds of a steady clock
 * since the server was created. */
typedef struct {
    int32_t k;            /* in: capacity of idx and val */
    int32_t n;            /* out: entries written (the request's k) */
    int32_t *idx;
    float *val;
    double t_submit_us;
    double t_admit_us;
    double t_done_us;     /* when the worker saw the micro-batch finish */
} cm_result;

typedef struct {
    int64_t submitted, completed, canceled;
    int64_t candidates, rows;    /* of completed requests */
    int64_t micro_batches;
    double wall_us;              /* first submission to last completion */
    double cands_per_s;          /* candidates / wall time */
    double p50_us, p99_us, max_us;  /* submit-to-done latency of completed requests */
    int32_t queue_depth;         /* queued now */
    int32_t in_flight;           /* admitted and unfinished now */
    int64_t arena_in_use, arena_high_water;
    double kernel_us;            /* GPU time of the step kernels of completed micro-batches
                                    (sum of each kernel's first-wave start to last-wave end) */
    int64_t kernel_bytes;        /* algorithmic bytes they read and wrote */
    double kernel_span_us;       /* earliest start to latest end of those kernels (device
                                    clock), gaps between them included */
    double kernel_busy_us;       /* device time during which at least one of the most
                                    recent kernel_busy_launches of them ran: the union of
                                    their [start, end] intervals, so consecutive
                                    micro-batches that overlap count once */
    int64_t kernel_busy_launches;  /* min(micro-batches since reset, 4096) */
} cm_server_stats;

/* Create a server on the current device for `model`, which must outlive it.
 * Allocates everything it will use (no allocation while serving) and starts
 * the worker.  Errors: CM_EINVAL, CM_EUNSUPPORTED (precision), CM_ENOMEM,
 * CM_EDEVICE. */
cm_status cm_server_create(const cm_model *model, const cm_server_cfg *cfg, cm_server **out);
/* Finishes every queued and admitted request, stops the worker and frees
 * the server.  Results not yet polled are dropped. */
cm_status cm_server_destroy(cm_server *server);

/* Open a session for a pipeline of n_stages stages with algorithm features
 * pipe_host (host float32 [n_stages][56]); its hoisted rows are computed on
 * the device before the call returns.  Errors: CM_EINVAL, CM_E2BIG (too many
 * stages), CM_EAGAIN (no free session), CM_EDEVICE. */
cm_status cm_session_open(cm_server *server, const float *pipe_host, int32_t n_stages,
                          int32_t *session_out);
/* Close a session: its queued requests are canceled (their poll returns
 * CM_ECANCELED), an admitted one still completes.  Errors: CM_ENOTFOUND. */
cm_status cm_session_close(cm_server *server, int32_t session);
/* The session's latest beam, from device memory: the server's k best
 * candidates of its most recently completed request ((-1, +inf) before the
 * first); the first k entries go into host arrays.  Errors: CM_EINVAL (k above the server's), CM_ENOTFOUND,
 * CM_EAGAIN (a request of the session is in flight), CM_EDEVICE. */
cm_status cm_session_beam(cm_server *server, int32_t session, int32_t k, int32_t *idx_host,
                          float *val_host);

/* Queue a request; returns with a ticket without waiting for the device (at
 * an idle server the call also launches the request, asynchronously).  A request takes
 * n_stages * n_cands * (80 + 32) + n_cands * 4 + k * 8 bytes of the arena
 * while admitted.  Errors: CM_EINVAL, CM_ENOTFOUND (session), CM_E2BIG (can
 * never be admitted: larger than the arena or a micro-batch, or above
 * cm_eval_batch's size limit for one query), CM_EAGAIN (queue full),
 * CM_EDEVICE (the server has failed). */
cm_status cm_serve_submit(cm_server *server, int32_t session, const cm_request *req,
                          uint64_t *ticket);
/* Non-blocking: CM_OK with the result (the ticket is then released),
 * CM_EAGAIN if not finished, CM_ECANCELED (released), CM_ENOTFOUND,
 * CM_EINVAL (result capacity too small), CM_EDEVICE (the server failed). */
cm_status cm_serve_poll(cm_server *server, uint64_t ticket, cm_result *out);
/* cm_serve_poll that waits up to timeout_ms for the result (CM_EAGAIN after). */
cm_status cm_serve_wait(cm_server *server, uint64_t ticket, int32_t timeout_ms, cm_result *out);

/* Queue n requests at once (request j for session sessions[j]), as n calls
 * of cm_serve_submit under one lock; tickets[j] receives each ticket.  All or
 * nothing: on an error no request is queued.  Errors: as cm_serve_submit. */
cm_status cm_serve_submit_batch(cm_server *server, int32_t n, const int32_t *sessions,
                                const cm_request *reqs, uint64_t *tickets);
/* Wait up to timeout_ms until every one of the n tickets has finished, then
 * release them, writing results into outs[j] (outs may be NULL to discard
 * them).  Returns CM_OK when all completed; the first CM_ECANCELED or
 * CM_EDEVICE otherwise (every finished ticket is still released); CM_EAGAIN
 * on time-out (nothing released); CM_ENOTFOUND for an unknown ticket;
 * CM_EINVAL when an outs[j] is too small. */
cm_status cm_serve_wait_all(cm_server *server, int32_t n, const uint64_t *tickets,
                            int32_t timeout_ms, cm_result *outs);

cm_status cm_server_get_stats(cm_server *server, cm_server_stats *out);
/* Clears the counters and latencies (not the queue or arena state). */
cm_status cm_server_reset_stats(cm_server *server);
/* Failure handling, forced from the host: the server's next micro-batch
 * launch fails as if the device had refused it (nothing is launched).  The
 * server then enters its failed state: every queued and admitted request
 * returns CM_EDEVICE from poll and wait, and later submissions and session
 * openings return CM_EDEVICE.  For tests of callers' error paths; a failed
 * server can only be destroyed.  Errors: CM_EINVAL. */
cm_status cm_server_fail_next_launch(cm_server *server);

/* Launch configuration of the server's steps (every slot; see
 * cm_step_config), for example the one cm_step_autotune or a short trial
 * of the caller picks for its traffic.  The default is the tuning cache's
 * entry for the server's max_batch_queries (cm_step_tuned_config), else
 * {grid 0 (two workgroups per compute unit), group_tiles 1, use_graph 1}; plain launches
 * (use_graph 0) cost a lone request less time per micro-batch.  Takes effect
 * for micro-batches launched afterwards; results never depend on it.
 * Errors: CM_EINVAL. */
cm_status cm_server_set_step_config(cm_server *server, const cm_step_config *cfg);
cm_status cm_server_get_step_config(const cm_server *server, cm_step_config *cfg);

/* Thread-local text of the last error on this thread ("" if none). */
const char *cm_last_error(void);
/* (major << 16) | minor */
int32_t cm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CM_H */
