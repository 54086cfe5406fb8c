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
#define CM_STAGE_CHUNK 16    /* sets the stage split of CM_BF16 (see cm_eval_batch) */

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
 *            float32; cost terms stay float32. */
typedef int32_t cm_precision;
enum { CM_FP32 = 0, CM_BF16 = 1 };

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
 * packed forms its kernels read.  params_host is not retained.  A model is
 * immutable and may be shared by concurrent calls.
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
 *                       float32 (CM_FP32) or bfloat16 bits (CM_BF16);
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
 * Errors: CM_EINVAL (bad descriptor, misaligned offset, NULL pointer),
 * CM_E2BIG (batch exceeds the workspace), CM_EUNSUPPORTED (precision),
 * CM_EDEVICE (launch failure). */
cm_status cm_eval_batch(const cm_model *model, cm_precision precision,
                        const cm_batch *batch, cm_workspace *ws, float *cost_out,
                        cm_stream stream);

/* Per-stage hoist (Sec. 5.2): the algorithm features of a stage are shared by
 * every candidate of its query, so their share of the first layer is
 * computed once per stage:
 *   U[row][j] = b_1[j] + sum_e W_1[j][e] (W_p log1p(pipe[s]) + b_p)[e]
 * (for CM_BF16 also + sum_e W_1[j][24 + e] b_s[e], since that form folds the
 * schedule embedding into the first layer).  Rows are written in batch order:
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

/* Thread-local text of the last error on this thread ("" if none). */
const char *cm_last_error(void);
/* (major << 16) | minor */
int32_t cm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CM_H */
