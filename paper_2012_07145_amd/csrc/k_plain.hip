// k_plain.hip -- per-stage hoist and the float32 evaluator.
//
// Hoist (one workgroup per stage): the algorithm features of a stage are the
// same for every candidate of the query, so their embedding and its share of
// the first layer are computed once per stage:
//   U[s] = W_1[:, :24] (W_p log1p(pipe[s]) + b_p) + b_1        (Sec. 5.2)
// plus W_1[:, 24:] b_s when the evaluator folds the schedule embedding into
// the first layer, times the hidden scale s_h of the FP8 form (1 else).
//
// Float32 evaluator: one thread per candidate walks the stages in ascending
// order, computing log1p of the 40 schedule features, the schedule embedding,
// the ReLU layer on the stacked embeddings, the ReLU coefficient layer and the
// dot product with the 8 cost terms (Sec. 5.2, App. B), and keeps a
// Kahan-compensated float32 sum over stages.
#include "cm_internal.h"

namespace cm {
namespace {

__device__ inline int find_query(const EvalLaunch &L, int t, bool by_stage)
{
    // Largest q with start(q) <= t.  Uniform across the workgroup.
    int q = 0;
    for (int j = 1; j < L.nq; ++j) {
        int start = by_stage ? L.q[j].hrow0 : L.q[j].task0;
        if (start <= t) q = j;
    }
    return q;
}

// One stage row of the hoist by a 64-thread workgroup: p = the stage's 56
// algorithm features, u = its 32 output floats.
__device__ inline void hoist_row(const float *__restrict__ params, const float *__restrict__ beta,
                                 int fold, float scale, const float *p, float *u, float *lp,
                                 float *ep)
{
    const int t = threadIdx.x;
    if (t < FP) lp[t] = log1pf(p[t]);
    __syncthreads();
    if (t < E) {
        const float *w = params + OFF_WP + t * FP;
        float a = params[OFF_BP + t];
        for (int f = 0; f < FP; ++f) a = fmaf(w[f], lp[f], a);
        ep[t] = a;
    }
    __syncthreads();
    if (t < H) {
        const float *w = params + OFF_W1 + t * 2 * E;
        float a = params[OFF_B1 + t];
        for (int e = 0; e < E; ++e) a = fmaf(w[e], ep[e], a);
        if (fold) a += beta[t];
        u[t] = a * scale;
    }
    __syncthreads();  // lp and ep are reused by the next row
}

__global__ __launch_bounds__(64) void k_hoist(EvalLaunch L, const float *__restrict__ params,
                                              const float *__restrict__ beta, int fold,
                                              float scale, const float *__restrict__ pipe,
                                              float *__restrict__ U)
{
    __shared__ float lp[FP];
    __shared__ float ep[E];
    const int q = find_query(L, blockIdx.x, true);
    const int s = blockIdx.x - L.q[q].hrow0;
    hoist_row(params, beta, fold, scale, pipe + L.q[q].pipe_off + (int64_t)s * FP,
              U + L.q[q].u_off + (int64_t)s * H, lp, ep);
}

// Hoist of a step: the rows of every query, grid-stride, from the device
// descriptors (the folded form of the bf16 and FP8 evaluators, with
// W_1[:, 24:] b_s folded in), times *scale when given (the FP8 form's s_h,
// read at run time so that a replayed graph follows the model's form).
__global__ __launch_bounds__(64) void k_hoist_step(const StepHead *__restrict__ h,
                                                   const StepQ *__restrict__ qs,
                                                   const float *__restrict__ params,
                                                   const float *__restrict__ beta,
                                                   const float *__restrict__ scale)
{
    __shared__ int32_t row0[STEP_MAX_QUERIES];
    __shared__ float lp[FP];
    __shared__ float ep[E];
    const int nq = h->nq, nrows = h->nrows;
    for (int j = threadIdx.x; j < nq; j += 64) row0[j] = qs[j].row0;
    __syncthreads();
    for (int r = blockIdx.x; r < nrows; r += gridDim.x) {
        // the last query whose first row is <= r
        int lo = 0, hi = nq - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (row0[mid] <= r) lo = mid;
            else hi = mid - 1;
        }
        const StepQ &D = qs[lo];
        const int s = r - row0[lo];
        hoist_row(params, beta, 1, scale ? *scale : 1.f, D.pipe + (int64_t)s * FP,
                  D.u + (int64_t)s * H, lp, ep);
    }
}

__global__ __launch_bounds__(64) void k_eval_fp32(EvalLaunch L, const float *__restrict__ params,
                                                  const float *__restrict__ sched,
                                                  const float *__restrict__ terms,
                                                  const float *__restrict__ U,
                                                  float *__restrict__ cost,
                                                  float *__restrict__ stage)
{
    const int q = find_query(L, blockIdx.x, false);
    const EvalQ Q = L.q[q];
    const int i = (blockIdx.x - Q.task0) * 64 + threadIdx.x;
    if (i >= Q.N) return;

    const float *Ws = params + OFF_WS;
    const float *bs = params + OFF_BS;
    const float *W1 = params + OFF_W1;
    const float *W2 = params + OFF_W2;
    const float *b2 = params + OFF_B2;

    float sum = 0.f, comp = 0.f;
    for (int s = 0; s < Q.S; ++s) {
        const int64_t r = (int64_t)s * Q.N + i;
        const float4 *xr = reinterpret_cast<const float4 *>(sched + Q.sched_off + r * FS);
        float x[FS];
#pragma unroll
        for (int v = 0; v < FS / 4; ++v) {
            float4 t4 = xr[v];
            x[4 * v + 0] = log1pf(t4.x);
            x[4 * v + 1] = log1pf(t4.y);
            x[4 * v + 2] = log1pf(t4.z);
            x[4 * v + 3] = log1pf(t4.w);
        }
        float es[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            float a = bs[e];
#pragma unroll
            for (int f = 0; f < FS; ++f) a = fmaf(Ws[e * FS + f], x[f], a);
            es[e] = a;
        }
        const float *u = U + Q.u_off + (int64_t)s * H;
        float h[H];
#pragma unroll
        for (int j = 0; j < H; ++j) {
            float a = u[j];
#pragma unroll
            for (int e = 0; e < E; ++e) a = fmaf(W1[j * 2 * E + E + e], es[e], a);
            h[j] = a < 0.f ? 0.f : a;  // ReLU; a NaN passes through
        }
        const float *tr = terms + Q.terms_off + r * C;
        float v = 0.f;
#pragma unroll
        for (int m = 0; m < C; ++m) {
            float a = b2[m];
#pragma unroll
            for (int j = 0; j < H; ++j) a = fmaf(W2[m * H + j], h[j], a);
            const float c = a < 0.f ? 0.f : a;
            v = fmaf(c, tr[m], v);
        }
        if (stage) stage[Q.stage_off + r] = v;
        // Kahan-compensated stage sum
        const float y = v - comp;
        const float t = sum + y;
        comp = (t - sum) - y;
        sum = t;
    }
    cost[Q.cost_off + i] = sum;
}

}  // namespace

hipError_t launch_hoist(const EvalLaunch &L, const Model &m, bool fold, float scale,
                        const float *pipe, float *U, hipStream_t st)
{
    if (L.nstages == 0) return hipSuccess;
    hipLaunchKernelGGL(k_hoist, dim3(L.nstages), dim3(64), 0, st, L, m.d_params, m.d_beta,
                       fold ? 1 : 0, scale, pipe, U);
    return hipGetLastError();
}

hipError_t launch_step_hoist(const StepHead *h, const StepQ *qs, const Model &m,
                             cm_precision prec, int grid, hipStream_t st)
{
    const float *scale = prec == CM_FP8 ? &m.d_fp8->uh : nullptr;
    hipLaunchKernelGGL(k_hoist_step, dim3(grid), dim3(64), 0, st, h, qs, m.d_params, m.d_beta,
                       scale);
    return hipGetLastError();
}

hipError_t launch_eval_fp32(const EvalLaunch &L, const Model &m, const float *sched,
                            const float *terms, const float *U, float *cost, float *stage,
                            hipStream_t st)
{
    if (L.ntasks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_eval_fp32, dim3(L.ntasks), dim3(64), 0, st, L, m.d_params, sched,
                       terms, U, cost, stage);
    return hipGetLastError();
}

}  // namespace cm
