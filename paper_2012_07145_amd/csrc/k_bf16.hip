// k_bf16.hip -- the bf16 matrix-core evaluator of the cost model (Sec. 5.2),
// one workgroup per row-tile group, query descriptors passed by value (up to
// QMAX queries per launch).  The arithmetic lives in eval_bf16.h and is the
// same as in the persistent step kernel.
#include "eval_bf16.h"

namespace cm {
namespace {

using namespace bf16eval;

__device__ inline int find_task_query(const EvalLaunch &L, int t)
{
    int q = 0;
    for (int j = 1; j < L.nq; ++j)
        if (L.q[j].task0 <= t) q = j;
    return q;
}

template <bool kStage, bool kIndexed>
__global__ __launch_bounds__(EVAL_WAVES * 64) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_eval_bf16(
    EvalLaunch L, const Bf16Pack *__restrict__ pk, const uint16_t *sched, const float *terms,
    const float *__restrict__ U, float *__restrict__ cost, float *__restrict__ stage,
    const int32_t *__restrict__ ridx, uint32_t rows)
{
    __shared__ GroupShared sh;
    __shared__ uint32_t tab[LOG_N];
    load_table(tab, pk);
    const int lane = threadIdx.x & 63;
    // wave-uniform values are kept in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int q = find_task_query(L, blockIdx.x);
    const EvalQ &E = L.q[q];
    QueryView Q;
    // memoized rows: sched is the row table and sched_off locates the row numbers
    Q.x = kIndexed ? sched : sched + E.sched_off;
    Q.ridx = kIndexed ? ridx + E.sched_off : nullptr;
    Q.rows = rows;
    Q.t = terms + E.terms_off;
    Q.u = U + E.u_off;
    Q.cost = cost + E.cost_off;
    Q.stage = kStage ? stage + E.stage_off : nullptr;
    Q.S = E.S;
    Q.N = E.N;
    Q.P = E.parts;
    const Weights w = load_weights(pk, lane);
    const Pairs kp = make_pairs();
    __syncthreads();  // the table is in LDS
    eval_group<false, kStage, kIndexed>(Q, blockIdx.x - E.task0, wave, lane, w, kp, tab, sh);
}

__global__ __launch_bounds__(256) void k_log_table(Bf16Pack *pk)
{
    const Pairs kp = make_pairs();
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < LOG_N) pk->logtab[i] = log_entry(LOG_BASE + (uint32_t)i, kp);
}

}  // namespace

hipError_t launch_log_table(Bf16Pack *pk, hipStream_t st)
{
    hipLaunchKernelGGL(k_log_table, dim3((LOG_N + 255) / 256), dim3(256), 0, st, pk);
    return hipGetLastError();
}

hipError_t launch_eval_bf16(const EvalLaunch &L, const Model &m, const uint16_t *sched,
                            const float *terms, const float *U, float *cost, float *stage,
                            hipStream_t st, const int32_t *ridx, uint32_t rows)
{
    if (L.ntasks == 0) return hipSuccess;
    const dim3 g(L.ntasks), b(EVAL_WAVES * 64);
    if (ridx) {
        if (stage)
            hipLaunchKernelGGL((k_eval_bf16<true, true>), g, b, 0, st, L, m.d_bf16, sched, terms,
                               U, cost, stage, ridx, rows);
        else
            hipLaunchKernelGGL((k_eval_bf16<false, true>), g, b, 0, st, L, m.d_bf16, sched, terms,
                               U, cost, stage, ridx, rows);
    } else if (stage) {
        hipLaunchKernelGGL((k_eval_bf16<true, false>), g, b, 0, st, L, m.d_bf16, sched, terms, U,
                           cost, stage, ridx, rows);
    } else {
        hipLaunchKernelGGL((k_eval_bf16<false, false>), g, b, 0, st, L, m.d_bf16, sched, terms, U,
                           cost, stage, ridx, rows);
    }
    return hipGetLastError();
}

}  // namespace cm
