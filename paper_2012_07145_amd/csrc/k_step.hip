// k_step.hip -- the persistent step kernel: bf16 or FP8 evaluation of many
// ragged queries (Sec. 5.2) and each query's beam selection (Sec. 4, Sec. 4.4)
// in one launch whose shape never depends on the batch.
//
// A fixed grid of workgroups (8 waves each) takes tasks from a device-wide
// queue (one atomic add per task, taken when the previous task ends).  A task is `gpt`
// consecutive row-tile groups of one query, evaluated exactly as the
// per-call kernels do (eval_bf16.h, eval_fp8.h), so the costs are
// bit-identical to them.
// Tasks never straddle a selection tile of TOPK_TILE candidates; the
// workgroup whose task completes a tile (an arrival count per tile) selects
// that tile's k best, and for a query of several tiles the last tile to
// finish merges their lists.  A query's selection therefore runs while other queries are
// still being evaluated.  All control words are left at zero when the
// kernel ends, so the next launch needs no clearing.
#include "eval_bf16.h"
#include "eval_fp8.h"
#include "topk_dev.h"

namespace cm {
namespace {

using namespace bf16eval;
using namespace topk;

constexpr int NT = EVAL_WAVES * 64;

// Selection of tile `tile` of query q after the last of its tasks has
// arrived, and for a query of several tiles, the merge by the last tile.
__device__ __forceinline__ void select_tile(const StepQ &D, int q, int tile, int k, uint32_t *qcnt,
                            uint64_t *tpart, TopkShared<NT> &tsh, int &s_query_last)
{
    const int tid = threadIdx.x;
    uint64_t key[TopkShared<NT>::PER];
    int nvalid;
    tile_keys<NT, true>(D.cost, D.N, tile, key, nvalid);
    int nbest = tile_select<NT>(key, nvalid, k, tsh);
    bool write = true;
    if (D.ntiles > 1) {
        publish_list<NT>(tsh, nbest, k, tpart + (int64_t)(D.tile0 + tile) * k);
        __syncthreads();
        if (tid == 0) s_query_last = atomicAdd(&qcnt[q], 1u) == (uint32_t)(D.ntiles - 1);
        __syncthreads();
        write = s_query_last;
        if (write) {
            if (tid == 0) atomicExch(&qcnt[q], 0u);
            nbest = merge_lists<NT>(tpart + (int64_t)D.tile0 * k, D.ntiles, D.N, k, tsh);
        }
    }
    if (write) {
        write_beam<NT, true>(tsh, nbest, k, D.cost, D.idx, D.val);
        if (D.sidx) write_beam<NT, true>(tsh, nbest, k, D.cost, D.sidx, D.sval);
    }
}

// One task's evaluation: gpt row-tile groups of one query.
__device__ __forceinline__ void eval_task(const StepQ &D, int tq, int gpt, int wave, int lane,
                                          const Bf16Pack *__restrict__ pk, const Pairs &kp,
                                          const uint32_t *tab, GroupShared &gsh)
{
    QueryView Q;
    Q.x = static_cast<const uint16_t *>(D.x);
    Q.t = D.t;
    Q.u = D.u;
    Q.cost = D.cost;
    Q.S = D.S;
    Q.N = D.N;
    Q.P = D.parts;
    const int group_rows = TILE_ROWS * (EVAL_WAVES / Q.P);
    const Weights w = load_weights(pk, lane);
    for (int g = 0; g < gpt; ++g) {
        const int group = tq * gpt + g;
        if (group * group_rows >= Q.N) break;  // uniform
        eval_group<true>(Q, group, wave, lane, w, kp, tab, gsh);
        __syncthreads();  // the group's LDS is reused by the next group
    }
}

__device__ __forceinline__ void eval_task(const StepQ &D, int tq, int gpt, int wave, int lane,
                                          const Fp8Pack *__restrict__ pk, const Pairs &,
                                          const uint32_t *, GroupShared &gsh)
{
    fp8eval::QueryView8 Q;
    Q.x = static_cast<const uint8_t *>(D.x);
    Q.t = D.t;
    Q.u = D.u;
    Q.cost = D.cost;
    Q.S = D.S;
    Q.N = D.N;
    Q.P = D.parts;
    const int group_rows = TILE_ROWS * (EVAL_WAVES / Q.P);
    const fp8eval::Weights8 w = fp8eval::load_weights8(pk, lane);
    for (int g = 0; g < gpt; ++g) {
        const int group = tq * gpt + g;
        if (group * group_rows >= Q.N) break;  // uniform
        fp8eval::eval_group8<true>(Q, group, wave, lane, w, gsh);
        __syncthreads();
    }
}

// LDS table of the log transform: the bf16 evaluator's only.
template <class Pack> struct LogTable { static constexpr int n = 1; };
template <> struct LogTable<Bf16Pack> { static constexpr int n = LOG_N; };

// The evaluation's and the selection's LDS are never in use at the same time
// (a workgroup-wide barrier separates every switch between them).
union StepShared {
    GroupShared g;
    TopkShared<NT> t;
};

template <class Pack>
__device__ __forceinline__ void step_body(const StepHead *__restrict__ h,
                                          const StepQ *__restrict__ qs, uint32_t *ctl,
                                          uint64_t *tpart, const Pack *__restrict__ pk)
{
    __shared__ StepShared ssh;
    __shared__ uint32_t tab[LogTable<Pack>::n];
    GroupShared &gsh = ssh.g;
    TopkShared<NT> &tsh = ssh.t;
    __shared__ int32_t task0[STEP_MAX_QUERIES];
    __shared__ int s_next, s_tail, s_query_last;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nq = h->nq, ntasks = h->ntasks, k = h->k, gpt = h->gpt;
    uint32_t *qcnt = ctl + CTL_QCNT;
    uint32_t *tcnt = ctl + CTL_TCNT;
    unsigned long long *clk = reinterpret_cast<unsigned long long *>(ctl + CTL_CLK);

    for (int j = tid; j < nq; j += NT) task0[j] = qs[j].task0;
    if constexpr (LogTable<Pack>::n > 1) load_table(tab, pk);
    if (tid == 0) {
        atomicMin(&clk[0], (unsigned long long)__builtin_amdgcn_s_memrealtime());
        s_next = (int)atomicAdd(&ctl[CTL_NEXT], 1u);
    }
    const Pairs kp = make_pairs();
    __syncthreads();
    int t = s_next;
    while (t < ntasks) {
        // the query of task t: the last q with task0[q] <= t
        int lo = 0, hi = nq - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (task0[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const int q = __builtin_amdgcn_readfirstlane(lo);
        const StepQ &D = qs[q];
        const int tq = t - D.task0;  // task within the query
        const int group_rows = TILE_ROWS * (EVAL_WAVES / D.parts);
        eval_task(D, tq, gpt, wave, lane, pk, kp, tab, gsh);
        // this task's costs (coherent stores) have completed before it counts
        // itself at its selection tile; the next task is taken only now, so
        // that the queue hands work to whichever workgroup is free first
        const int tpt = TOPK_TILE / (group_rows * gpt);  // tasks per tile
        const int tile = tq / tpt;
        wait_stores();
        __syncthreads();
        if (tid == 0) {
            const uint32_t need = (uint32_t)min(tpt, D.ntasks - tile * tpt);
            const uint32_t next = atomicAdd(&ctl[CTL_NEXT], 1u);
            const uint32_t arrived = atomicAdd(&tcnt[D.tile0 + tile], 1u);
            s_next = (int)next;
            s_tail = arrived == need - 1;
        }
        __syncthreads();
        if (s_tail) {
            if (tid == 0) atomicExch(&tcnt[D.tile0 + tile], 0u);
            select_tile(D, q, tile, k, qcnt, tpart, tsh, s_query_last);
        }
        t = s_next;
        __syncthreads();  // s_next and s_tail are read; the selection's LDS is free
    }
    // the last workgroup to leave resets the queue for the next launch (every
    // other workgroup has made its final queue fetch before counting itself)
    // and publishes the launch's clock pair
    if (tid == 0) {
        atomicMax(&clk[1], (unsigned long long)__builtin_amdgcn_s_memrealtime());
        wait_stores();
        if (atomicAdd(&ctl[CTL_DONE], 1u) == gridDim.x - 1) {
            unsigned long long *out = reinterpret_cast<unsigned long long *>(ctl + CTL_CLKOUT);
            const unsigned long long c0 = atomicExch(&clk[0], ~0ull);
            const unsigned long long c1 = atomicExch(&clk[1], 0ull);
            store_shared(&out[0], c0);
            store_shared(&out[1], c1);
            if (h->clk_out) {
                __hip_atomic_store(&h->clk_out[0], (uint64_t)c0, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(&h->clk_out[1], (uint64_t)c1, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_SYSTEM);
            }
            atomicExch(&ctl[CTL_NEXT], 0u);
            atomicExch(&ctl[CTL_DONE], 0u);
        }
    }
}

__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_step_bf16(
    const StepHead *__restrict__ h, const StepQ *__restrict__ qs, uint32_t *ctl,
    uint64_t *tpart, const Bf16Pack *__restrict__ pk)
{
    step_body(h, qs, ctl, tpart, pk);
}

__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_step_fp8(
    const StepHead *__restrict__ h, const StepQ *__restrict__ qs, uint32_t *ctl,
    uint64_t *tpart, const Fp8Pack *__restrict__ pk)
{
    step_body(h, qs, ctl, tpart, pk);
}

}  // namespace

hipError_t launch_step(const StepHead *h, const StepQ *qs, uint32_t *ctl, uint64_t *tpart,
                       const Model &m, cm_precision prec, int grid, hipStream_t st)
{
    if (prec == CM_FP8)
        hipLaunchKernelGGL(k_step_fp8, dim3(grid), dim3(NT), 0, st, h, qs, ctl, tpart, m.d_fp8);
    else
        hipLaunchKernelGGL(k_step_bf16, dim3(grid), dim3(NT), 0, st, h, qs, ctl, tpart,
                           m.d_bf16);
    return hipGetLastError();
}

}  // namespace cm
