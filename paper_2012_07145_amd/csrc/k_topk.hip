// k_topk.hip -- per-query beam selection kernel (Sec. 4, Sec. 4.4): one
// 256-thread workgroup per tile of up to TOPK_TILE candidates, query
// descriptors passed by value; the selection itself is in topk_dev.h.
#include "topk_dev.h"

namespace cm {
namespace {

using namespace topk;

constexpr int TK_THREADS = 256;

__device__ inline int find_tile_query(const TopkLaunch &L, int t)
{
    int q = 0;
    for (int j = 1; j < L.nq; ++j)
        if (L.q[j].tile0 <= t) q = j;
    return q;
}

__global__ __launch_bounds__(TK_THREADS) void k_topk(TopkLaunch L, const float *__restrict__ cost,
                                                     uint64_t *__restrict__ tpart,
                                                     int32_t *__restrict__ tcnt,
                                                     int32_t *__restrict__ idx_out,
                                                     float *__restrict__ val_out)
{
    __shared__ TopkShared<TK_THREADS> sh;
    __shared__ int last;
    const int t = threadIdx.x;
    const int task = blockIdx.x;
    const int q = find_tile_query(L, task);
    const TopkQ Q = L.q[q];
    const int tile = task - Q.tile0;
    const int k = L.k;
    const float *c = cost + Q.cost_off;

    uint64_t key[TopkShared<TK_THREADS>::PER];
    int nvalid;
    tile_keys<TK_THREADS, false>(c, Q.N, tile, key, nvalid);
    int nbest = tile_select<TK_THREADS>(key, nvalid, k, sh);

    if (Q.ntiles > 1) {
        publish_list<TK_THREADS>(sh, nbest, k, tpart + (int64_t)task * k);
        __syncthreads();
        if (t == 0) last = atomicAdd(&tcnt[q], 1) == Q.ntiles - 1;
        __syncthreads();
        if (!last) return;
        nbest = merge_lists<TK_THREADS>(tpart + (int64_t)Q.tile0 * k, Q.ntiles, Q.N, k, sh);
        if (t == 0) atomicExch(&tcnt[q], 0);
    }
    write_beam<TK_THREADS, false>(sh, nbest, k, c, idx_out + (int64_t)Q.out_q * k,
                           val_out + (int64_t)Q.out_q * k);
}

}  // namespace

hipError_t launch_topk(const TopkLaunch &L, const float *cost, uint64_t *tpart, int32_t *tcnt,
                       int32_t *idx_out, float *val_out, hipStream_t st)
{
    if (L.ntasks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_topk, dim3(L.ntasks), dim3(TK_THREADS), 0, st, L, cost, tpart, tcnt,
                       idx_out, val_out);
    return hipGetLastError();
}

}  // namespace cm
