// k_penalty.hip -- the known-bad-state penalty of the multi-pass search
// (Sec. 4.5): a candidate whose structural hash at the current pass's depth
// was seen before and judged unpromising gets a cost penalty, which moves it
// back in the beam before selection.
#include <algorithm>

#include "cm_internal.h"

namespace cm {
namespace {

constexpr int PENALTY_THREADS = 256;

// Is h in bad[0, n) (ascending)?  Lower bound by bisection.
__device__ inline bool contains(const uint64_t *__restrict__ bad, int64_t n, uint64_t h)
{
    int64_t lo = 0, len = n;
    while (len > 0) {
        const int64_t half = len >> 1;
        if (bad[lo + half] < h) {
            lo += half + 1;
            len -= half + 1;
        } else {
            len = half;
        }
    }
    return lo < n && bad[lo] == h;
}

// One thread per candidate of the launch's queries (grid-stride over a
// prefix of candidate counts in the descriptors).
__global__ __launch_bounds__(PENALTY_THREADS) void k_penalty(PenaltyLaunch L,
                                                             const uint64_t *__restrict__ hashes,
                                                             const uint64_t *__restrict__ bad,
                                                             int64_t n_bad, float penalty,
                                                             float *__restrict__ cost)
{
    const int64_t total = L.q[L.nq - 1].cand0 + L.q[L.nq - 1].N;
    for (int64_t t = (int64_t)blockIdx.x * PENALTY_THREADS + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * PENALTY_THREADS) {
        int q = 0;
        for (int j = 1; j < L.nq; ++j)
            if (L.q[j].cand0 <= t) q = j;
        const int64_t i = L.q[q].cost_off + (t - L.q[q].cand0);
        if (contains(bad, n_bad, hashes[i])) cost[i] = cost[i] + penalty;
    }
}

}  // namespace

hipError_t launch_penalty(const PenaltyLaunch &L, const uint64_t *hashes, const uint64_t *bad,
                          int64_t n_bad, float penalty, float *cost, hipStream_t st)
{
    if (L.nq == 0) return hipSuccess;
    const int64_t total = L.q[L.nq - 1].cand0 + L.q[L.nq - 1].N;
    if (total == 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((total + PENALTY_THREADS - 1) / PENALTY_THREADS, 4096);
    hipLaunchKernelGGL(k_penalty, dim3((unsigned)blocks), dim3(PENALTY_THREADS), 0, st, L,
                       hashes, bad, n_bad, penalty, cost);
    return hipGetLastError();
}

}  // namespace cm
