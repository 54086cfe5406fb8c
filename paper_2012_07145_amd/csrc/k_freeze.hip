// k_freeze.hip -- freezing of the lowest-cost stages (Sec. 3.2): for the
// candidate a search kept, every stage except the ceil(log2 S) most costly
// ones has its schedule options frozen.  One workgroup per query ranks the
// candidate's per-stage costs by counting.
#include "cm_internal.h"

namespace cm {
namespace {

constexpr int FREEZE_THREADS = 256;
constexpr int FREEZE_CHUNK = 2048;  // stage keys staged in LDS at a time

// Order-preserving key of a stage cost: ascending cost, -0 == +0, NaN after
// every number (all NaNs equal).
__device__ inline uint32_t cost_key(float v)
{
    if (v != v) return 0xffffffffu;
    if (v == 0.f) v = 0.f;
    const uint32_t u = __float_as_uint(v);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__global__ __launch_bounds__(FREEZE_THREADS) void k_freeze(FreezeLaunch L,
                                                           const float *__restrict__ stage,
                                                           const int32_t *__restrict__ cand,
                                                           int64_t cand_stride,
                                                           uint8_t *__restrict__ frozen)
{
    __shared__ uint32_t keys[FREEZE_CHUNK];
    const FreezeQ Q = L.q[blockIdx.x];
    const int c = cand[Q.cand_q * cand_stride];
    uint8_t *out = frozen + Q.flag_off;
    if (c < 0 || c >= Q.N) {  // no candidate kept: nothing is frozen
        for (int s = threadIdx.x; s < Q.S; s += FREEZE_THREADS) out[s] = 0;
        return;
    }
    int lg = 0;  // ceil(log2 S): the stages left unfrozen
    while ((1 << lg) < Q.S) ++lg;
    const int nfreeze = Q.S - lg;
    const float *v = stage + Q.stage_off + c;  // v[s * N]

    // each thread ranks up to FREEZE_CHUNK / FREEZE_THREADS stages per round
    constexpr int PER = FREEZE_CHUNK / FREEZE_THREADS;
    for (int base = 0; base < Q.S; base += FREEZE_CHUNK) {
        uint32_t mine[PER];
        int rank[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int s = base + j * FREEZE_THREADS + threadIdx.x;
            mine[j] = s < Q.S ? cost_key(v[(int64_t)s * Q.N]) : 0u;
            rank[j] = 0;
        }
        // count the stages ahead of each of mine: lower key, or equal key and
        // lower index
        for (int t0 = 0; t0 < Q.S; t0 += FREEZE_CHUNK) {
            __syncthreads();
            for (int t = threadIdx.x; t < FREEZE_CHUNK; t += FREEZE_THREADS)
                keys[t] = t0 + t < Q.S ? cost_key(v[(int64_t)(t0 + t) * Q.N]) : 0u;
            __syncthreads();
            const int nt = min(FREEZE_CHUNK, Q.S - t0);
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                const int s = base + j * FREEZE_THREADS + threadIdx.x;
                int r = 0;
                for (int t = 0; t < nt; ++t) {
                    const uint32_t k = keys[t];
                    r += (k < mine[j]) || (k == mine[j] && t0 + t < s);
                }
                rank[j] += r;
            }
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int s = base + j * FREEZE_THREADS + threadIdx.x;
            if (s < Q.S) out[s] = rank[j] < nfreeze ? 1 : 0;
        }
    }
}

}  // namespace

hipError_t launch_freeze(const FreezeLaunch &L, const float *stage, const int32_t *cand,
                         int64_t cand_stride, uint8_t *frozen, hipStream_t st)
{
    if (L.nq == 0) return hipSuccess;
    hipLaunchKernelGGL(k_freeze, dim3(L.nq), dim3(FREEZE_THREADS), 0, st, L, stage, cand,
                       cand_stride, frozen);
    return hipGetLastError();
}

}  // namespace cm
