// k_topk.hip -- per-query beam selection (Sec. 4: the search keeps the k best
// candidate states; Sec. 4.4: evaluated candidates are added to the beam).
//
// Ranking key: 64 bits = (order-preserving image of the float32 cost) << 32 |
// candidate index.  -0 is mapped to +0 and every NaN to one quiet NaN that
// ranks after +inf, so the unsigned order of the keys is exactly "ascending
// cost, ties by lower index, NaN last", and keys are unique.
//
// One wavefront per tile of TOPK_TILE candidates keeps a sorted list of the
// 64*M smallest keys seen (M registers per lane, element e = r*64 + lane).
// Each batch of 64 keys (one per lane) is skipped when no key beats the
// current k-th best; otherwise it is bitonic-sorted across the wave, reversed
// and min-merged into the list's last register, and a bitonic merge restores
// the order.  A query with several tiles writes each tile's k best to the
// workspace; the last tile to finish merges them with the same routine.
#include "cm_internal.h"

namespace cm {
namespace {

constexpr uint64_t SENT = ~0ull;  // empty slot: ranks after every real key

__device__ inline uint64_t make_key(float c, uint32_t idx)
{
    uint32_t b = __float_as_uint(c);
    const uint32_t mag = b & 0x7fffffffu;
    if (mag == 0) b = 0;                        // -0 -> +0
    else if (mag > 0x7f800000u) b = 0x7fc00000u;  // any NaN -> one quiet NaN
    b = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    return ((uint64_t)b << 32) | idx;
}

__device__ inline uint64_t shfl_xor64(uint64_t v, int m)
{
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m);
    return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint64_t shfl64(uint64_t v, int src)
{
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }
__device__ inline uint64_t umax64(uint64_t a, uint64_t b) { return a < b ? b : a; }

template <int M>
struct Beam {
    uint64_t R[M];

    __device__ void clear()
    {
#pragma unroll
        for (int r = 0; r < M; ++r) R[r] = SENT;
    }

    // element e = k-1 of the sorted list, broadcast to the wave
    __device__ uint64_t kth(int k) const
    {
        const int e = k - 1;
        const int rr = e >> 6;
        uint64_t v = R[0];
#pragma unroll
        for (int r = 1; r < M; ++r)
            if (r == rr) v = R[r];
        return shfl64(v, e & 63);
    }

    __device__ void insert(uint64_t key, int lane)
    {
        // bitonic sort of the 64 incoming keys, ascending
#pragma unroll
        for (int kk = 2; kk <= 64; kk <<= 1) {
#pragma unroll
            for (int j = kk >> 1; j > 0; j >>= 1) {
                const uint64_t o = shfl_xor64(key, j);
                const bool asc = (lane & kk) == 0;
                const bool low = (lane & j) == 0;
                key = (low == asc) ? umin64(key, o) : umax64(key, o);
            }
        }
        // the smallest 64*M of list + batch form a bitonic sequence
        R[M - 1] = umin64(R[M - 1], shfl64(key, 63 - lane));
#pragma unroll
        for (int j = 32 * M; j >= 64; j >>= 1) {
            const int d = j >> 6;
#pragma unroll
            for (int r = 0; r < M; ++r) {
                if ((r & d) == 0) {
                    const uint64_t a = R[r], b = R[r | d];
                    R[r] = umin64(a, b);
                    R[r | d] = umax64(a, b);
                }
            }
        }
#pragma unroll
        for (int j = 32; j > 0; j >>= 1) {
#pragma unroll
            for (int r = 0; r < M; ++r) {
                const uint64_t o = shfl_xor64(R[r], j);
                R[r] = ((lane & j) == 0) ? umin64(R[r], o) : umax64(R[r], o);
            }
        }
    }

    // stream keys src[0..n) through the list
    __device__ void absorb(const uint64_t *src, int n, int k, int lane)
    {
        uint64_t thr = kth(k);
        for (int base = 0; base < n; base += 64) {
            const int e = base + lane;
            const uint64_t key = e < n ? src[e] : SENT;
            if (!__any(key < thr)) continue;
            insert(key, lane);
            thr = kth(k);
        }
    }
};

__device__ inline int find_tile_query(const TopkLaunch &L, int t)
{
    int q = 0;
    for (int j = 1; j < L.nq; ++j)
        if (L.q[j].tile0 <= t) q = j;
    return q;
}

template <int M>
__global__ __launch_bounds__(64) void k_topk(TopkLaunch L, const float *__restrict__ cost,
                                             uint64_t *__restrict__ tpart,
                                             int32_t *__restrict__ tcnt,
                                             int32_t *__restrict__ idx_out,
                                             float *__restrict__ val_out)
{
    const int lane = threadIdx.x;
    const int task = blockIdx.x;
    const int q = find_tile_query(L, task);
    const TopkQ Q = L.q[q];
    const int tile = task - Q.tile0;
    const int k = L.k;
    const float *c = cost + Q.cost_off;

    Beam<M> B;
    B.clear();
    const int beg = tile * TOPK_TILE;
    const int end = min(Q.N, beg + TOPK_TILE);
    uint64_t thr = SENT;
    for (int base = beg; base < end; base += 64) {
        const int i = base + lane;
        const uint64_t key = i < end ? make_key(c[i], (uint32_t)i) : SENT;
        if (!__any(key < thr)) continue;
        B.insert(key, lane);
        thr = B.kth(k);
    }

    if (Q.ntiles > 1) {
        uint64_t *mine = tpart + (int64_t)task * k;
#pragma unroll
        for (int r = 0; r < M; ++r) {
            const int e = r * 64 + lane;
            if (e < k) mine[e] = B.R[r];
        }
        __threadfence();
        int old = 0;
        if (lane == 0) old = atomicAdd(&tcnt[q], 1);
        old = __shfl(old, 0);
        if (old != Q.ntiles - 1) return;
        __threadfence();
        B.clear();
        B.absorb(tpart + (int64_t)Q.tile0 * k, Q.ntiles * k, k, lane);
        if (lane == 0) atomicExch(&tcnt[q], 0);
    }

#pragma unroll
    for (int r = 0; r < M; ++r) {
        const int e = r * 64 + lane;
        if (e < k) {
            const uint64_t key = B.R[r];
            int32_t id = -1;
            float v = __builtin_inff();
            if (key != SENT) {
                id = (int32_t)(uint32_t)key;
                v = c[id];
            }
            idx_out[(int64_t)Q.out_q * k + e] = id;
            val_out[(int64_t)Q.out_q * k + e] = v;
        }
    }
}

}  // namespace

hipError_t launch_topk(const TopkLaunch &L, const float *cost, uint64_t *tpart, int32_t *tcnt,
                       int32_t *idx_out, float *val_out, hipStream_t st)
{
    if (L.ntasks == 0) return hipSuccess;
    if (L.k <= 64)
        hipLaunchKernelGGL(k_topk<1>, dim3(L.ntasks), dim3(64), 0, st, L, cost, tpart, tcnt,
                           idx_out, val_out);
    else if (L.k <= 128)
        hipLaunchKernelGGL(k_topk<2>, dim3(L.ntasks), dim3(64), 0, st, L, cost, tpart, tcnt,
                           idx_out, val_out);
    else
        hipLaunchKernelGGL(k_topk<4>, dim3(L.ntasks), dim3(64), 0, st, L, cost, tpart, tcnt,
                           idx_out, val_out);
    return hipGetLastError();
}

}  // namespace cm
