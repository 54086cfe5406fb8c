// topk_dev.h -- device code of per-query beam selection (Sec. 4: the search
// keeps the k best candidate states; Sec. 4.4: evaluated candidates are added
// to the beam), shared by the selection kernel and the tail of the
// persistent step kernel.
//
// Ranking key: 64 bits = (order-preserving image of the float32 cost) << 32 |
// candidate index.  -0 is mapped to +0 and every NaN to one quiet NaN that
// ranks after +inf, so the unsigned order of the keys is exactly "ascending
// cost, ties by lower index, NaN last", and keys are unique.
//
// One workgroup of NT threads selects over a tile of up to TOPK_TILE
// candidates (TOPK_TILE / NT keys per thread, element e = j*NT + thread):
//   1. every thread takes the minimum of its keys; the k-th smallest of these
//      NT minima (a bitonic sort of the minima across the workgroup) is a
//      threshold T with at least k keys <= T (the k minima themselves), and
//      for unordered costs only slightly more than k;
//   2. keys <= T are compacted into LDS with one atomic per wave and key slot;
//   3. each compacted key is placed by counting the compacted keys below it;
//      keys placed at rank < k are the k best, already in order.
// If more than 1024 keys pass the threshold (only possible for large k), a
// workgroup-wide bitwise radix search over them takes the place of step 3.
// A query with several tiles has each tile's sorted k best written to a
// device list; the last tile to finish selects again over those lists.
#pragma once

#include "cm_internal.h"

namespace cm {
namespace topk {

constexpr uint64_t SENT = ~0ull;  // empty slot: ranks after every real key
constexpr int RANK_MAX = 1024;  // largest compacted set placed by counting
static_assert(TOPK_TILE > CM_MAX_K, "a merge pass must make progress");

__device__ inline uint64_t make_key(float c, uint32_t idx)
{
    uint32_t b = __float_as_uint(c);
    const uint32_t mag = b & 0x7fffffffu;
    if (mag == 0) b = 0;                          // -0 -> +0
    else if (mag > 0x7f800000u) b = 0x7fc00000u;  // any NaN -> one quiet NaN
    b = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    return ((uint64_t)b << 32) | idx;
}

// NT = threads of the workgroup that selects (256 or 512); element e of a
// tile is held by thread e % NT as its key e / NT.
template <int NT>
struct TopkShared {
    static constexpr int WAVES = NT / 64;
    static constexpr int PER = TOPK_TILE / NT;
    static_assert(PER * NT == TOPK_TILE, "tile split");
    static_assert(NT >= CM_MAX_K, "one thread per output slot");
    uint64_t mins[NT];
    uint64_t filt[TOPK_TILE];
    uint64_t best[CM_MAX_K];
    uint64_t thr;
    uint32_t nfilt;
    uint32_t cnt[2][WAVES];
    uint32_t red_and[WAVES], red_or[WAVES];
};

__device__ inline uint32_t wave_count(bool p) { return (uint32_t)__popcll(__ballot(p)); }

// The thread's index, opaque to the compiler: values derived from it (lane
// masks, partner addresses of the sort) are recomputed where they are used
// instead of being hoisted out of the persistent kernel's task loop, where
// they would stay live through the evaluation and spill.
__device__ inline int sel_tid()
{
    int t = (int)threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// ---------------------------------------------------------------- sorting
__device__ inline uint64_t shfl_xor64(uint64_t v, int mask)
{
    const int lo = __shfl_xor((int)(uint32_t)v, mask);
    const int hi = __shfl_xor((int)(uint32_t)(v >> 32), mask);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// Ascending bitonic sort of one key per thread across the NT-thread
// workgroup: thread t returns the key of rank t.  Pairs closer than a wave
// exchange by shuffles; farther ones through x (NT keys of LDS).
template <int NT>
__device__ uint64_t block_sort1(uint64_t key, uint64_t *x)
{
    const int t = sel_tid();
#pragma unroll
    for (int size = 2; size <= NT; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            uint64_t other;
            if (stride >= 64) {
                x[t] = key;
                __syncthreads();
                other = x[t ^ stride];
                __syncthreads();
            } else {
                other = shfl_xor64(key, stride);
            }
            const bool up = (t & size) == 0;       // this run ascends
            const bool lower = (t & stride) == 0;  // t is the first of its pair
            const uint64_t mn = key < other ? key : other;
            const uint64_t mx = key < other ? other : key;
            key = lower == up ? mn : mx;
        }
    }
    return key;
}

// ---------------------------------------------------------------- workgroup
template <int NT>
__device__ inline uint32_t block_sum(uint32_t wave_value, TopkShared<NT> &sh, int &buf)
{
    const int tid = sel_tid();
    const int w = tid >> 6;
    if ((tid & 63) == 0) sh.cnt[buf][w] = wave_value;
    __syncthreads();
    uint32_t tot = 0;
#pragma unroll
    for (int j = 0; j < NT / 64; ++j) tot += sh.cnt[buf][j];
    buf ^= 1;
    return tot;
}

template <int NT, int PER>
__device__ uint32_t block_radix(const uint32_t (&val)[PER], const bool (&sel)[PER],
                                uint32_t &rank, TopkShared<NT> &sh, int &buf)
{
    uint32_t a = 0xffffffffu, o = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j)
        if (sel[j]) {
            a &= val[j];
            o |= val[j];
        }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        a &= (uint32_t)__shfl_xor((int)a, d);
        o |= (uint32_t)__shfl_xor((int)o, d);
    }
    const int tid = sel_tid();
    const int w = tid >> 6;
    if ((tid & 63) == 0) {
        sh.red_and[w] = a;
        sh.red_or[w] = o;
    }
    __syncthreads();
    a = 0xffffffffu;
    o = 0;
#pragma unroll
    for (int j = 0; j < NT / 64; ++j) {
        a &= sh.red_and[j];
        o |= sh.red_or[j];
    }
    __syncthreads();
    const uint32_t diff = a ^ o;
    if (diff == 0) return a;
    const int hb = 31 - __clz(diff);
    uint32_t prefix = a & ~((2u << hb) - 1u);
    for (int b = hb; b >= 0; --b) {
        const uint32_t hmask = ~((2u << b) - 1u);
        uint32_t c = 0;
#pragma unroll
        for (int j = 0; j < PER; ++j)
            c += wave_count(sel[j] && ((val[j] ^ prefix) & hmask) == 0 && !((val[j] >> b) & 1u));
        const uint32_t cnt = block_sum(c, sh, buf);
        if (cnt < rank) {
            rank -= cnt;
            prefix |= 1u << b;
        }
    }
    return prefix;
}

// Threshold over the compacted keys when too many passed to place by counting.
template <int NT>
__device__ uint64_t block_threshold(int nf, uint32_t rank, TopkShared<NT> &sh)
{
    constexpr int PER = TopkShared<NT>::PER;
    int buf = 0;
    uint32_t hi[PER], lo[PER];
    bool sel[PER], eq[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int e = j * NT + sel_tid();
        const uint64_t key = e < nf ? sh.filt[e] : SENT;
        hi[j] = (uint32_t)(key >> 32);
        lo[j] = (uint32_t)key;
        sel[j] = key != SENT;
    }
    const uint32_t thi = block_radix(hi, sel, rank, sh, buf);
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        eq[j] = sel[j] && hi[j] == thi;
        c += wave_count(eq[j]);
    }
    const uint32_t neq = block_sum(c, sh, buf);
    const uint32_t tlo = neq > rank ? block_radix(lo, eq, rank, sh, buf) : 0xffffffffu;
    return ((uint64_t)thi << 32) | tlo;
}

// Select the k smallest keys of the workgroup (element e = j*NT + thread;
// the nvalid real keys occupy elements 0..nvalid-1, the rest are SENT) into
// sh.best, ascending.  Returns min(k, nvalid).
template <int NT>
__device__ int tile_select(const uint64_t (&key)[TopkShared<NT>::PER], int nvalid, int k,
                           TopkShared<NT> &sh)
{
    constexpr int PER = TopkShared<NT>::PER;
    const int t = sel_tid();
    const int lane = t & 63;
    if (t == 0) sh.nfilt = 0;
    uint64_t T = SENT - 1;  // at most k keys: all of them
    if (nvalid > k) {
        uint64_t m = key[0];
#pragma unroll
        for (int j = 1; j < PER; ++j) m = key[j] < m ? key[j] : m;
        // min(nvalid, NT) >= k + 1 threads hold a real key, so the minimum of
        // rank k - 1 is a real key
        m = block_sort1<NT>(m, sh.mins);
        if (t == k - 1) sh.thr = m;
    }
    __syncthreads();
    if (nvalid > k) T = sh.thr;
    // compact the keys <= T
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const bool p = key[j] <= T && key[j] != SENT;
        const uint64_t mask = __ballot(p);
        if (mask) {
            const int first = __ffsll((unsigned long long)mask) - 1;
            uint32_t base = 0;
            if (lane == first) base = atomicAdd(&sh.nfilt, (uint32_t)__popcll(mask));
            base = (uint32_t)__shfl((int)base, first);
            if (p) {
                const uint32_t below = (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
                sh.filt[base + below] = key[j];
            }
        }
    }
    __syncthreads();
    const int nf = (int)sh.nfilt;
    if (nf > RANK_MAX) {
        // many ties at the threshold's cost: exact threshold over the compacted set
        const uint64_t T2 = block_threshold(nf, (uint32_t)k, sh);
        __syncthreads();
        if (t == 0) sh.nfilt = 0;
        __syncthreads();
        uint64_t mine[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int e = j * NT + t;
            mine[j] = e < nf ? sh.filt[e] : SENT;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PER; ++j)
            if (mine[j] <= T2 && mine[j] != SENT) sh.filt[atomicAdd(&sh.nfilt, 1u)] = mine[j];
        __syncthreads();
    }
    const int n = min((int)sh.nfilt, RANK_MAX);
    // place by counting; ranks >= k are dropped
    for (int e = t; e < n; e += NT) {
        const uint64_t mine = sh.filt[e];
        int r = 0;
        for (int j = 0; j < n; ++j) r += sh.filt[j] < mine;
        if (r < k) sh.best[r] = mine;
    }
    __syncthreads();
    return min(n, k);
}

// This workgroup's tile list for the merge: k sorted keys (SENT past nbest),
// made visible to the merging workgroup.
template <int NT>
__device__ inline void publish_list(const TopkShared<NT> &sh, int nbest, int k, uint64_t *dst)
{
    const int t = sel_tid();
    if (t < k) store_shared(dst + t, t < nbest ? sh.best[t] : SENT);
    wait_stores();
}

// Select again over `ntiles` sorted per-tile lists of k keys at src (every
// list but the last is full; the last holds min(k, N - (ntiles - 1) *
// TOPK_TILE) real keys; written by other workgroups with store_shared) into
// sh.best.  Returns min(k, N).
template <int NT>
__device__ int merge_lists(const uint64_t *src, int ntiles, int N, int k, TopkShared<NT> &sh)
{
    constexpr int PER = TopkShared<NT>::PER;
    const int t = sel_tid();
    const int total = ntiles * k;
    const int total_valid = (ntiles - 1) * k + min(k, N - (ntiles - 1) * TOPK_TILE);
    const int fresh = TOPK_TILE - k;
    int nbest = 0;
    uint64_t key[PER];
    for (int base = 0; base < total; base += fresh) {
        const int nnew = max(0, min(fresh, total_valid - base));
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int e = j * NT + t;
            if (e < nbest)
                key[j] = sh.best[e];
            else if (e < nbest + nnew)
                key[j] = load_shared(src + base + e - nbest);
            else
                key[j] = SENT;
        }
        __syncthreads();
        nbest = tile_select<NT>(key, nbest + nnew, k, sh);
    }
    return nbest;
}

// Keys of tile `tile` of a query's costs c[0..N) (kShared: written by other
// workgroups of the same launch).
template <int NT, bool kShared>
__device__ inline void tile_keys(const float *c, int N, int tile, uint64_t (&key)[TopkShared<NT>::PER],
                                 int &nvalid)
{
    constexpr int PER = TopkShared<NT>::PER;
    const int beg = tile * TOPK_TILE;
    nvalid = max(0, min(TOPK_TILE, N - beg));
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int e = j * NT + sel_tid();
        if (e < nvalid) {
            const float v = kShared ? load_shared(c + beg + e) : c[beg + e];
            key[j] = make_key(v, (uint32_t)(beg + e));
        } else {
            key[j] = SENT;
        }
    }
}

// Write the beam: idx[j] = query-local index, val[j] = its cost bit for bit,
// padded with (-1, +inf) past nbest.
template <int NT, bool kShared>
__device__ inline void write_beam(const TopkShared<NT> &sh, int nbest, int k, const float *c,
                                  int32_t *idx, float *val)
{
    const int t = sel_tid();
    if (t < k) {
        int32_t id = -1;
        float v = __builtin_inff();
        if (t < nbest) {
            id = (int32_t)(uint32_t)sh.best[t];
            v = kShared ? load_shared(c + id) : c[id];
        }
        idx[t] = id;
        val[t] = v;
    }
}

}  // namespace topk
}  // namespace cm
