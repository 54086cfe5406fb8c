// cm_sample.hip -- hierarchical sampling (Sec. 3.1, Sec. 4.4): the options of
// every query are grouped into buckets of equal structural hash, and from a
// bucket of B options max(1, ceil(log2 B)) representatives are drawn at
// random without replacement -- the members with the smallest random keys,
// key i being the high 32 bits of output i of SplitMix64 (Steele, Lea and
// Flood 2014) seeded per query, equal keys by lower index.  The
// representatives' indices are written ascending, per query.
//
// On the device: three stable radix sorts (by key, by hash, by query; least
// significant first) put every option at its rank in (query, hash, key,
// index) order; a scan over bucket heads numbers the buckets; each option's
// rank inside its bucket decides whether it is kept; a scan over the kept
// flags compacts them back into index order.  Sorts and scans are rocPRIM's.
#include <algorithm>
#include <cstring>
#include <new>

#include <rocprim/rocprim.hpp>

#include "cm_internal.h"

namespace cm {
namespace {

struct SampleQ {
    int64_t base;   // first global option of the query
    int64_t off;    // hashes, selected indices at off
    uint64_t seed;
    int32_t n;
    int32_t pad;
};

constexpr int ST = 256;  // threads per block of the sampling kernels

__device__ inline uint64_t splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// The query holding global option g: the last one whose base is <= g (an
// empty query never follows the query of g with a base <= g).
__device__ inline int query_of(const SampleQ *__restrict__ q, int nq, int64_t g)
{
    int lo = 0, hi = nq - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (q[mid].base <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ inline uint64_t hash_of(const SampleQ *__restrict__ q, const uint64_t *__restrict__ h,
                                   int qi, int64_t g)
{
    return h[q[qi].off + (g - q[qi].base)];
}

#define GRID_STRIDE(j, n) \
    for (int64_t j = (int64_t)blockIdx.x * ST + threadIdx.x; j < (n); j += (int64_t)gridDim.x * ST)

__global__ __launch_bounds__(ST) void k_s_keys(const SampleQ *__restrict__ q, int nq, int64_t T,
                                               uint32_t *__restrict__ key,
                                               uint32_t *__restrict__ val)
{
    GRID_STRIDE(g, T)
    {
        const int qi = query_of(q, nq, g);
        key[g] = (uint32_t)(splitmix64(q[qi].seed, (uint64_t)(g - q[qi].base)) >> 32);
        val[g] = (uint32_t)g;
    }
}

__global__ __launch_bounds__(ST) void k_s_hashes(const SampleQ *__restrict__ q, int nq, int64_t T,
                                                 const uint64_t *__restrict__ hashes,
                                                 const uint32_t *__restrict__ val,
                                                 uint64_t *__restrict__ hkey)
{
    GRID_STRIDE(j, T)
    {
        const int64_t g = val[j];
        hkey[j] = hash_of(q, hashes, query_of(q, nq, g), g);
    }
}

__global__ __launch_bounds__(ST) void k_s_queries(const SampleQ *__restrict__ q, int nq, int64_t T,
                                                  const uint32_t *__restrict__ val,
                                                  uint32_t *__restrict__ qkey)
{
    GRID_STRIDE(j, T) qkey[j] = (uint32_t)query_of(q, nq, val[j]);
}

// head[j] = 1 where a bucket starts in (query, hash, key, index) order
__global__ __launch_bounds__(ST) void k_s_heads(const SampleQ *__restrict__ q, int64_t T,
                                                const uint64_t *__restrict__ hashes,
                                                const uint32_t *__restrict__ qkey,
                                                const uint32_t *__restrict__ val,
                                                int32_t *__restrict__ head)
{
    GRID_STRIDE(j, T)
    {
        bool h = j == 0;
        if (!h) {
            const int qa = (int)qkey[j], qb = (int)qkey[j - 1];
            h = qa != qb || hash_of(q, hashes, qa, val[j]) != hash_of(q, hashes, qb, val[j - 1]);
        }
        head[j] = h ? 1 : 0;
    }
}

// bucket b (from 0) starts at start[b]; nb = number of buckets
__global__ __launch_bounds__(ST) void k_s_starts(int64_t T, const int32_t *__restrict__ head,
                                                 const int32_t *__restrict__ bid,
                                                 int64_t *__restrict__ start,
                                                 int32_t *__restrict__ nb)
{
    GRID_STRIDE(j, T)
    {
        if (head[j]) start[bid[j] - 1] = j;
        if (j == T - 1) *nb = bid[j];
    }
}

// keep[g] = 1 for the first max(1, ceil(log2 B)) members of every bucket
__global__ __launch_bounds__(ST) void k_s_keep(int64_t T, const int32_t *__restrict__ bid,
                                               const int64_t *__restrict__ start,
                                               const int32_t *__restrict__ nb,
                                               const uint32_t *__restrict__ val,
                                               int32_t *__restrict__ keep)
{
    const int32_t nbk = *nb;
    GRID_STRIDE(j, T)
    {
        const int32_t b = bid[j] - 1;
        const int64_t st = start[b];
        const int64_t B = (b + 1 < nbk ? start[b + 1] : T) - st;
        int r = 0;
        while (((int64_t)1 << r) < B) ++r;
        keep[val[j]] = (j - st) < max(r, 1) ? 1 : 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) keep[T] = 0;
}

__global__ __launch_bounds__(ST) void k_s_compact(const SampleQ *__restrict__ q, int nq, int64_t T,
                                                  const int32_t *__restrict__ keep,
                                                  const int32_t *__restrict__ pos,
                                                  int32_t *__restrict__ out)
{
    GRID_STRIDE(g, T)
    {
        if (!keep[g]) continue;
        const int qi = query_of(q, nq, g);
        out[q[qi].off + (pos[g] - pos[q[qi].base])] = (int32_t)(g - q[qi].base);
    }
}

__global__ __launch_bounds__(ST) void k_s_counts(const SampleQ *__restrict__ q, int nq,
                                                 const int32_t *__restrict__ pos,
                                                 int32_t *__restrict__ count)
{
    for (int i = blockIdx.x * ST + threadIdx.x; i < nq; i += gridDim.x * ST)
        count[i] = pos[q[i].base + q[i].n] - pos[q[i].base];
}

unsigned blocks_for(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + ST - 1) / ST, 8192)); }

}  // namespace
}  // namespace cm

struct cm_sampler {
    int device = 0;
    int32_t max_queries = 0;
    int64_t max_options = 0;
    cm::SampleQ *h_q = nullptr;  // pinned staging of the descriptors
    cm::SampleQ *d_q = nullptr;
    hipEvent_t staged = nullptr;  // the last copy out of h_q has been done
    uint32_t *key[2] = {nullptr, nullptr};
    uint32_t *val[2] = {nullptr, nullptr};
    uint32_t *qkey[2] = {nullptr, nullptr};
    uint64_t *hkey[2] = {nullptr, nullptr};
    int32_t *head = nullptr, *bid = nullptr, *keep = nullptr, *pos = nullptr, *nb = nullptr;
    int64_t *start = nullptr;
    void *temp = nullptr;
    size_t temp_bytes = 0;
};

namespace {

using cm::fail;

void free_sampler(cm_sampler *s)
{
    auto f = [](void *p) {
        if (p) (void)hipFree(p);
    };
    if (s->h_q) (void)hipHostFree(s->h_q);
    f(s->d_q);
    if (s->staged) (void)hipEventDestroy(s->staged);
    for (int i = 0; i < 2; ++i) {
        f(s->key[i]);
        f(s->val[i]);
        f(s->qkey[i]);
        f(s->hkey[i]);
    }
    f(s->head);
    f(s->bid);
    f(s->keep);
    f(s->pos);
    f(s->nb);
    f(s->start);
    f(s->temp);
}

}  // namespace

extern "C" {

cm_status cm_sampler_create(int32_t max_queries, int64_t max_options, cm_sampler **out)
{
    using namespace cm;
    if (!out) return fail(CM_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_queries < 1 || max_options < 1 || max_options > INT32_MAX - 1)
        return fail(CM_EINVAL, "max_queries must be >= 1 and max_options in [1, 2^31 - 2]");
    cm_sampler *s = new (std::nothrow) cm_sampler;
    if (!s) return fail(CM_ENOMEM, "host allocation failed");
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return fail(CM_EDEVICE, "no HIP device");
    }
    s->max_queries = max_queries;
    s->max_options = max_options;
    const size_t T = (size_t)max_options + 1;
    bool ok = hipHostMalloc((void **)&s->h_q, sizeof(SampleQ) * max_queries, 0) == hipSuccess &&
              hipMalloc((void **)&s->d_q, sizeof(SampleQ) * max_queries) == hipSuccess &&
              hipEventCreateWithFlags(&s->staged, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; ok && i < 2; ++i)
        ok = hipMalloc((void **)&s->key[i], T * 4) == hipSuccess &&
             hipMalloc((void **)&s->val[i], T * 4) == hipSuccess &&
             hipMalloc((void **)&s->qkey[i], T * 4) == hipSuccess &&
             hipMalloc((void **)&s->hkey[i], T * 8) == hipSuccess;
    ok = ok && hipMalloc((void **)&s->head, T * 4) == hipSuccess &&
         hipMalloc((void **)&s->bid, T * 4) == hipSuccess &&
         hipMalloc((void **)&s->keep, T * 4) == hipSuccess &&
         hipMalloc((void **)&s->pos, T * 4) == hipSuccess &&
         hipMalloc((void **)&s->nb, 4) == hipSuccess &&
         hipMalloc((void **)&s->start, T * 8) == hipSuccess;
    if (ok) {  // the largest scratch any of the sorts and scans asks for
        size_t b1 = 0, b2 = 0, b3 = 0, b4 = 0, b5 = 0;
        ok = rocprim::radix_sort_pairs(nullptr, b1, s->key[0], s->key[1], s->val[0], s->val[1],
                                       T, 0, 32) == hipSuccess &&
             rocprim::radix_sort_pairs(nullptr, b2, s->hkey[0], s->hkey[1], s->val[0], s->val[1],
                                       T, 0, 64) == hipSuccess &&
             rocprim::radix_sort_pairs(nullptr, b3, s->qkey[0], s->qkey[1], s->val[0], s->val[1],
                                       T, 0, 32) == hipSuccess &&
             rocprim::inclusive_scan(nullptr, b4, s->head, s->bid, T,
                                     rocprim::plus<int32_t>()) == hipSuccess &&
             rocprim::exclusive_scan(nullptr, b5, s->keep, s->pos, 0, T,
                                     rocprim::plus<int32_t>()) == hipSuccess;
        s->temp_bytes = std::max({b1, b2, b3, b4, b5, (size_t)256});
        ok = ok && hipMalloc(&s->temp, s->temp_bytes) == hipSuccess;
    }
    if (!ok) {
        (void)hipGetLastError();
        free_sampler(s);
        delete s;
        return fail(CM_ENOMEM, "sampler allocation failed");
    }
    *out = s;
    return CM_OK;
}

cm_status cm_sampler_destroy(cm_sampler *s)
{
    if (!s) return fail(CM_EINVAL, "sampler is NULL");
    (void)hipDeviceSynchronize();
    free_sampler(s);
    delete s;
    return CM_OK;
}

cm_status cm_sample_buckets(cm_sampler *sp, const cm_batch *b, const uint64_t *hashes,
                            const uint64_t *seeds, int32_t *sel_idx, int32_t *sel_count,
                            cm_stream stream)
{
    using namespace cm;
    if (!sp || !b) return fail(CM_EINVAL, "sampler or batch is NULL");
    if (b->n_queries < 0) return fail(CM_EINVAL, "n_queries < 0");
    if (b->n_queries == 0) return CM_OK;
    if (!b->queries || !seeds) return fail(CM_EINVAL, "queries or seeds is NULL");
    if (b->n_queries > sp->max_queries)
        return fail(CM_E2BIG, "batch has %d queries, sampler holds %d", b->n_queries,
                    sp->max_queries);
    if (!sel_count) return fail(CM_EINVAL, "sel_count is NULL");
    int64_t T = 0;
    for (int32_t q = 0; q < b->n_queries; ++q) {
        const cm_query &Q = b->queries[q];
        if (Q.n_cands < 0) return fail(CM_EINVAL, "query %d: n_cands %d < 0", q, Q.n_cands);
        if (Q.cost_off < 0) return fail(CM_EINVAL, "query %d: negative cost_off", q);
        T += Q.n_cands;
    }
    if (T > sp->max_options)
        return fail(CM_E2BIG, "batch has %lld options, sampler holds %lld", (long long)T,
                    (long long)sp->max_options);
    if (T > 0 && (!hashes || !sel_idx)) return fail(CM_EINVAL, "hashes or sel_idx is NULL");
    int dev = -1;
    CM_HIP(hipGetDevice(&dev));
    if (dev != sp->device)
        return fail(CM_EINVAL, "sampler lives on device %d but device %d is current", sp->device,
                    dev);

    hipStream_t s = (hipStream_t)stream;
    const int nq = b->n_queries;
    CM_HIP(hipEventSynchronize(sp->staged));  // the previous call's copy has left h_q
    int64_t base = 0;
    for (int q = 0; q < nq; ++q) {
        const cm_query &Q = b->queries[q];
        sp->h_q[q] = SampleQ{base, Q.cost_off, seeds[q], Q.n_cands, 0};
        base += Q.n_cands;
    }
    CM_HIP(hipMemcpyAsync(sp->d_q, sp->h_q, sizeof(SampleQ) * nq, hipMemcpyHostToDevice, s));
    CM_HIP(hipEventRecord(sp->staged, s));

    const unsigned gT = blocks_for(T);
    if (T > 0) {
        int qbits = 1;
        while (qbits < 32 && ((int64_t)1 << qbits) < nq) ++qbits;
        size_t tb = sp->temp_bytes;
        hipLaunchKernelGGL(k_s_keys, dim3(gT), dim3(ST), 0, s, sp->d_q, nq, T, sp->key[0],
                           sp->val[0]);
        CM_HIP(hipGetLastError());
        // (key, index) order: the indices start ascending and the sort is stable
        CM_HIP(rocprim::radix_sort_pairs(sp->temp, tb, sp->key[0], sp->key[1], sp->val[0],
                                         sp->val[1], (size_t)T, 0, 32, s));
        hipLaunchKernelGGL(k_s_hashes, dim3(gT), dim3(ST), 0, s, sp->d_q, nq, T, hashes,
                           sp->val[1], sp->hkey[0]);
        CM_HIP(hipGetLastError());
        tb = sp->temp_bytes;
        CM_HIP(rocprim::radix_sort_pairs(sp->temp, tb, sp->hkey[0], sp->hkey[1], sp->val[1],
                                         sp->val[0], (size_t)T, 0, 64, s));
        hipLaunchKernelGGL(k_s_queries, dim3(gT), dim3(ST), 0, s, sp->d_q, nq, T, sp->val[0],
                           sp->qkey[0]);
        CM_HIP(hipGetLastError());
        tb = sp->temp_bytes;
        CM_HIP(rocprim::radix_sort_pairs(sp->temp, tb, sp->qkey[0], sp->qkey[1], sp->val[0],
                                         sp->val[1], (size_t)T, 0, (unsigned)qbits, s));
        // now in (query, hash, key, index) order: buckets are runs
        hipLaunchKernelGGL(k_s_heads, dim3(gT), dim3(ST), 0, s, sp->d_q, T, hashes,
                           sp->qkey[1], sp->val[1], sp->head);
        CM_HIP(hipGetLastError());
        tb = sp->temp_bytes;
        CM_HIP(rocprim::inclusive_scan(sp->temp, tb, sp->head, sp->bid, (size_t)T,
                                       rocprim::plus<int32_t>(), s));
        hipLaunchKernelGGL(k_s_starts, dim3(gT), dim3(ST), 0, s, T, sp->head, sp->bid,
                           sp->start, sp->nb);
        CM_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_s_keep, dim3(gT), dim3(ST), 0, s, T, sp->bid, sp->start, sp->nb,
                           sp->val[1], sp->keep);
        CM_HIP(hipGetLastError());
        tb = sp->temp_bytes;
        CM_HIP(rocprim::exclusive_scan(sp->temp, tb, sp->keep, sp->pos, 0, (size_t)T + 1,
                                       rocprim::plus<int32_t>(), s));
        hipLaunchKernelGGL(k_s_compact, dim3(gT), dim3(ST), 0, s, sp->d_q, nq, T, sp->keep,
                           sp->pos, sel_idx);
        CM_HIP(hipGetLastError());
    } else {
        // no options: every count is 0 (pos[0] = 0 by the fill below)
        hipLaunchKernelGGL(k_s_keep, dim3(1), dim3(ST), 0, s, (int64_t)0, sp->bid, sp->start,
                           sp->nb, sp->val[1], sp->keep);
        CM_HIP(hipGetLastError());
        size_t tb = sp->temp_bytes;
        CM_HIP(rocprim::exclusive_scan(sp->temp, tb, sp->keep, sp->pos, 0, (size_t)1,
                                       rocprim::plus<int32_t>(), s));
    }
    hipLaunchKernelGGL(k_s_counts, dim3(blocks_for(nq)), dim3(ST), 0, s, sp->d_q, nq, sp->pos,
                       sel_count);
    CM_HIP(hipGetLastError());
    return CM_OK;
}

}  // extern "C"
