// k_bf16.hip -- the bf16 matrix-core evaluator of the cost model (Sec. 5.2).
//
// Work unit ("task") = one wavefront x (32 candidates of one query) x (one
// chunk of up to CM_STAGE_CHUNK consecutive stages).  Per stage the wave
//   1. loads the 32 candidates' bf16 schedule features (stage-major rows of
//      80 bytes, 16 bytes per lane per load) and their float32 cost terms;
//   2. takes log2(1 + x) in float32 (ln 2 is folded into the weights, so the
//      layer sees log1p(x)) and splits it into high and low bf16 parts;
//   3. runs the first layer as D[hidden][cand] = Wf . X^T on the 32x32x16 bf16
//      matrix core: Wf = W_1[:, 24:] W_s is the schedule embedding folded into
//      the first layer (no activation sits between them), the accumulator
//      starts from the hoisted per-stage vector U[s] (algorithm embedding,
//      biases), and each product is hi*hi + lo*hi + hi*lo;
//   4. applies the ReLU, splits the hidden activations the same way and runs
//      the coefficient layer (8 outputs padded to 32) on the matrix core; the
//      hidden order is permuted in the packed weights so that the first
//      layer's output registers are already the second layer's operands;
//   5. applies the ReLU to the 8 coefficients, dots them with the 8 cost
//      terms (two lanes hold four each and exchange halves) and adds the
//      stage prediction to a Kahan-compensated float32 sum (App. B).
// A chunk's (sum, compensation) pair goes to the workspace; the last wave to
// finish a row tile combines the chunks in ascending order, so the result of
// a candidate depends only on its query, never on the batch or on timing.
#include "cm_internal.h"

namespace cm {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ inline uint32_t pack_bf16x2(float a, float b)
{
    bf16x2 v = {(__bf16)a, (__bf16)b};  // round to nearest even
    return __builtin_bit_cast(uint32_t, v);
}

__device__ inline float bf16lo_to_f32(uint32_t w) { return __uint_as_float(w << 16); }
__device__ inline float bf16hi_to_f32(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

// Two float values -> (high bf16 pair, low bf16 pair) with a ~= hi + lo.
__device__ inline void split2(float a, float b, uint32_t &hi, uint32_t &lo)
{
    hi = pack_bf16x2(a, b);
    lo = pack_bf16x2(a - bf16lo_to_f32(hi), b - bf16hi_to_f32(hi));
}

// 8 raw bf16 features -> high/low bf16 operands of log2(1 + x).
__device__ inline void log_split(uint4 raw, bf16x8 &hi, bf16x8 &lo)
{
    uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
    uint32_t h[4], l[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const float y0 = __builtin_amdgcn_logf(1.0f + bf16lo_to_f32(w[d]));
        const float y1 = __builtin_amdgcn_logf(1.0f + bf16hi_to_f32(w[d]));
        split2(y0, y1, h[d], l[d]);
    }
    hi = __builtin_bit_cast(bf16x8, make_uint4(h[0], h[1], h[2], h[3]));
    lo = __builtin_bit_cast(bf16x8, make_uint4(l[0], l[1], l[2], l[3]));
}

__device__ inline void kahan_add(float &s, float &c, float v)
{
    const float y = v - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

__device__ inline f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ inline int find_task_query(const EvalLaunch &L, int t)
{
    int q = 0;
    for (int j = 1; j < L.nq; ++j)
        if (L.q[j].task0 <= t) q = j;
    return q;
}

__global__ __launch_bounds__(256) void k_eval_bf16(EvalLaunch L, const Bf16Pack *__restrict__ pk,
                                                   const uint16_t *__restrict__ sched,
                                                   const float *__restrict__ terms,
                                                   const float *__restrict__ U,
                                                   float2 *__restrict__ part,
                                                   int32_t *__restrict__ cnt,
                                                   float *__restrict__ cost)
{
    const int lane = threadIdx.x & 63;
    const int task = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (task >= L.ntasks) return;
    const int q = find_task_query(L, task);
    const EvalQ Q = L.q[q];
    const int local = task - Q.task0;
    const int tile = local / Q.nchunk;
    const int chunk = local - tile * Q.nchunk;
    const int n = lane & 31;
    const int hf = lane >> 5;
    const int i = tile * TILE_ROWS + n;
    const bool valid = i < Q.N;
    const int s0 = chunk * SCHUNK;
    const int s1 = min(Q.S, s0 + SCHUNK);

    bf16x8 A1h[3], A1l[3], A2h[2], A2l[2];
#pragma unroll
    for (int st = 0; st < 3; ++st) {
        A1h[st] = __builtin_bit_cast(bf16x8, pk->a1[0][st][lane]);
        A1l[st] = __builtin_bit_cast(bf16x8, pk->a1[1][st][lane]);
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        A2h[t] = __builtin_bit_cast(bf16x8, pk->a2[0][t][lane]);
        A2l[t] = __builtin_bit_cast(bf16x8, pk->a2[1][t][lane]);
    }
    float b2v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) b2v[r] = pk->b2[hf * 4 + r];

    const uint4 zero4 = make_uint4(0, 0, 0, 0);
    float sum = 0.f, comp = 0.f;
    for (int s = s0; s < s1; ++s) {
        const int64_t r = (int64_t)s * Q.N + i;
        const uint4 *xr = reinterpret_cast<const uint4 *>(sched + Q.sched_off + r * FS);
        const uint4 x0 = valid ? xr[hf] : zero4;
        const uint4 x1 = valid ? xr[2 + hf] : zero4;
        const uint4 x2 = (valid && hf == 0) ? xr[4] : zero4;
        float4 tv = make_float4(0.f, 0.f, 0.f, 0.f);
        if (valid) tv = *reinterpret_cast<const float4 *>(terms + Q.terms_off + r * C + hf * 4);

        // accumulator starts from the hoisted per-stage vector, in the
        // matrix core's output order: register g*4+j <-> hidden g*8 + hf*4 + j
        const float4 *up = reinterpret_cast<const float4 *>(U + (int64_t)(Q.stage0 + s) * H);
        f32x16 acc;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const float4 u4 = up[g * 2 + hf];
            acc[g * 4 + 0] = u4.x;
            acc[g * 4 + 1] = u4.y;
            acc[g * 4 + 2] = u4.z;
            acc[g * 4 + 3] = u4.w;
        }
        bf16x8 bh, bl;
        log_split(x0, bh, bl);
        acc = mfma(A1h[0], bh, acc);
        acc = mfma(A1l[0], bh, acc);
        acc = mfma(A1h[0], bl, acc);
        log_split(x1, bh, bl);
        acc = mfma(A1h[1], bh, acc);
        acc = mfma(A1l[1], bh, acc);
        acc = mfma(A1h[1], bl, acc);
        log_split(x2, bh, bl);
        acc = mfma(A1h[2], bh, acc);
        acc = mfma(A1l[2], bh, acc);
        acc = mfma(A1h[2], bl, acc);

        f32x16 acc2;
#pragma unroll
        for (int k = 0; k < 16; ++k) acc2[k] = 0.f;
#pragma unroll
        for (int k = 0; k < 4; ++k) acc2[k] = b2v[k];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            uint32_t hh[4], hl[4];
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const float a = fmaxf(acc[t * 8 + 2 * d], 0.f);
                const float b = fmaxf(acc[t * 8 + 2 * d + 1], 0.f);
                split2(a, b, hh[d], hl[d]);
            }
            const bf16x8 Hh = __builtin_bit_cast(bf16x8, make_uint4(hh[0], hh[1], hh[2], hh[3]));
            const bf16x8 Hl = __builtin_bit_cast(bf16x8, make_uint4(hl[0], hl[1], hl[2], hl[3]));
            acc2 = mfma(A2h[t], Hh, acc2);
            acc2 = mfma(A2l[t], Hh, acc2);
            acc2 = mfma(A2h[t], Hl, acc2);
        }
        // lanes hf=0 hold coefficients 0..3 of their candidate, hf=1 hold 4..7
        float v = fmaxf(acc2[0], 0.f) * tv.x;
        v = fmaf(fmaxf(acc2[1], 0.f), tv.y, v);
        v = fmaf(fmaxf(acc2[2], 0.f), tv.z, v);
        v = fmaf(fmaxf(acc2[3], 0.f), tv.w, v);
        v += __shfl_xor(v, 32);
        kahan_add(sum, comp, v);
    }

    const int64_t cidx = Q.cost_off + i;
    if (Q.nchunk == 1) {
        if (hf == 0 && valid) {
            float S = 0.f, Cc = 0.f;
            kahan_add(S, Cc, sum);
            kahan_add(S, Cc, -comp);
            cost[cidx] = S - Cc;
        }
        return;
    }
    if (hf == 0 && valid) part[Q.part0 + (int64_t)chunk * Q.N + i] = make_float2(sum, comp);
    __threadfence();
    int old = 0;
    if (lane == 0) old = atomicAdd(&cnt[Q.cnt0 + tile], 1);
    old = __shfl(old, 0);
    if (old != Q.nchunk - 1) return;
    __threadfence();
    if (hf == 0 && valid) {
        float S = 0.f, Cc = 0.f;
        for (int ch = 0; ch < Q.nchunk; ++ch) {
            const float2 p = part[Q.part0 + (int64_t)ch * Q.N + i];
            kahan_add(S, Cc, p.x);
            kahan_add(S, Cc, -p.y);
        }
        cost[cidx] = S - Cc;
    }
    if (lane == 0) atomicExch(&cnt[Q.cnt0 + tile], 0);
}

}  // namespace

hipError_t launch_eval_bf16(const EvalLaunch &L, const Model &m, const uint16_t *sched,
                            const float *terms, const float *U, float2 *part, int32_t *cnt,
                            float *cost, hipStream_t st)
{
    if (L.ntasks == 0) return hipSuccess;
    const int blocks = (L.ntasks + 3) / 4;
    hipLaunchKernelGGL(k_eval_bf16, dim3(blocks), dim3(256), 0, st, L, m.d_bf16, sched, terms, U,
                       part, cnt, cost);
    return hipGetLastError();
}

}  // namespace cm
