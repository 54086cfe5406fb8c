// k_fp8.hip -- the FP8 (e4m3) form of the cost model (Sec. 5.2) on the fp8
// matrix cores, and the encoder that turns raw schedule features into its
// e4m3 input codes (the log transform of Sec. 5.2 happens there, once per
// feature value).  The arithmetic lives in eval_fp8.h.
#include <algorithm>

#include "eval_fp8.h"

namespace cm {
namespace {

using namespace fp8eval;

__device__ inline int find_task_query(const EvalLaunch &L, int t)
{
    int q = 0;
    for (int j = 1; j < L.nq; ++j)
        if (L.q[j].task0 <= t) q = j;
    return q;
}

template <bool kStage, bool kIndexed>
__global__ __launch_bounds__(EVAL_WAVES * 64) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_eval_fp8(
    EvalLaunch L, const Fp8Pack *__restrict__ pk, const uint8_t *codes, const float *terms,
    const float *__restrict__ U, float *__restrict__ cost, float *__restrict__ stage,
    const int32_t *__restrict__ ridx, uint32_t rows)
{
    __shared__ bf16eval::GroupShared sh;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int q = find_task_query(L, blockIdx.x);
    const EvalQ &E = L.q[q];
    QueryView8 Q;
    // memoized rows: codes is the row table and sched_off locates the row numbers
    Q.x = kIndexed ? codes : codes + E.sched_off;
    Q.ridx = kIndexed ? ridx + E.sched_off : nullptr;
    Q.rows = rows;
    Q.t = terms + E.terms_off;
    Q.u = U + E.u_off;
    Q.cost = cost + E.cost_off;
    Q.stage = kStage ? stage + E.stage_off : nullptr;
    Q.S = E.S;
    Q.N = E.N;
    Q.P = E.parts;
    const Weights8 w = load_weights8(pk, lane);
    eval_group8<false, kStage, kIndexed>(Q, blockIdx.x - E.task0, wave, lane, w, sh);
}

// e4m3 code of v: NaN -> 0x7F, magnitudes beyond 448 saturate (the
// conversion instruction itself gives NaN there), round to nearest even.
__device__ inline uint32_t e4m3_pair(float a, float b)
{
    const float ca = __builtin_amdgcn_fmed3f(a, -448.f, 448.f);
    const float cb = __builtin_amdgcn_fmed3f(b, -448.f, 448.f);
    uint32_t w = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(ca, cb, 0, false) & 0xffffu;
    if (a != a) w = (w & 0xff00u) | 0x7fu;
    if (b != b) w = (w & 0x00ffu) | 0x7f00u;
    return w;
}

// log1p(x) in float32 within a few ulps, from the hardware base-2 logarithm:
// with u = 1 + x rounded, log(u) * x / (u - 1) cancels the rounding of u to
// first order (Goldberg's method, "What every computer scientist should know
// about floating-point arithmetic", 1991); u == 1 means log1p(x) = x to
// float32 precision, and for huge |u - 1| (whose reciprocal would underflow)
// the rounding of u no longer matters.  -1 gives -inf, below -1 NaN, +inf
// stays +inf.
__device__ inline float log1p_fast(float x)
{
    const float u = 1.f + x;
    const float d = u - 1.f;
    if (d == 0.f) return x;
    const float l = __builtin_amdgcn_logf(u) * 0.6931471805599453f;
    if (!(fabsf(d) < 0x1p100f)) return l;
    return l * (x * __builtin_amdgcn_rcpf(d));
}

__device__ inline uint32_t encode4(float4 x, float s)
{
    const uint32_t lo = e4m3_pair(log1p_fast(x.x) * s, log1p_fast(x.y) * s);
    const uint32_t hi = e4m3_pair(log1p_fast(x.z) * s, log1p_fast(x.w) * s);
    return lo | (hi << 16);
}

// n values, 16 per thread (one 16-byte store of codes); the last thread
// handles the tail one value at a time.
__global__ __launch_bounds__(256) void k_fp8_encode(const float *__restrict__ x, int64_t n,
                                                     float s, uint8_t *__restrict__ codes)
{
    const int64_t n16 = n / 16;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const float4 *x4 = reinterpret_cast<const float4 *>(x);
    uint4 *c4 = reinterpret_cast<uint4 *>(codes);
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n16; g += stride) {
        uint4 o;
        o.x = encode4(x4[g * 4 + 0], s);
        o.y = encode4(x4[g * 4 + 1], s);
        o.z = encode4(x4[g * 4 + 2], s);
        o.w = encode4(x4[g * 4 + 3], s);
        c4[g] = o;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (int64_t i = n16 * 16; i < n; ++i)
            codes[i] = (uint8_t)(e4m3_pair(log1p_fast(x[i]) * s, 0.f) & 0xffu);
}

}  // namespace

hipError_t launch_eval_fp8(const EvalLaunch &L, const Model &m, const uint8_t *codes,
                           const float *terms, const float *U, float *cost, float *stage,
                           hipStream_t st, const int32_t *ridx, uint32_t rows)
{
    if (L.ntasks == 0) return hipSuccess;
    const dim3 g(L.ntasks), b(EVAL_WAVES * 64);
    if (ridx) {
        if (stage)
            hipLaunchKernelGGL((k_eval_fp8<true, true>), g, b, 0, st, L, m.d_fp8, codes, terms, U,
                               cost, stage, ridx, rows);
        else
            hipLaunchKernelGGL((k_eval_fp8<false, true>), g, b, 0, st, L, m.d_fp8, codes, terms, U,
                               cost, stage, ridx, rows);
    } else if (stage) {
        hipLaunchKernelGGL((k_eval_fp8<true, false>), g, b, 0, st, L, m.d_fp8, codes, terms, U,
                           cost, stage, ridx, rows);
    } else {
        hipLaunchKernelGGL((k_eval_fp8<false, false>), g, b, 0, st, L, m.d_fp8, codes, terms, U,
                           cost, stage, ridx, rows);
    }
    return hipGetLastError();
}

// x and codes must be 16-byte aligned (checked by the caller).
hipError_t launch_fp8_encode(const float *x, int64_t n, float in_scale, uint8_t *codes,
                             hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const int64_t groups = std::max<int64_t>(1, n / 16);
    const int64_t blocks = std::min<int64_t>((groups + 255) / 256, 8192);
    hipLaunchKernelGGL(k_fp8_encode, dim3((unsigned)blocks), dim3(256), 0, st, x, n, in_scale,
                       codes);
    return hipGetLastError();
}

}  // namespace cm
