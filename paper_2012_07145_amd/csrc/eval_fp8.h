// eval_fp8.h -- device code of the FP8 (e4m3) form of the evaluator: the
// cost model of Sec. 5.2 with 8-bit inputs, weights and hidden activations
// on the 32x32x64 fp8 matrix core, float32 accumulation, float32 cost terms
// and a Kahan-compensated float32 stage sum (App. B).
//
// Inputs are e4m3 codes of log1p(x) * s_in (40 bytes per row), so there is no
// log on the device.  Per stage a wave of 32 candidates
//   1. loads 20 code bytes per lane (lanes l and l + 32 hold features 0..19
//      and 20..39 of candidate l % 32) and the float32 cost terms;
//   2. runs the first layer's product sum as one fp8 matrix instruction: the
//      A operand holds e4m3(W_1[:, 24:] W_s * s_w1) in the same (lane half,
//      byte) slots as the features it multiplies;
//   3. adds the hoisted row U[s] * s_h in float32 (one fma with the unscale:
//      the matrix instruction sums with less than float32 precision, relative
//      to its largest term, so the hoisted row stays out of it), takes the
//      ReLU, clamps to 448 (the conversion gives NaN above the e4m3 range
//      instead of saturating) and packs to e4m3; the accumulator register
//      order is the byte order the second layer needs;
//   4. runs the coefficient layer as one fp8 matrix instruction with
//      e4m3(W_2 * s_w2), undoes the scales, adds b_2, applies the ReLU and
//      dots the 8 coefficients with the cost terms;
//   5. adds the stage prediction to the compensated sum.
// A NaN input (a code 0x7F or 0xFF) makes every hidden pre-activation of its
// candidate NaN; one ordered compare per stage keeps it in the cost.
// Stage parts and their combination are those of the bf16 form.
#pragma once

#include "eval_bf16.h"

namespace cm {
namespace fp8eval {

using bf16eval::add_halves;
using bf16eval::buffer_over;
using bf16eval::kahan_add;
using bf16eval::refill_u;
using bf16eval::relu;
using bf16eval::u32x4;
using bf16eval::USTAGE;

typedef int i32x8 __attribute__((ext_vector_type(8)));

struct QueryView8 {
    const uint8_t *x;  // e4m3 codes [S][N][40]
    const float *t;    // cost terms [S][N][8]
    const float *u;    // hoisted rows [S][32], already times s_h
    float *cost;       // [N]
    float *stage;      // per-stage costs [S][N] (only with kStage)
    const int32_t *ridx;  // memoized rows: row numbers [S][N] into x (only with kIndexed)
    uint32_t rows;        // rows in the table x (only with kIndexed)
    int S, N, P;
};
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ inline f32x16 mfma8(i32x8 a, i32x8 b, f32x16 c)
{
    // the scaled form with zero scale operands is the unscaled instruction
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 0, 0, 0);
}

struct Weights8 {
    i32x8 A1, A2;
    float b2v[4];
    float r1, r2;  // s_h / (s_w1 s_in), 1 / (s_w2 s_h)
};

__device__ inline Weights8 load_weights8(const Fp8Pack *__restrict__ pk, int lane)
{
    Weights8 w;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        w.A1[j] = (int)pk->a1[lane][j];
        w.A2[j] = (int)pk->a2[lane][j];
    }
    const int hf = lane >> 5;
#pragma unroll
    for (int r = 0; r < 4; ++r) w.b2v[r] = pk->b2[hf * 4 + r];
    w.r1 = pk->r1;
    w.r2 = pk->r2;
    return w;
}

struct StageIn8 {
    uint4 x0;     // code bytes 0..15 of this lane's 20
    uint32_t x1;  // bytes 16..19
    float4 t;
    bool bad;     // memoized rows: the stage's row number is outside the table
};

__device__ inline void load_stage8(StageIn8 &in, __amdgpu_buffer_rsrc_t xr,
                                   __amdgpu_buffer_rsrc_t tr, uint32_t xsoff, uint32_t tsoff,
                                   uint32_t xo, uint32_t to)
{
    in.x0 = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(xr, xo, xsoff, 0));
    in.x1 = __builtin_amdgcn_raw_buffer_load_b32(xr, xo + 16, xsoff, 0);
    in.t = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(tr, to, tsoff, 0));
}

__device__ __forceinline__ float stage_math8(const StageIn8 &in, const float4 *us, int hf,
                                             const Weights8 &w, float &sum, float &comp)
{
    i32x8 B;
    B[0] = (int)in.x0.x;
    B[1] = (int)in.x0.y;
    B[2] = (int)in.x0.z;
    B[3] = (int)in.x0.w;
    B[4] = (int)in.x1;
    B[5] = 0;
    B[6] = 0;
    B[7] = 0;
    f32x16 acc;
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = 0.f;
    acc = mfma8(w.A1, B, acc);
    const bool invalid = acc[0] != acc[0];  // NaN: an invalid input code

    // hidden activations: unscale and add the hoisted row in one fma, ReLU
    // and the clamp to the e4m3 range in one median, then e4m3 with round to
    // nearest even, packed in accumulator register order
    i32x8 Hb;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const float4 u4 = us[d * 2 + hf];
        const float a0 = __builtin_amdgcn_fmed3f(fmaf(acc[4 * d + 0], w.r1, u4.x), 0.f, 448.f);
        const float a1 = __builtin_amdgcn_fmed3f(fmaf(acc[4 * d + 1], w.r1, u4.y), 0.f, 448.f);
        const float a2 = __builtin_amdgcn_fmed3f(fmaf(acc[4 * d + 2], w.r1, u4.z), 0.f, 448.f);
        const float a3 = __builtin_amdgcn_fmed3f(fmaf(acc[4 * d + 3], w.r1, u4.w), 0.f, 448.f);
        Hb[d] = __builtin_amdgcn_cvt_pk_fp8_f32(
            a2, a3, __builtin_amdgcn_cvt_pk_fp8_f32(a0, a1, 0, false), true);
    }
    Hb[4] = 0;
    Hb[5] = 0;
    Hb[6] = 0;
    Hb[7] = 0;
    f32x16 acc2;
#pragma unroll
    for (int k = 0; k < 16; ++k) acc2[k] = 0.f;
    acc2 = mfma8(w.A2, Hb, acc2);
    // lanes hf=0 hold coefficients 0..3 of their candidate, hf=1 hold 4..7
    float v = relu(fmaf(acc2[0], w.r2, w.b2v[0])) * in.t.x;
    v = fmaf(relu(fmaf(acc2[1], w.r2, w.b2v[1])), in.t.y, v);
    v = fmaf(relu(fmaf(acc2[2], w.r2, w.b2v[2])), in.t.z, v);
    v = fmaf(relu(fmaf(acc2[3], w.r2, w.b2v[3])), in.t.w, v);
    if (invalid || in.bad) v = __builtin_nanf("");
    const float vs = add_halves(v);
    kahan_add(sum, comp, vs);
    return vs;
}

// eval_group of the FP8 form (see eval_bf16.h for the work split).  Q.x
// points at the query's code bytes [S][N][40], or with kIndexed at a table of
// code rows that Q.ridx[s][i] numbers (memoized rows).
template <bool kShared, bool kStage = false, bool kIndexed = false>
__device__ __forceinline__ void eval_group8(const QueryView8 &Q, int group, int wave, int lane,
                                            const Weights8 &w, bf16eval::GroupShared &sh)
{
    const int P = Q.P;
    const int tile = group * (EVAL_WAVES / P) + wave / P;
    const int part = wave % P;
    const int n = lane & 31;
    const int hf = lane >> 5;
    const int i = tile * TILE_ROWS + n;
    const bool valid = i < Q.N;
    const int ic = valid ? i : Q.N - 1;
    const int s0 = tile * TILE_ROWS < Q.N ? (Q.S * part) / P : 0;
    const int s1 = tile * TILE_ROWS < Q.N ? (Q.S * (part + 1)) / P : 0;

    // 32-bit byte offsets: the host keeps a query's codes and terms below
    // MAX_QUERY_BYTES (check_query_bytes)
    const uint32_t xstep = kIndexed ? 0u : (uint32_t)Q.N * FS;
    const uint32_t tstep = (uint32_t)Q.N * C * 4;
    const uint32_t xbytes = kIndexed ? Q.rows * FS : xstep * (uint32_t)Q.S;
    const __amdgpu_buffer_rsrc_t xr = buffer_over(Q.x, xbytes);
    const __amdgpu_buffer_rsrc_t tr = buffer_over(Q.t, tstep * (uint32_t)Q.S);
    uint32_t xsoff = (uint32_t)s0 * xstep;
    uint32_t tsoff = (uint32_t)s0 * tstep;
    uint32_t xo = (uint32_t)ic * FS + hf * 20;  // code bytes 20*hf .. +20
    const uint32_t to = (uint32_t)ic * (C * 4) + hf * 16;
    // memoized rows (as in the bf16 evaluator): row numbers read one stage
    // ahead; a row outside the table reads zeros and is flagged
    int32_t rnext = 0;
    bool bad = false;
    auto point_at = [&](int32_t r) {
        const bool ok = (uint32_t)r < Q.rows;
        xo = (ok ? (uint32_t)r * FS : xbytes) + hf * 20;
        bad = !ok;
    };
    auto row_of = [&](int s) { return Q.ridx[(int64_t)s * Q.N + ic]; };
    const float4 *ug = reinterpret_cast<const float4 *>(Q.u);
    float4 *ur = sh.u[wave];

    float sum = 0.f, comp = 0.f;
    if (s0 < s1) {
        StageIn8 A, B;
        if (kIndexed) {
            point_at(row_of(s0));
            if (s0 + 1 < s1) rnext = row_of(s0 + 1);
        }
        load_stage8(A, xr, tr, xsoff, tsoff, xo, to);
        A.bad = bad;
        for (int s = s0; s < s1; s += 2) {
            if ((s - s0) % USTAGE == 0) refill_u(ur, ug, s, min(USTAGE, s1 - s), lane);
            if (s + 1 < s1) {
                xsoff += xstep;
                tsoff += tstep;
                if (kIndexed) {
                    point_at(rnext);
                    if (s + 2 < s1) rnext = row_of(s + 2);
                }
            }
            load_stage8(B, xr, tr, xsoff, tsoff, xo, to);
            B.bad = bad;
            asm volatile("" ::: "memory");
            const float va = stage_math8(A, ur + ((s - s0) % USTAGE) * (H / 4), hf, w, sum, comp);
            if (kStage && hf == 0 && valid) Q.stage[(int64_t)s * Q.N + i] = va;
            if (s + 1 >= s1) break;

            if ((s + 1 - s0) % USTAGE == 0) refill_u(ur, ug, s + 1, min(USTAGE, s1 - s - 1), lane);
            if (s + 2 < s1) {
                xsoff += xstep;
                tsoff += tstep;
                if (kIndexed) {
                    point_at(rnext);
                    if (s + 3 < s1) rnext = row_of(s + 3);
                }
            }
            load_stage8(A, xr, tr, xsoff, tsoff, xo, to);
            A.bad = bad;
            asm volatile("" ::: "memory");
            const float vb =
                stage_math8(B, ur + ((s + 1 - s0) % USTAGE) * (H / 4), hf, w, sum, comp);
            if (kStage && hf == 0 && valid) Q.stage[(int64_t)(s + 1) * Q.N + i] = vb;
        }
    }

    if (P > 1) {
        if (hf == 0) sh.part[wave][n] = make_float2(sum, comp);
        __syncthreads();
    }
    if (part == 0 && hf == 0 && valid) {
        float S = 0.f, Cc = 0.f;
        for (int p = 0; p < P; ++p) {
            const float2 pc = P > 1 ? sh.part[wave + p][n] : make_float2(sum, comp);
            kahan_add(S, Cc, pc.x);
            kahan_add(S, Cc, -pc.y);
        }
        if (kShared) store_shared(Q.cost + i, S - Cc);
        else Q.cost[i] = S - Cc;
    }
}

}  // namespace fp8eval
}  // namespace cm
