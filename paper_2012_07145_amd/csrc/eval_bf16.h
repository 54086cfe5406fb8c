// eval_bf16.h -- device code of the bf16 matrix-core evaluator of the cost
// model (Sec. 5.2), shared by the per-call kernel and the persistent step
// kernel so that both give bit-identical results.
//
// Work unit = one wavefront x (32 candidates of one query) x (one part of the
// query's stages; stage_parts() splits them into 1, 2, 4 or 8 contiguous
// parts by stage count alone).  A group of 8 waves holds every part of its
// row tiles.  The matrix work runs on the 16x16x32 bf16 matrix core, whose
// operands give lane l the row or column l mod 16 and the k-slots
// 8 (l / 16) .. +7, and whose output gives lane l column l mod 16, rows
// 4 (l / 16) .. +3.  The wave's 32 candidates are two halves of 16 (columns).
// Per stage the wave
//   1. loads the 32 candidates' bf16 schedule features (stage-major rows of
//      80 bytes) and their float32 cost terms, one stage ahead of the
//      arithmetic: the features as three whole-line copies from memory into
//      the wave's LDS block (read into registers when the stage starts:
//      lane l takes features 8g .. 8g+7 and 32+2g, 33+2g, g = l / 16, of
//      candidates l mod 16 and 16 + l mod 16), the terms into registers
//      (memoized rows, which are gathered by number, are loaded straight into
//      registers);
//   2. takes log2(1 + x) in float32 (ln 2 is folded into the weights, so the
//      layer sees log1p(x)) and splits it into high and low bf16 parts: by
//      lookup in an LDS table of both parts per feature code, or, for a
//      stage whose wave holds a code outside the table, by computing it;
//   3. runs the first layer as D[hidden][cand] = Wf . X^T in four 16x16 tiles
//      (two hidden halves x two candidate halves): Wf = W_1[:, 24:] W_s is the
//      schedule embedding folded into the first layer (no activation sits
//      between them), the accumulators start from the hoisted per-stage
//      vector U[s] (algorithm embedding, biases), and each product is
//      hi*hi + lo*hi + hi*lo;
//   4. applies the ReLU, splits the hidden activations the same way and runs
//      the coefficient layer per candidate half as one 16-row product: rows
//      0..7 take the 8 coefficients against the high weights, rows 8..15
//      against the low weights, so both weight parts share one instruction;
//      the two hidden tiles of a candidate half are already the layer's
//      32-slot operand (the packed weights follow their order);
//   5. adds the two weight parts of each coefficient across lane halves,
//      applies the ReLU, dots the 8 coefficients with the 8 cost terms (two
//      lanes hold four each and exchange halves) and adds the stage
//      prediction to a Kahan-compensated float32 sum (App. B).
// Each part's (sum, compensation) pair goes through LDS and the first wave of
// the tile combines the parts in ascending order, so the result of a
// candidate depends only on its query, never on the batch, the launch shape
// or timing, and no device-wide synchronisation is needed.
#pragma once

#include "cm_internal.h"

namespace cm {
namespace bf16eval {


constexpr int USTAGE = 16;  // hoisted rows staged in LDS per refill

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline uint32_t pack_bf16x2(float a, float b)
{
    bf16x2 v = {(__bf16)a, (__bf16)b};  // round to nearest even
    return __builtin_bit_cast(uint32_t, v);
}

// A packed pair of bf16 constants kept in a register.  The dot instruction
// below must not see them as inline constants: an inline constant in a
// packed-bf16 operand does not select the same halves as the compiler
// assumes, so the value is hidden from constant folding.
__device__ inline bf16x2 pair_reg(uint32_t bits)
{
    uint32_t v;
    asm volatile("s_mov_b32 %0, %1" : "=s"(v) : "i"(bits));
    return __builtin_bit_cast(bf16x2, v);
}

// c + (one bf16 of w) * (the matching bf16 of m): the product of two bf16
// values is exact in float32 and the sum is rounded once.
__device__ inline float dot(uint32_t w, bf16x2 m, float c)
{
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, w), m, c, false);
}

struct Pairs {
    bf16x2 one_lo, one_hi, neg_lo, neg_hi;  // (1,0) (0,1) (-1,0) (0,-1)
};

__device__ inline Pairs make_pairs()
{
    return Pairs{pair_reg(0x00003f80u), pair_reg(0x3f800000u), pair_reg(0x0000bf80u),
                 pair_reg(0xbf800000u)};
}

// Two float values -> (high bf16 pair, low bf16 pair) with a ~= hi + lo:
// hi rounds to nearest, lo = a - hi is exact in float32 before its rounding.
__device__ inline void split2(float a, float b, uint32_t &hi, uint32_t &lo, const Pairs &k)
{
    hi = pack_bf16x2(a, b);
    lo = pack_bf16x2(dot(hi, k.neg_lo, a), dot(hi, k.neg_hi, b));
}

// 8 raw bf16 features -> high/low bf16 operands of log2(1 + x).
__device__ inline void log_split(uint4 raw, bf16x8 &hi, bf16x8 &lo, const Pairs &k)
{
    uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
    uint32_t h[4], l[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const float y0 = __builtin_amdgcn_logf(dot(w[d], k.one_lo, 1.0f));
        const float y1 = __builtin_amdgcn_logf(dot(w[d], k.one_hi, 1.0f));
        split2(y0, y1, h[d], l[d], k);
    }
    hi = __builtin_bit_cast(bf16x8, make_uint4(h[0], h[1], h[2], h[3]));
    lo = __builtin_bit_cast(bf16x8, make_uint4(l[0], l[1], l[2], l[3]));
}

// The last-block operand of a word of two raw bf16 features a, b: slots
// (hi a, hi b, lo a, lo b, hi a, hi b, lo a, lo b).  Its packed weights are
// (Wh a, Wh b, Wh a, Wh b, Wl a, Wl b, 0, 0): one product takes
// hi*hi + lo*hi + hi*lo of both features.
__device__ inline bf16x8 last_operand(uint32_t h, uint32_t l)
{
    return __builtin_bit_cast(bf16x8, make_uint4(h, l, h, l));
}

__device__ inline bf16x8 log_last(uint32_t raw, const Pairs &k)
{
    const float y0 = __builtin_amdgcn_logf(dot(raw, k.one_lo, 1.0f));
    const float y1 = __builtin_amdgcn_logf(dot(raw, k.one_hi, 1.0f));
    uint32_t h, l;
    split2(y0, y1, h, l, k);
    return last_operand(h, l);
}

// ---- the log transform by table lookup ----
// A bf16 feature has one of 2^16 codes, so the (high, low) bf16 parts of its
// log2(1 + x) can be looked up instead of computed.  The table holds the codes
// LOG_BASE .. LOG_BASE + LOG_N - 1 and is filled with log_entry, i.e. with
// exactly the instructions of log_split, so a lookup gives the same bits.
// A saturating subtraction maps every smaller non-negative code (1 + x == 1
// in float32, value 0) to entry 0, which is 0.  A stage whose wave holds any
// code above the table (features of 2^40 or more, infinities, NaNs, negative
// values) takes log_split instead.

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// Table entry of one code: (high bf16 | low bf16 << 16).
__device__ inline uint32_t log_entry(uint32_t code, const Pairs &k)
{
    const float y = __builtin_amdgcn_logf(dot(code, k.one_lo, 1.0f));
    uint32_t h, l;
    split2(y, 0.f, h, l, k);
    return (h & 0xffffu) | (l << 16);
}

// The two table indices of a word of two codes (saturated at 0 below the
// table; an index of LOG_N or more is outside it).
__device__ inline uint32_t tab_index(uint32_t w)
{
    const u16x2 b = {(unsigned short)LOG_BASE, (unsigned short)LOG_BASE};
    return __builtin_bit_cast(uint32_t,
                              __builtin_elementwise_sub_sat(__builtin_bit_cast(u16x2, w), b));
}
static_assert(LOG_N == 8192, "in-table test: bits 13..15 of each index clear");
constexpr uint32_t TAB_OUT = 0xe000e000u;

// High and low operand pairs of the two codes behind index word ix.
__device__ inline void tab_pair(const uint32_t *tab, uint32_t ix, uint32_t &h, uint32_t &l)
{
    const uint32_t e0 = tab[ix & 0xffffu], e1 = tab[ix >> 16];
    h = __builtin_amdgcn_perm(e1, e0, 0x05040100u);
    l = __builtin_amdgcn_perm(e1, e0, 0x07060302u);
}

__device__ inline void tab_split(const uint32_t *tab, uint32_t i0, uint32_t i1, uint32_t i2,
                                 uint32_t i3, bf16x8 &hi, bf16x8 &lo)
{
    uint32_t h[4], l[4];
    tab_pair(tab, i0, h[0], l[0]);
    tab_pair(tab, i1, h[1], l[1]);
    tab_pair(tab, i2, h[2], l[2]);
    tab_pair(tab, i3, h[3], l[3]);
    hi = __builtin_bit_cast(bf16x8, make_uint4(h[0], h[1], h[2], h[3]));
    lo = __builtin_bit_cast(bf16x8, make_uint4(l[0], l[1], l[2], l[3]));
}

__device__ inline bf16x8 tab_last(const uint32_t *tab, uint32_t ix)
{
    uint32_t h, l;
    tab_pair(tab, ix, h, l);
    return last_operand(h, l);
}

// Copy the table into LDS (every thread of the workgroup; the caller
// synchronises before the first lookup).
__device__ inline void load_table(uint32_t *tab, const Bf16Pack *__restrict__ pk)
{
    const uint4 *src = reinterpret_cast<const uint4 *>(pk->logtab);
    uint4 *dst = reinterpret_cast<uint4 *>(tab);
    for (int i = threadIdx.x; i < LOG_N / 4; i += blockDim.x) dst[i] = src[i];
}

// max(x, 0) on the bit pattern (negative floats are negative integers): one
// instruction.  It maps a NaN with the sign bit set to 0; stage_math restores
// NaN propagation by testing one hidden pre-activation per stage, since an
// invalid input makes every hidden unit of its candidate NaN (each sums every
// feature times a weight, and 0 * NaN is NaN).
__device__ inline float relu(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

__device__ inline void kahan_add(float &s, float &c, float v)
{
    const float y = v - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

__device__ inline f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Sum of a value held by lane l and lane l ^ 32, identical in both lanes.
__device__ inline float add_halves(float v)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v),
                                                    false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Sum of a value held by lane l and lane l ^ 16, identical in both lanes.
__device__ inline float add_pairs16(float v)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v),
                                                    false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// One stage's operands for one lane (g = lane / 16): x0, x1 = features
// 8g .. 8g+7 of candidates lane % 16 and 16 + lane % 16; x2 = features 32+2g
// and 33+2g of the same two candidates; t = cost terms 4q .. 4q+3
// (q = (lane / 16) % 2) of the lane's own candidate 16 (lane / 32) + lane % 16.
struct StageIn {
    uint4 x0, x1;
    uint2 x2;
    float4 t;
    bool bad;  // memoized rows: the row number of the lane's own candidate is outside the table
};

// This lane's part of a stage's hoisted row (the first layer's accumulator
// seed): hidden units 4g .. 4g+3 and 16+4g .. 16+4g+3, from the wave's LDS
// slice.
__device__ inline void read_u(float4 (&u)[2], const float4 *us, int g)
{
    u[0] = us[g];
    u[1] = us[4 + g];
}

// Buffer descriptor over n bytes at p (raw, untyped dword access; loads at
// or past n bytes return 0).
__device__ inline __amdgpu_buffer_rsrc_t buffer_over(const void *p, uint32_t n)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)n,
                                             0x00020000);
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// One stage's loads from memoized rows: xsoff, tsoff = byte offsets of the
// stage's rows (uniform); xo0, xo1 = byte offsets of the two candidates' rows,
// to = of this lane's terms inside the stage; g = lane / 16.
__device__ inline void load_stage(StageIn &in, __amdgpu_buffer_rsrc_t xr, __amdgpu_buffer_rsrc_t tr,
                                  uint32_t xsoff, uint32_t tsoff, uint32_t xo0, uint32_t xo1,
                                  int g, uint32_t to)
{
    in.x0 = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(xr, xo0 + 16 * g, xsoff, 0));
    in.x1 = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(xr, xo1 + 16 * g, xsoff, 0));
    in.x2.x = __builtin_amdgcn_raw_buffer_load_b32(xr, xo0 + 64 + 4 * g, xsoff, 0);
    in.x2.y = __builtin_amdgcn_raw_buffer_load_b32(xr, xo1 + 64 + 4 * g, xsoff, 0);
    in.t = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(tr, to, tsoff, 0));
}

// Packed weights held by a lane for the whole wave: per hidden half hh, the
// first layer's high and low weights of features 0..31 and its last-block
// operand; the coefficient layer's [high; low] and [high; 0] operands; the
// coefficient biases 4q .. 4q+3.
struct Weights {
    bf16x8 A1h[2], A1l[2], A1x[2], A2s, A2h;
    float b2v[4];
};

// Refill this wave's LDS slice with the hoisted rows of stages s .. s+n-1.
// Only this wave reads its slice and its LDS operations complete in order.
__device__ inline void refill_u(float4 *ur, const float4 *ug, int s, int n, int lane)
{
    const int nv = n * (H / 4);
    for (int v = lane; v < nv; v += 64) ur[v] = ug[(int64_t)s * (H / 4) + v];
    __builtin_amdgcn_wave_barrier();
}

// One candidate half's coefficient layer: t0, t1 = its first-layer tiles
// (hidden 4g .. 4g+3 and 16+4g .. 16+4g+3 of the lane's column), ReLU, split
// into high and low bf16 parts, then rows 0..7 = W_2,hi (h_hi + h_lo) and
// rows 8..15 = W_2,lo h_hi.
__device__ __forceinline__ f32x4 coef_layer(const f32x4 &t0, const f32x4 &t1, const Weights &w,
                                            const Pairs &kp)
{
    uint32_t hh[4], hl[4];
    split2(relu(t0[0]), relu(t0[1]), hh[0], hl[0], kp);
    split2(relu(t0[2]), relu(t0[3]), hh[1], hl[1], kp);
    split2(relu(t1[0]), relu(t1[1]), hh[2], hl[2], kp);
    split2(relu(t1[2]), relu(t1[3]), hh[3], hl[3], kp);
    const bf16x8 Hh = __builtin_bit_cast(bf16x8, make_uint4(hh[0], hh[1], hh[2], hh[3]));
    const bf16x8 Hl = __builtin_bit_cast(bf16x8, make_uint4(hl[0], hl[1], hl[2], hl[3]));
    const f32x4 z = {0.f, 0.f, 0.f, 0.f};
    return mfma(w.A2h, Hl, mfma(w.A2s, Hh, z));
}

// One stage of 32 candidates: both dense layers on the matrix cores, the
// coefficient dot product with the cost terms, and the compensated sum.
// g = lane / 16, upper = lane >= 32.  Returns the stage's cost (in both lanes
// of the lane's own candidate).
__device__ __forceinline__ float stage_math(const StageIn &in, const float4 (&u)[2], bool upper,
                                            const Weights &w, const Pairs &kp,
                                            const uint32_t *tab, float &sum, float &comp)
{
    // first layer: tile t<hh><c> = hidden 16hh + 4g .. +3 of candidate
    // 16c + lane % 16, seeded with U[s]
    const f32x4 u0 = {u[0].x, u[0].y, u[0].z, u[0].w};
    const f32x4 u1 = {u[1].x, u[1].y, u[1].z, u[1].w};
    f32x4 t00 = u0, t10 = u1, t01 = u0, t11 = u1;
    // table indices of the stage's 20 codes, and whether every code of the
    // wave is in the table (one uniform branch per stage)
    const uint32_t ix[10] = {tab_index(in.x0.x), tab_index(in.x0.y), tab_index(in.x0.z),
                             tab_index(in.x0.w), tab_index(in.x1.x), tab_index(in.x1.y),
                             tab_index(in.x1.z), tab_index(in.x1.w), tab_index(in.x2.x),
                             tab_index(in.x2.y)};
    const uint32_t all = ix[0] | ix[1] | ix[2] | ix[3] | ix[4] | ix[5] | ix[6] | ix[7] | ix[8] |
                         ix[9];
    const bool fast = __builtin_amdgcn_ballot_w64((all & TAB_OUT) != 0u) == 0;
    bf16x8 bh, bl, bx;
    // candidates 0..15 (both hidden halves share the operands)
    if (fast) {
        tab_split(tab, ix[0], ix[1], ix[2], ix[3], bh, bl);
        bx = tab_last(tab, ix[8]);
    } else {
        log_split(in.x0, bh, bl, kp);
        bx = log_last(in.x2.x, kp);
    }
    t00 = mfma(w.A1h[0], bh, t00);
    t10 = mfma(w.A1h[1], bh, t10);
    t00 = mfma(w.A1l[0], bh, t00);
    t10 = mfma(w.A1l[1], bh, t10);
    t00 = mfma(w.A1h[0], bl, t00);
    t10 = mfma(w.A1h[1], bl, t10);
    t00 = mfma(w.A1x[0], bx, t00);
    t10 = mfma(w.A1x[1], bx, t10);
    // candidates 16..31
    if (fast) {
        tab_split(tab, ix[4], ix[5], ix[6], ix[7], bh, bl);
        bx = tab_last(tab, ix[9]);
    } else {
        log_split(in.x1, bh, bl, kp);
        bx = log_last(in.x2.y, kp);
    }
    t01 = mfma(w.A1h[0], bh, t01);
    t11 = mfma(w.A1h[1], bh, t11);
    t01 = mfma(w.A1l[0], bh, t01);
    t11 = mfma(w.A1l[1], bh, t11);
    t01 = mfma(w.A1h[0], bl, t01);
    t11 = mfma(w.A1h[1], bl, t11);
    t01 = mfma(w.A1x[0], bx, t01);
    t11 = mfma(w.A1x[1], bx, t11);

    // NaN: an input outside log1p's domain (the lane's own candidate is in
    // the first tile of its half)
    const float pre = upper ? t01[0] : t00[0];
    const bool invalid = pre != pre;

    const f32x4 d0 = coef_layer(t00, t10, w, kp);
    const f32x4 d1 = coef_layer(t01, t11, w, kp);
    // rows 4g .. 4g+3 of d_c: lanes 0..31 hold the high-weight parts of
    // coefficients, lanes 32..63 the low-weight parts of the same ones.  The
    // swap gathers, in lanes 0..31, candidate half 0 and in lanes 32..63 half
    // 1, with the high parts in its first result and the low parts in its
    // second: lane l then holds coefficients 4q .. 4q+3 of its own candidate.
    float cf[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(d0[j]),
                                                        __float_as_uint(d1[j]), false, false);
        cf[j] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    float v = relu(cf[0] + w.b2v[0]) * in.t.x;
    v = fmaf(relu(cf[1] + w.b2v[1]), in.t.y, v);
    v = fmaf(relu(cf[2] + w.b2v[2]), in.t.z, v);
    v = fmaf(relu(cf[3] + w.b2v[3]), in.t.w, v);
    if (invalid || in.bad) v = __builtin_nanf("");
    const float vs = add_pairs16(v);
    kahan_add(sum, comp, vs);
    return vs;
}

// Load this lane's packed operands of both layers (held for the whole wave).
__device__ inline Weights load_weights(const Bf16Pack *__restrict__ pk, int lane)
{
    Weights w;
    const int q = (lane >> 4) & 1;
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
        w.A1h[hh] = __builtin_bit_cast(bf16x8, pk->a1[hh][0][lane]);
        w.A1l[hh] = __builtin_bit_cast(bf16x8, pk->a1[hh][1][lane]);
        w.A1x[hh] = __builtin_bit_cast(bf16x8, pk->a1[hh][2][lane]);
    }
    w.A2s = __builtin_bit_cast(bf16x8, pk->a2[0][lane]);
    w.A2h = __builtin_bit_cast(bf16x8, pk->a2[1][lane]);
#pragma unroll
    for (int r = 0; r < 4; ++r) w.b2v[r] = pk->b2[q * 4 + r];
    return w;
}

// One query as the evaluator reads it.
struct QueryView {
    const uint16_t *x;  // schedule features [S][N][40], bf16
    const float *t;     // cost terms [S][N][8]
    const float *u;     // hoisted rows [S][32]
    float *cost;        // [N]
    float *stage;       // per-stage costs [S][N] (only with kStage)
    const int32_t *ridx;  // memoized rows: row numbers [S][N] into x (only with kIndexed)
    uint32_t rows;        // rows in the table x (only with kIndexed)
    int S, N, P;
};

// LDS of one group of EVAL_WAVES waves.
struct GroupShared {
    float2 part[EVAL_WAVES][TILE_ROWS];
    float4 u[EVAL_WAVES][USTAGE * H / 4];
    // one stage of each wave's feature rows (32 rows x 80 bytes), copied
    // from memory straight into LDS
    uint4 xs[EVAL_WAVES][TILE_ROWS * FS * 2 / 16];
};

typedef __attribute__((address_space(3))) void lds_void;
// Views of a copy block in other element types (may_alias: no type-based
// alias analysis between them and the block's own type).
typedef uint32_t __attribute__((may_alias)) lds_u1;

// The 2,560 contiguous bytes of a wave's 32 feature rows of one stage into
// its LDS block: three 16-byte-per-lane copies that each cover whole cache
// lines (lane l's bytes land at 16 l), so every line is requested once.  Bytes
// past the end of the buffer read as zero.
// Cache policy of loads of data read exactly once (features and terms of a
// materialized batch): non-temporal, so streaming them does not evict what
// is reused (the log table, weights, hoisted rows, descriptors) from the
// caches.
constexpr int STREAM = 2;  // the nt bit of the buffer instructions' cache policy

__device__ inline void dma_rows(uint4 *xsw, __amdgpu_buffer_rsrc_t xr, uint32_t row0, uint32_t soff,
                                int lane)
{
    const uint32_t vo = row0 + (uint32_t)lane * 16;
    __builtin_amdgcn_raw_ptr_buffer_load_lds(xr, (lds_void *)xsw, 16, vo, soff, 0, STREAM);
    __builtin_amdgcn_raw_ptr_buffer_load_lds(xr, (lds_void *)(xsw + 64), 16, vo + 1024, soff, 0,
                                             STREAM);
    if (lane < 32)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(xr, (lds_void *)(xsw + 128), 16, vo + 2048, soff, 0,
                                                 STREAM);
}
static_assert(TILE_ROWS * FS * 2 == 2560, "three copies of 1,024 + 1,024 + 512 bytes");

// Evaluate row-tile group `group` of a query: EVAL_WAVES / P tiles of 32
// candidates, every wave one (tile, stage part).  Every thread of the
// EVAL_WAVES-wave workgroup must call this with the same arguments (it
// synchronises the workgroup when P > 1).  kShared: the costs are read by
// another workgroup of the same launch (coherent stores).  kStage: also write
// every stage's cost to Q.stage[s][i].  kIndexed: the feature row of (s, i)
// is row Q.ridx[s][i] of the table Q.x (memoized rows); a row number outside
// the table makes that stage's cost NaN.
template <bool kShared, bool kStage = false, bool kIndexed = false>
__device__ __forceinline__ void eval_group(const QueryView &Q, int group, int wave, int lane,
                                           const Weights &w, const Pairs &kp,
                                           const uint32_t *tab, GroupShared &sh)
{
    const int P = Q.P;
    const int tile = group * (EVAL_WAVES / P) + wave / P;
    const int part = wave % P;
    // lane l: g = l / 16 selects the features and hoisted units it feeds to
    // the matrix core for candidates r = l % 16 and 16 + r; its own candidate
    // (terms, sum, result) is n = 16 (l / 32) + r, of which it holds
    // coefficients 4q .. 4q+3; the lane with q = 0 stores
    const int g = lane >> 4;
    const int r = lane & 15;
    const bool upper = lane >= 32;
    const int q = g & 1;
    const int n = (upper ? 16 : 0) + r;
    const int i = tile * TILE_ROWS + n;
    const bool valid = i < Q.N;
    // rows past the end of the query compute on other bytes (the last row's
    // terms, and whatever features follow the query's rows, or zeros past the
    // buffer's end); every load stays in bounds and their results are never
    // stored
    const int ic = valid ? i : Q.N - 1;
    // stages [s0, s1) of this part; a tile past the query's end does no work
    const int s0 = tile * TILE_ROWS < Q.N ? (Q.S * part) / P : 0;
    const int s1 = tile * TILE_ROWS < Q.N ? (Q.S * (part + 1)) / P : 0;

    // byte offsets: stage rows are N * 80 (features) and N * 32 (terms) apart;
    // the host rejects a query whose features or terms reach MAX_QUERY_BYTES
    // (check_query_bytes), so these 32-bit offsets, the last tile's reads
    // past the end included, never wrap
    const uint32_t xstep = kIndexed ? 0u : (uint32_t)Q.N * FS * 2;
    const uint32_t tstep = (uint32_t)Q.N * C * 4;
    // memoized rows: the table's rows * 80 bytes fit in 32 bits (host check)
    const uint32_t xbytes = kIndexed ? Q.rows * (FS * 2) : xstep * (uint32_t)Q.S;
    const __amdgpu_buffer_rsrc_t xr = buffer_over(Q.x, xbytes);
    const __amdgpu_buffer_rsrc_t tr = buffer_over(Q.t, tstep * (uint32_t)Q.S);
    uint32_t xsoff = (uint32_t)s0 * xstep;
    uint32_t tsoff = (uint32_t)s0 * tstep;
    const uint32_t to = (uint32_t)ic * (C * 4) + q * 16;
    // memoized rows: the row numbers of the stage loaded next (candidates r
    // and 16 + r), read one stage ahead of their feature loads; a row outside
    // the table reads past the buffer's end (zeros) and flags the lane's own
    // candidate when it is that one
    const int ic0 = min(tile * TILE_ROWS + r, Q.N - 1);
    const int ic1 = min(tile * TILE_ROWS + 16 + r, Q.N - 1);
    uint32_t xo0 = 0, xo1 = 0;
    int32_t rnext0 = 0, rnext1 = 0;
    bool bad = false;
    auto point_at = [&](int32_t r0, int32_t r1) {
        const bool ok0 = (uint32_t)r0 < Q.rows, ok1 = (uint32_t)r1 < Q.rows;
        xo0 = ok0 ? (uint32_t)r0 * (FS * 2) : xbytes;
        xo1 = ok1 ? (uint32_t)r1 * (FS * 2) : xbytes;
        bad = upper ? !ok1 : !ok0;
    };
    auto row_of = [&](int s, int c) { return Q.ridx[(int64_t)s * Q.N + c]; };
    const float4 *ug = reinterpret_cast<const float4 *>(Q.u);
    // this wave's slice of LDS holds the hoisted rows of up to USTAGE stages
    float4 *ur = sh.u[wave];

    float sum = 0.f, comp = 0.f;
    if (!kIndexed && s0 < s1) {
        // features: copied into this wave's LDS block one stage ahead of the
        // arithmetic and read from there into registers at the stage's start
        // (of each 80-byte row, lane l reads bytes 16g .. 16g+15 and
        // 64+4g .. 64+4g+3 of rows r and 16 + r); terms: loaded into two
        // alternating register buffers
        uint4 *xsw = sh.xs[wave];
        const uint32_t row0 = (uint32_t)tile * TILE_ROWS * (FS * 2);
        const lds_u1 *xs4 = reinterpret_cast<const lds_u1 *>(xsw);
        float4 tA, tB;
        auto load_t = [&](float4 &t) {
            t = __builtin_bit_cast(float4,
                                   __builtin_amdgcn_raw_buffer_load_b128(tr, to, tsoff, STREAM));
        };
        auto stage_in = [&](StageIn &in, const float4 &t) {
            // the stage's copy (and its terms, issued before it) have landed:
            // an explicit wait, since the compiler's own waits for copies into
            // LDS follow its alias analysis, which need not see this read
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            in.x0 = xsw[5 * r + g];
            in.x1 = xsw[5 * (16 + r) + g];
            in.x2.x = xs4[20 * r + 16 + g];
            in.x2.y = xs4[20 * (16 + r) + 16 + g];
            in.t = t;
            in.bad = false;
            // the rows are in registers before the block is refilled
            asm volatile("" ::"v"(in.x0.x), "v"(in.x0.y), "v"(in.x0.z), "v"(in.x0.w),
                         "v"(in.x1.x), "v"(in.x1.y), "v"(in.x1.z), "v"(in.x1.w), "v"(in.x2.x),
                         "v"(in.x2.y)
                         : "memory");
        };
        // the terms go first: waiting for a stage's copy then covers them
        load_t(tA);
        dma_rows(xsw, xr, row0, xsoff, lane);
        for (int s = s0; s < s1; s += 2) {
            if ((s - s0) % USTAGE == 0) refill_u(ur, ug, s, min(USTAGE, s1 - s), lane);
            StageIn in;
            float4 u[2];
            read_u(u, ur + ((s - s0) % USTAGE) * (H / 4), g);
            stage_in(in, tA);
            if (s + 1 < s1) {
                xsoff += xstep;
                tsoff += tstep;
                load_t(tB);
                dma_rows(xsw, xr, row0, xsoff, lane);
            }
            asm volatile("" ::: "memory");
            const float va = stage_math(in, u, upper, w, kp, tab, sum, comp);
            if (kStage && q == 0 && valid) Q.stage[(int64_t)s * Q.N + i] = va;
            if (s + 1 >= s1) break;

            if ((s + 1 - s0) % USTAGE == 0) refill_u(ur, ug, s + 1, min(USTAGE, s1 - s - 1), lane);
            read_u(u, ur + ((s + 1 - s0) % USTAGE) * (H / 4), g);
            stage_in(in, tB);
            if (s + 2 < s1) {
                xsoff += xstep;
                tsoff += tstep;
                load_t(tA);
                dma_rows(xsw, xr, row0, xsoff, lane);
            }
            asm volatile("" ::: "memory");
            const float vb = stage_math(in, u, upper, w, kp, tab, sum, comp);
            if (kStage && q == 0 && valid) Q.stage[(int64_t)(s + 1) * Q.N + i] = vb;
        }
    }
    if (kIndexed && s0 < s1) {
        // two register buffers alternate so that a stage's loads stay in
        // flight during the previous stage's arithmetic without copies
        StageIn A, B;
        if (kIndexed) {
            point_at(row_of(s0, ic0), row_of(s0, ic1));
            if (s0 + 1 < s1) {
                rnext0 = row_of(s0 + 1, ic0);
                rnext1 = row_of(s0 + 1, ic1);
            }
        }
        load_stage(A, xr, tr, xsoff, tsoff, xo0, xo1, g, to);
        A.bad = bad;
        for (int s = s0; s < s1; s += 2) {
            if ((s - s0) % USTAGE == 0) refill_u(ur, ug, s, min(USTAGE, s1 - s), lane);
            if (s + 1 < s1) {
                xsoff += xstep;
                tsoff += tstep;
                if (kIndexed) {
                    point_at(rnext0, rnext1);
                    if (s + 2 < s1) {
                        rnext0 = row_of(s + 2, ic0);
                        rnext1 = row_of(s + 2, ic1);
                    }
                }
            }
            load_stage(B, xr, tr, xsoff, tsoff, xo0, xo1, g, to);
            B.bad = bad;
            // keep the loads here, ahead of their use
            asm volatile("" ::: "memory");
            float4 u[2];
            read_u(u, ur + ((s - s0) % USTAGE) * (H / 4), g);
            const float va = stage_math(A, u, upper, w, kp, tab, sum, comp);
            if (kStage && q == 0 && valid) Q.stage[(int64_t)s * Q.N + i] = va;
            if (s + 1 >= s1) break;

            if ((s + 1 - s0) % USTAGE == 0) refill_u(ur, ug, s + 1, min(USTAGE, s1 - s - 1), lane);
            if (s + 2 < s1) {
                xsoff += xstep;
                tsoff += tstep;
                if (kIndexed) {
                    point_at(rnext0, rnext1);
                    if (s + 3 < s1) {
                        rnext0 = row_of(s + 3, ic0);
                        rnext1 = row_of(s + 3, ic1);
                    }
                }
            }
            load_stage(A, xr, tr, xsoff, tsoff, xo0, xo1, g, to);
            A.bad = bad;
            asm volatile("" ::: "memory");
            read_u(u, ur + ((s + 1 - s0) % USTAGE) * (H / 4), g);
            const float vb = stage_math(B, u, upper, w, kp, tab, sum, comp);
            if (kStage && q == 0 && valid) Q.stage[(int64_t)(s + 1) * Q.N + i] = vb;
        }
    }

    // combine the parts of each tile in ascending order
    if (P > 1) {
        if (q == 0) sh.part[wave][n] = make_float2(sum, comp);
        __syncthreads();
    }
    if (part == 0 && q == 0 && valid) {
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

}  // namespace bf16eval
}  // namespace cm
