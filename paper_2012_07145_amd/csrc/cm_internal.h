// cm_internal.h -- shared definitions of the gfx950 library: model and
// workspace objects, per-launch query descriptors, launcher prototypes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cm.h"

namespace cm {

constexpr int FP = CM_N_PIPE_FEATURES;   // 56 algorithm features per stage
constexpr int FS = CM_N_SCHED_FEATURES;  // 40 schedule features per (stage, candidate)
constexpr int E = CM_EMBED;              // 24
constexpr int H = CM_HIDDEN;             // 32
constexpr int C = CM_N_COEFS;            // 8 coefficients / cost terms

// Offsets (floats) of each tensor in the parameter blob.
constexpr int OFF_WP = 0;
constexpr int OFF_BP = OFF_WP + E * FP;
constexpr int OFF_WS = OFF_BP + E;
constexpr int OFF_BS = OFF_WS + E * FS;
constexpr int OFF_W1 = OFF_BS + E;
constexpr int OFF_B1 = OFF_W1 + H * 2 * E;
constexpr int OFF_W2 = OFF_B1 + H;
constexpr int OFF_B2 = OFF_W2 + C * H;
constexpr int N_PARAMS = OFF_B2 + C;
static_assert(N_PARAMS == CM_N_PARAMS, "parameter layout");

constexpr int QMAX = 32;            // queries per kernel launch (descriptors by value)
constexpr int TILE_ROWS = 32;       // candidates per wave of the bf16 evaluator
constexpr int EVAL_WAVES = 8;       // waves per workgroup of the bf16 evaluator

// Stage parts of the bf16 evaluator: a query's stages are split into P
// contiguous, near-equal parts, one wave each; the parts' compensated sums
// are combined in ascending order inside the workgroup.  P depends only on
// the query's stage count, so results never depend on the batch.
__host__ __device__ constexpr int stage_parts(int S)
{
    return S <= CM_STAGE_CHUNK / 2 ? 1 : S <= CM_STAGE_CHUNK ? 2 : S <= 2 * CM_STAGE_CHUNK ? 4 : 8;
}
constexpr int TOPK_TILE = 4096;     // candidates per workgroup of the selection

// bf16 split-product operands of the two dense layers, laid out as the
// 16x16x32 bf16 matrix-core instruction reads them: 8 bf16 (16 bytes) per
// lane per operand.
// The bf16 evaluator looks up log2(1 + x) of a feature code in a table of
// the codes LOG_BASE .. LOG_BASE + LOG_N - 1 (x from 2^-24 to just below
// 2^40).  Below LOG_BASE, 1 + x rounds to 1 in float32.
constexpr uint32_t LOG_BASE = 0x3380u;
constexpr int LOG_N = 8192;

struct Bf16Pack {
    // 16x16x32 operands (lane l: row l % 16, k-slots 8 (l / 16) .. +7)
    uint4 a1[2][3][64];  // folded first layer per hidden half: high and low
                         // weights of features 0..31, last-block operand
    uint4 a2[2][64];     // coefficient layer: rows [W_2 high; W_2 low] and [W_2 high; 0]
    float b2[8];
    float pad[4];
    // (high bf16 | low bf16 << 16) of log2(1 + x) for code LOG_BASE + i,
    // filled on the device by launch_log_table
    uint32_t logtab[LOG_N];
};
static_assert(offsetof(Bf16Pack, logtab) % 16 == 0, "table copied in 16-byte units");

// e4m3 operands of the FP8 form, laid out as the 32x32x64 fp8 matrix core
// reads them (32 bytes per lane and operand), and its scales.
struct Fp8Pack {
    uint32_t a1[64][8];  // first layer: lane m + 32h, byte j < 20 = e4m3(Wf[m][20h + j] s_w1)
    uint32_t a2[64][8];  // coefficient layer: byte j < 16 = e4m3(W_2[m][unit(h, j)] s_w2)
    float b2[8];
    float r1;            // s_h / (s_w1 s_in): first-layer accumulator -> scaled hidden
    float r2;            // 1 / (s_w2 s_h): second-layer accumulator -> coefficient
    float uh;            // s_h: scale of the hoisted rows
    float pad;
};

struct Model {
    int device = 0;
    float *d_params = nullptr;   // float32 blob as given
    float *d_beta = nullptr;     // W_1[:, 24:] b_s (32), added when folding
    Bf16Pack *d_bf16 = nullptr;  // packed operands of the bf16 evaluator
    Fp8Pack *d_fp8 = nullptr;    // operands of the FP8 form (after cm_model_prepare_fp8)
    float fp8_uscale = 0.f;      // Fp8Pack::uh, kept on the host for the hoist
    float *h_params = nullptr;   // host copy of the blob (FP8 preparation, calibration)
};

struct Workspace {
    int device = 0;
    cm_workspace_desc cap{};
    float *d_U = nullptr;          // [stages][32] hoisted first-layer input
    uint64_t *d_tpart = nullptr;   // per-tile beam lists
    int64_t tpart_cap = 0;
    int32_t *d_tcnt = nullptr;     // arrival counters per query (selection)
};

// Per-query data of one launch of the evaluator.
struct EvalQ {
    int32_t S, N;
    int64_t pipe_off, sched_off, terms_off, cost_off;
    int64_t u_off;     // offset (floats) of this query's hoisted rows U[S][32]
    int32_t hrow0;     // first hoist block of this query in the launch
    int32_t task0;     // first workgroup (bf16) or thread block (fp32) of this query
    int32_t parts;     // stage parts P (bf16)
    int32_t pad;
    int64_t stage_off; // offset (floats) of this query's per-stage costs [S][N] (terms_off / 8)
};

struct EvalLaunch {
    int32_t nq;
    int32_t ntasks;    // workgroups (bf16) or thread blocks (fp32)
    int32_t nstages;   // hoist blocks
    int32_t pad;
    EvalQ q[QMAX];
};

struct FreezeQ {
    int32_t S, N;
    int64_t stage_off;  // per-stage costs [S][N] of the query (floats)
    int64_t flag_off;   // its S flags in the output (batch order)
    int64_t cand_q;     // index of the query in the caller's batch (cand[cand_q * stride])
};

struct FreezeLaunch {
    int32_t nq;
    int32_t pad;
    FreezeQ q[QMAX];
};

struct PenaltyQ {
    int32_t N;
    int32_t pad;
    int64_t cost_off;  // costs (and hashes) of the query
    int64_t cand0;     // candidates of the launch's earlier queries
};

struct PenaltyLaunch {
    int32_t nq;
    int32_t pad;
    PenaltyQ q[QMAX];
};

struct TopkQ {
    int32_t N;
    int32_t out_q;     // index of the query in the caller's batch
    int64_t cost_off;
    int32_t tile0;     // first tile of this query
    int32_t ntiles;
};

struct TopkLaunch {
    int32_t nq;
    int32_t ntasks;
    int32_t k;
    int32_t pad;
    TopkQ q[QMAX];
};

// ------------------------------------------------------------------ step
// Device-resident descriptors of one persistent step (hoist + evaluate +
// select).  The host writes them into pinned memory and one copy moves them
// to the device ahead of the kernels, so the launch configuration never
// depends on the batch and the whole step can be replayed as a graph.
constexpr int STEP_MAX_QUERIES = CM_STEP_MAX_QUERIES;

struct StepQ {
    const void *x;      // schedule features [S][N][40]: bf16 bits or e4m3 codes
    const float *t;     // cost terms [S][N][8]
    float *u;           // hoisted rows [S][32] (written by the hoist when it runs)
    const float *pipe;  // algorithm features [S][56] (hoist only)
    float *cost;        // [N]
    int32_t *idx;       // beam [k]
    float *val;         // beam costs [k]
    int32_t *sidx;      // second copy of the beam (a session's), or null
    float *sval;
    int32_t S, N;
    int32_t task0;      // first task of this query
    int32_t ntasks;     // >= 1 (a query with no candidates still writes its padding)
    int32_t parts;      // stage parts P
    int32_t row0;       // first hoist row of this query
    int32_t tile0;      // first selection tile (global numbering)
    int32_t ntiles;     // selection tiles of TOPK_TILE candidates, >= 1
};

struct StepHead {
    int32_t nq;        // queries
    int32_t ntasks;    // tasks over all queries
    int32_t nrows;     // hoist rows over all queries
    int32_t k;         // beam width
    int32_t gpt;       // row-tile groups per task (1, 2 or 4)
    int32_t pad;
    // where the launch's (first start, last end) clock pair also goes, or
    // null: host memory mapped for the device, so a server learns it without
    // a copy
    uint64_t *clk_out;
};
static_assert(sizeof(StepHead) == 32, "step head layout");

// Control words of a step, zero between steps (the step kernel leaves them
// zero when it ends): task queue head, exit count, per-query and per-tile
// arrival counts.
// CTL_CLK: running (first start, last end) of the launch's workgroups and
// CTL_CLKOUT: the last finished launch's pair, as 64-bit words of the
// constant-rate real-time counter (100 MHz).
constexpr int CTL_NEXT = 0;
constexpr int CTL_CLK = 16;
constexpr int CTL_CLKOUT = 24;
constexpr int CTL_DONE = 32;
constexpr double CLOCK_MHZ = 100.0;
constexpr int CTL_QCNT = 64;
constexpr int CTL_TCNT = CTL_QCNT + STEP_MAX_QUERIES;

// One query of a step, as absolute device pointers (host side).
struct StepReq {
    const void *x;      // bf16 bits or e4m3 codes, as the step's precision
    const float *t;
    float *u;
    const float *pipe;  // needed only when the step hoists
    float *cost;
    int32_t *idx;
    float *val;
    int32_t *sidx;      // optional second beam destination
    float *sval;
    int32_t S, N;
};

// Queue one step over `n` queries on `st` (validated by the caller against
// the step's capacities; n <= max_queries, sum N <= max_cands, sum S <=
// max_stages when hoisting).
// clk_out: optional device-visible address (host memory mapped for the
// device) that also receives the launch's clock pair.
cm_status step_launch(cm_step *S, const StepReq *r, int n, int k, bool hoist, hipStream_t st,
                      uint64_t *clk_out = nullptr);
// Capacities of a step.
const cm_step_desc &step_caps(const cm_step *S);
// Kernel-only GPU time (microseconds) of the step's most recent launch,
// waiting for it if it is still running.
cm_status step_kernel_us(cm_step *S, float *us);
// Device address of the (first start, last end) clock pair that the step's
// most recent launch leaves behind (two uint64 words; see CTL_CLKOUT).
const uint64_t *step_clock(const cm_step *S);

// Kernel launchers (one per translation unit).
hipError_t launch_hoist(const EvalLaunch &L, const Model &m, bool fold, float scale,
                        const float *pipe, float *U, hipStream_t st);
// ridx, rows: memoized rows (sched is then a table of `rows` rows and each
// query's sched_off locates its row numbers in ridx), or nullptr.
hipError_t launch_eval_fp8(const EvalLaunch &L, const Model &m, const uint8_t *codes,
                           const float *terms, const float *U, float *cost, float *stage,
                           hipStream_t st, const int32_t *ridx = nullptr, uint32_t rows = 0);
hipError_t launch_fp8_encode(const float *x, int64_t n, float in_scale, uint8_t *codes,
                             hipStream_t st);
// stage: per-stage costs [S][N] at each query's stage_off, or nullptr.
hipError_t launch_eval_fp32(const EvalLaunch &L, const Model &m, const float *sched,
                            const float *terms, const float *U, float *cost, float *stage,
                            hipStream_t st);
// Fill pk->logtab (the device's own arithmetic of the bf16 evaluator).
hipError_t launch_log_table(Bf16Pack *pk, hipStream_t st);
hipError_t launch_eval_bf16(const EvalLaunch &L, const Model &m, const uint16_t *sched,
                            const float *terms, const float *U, float *cost, float *stage,
                            hipStream_t st, const int32_t *ridx = nullptr, uint32_t rows = 0);
hipError_t launch_freeze(const FreezeLaunch &L, const float *stage, const int32_t *cand,
                         int64_t cand_stride, uint8_t *frozen, hipStream_t st);
hipError_t launch_penalty(const PenaltyLaunch &L, const uint64_t *hashes, const uint64_t *bad,
                          int64_t n_bad, float penalty, float *cost, hipStream_t st);
hipError_t launch_topk(const TopkLaunch &L, const float *cost, uint64_t *tpart, int32_t *tcnt,
                       int32_t *idx_out, float *val_out, hipStream_t st);
hipError_t launch_step_hoist(const StepHead *h, const StepQ *qs, const Model &m,
                             cm_precision prec, int grid, hipStream_t st);
hipError_t launch_step(const StepHead *h, const StepQ *qs, uint32_t *ctl, uint64_t *tpart,
                       const Model &m, cm_precision prec, int grid, hipStream_t st);

// Device side: data one workgroup hands to another inside a launch (costs
// read by the selecting workgroup, per-tile beam lists) is stored and loaded
// with agent-scope atomic accesses, which bypass the per-XCD L2's
// non-coherent copies, and the producer waits for its stores to complete
// before its arrival count.  This replaces device-wide fences, which write
// back and invalidate the whole L2.
// (Pointers are taken as global memory, so the accesses are global, not
// flat, instructions and the store wait below covers them.)
template <class T>
__device__ inline void store_shared(T *p, T v)
{
    __hip_atomic_store((__attribute__((address_space(1))) T *)p, v, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ inline T load_shared(const T *p)
{
    return __hip_atomic_load((__attribute__((address_space(1))) T *)const_cast<T *>(p),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Wait until this wave's stores have completed.
__device__ inline void wait_stores() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Host side: record a thread-local error message and return `st`.
cm_status fail(cm_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

// The bf16 and FP8 evaluators address one query's schedule features and
// cost terms through buffer resources with 32-bit byte offsets.  A query
// whose features (S * N * 80 bytes in bf16, S * N * 40 in FP8) or terms
// (S * N * 32 bytes) would reach this size is rejected on the host; the
// margin covers the last row tile's reads past the query's end.
constexpr int64_t MAX_QUERY_BYTES = ((int64_t)1 << 32) - ((int64_t)1 << 16);
// CM_E2BIG (with a message naming query q) unless a query of S stages and N
// candidates fits those offsets in `prec`; CM_FP32 addresses with 64-bit
// offsets and always fits.  table: the features come from a row table
// (memoized rows, checked against its own size), so only the terms count.
cm_status check_query_bytes(int64_t q, int64_t S, int64_t N, cm_precision prec, bool table);

#define CM_HIP(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return ::cm::fail(CM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

}  // namespace cm

struct cm_model {
    cm::Model m;
};
