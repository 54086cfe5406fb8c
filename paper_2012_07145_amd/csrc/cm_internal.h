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
// 32x32x16 bf16 matrix-core instruction reads them: 8 bf16 (16 bytes) per
// lane per operand.  [hi/lo][k-step][lane].
struct Bf16Pack {
    uint4 a1[2][3][64];  // folded first layer (32 hidden x 48 padded features)
    uint4 a2[2][2][64];  // coefficient layer (32 padded outputs x 32 hidden)
    float b2[8];
};

struct Model {
    int device = 0;
    float *d_params = nullptr;   // float32 blob as given
    float *d_beta = nullptr;     // W_1[:, 24:] b_s (32), added when folding
    Bf16Pack *d_bf16 = nullptr;  // packed operands of the bf16 evaluator
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
};

struct EvalLaunch {
    int32_t nq;
    int32_t ntasks;    // workgroups (bf16) or thread blocks (fp32)
    int32_t nstages;   // hoist blocks
    int32_t pad;
    EvalQ q[QMAX];
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

// Kernel launchers (one per translation unit).
hipError_t launch_hoist(const EvalLaunch &L, const Model &m, bool fold, const float *pipe,
                        float *U, hipStream_t st);
hipError_t launch_eval_fp32(const EvalLaunch &L, const Model &m, const float *sched,
                            const float *terms, const float *U, float *cost, hipStream_t st);
hipError_t launch_eval_bf16(const EvalLaunch &L, const Model &m, const uint16_t *sched,
                            const float *terms, const float *U, float *cost, hipStream_t st);
hipError_t launch_topk(const TopkLaunch &L, const float *cost, uint64_t *tpart, int32_t *tcnt,
                       int32_t *idx_out, float *val_out, hipStream_t st);

}  // namespace cm
