// cm_step.hip -- host side of the persistent beam step (include/cm.h):
// descriptor slots in pinned memory, graph capture and replay, autotuner.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "cm_internal.h"

namespace {

using cm::fail;

constexpr int MAX_SLOTS = 8;

struct Slot {
    unsigned char *h_block = nullptr;  // pinned host descriptors
    unsigned char *d_block = nullptr;  // their device copy
    uint32_t *d_ctl = nullptr;         // control words (zero between steps)
    uint64_t *d_tpart = nullptr;       // per-tile beam lists
    float *d_U = nullptr;              // hoisted rows when the caller gives none
    hipGraphExec_t exec[2] = {nullptr, nullptr};  // [with hoist]
    int exec_grid[2] = {0, 0};
    hipEvent_t done = nullptr;         // recorded after the slot's last step
    bool pending = false;
};

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

}  // namespace

struct cm_step {
    const cm_model *model = nullptr;
    cm_precision prec = CM_BF16;  // CM_BF16 or CM_FP8
    int device = 0;
    cm_step_desc cap{};
    cm_step_config cfg{};
    int cus = 0;
    char arch[64] = {0};  // the device's gcnArchName (key of the tuning cache)
    int64_t max_tiles = 0;
    size_t block_bytes = 0;
    hipStream_t cs = nullptr;  // capture stream
    Slot slot[MAX_SLOTS];
    int next = 0;
    int last = -1;  // slot of the most recent step
    std::mutex mu;
};

namespace {

size_t ctl_words(const cm_step &S) { return (size_t)cm::CTL_TCNT + (size_t)S.max_tiles; }

int grid_of(const cm_step &S) { return S.cfg.grid > 0 ? S.cfg.grid : 2 * S.cus; }

int hoist_grid(const cm_step &S) { return (int)std::min<int64_t>(S.cap.max_stages, 4 * S.cus); }

cm::StepHead *head_of(unsigned char *block) { return reinterpret_cast<cm::StepHead *>(block); }
cm::StepQ *queries_of(unsigned char *block)
{
    return reinterpret_cast<cm::StepQ *>(block + sizeof(cm::StepHead));
}

void free_slot(Slot &s)
{
    for (auto &e : s.exec)
        if (e) (void)hipGraphExecDestroy(e);
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.h_block) (void)hipHostFree(s.h_block);
    if (s.d_block) (void)hipFree(s.d_block);
    if (s.d_ctl) (void)hipFree(s.d_ctl);
    if (s.d_tpart) (void)hipFree(s.d_tpart);
    if (s.d_U) (void)hipFree(s.d_U);
    s = Slot{};
}

void free_step(cm_step *S)
{
    for (auto &s : S->slot) free_slot(s);
    if (S->cs) (void)hipStreamDestroy(S->cs);
    delete S;
}

cm_status check_step_batch(const cm_step &S, const cm_batch *b, const float *U, int32_t k,
                           const float *cost_out, const int32_t *idx_out, const float *val_out)
{
    if (!b) return fail(CM_EINVAL, "batch is NULL");
    if (k < 1 || k > S.cap.max_k)
        return fail(CM_EINVAL, "k=%d outside [1, %d]", k, S.cap.max_k);
    if (b->n_queries < 0) return fail(CM_EINVAL, "n_queries < 0");
    if (b->n_queries > 0 && !b->queries) return fail(CM_EINVAL, "queries is NULL");
    if (b->n_queries > S.cap.max_queries)
        return fail(CM_E2BIG, "batch has %d queries, the step holds %d", b->n_queries,
                    S.cap.max_queries);
    int64_t stages = 0, cands = 0;
    for (int32_t q = 0; q < b->n_queries; ++q) {
        const cm_query &Q = b->queries[q];
        if (Q.n_stages < 1) return fail(CM_EINVAL, "query %d: n_stages %d < 1", q, Q.n_stages);
        if (Q.n_cands < 0) return fail(CM_EINVAL, "query %d: n_cands %d < 0", q, Q.n_cands);
        if (Q.pipe_off < 0 || Q.sched_off < 0 || Q.terms_off < 0 || Q.cost_off < 0)
            return fail(CM_EINVAL, "query %d: negative offset", q);
        if (Q.sched_off % 8 != 0)
            return fail(CM_EINVAL, "query %d: sched_off %lld is not a multiple of 8", q,
                        (long long)Q.sched_off);
        if (Q.terms_off % 4 != 0)
            return fail(CM_EINVAL, "query %d: terms_off %lld is not a multiple of 4", q,
                        (long long)Q.terms_off);
        const cm_status st = cm::check_query_bytes(q, Q.n_stages, Q.n_cands, S.prec, false);
        if (st != CM_OK) return st;
        stages += Q.n_stages;
        cands += Q.n_cands;
    }
    if (stages > S.cap.max_stages)
        return fail(CM_E2BIG, "batch has %lld stages, the step holds %lld", (long long)stages,
                    (long long)S.cap.max_stages);
    if (cands > S.cap.max_cands)
        return fail(CM_E2BIG, "batch has %lld candidates, the step holds %lld",
                    (long long)cands, (long long)S.cap.max_cands);
    if (b->n_queries > 0 && (!idx_out || !val_out))
        return fail(CM_EINVAL, "idx_out or val_out is NULL");
    if (cands > 0) {
        if (!cost_out) return fail(CM_EINVAL, "cost_out is NULL");
        if (!b->sched || !b->terms) return fail(CM_EINVAL, "batch sched/terms pointer is NULL");
        if (!aligned(b->sched, 16) || !aligned(b->terms, 16))
            return fail(CM_EINVAL, "sched and terms must be 16-byte aligned");
    }
    if (b->n_queries > 0) {
        if (U && !aligned(U, 16)) return fail(CM_EINVAL, "U must be 16-byte aligned");
        if (!U && !b->pipe) return fail(CM_EINVAL, "pipe is NULL and no U was given");
        if (!U && !aligned(b->pipe, 4)) return fail(CM_EINVAL, "pipe is misaligned");
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(CM_EDEVICE, "hipGetDevice failed");
    if (dev != S.device)
        return fail(CM_EINVAL, "step lives on device %d but device %d is current", S.device, dev);
    return CM_OK;
}

// Descriptors of the queries into the slot's pinned block.  Tasks are issued
// longest stage part first; each query's outputs stay where its request
// points.
void fill_descriptors(const cm_step &S, Slot &sl, const cm::StepReq *r, int nq, int32_t k,
                      bool hoist, uint64_t *clk_out)
{
    using namespace cm;
    std::vector<int32_t> order(nq);
    for (int q = 0; q < nq; ++q) order[q] = q;
    auto per_wave = [&](int32_t q) {
        const int Sq = r[q].S;
        return (Sq + stage_parts(Sq) - 1) / stage_parts(Sq);
    };
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t x, int32_t y) { return per_wave(x) > per_wave(y); });

    const int gpt = S.cfg.group_tiles;
    StepHead *h = head_of(sl.h_block);
    StepQ *qs = queries_of(sl.h_block);
    std::memset(h, 0, sizeof *h);
    int64_t task = 0, row = 0, tile = 0;
    for (int j = 0; j < nq; ++j) {
        const StepReq &R = r[order[j]];
        StepQ &d = qs[j];
        std::memset(&d, 0, sizeof d);
        d.x = R.x;
        d.t = R.t;
        d.u = R.u;
        d.pipe = R.pipe;
        d.cost = R.cost;
        d.idx = R.idx;
        d.val = R.val;
        d.sidx = R.sidx;
        d.sval = R.sval;
        d.S = R.S;
        d.N = R.N;
        d.parts = stage_parts(R.S);
        const int64_t groups = cdiv(cdiv(R.N, TILE_ROWS), EVAL_WAVES / d.parts);
        d.task0 = (int32_t)task;
        d.ntasks = (int32_t)std::max<int64_t>(1, cdiv(groups, gpt));
        d.row0 = (int32_t)row;
        d.tile0 = (int32_t)tile;
        d.ntiles = (int32_t)std::max<int64_t>(1, cdiv(R.N, TOPK_TILE));
        task += d.ntasks;
        row += R.S;
        tile += d.ntiles;
    }
    h->nq = nq;
    h->ntasks = (int32_t)task;
    h->nrows = hoist ? (int32_t)row : 0;
    h->k = k;
    h->gpt = gpt;
    h->clk_out = clk_out;
}

// The device work of one step on `st`: descriptor copy, hoist, step kernel.
hipError_t issue(const cm_step &S, Slot &sl, bool hoist, size_t bytes, hipStream_t st)
{
    using namespace cm;
    const StepHead *h = reinterpret_cast<const StepHead *>(sl.d_block);
    const StepQ *qs = reinterpret_cast<const StepQ *>(sl.d_block + sizeof(StepHead));
    hipError_t e = hipMemcpyAsync(sl.d_block, sl.h_block, bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    if (hoist &&
        (e = launch_step_hoist(h, qs, S.model->m, S.prec, hoist_grid(S), st)) != hipSuccess)
        return e;
    return launch_step(h, qs, sl.d_ctl, sl.d_tpart, S.model->m, S.prec, grid_of(S), st);
}

cm_status get_exec(cm_step &S, Slot &sl, bool hoist, hipGraphExec_t *out)
{
    const int g = grid_of(S);
    hipGraphExec_t &ex = sl.exec[hoist ? 1 : 0];
    if (ex && sl.exec_grid[hoist ? 1 : 0] == g) {
        *out = ex;
        return CM_OK;
    }
    if (ex) {
        (void)hipGraphExecDestroy(ex);
        ex = nullptr;
    }
    CM_HIP(hipStreamBeginCapture(S.cs, hipStreamCaptureModeThreadLocal));
    const hipError_t e = issue(S, sl, hoist, S.block_bytes, S.cs);
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(S.cs, &graph);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(CM_EDEVICE, "step capture failed: %s",
                    hipGetErrorString(e != hipSuccess ? e : e2));
    }
    const hipError_t e3 = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) {
        ex = nullptr;
        return fail(CM_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e3));
    }
    sl.exec_grid[hoist ? 1 : 0] = g;
    *out = ex;
    return CM_OK;
}

cm_status launch_locked(cm_step &S, const cm::StepReq *r, int n, int32_t k, bool hoist,
                        hipStream_t st, uint64_t *clk_out = nullptr)
{
    if (n == 0) return CM_OK;
    Slot &sl = S.slot[S.next];
    if (sl.pending) CM_HIP(hipEventSynchronize(sl.done));  // its descriptors are still read
    sl.pending = false;
    fill_descriptors(S, sl, r, n, k, hoist, clk_out);
    if (S.cfg.use_graph) {
        hipGraphExec_t ex = nullptr;
        cm_status rc = get_exec(S, sl, hoist, &ex);
        if (rc != CM_OK) return rc;
        CM_HIP(hipGraphLaunch(ex, st));
    } else {
        const size_t bytes = sizeof(cm::StepHead) + (size_t)n * sizeof(cm::StepQ);
        CM_HIP(issue(S, sl, hoist, bytes, st));
    }
    CM_HIP(hipEventRecord(sl.done, st));
    sl.pending = true;
    S.last = S.next;
    S.next = (S.next + 1) % S.cap.slots;
    return CM_OK;
}

// A cm_batch as step requests: outputs of query q at idx_out + q*k.
void batch_requests(const cm_step &S, const cm_batch *b, const float *U, int32_t k,
                    float *cost_out, int32_t *idx_out, float *val_out,
                    std::vector<cm::StepReq> &r)
{
    using namespace cm;
    const Slot &sl = S.slot[S.next];
    float *ubase = U ? const_cast<float *>(U) : sl.d_U;
    r.resize(b->n_queries);
    int64_t urow = 0;
    for (int q = 0; q < b->n_queries; ++q) {
        const cm_query &Q = b->queries[q];
        StepReq &R = r[q];
        R.x = static_cast<const unsigned char *>(b->sched) +
              Q.sched_off * (S.prec == CM_FP8 ? 1 : 2);
        R.t = b->terms + Q.terms_off;
        R.u = ubase + urow * H;
        R.pipe = U ? nullptr : b->pipe + Q.pipe_off;
        R.cost = cost_out + Q.cost_off;
        R.idx = idx_out + (int64_t)q * k;
        R.val = val_out + (int64_t)q * k;
        R.sidx = nullptr;
        R.sval = nullptr;
        R.S = Q.n_stages;
        R.N = Q.n_cands;
        urow += Q.n_stages;
    }
}

cm_status run_locked(cm_step &S, const cm_batch *b, const float *U, int32_t k, float *cost_out,
                     int32_t *idx_out, float *val_out, hipStream_t st)
{
    cm_status rc = check_step_batch(S, b, U, k, cost_out, idx_out, val_out);
    if (rc != CM_OK) return rc;
    std::vector<cm::StepReq> r;
    batch_requests(S, b, U, k, cost_out, idx_out, val_out, r);
    return launch_locked(S, r.data(), (int)r.size(), k, U == nullptr, st);
}

cm_status check_config(const cm_step_config *c)
{
    if (!c) return fail(CM_EINVAL, "config is NULL");
    if (c->grid < 0 || c->grid > 65535) return fail(CM_EINVAL, "grid %d outside [0, 65535]", c->grid);
    if (c->group_tiles != 1 && c->group_tiles != 2 && c->group_tiles != 4 && c->group_tiles != 8)
        return fail(CM_EINVAL, "group_tiles must be 1, 2, 4 or 8");
    if (c->use_graph != 0 && c->use_graph != 1) return fail(CM_EINVAL, "use_graph must be 0 or 1");
    return CM_OK;
}

}  // namespace

// ---- tuning cache: the autotuner's pick per (GPU architecture, precision,
// shape bucket), shape bucket = (ceil log2 of the queries, ceil log2 of the
// rows) of the batch it was tuned on.  Process-wide; loaded from and saved
// to the text file named by the environment variable CM_TUNE_CACHE when it
// is set (one entry per line: arch precision qbucket rbucket grid
// group_tiles use_graph microseconds).
namespace {

struct TuneEntry {
    cm_step_config cfg;
    float us;
};

std::mutex g_tune_mu;
std::map<std::string, TuneEntry> g_tune;  // key: "arch precision qb rb"
bool g_tune_loaded = false;

int ceil_log2(int64_t v)
{
    int b = 0;
    while (((int64_t)1 << b) < v) ++b;
    return b;
}

std::string tune_key(const char *arch, cm_precision prec, int qb, int rb)
{
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s %d %d %d", arch, (int)prec, qb, rb);
    return buf;
}

// (mutex held)
void tune_load_locked()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("CM_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char arch[64];
    int prec, qb, rb, grid, gt, graph;
    float us;
    while (std::fscanf(f, "%63s %d %d %d %d %d %d %f", arch, &prec, &qb, &rb, &grid, &gt, &graph,
                       &us) == 8) {
        const cm_step_config c{grid, gt, graph};
        if (grid >= 0 && grid <= 65535 && (gt == 1 || gt == 2 || gt == 4 || gt == 8) &&
            (graph == 0 || graph == 1))
            g_tune[tune_key(arch, prec, qb, rb)] = TuneEntry{c, us};
    }
    std::fclose(f);
}

// (mutex held)
void tune_save_locked()
{
    const char *path = std::getenv("CM_TUNE_CACHE");
    if (!path || !*path) return;
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    for (const auto &kv : g_tune)
        std::fprintf(f, "%s %d %d %d %.3f\n", kv.first.c_str(), kv.second.cfg.grid,
                     kv.second.cfg.group_tiles, kv.second.cfg.use_graph, kv.second.us);
    const bool ok = std::fclose(f) == 0;
    if (ok) std::rename(tmp.c_str(), path);
}

}  // namespace

namespace cm {

cm_status step_launch(cm_step *S, const StepReq *r, int n, int k, bool hoist, hipStream_t st,
                      uint64_t *clk_out)
{
    std::lock_guard<std::mutex> lk(S->mu);
    return launch_locked(*S, r, n, k, hoist, st, clk_out);
}

const cm_step_desc &step_caps(const cm_step *S) { return S->cap; }

cm_status step_kernel_us(cm_step *S, float *us)
{
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->last < 0) return fail(CM_ENOTFOUND, "the step has not run yet");
    Slot &sl = S->slot[S->last];
    CM_HIP(hipEventSynchronize(sl.done));
    uint64_t clk[2];
    CM_HIP(hipMemcpy(clk, sl.d_ctl + CTL_CLKOUT, sizeof clk, hipMemcpyDeviceToHost));
    *us = (float)((double)(clk[1] - clk[0]) / CLOCK_MHZ);
    return CM_OK;
}

const uint64_t *step_clock(const cm_step *S)
{
    const int s = S->last < 0 ? 0 : S->last;
    return reinterpret_cast<const uint64_t *>(S->slot[s].d_ctl + CTL_CLKOUT);
}

}  // namespace cm

extern "C" {

cm_status cm_step_kernel_time(cm_step *S, float *us)
{
    if (!S || !us) return fail(CM_EINVAL, "NULL argument");
    return cm::step_kernel_us(S, us);
}

cm_status cm_step_create(const cm_model *model, cm_precision prec, const cm_step_desc *d,
                         cm_step **out)
{
    using namespace cm;
    if (!model || !d || !out) return fail(CM_EINVAL, "NULL argument");
    *out = nullptr;
    if (prec != CM_BF16 && prec != CM_FP8)
        return fail(CM_EUNSUPPORTED, "the step supports CM_BF16 and CM_FP8 only");
    if (prec == CM_FP8 && !model->m.d_fp8)
        return fail(CM_EINVAL, "model has no FP8 form (cm_model_prepare_fp8)");
    if (d->max_queries < 1 || d->max_queries > CM_STEP_MAX_QUERIES || d->max_stages < 1 ||
        d->max_cands < 0 || d->max_k < 1 || d->max_k > CM_MAX_K || d->slots < 1 ||
        d->slots > MAX_SLOTS)
        return fail(CM_EINVAL, "bad step capacities");
    if (d->max_cands > INT32_MAX || d->max_stages > INT32_MAX / 2)
        return fail(CM_EINVAL, "step capacities too large");
    cm_step *S = new (std::nothrow) cm_step;
    if (!S) return fail(CM_ENOMEM, "host allocation failed");
    S->model = model;
    S->prec = prec;
    S->cap = *d;
    S->cfg = cm_step_config{0, 1, 1};
    S->max_tiles = d->max_cands / TOPK_TILE + d->max_queries;
    S->block_bytes = sizeof(StepHead) + (size_t)d->max_queries * sizeof(StepQ);
    hipDeviceProp_t prop;
    if (hipGetDevice(&S->device) != hipSuccess ||
        hipGetDeviceProperties(&prop, S->device) != hipSuccess) {
        free_step(S);
        return fail(CM_EDEVICE, "no HIP device");
    }
    if (S->device != model->m.device) {
        free_step(S);
        return fail(CM_EINVAL, "model lives on device %d, current device is %d", model->m.device,
                    S->device);
    }
    S->cus = prop.multiProcessorCount;
    std::snprintf(S->arch, sizeof S->arch, "%s", prop.gcnArchName);
    if (hipStreamCreateWithFlags(&S->cs, hipStreamNonBlocking) != hipSuccess) {
        S->cs = nullptr;
        free_step(S);
        return fail(CM_EDEVICE, "stream creation failed");
    }
    for (int i = 0; i < d->slots; ++i) {
        Slot &sl = S->slot[i];
        bool ok = hipHostMalloc((void **)&sl.h_block, S->block_bytes, hipHostMallocDefault) ==
                  hipSuccess;
        ok = ok && hipMalloc((void **)&sl.d_block, S->block_bytes) == hipSuccess;
        ok = ok && hipMalloc((void **)&sl.d_ctl, ctl_words(*S) * sizeof(uint32_t)) == hipSuccess;
        ok = ok && hipMalloc((void **)&sl.d_tpart,
                             (size_t)S->max_tiles * d->max_k * sizeof(uint64_t)) == hipSuccess;
        ok = ok && hipMalloc((void **)&sl.d_U, (size_t)d->max_stages * H * sizeof(float)) ==
                       hipSuccess;
        ok = ok && hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            free_step(S);
            return fail(CM_ENOMEM, "step allocation failed");
        }
        std::memset(sl.h_block, 0, S->block_bytes);
        const uint64_t clk_init[2] = {~0ull, 0ull};  // (first start, last end)
        if (hipMemset(sl.d_ctl, 0, ctl_words(*S) * sizeof(uint32_t)) != hipSuccess ||
            hipMemcpy(sl.d_ctl + CTL_CLK, clk_init, sizeof clk_init, hipMemcpyHostToDevice) !=
                hipSuccess) {
            free_step(S);
            return fail(CM_EDEVICE, "step initialisation failed");
        }
    }
    if (hipDeviceSynchronize() != hipSuccess) {
        free_step(S);
        return fail(CM_EDEVICE, "step initialisation failed");
    }
    *out = S;
    return CM_OK;
}

cm_status cm_step_destroy(cm_step *S)
{
    if (!S) return fail(CM_EINVAL, "step is NULL");
    cm_status rc = CM_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        for (auto &sl : S->slot)
            if (sl.pending && hipEventSynchronize(sl.done) != hipSuccess)
                rc = fail(CM_EDEVICE, "waiting for the step's work failed");
    }
    free_step(S);
    return rc;
}

cm_status cm_step_run(cm_step *S, const cm_batch *b, const float *U, int32_t k, float *cost_out,
                      int32_t *idx_out, float *val_out, cm_stream stream)
{
    if (!S) return fail(CM_EINVAL, "step is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    return run_locked(*S, b, U, k, cost_out, idx_out, val_out, (hipStream_t)stream);
}

cm_status cm_step_set_config(cm_step *S, const cm_step_config *c)
{
    if (!S) return fail(CM_EINVAL, "step is NULL");
    cm_status rc = check_config(c);
    if (rc != CM_OK) return rc;
    std::lock_guard<std::mutex> lk(S->mu);
    S->cfg = *c;
    return CM_OK;
}

cm_status cm_step_get_config(const cm_step *S, cm_step_config *c)
{
    if (!S || !c) return fail(CM_EINVAL, "NULL argument");
    *c = S->cfg;
    if (c->grid == 0) c->grid = grid_of(*S);
    return CM_OK;
}

cm_status cm_step_autotune(cm_step *S, const cm_batch *b, const float *U, int32_t k,
                           float *cost_out, int32_t *idx_out, float *val_out, cm_stream stream,
                           int32_t reps, cm_step_config *best, float *best_us)
{
    if (!S) return fail(CM_EINVAL, "step is NULL");
    if (reps < 1 || reps > 1000) return fail(CM_EINVAL, "reps %d outside [1, 1000]", reps);
    hipStream_t st = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(S->mu);
    cm_status rc = check_step_batch(*S, b, U, k, cost_out, idx_out, val_out);
    if (rc != CM_OK) return rc;
    const cm_step_config saved = S->cfg;
    std::vector<cm_step_config> cands;
    for (int graph : {1, 0})
        for (int gm : {1, 2, 4})
            for (int gt : {1, 2, 4, 8}) cands.push_back(cm_step_config{gm * S->cus, gt, graph});
    std::vector<hipEvent_t> ev(2 * (size_t)reps, nullptr);
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
            rc = fail(CM_EDEVICE, "event creation failed");
        }
    float best_t = 0.f;
    cm_step_config best_c = saved;
    for (size_t c = 0; c < cands.size() && rc == CM_OK; ++c) {
        S->cfg = cands[c];
        if ((rc = run_locked(*S, b, U, k, cost_out, idx_out, val_out, st)) != CM_OK) break;
        for (int r = 0; r < reps && rc == CM_OK; ++r) {
            if (hipEventRecord(ev[2 * r], st) != hipSuccess)
                rc = fail(CM_EDEVICE, "event record failed");
            else if ((rc = run_locked(*S, b, U, k, cost_out, idx_out, val_out, st)) == CM_OK &&
                     hipEventRecord(ev[2 * r + 1], st) != hipSuccess)
                rc = fail(CM_EDEVICE, "event record failed");
        }
        if (rc != CM_OK) break;
        if (hipStreamSynchronize(st) != hipSuccess) {
            rc = fail(CM_EDEVICE, "stream synchronisation failed");
            break;
        }
        std::vector<float> ts(reps);
        for (int r = 0; r < reps; ++r)
            if (hipEventElapsedTime(&ts[r], ev[2 * r], ev[2 * r + 1]) != hipSuccess)
                rc = fail(CM_EDEVICE, "event timing failed");
        if (rc != CM_OK) break;
        std::nth_element(ts.begin(), ts.begin() + reps / 2, ts.end());
        const float med = ts[reps / 2] * 1000.f;
        if (c == 0 || med < best_t) {
            best_t = med;
            best_c = cands[c];
        }
    }
    for (auto e : ev)
        if (e) (void)hipEventDestroy(e);
    S->cfg = rc == CM_OK ? best_c : saved;
    if (rc == CM_OK) {
        if (best) *best = best_c;
        if (best_us) *best_us = best_t;
        int64_t rows = 0;
        for (int32_t q = 0; q < b->n_queries; ++q)
            rows += (int64_t)b->queries[q].n_stages * b->queries[q].n_cands;
        std::lock_guard<std::mutex> tl(g_tune_mu);
        tune_load_locked();
        g_tune[tune_key(S->arch, S->prec, ceil_log2(b->n_queries), ceil_log2(rows))] =
            TuneEntry{best_c, best_t};
        tune_save_locked();
    }
    return rc;
}

cm_status cm_step_tuned_config(const cm_step *S, int32_t n_queries, int64_t rows,
                               cm_step_config *out)
{
    if (!S || !out) return fail(CM_EINVAL, "NULL argument");
    if (n_queries < 1) return fail(CM_EINVAL, "n_queries %d < 1", n_queries);
    const int qb = ceil_log2(n_queries), rb = rows > 0 ? ceil_log2(rows) : -1;
    std::lock_guard<std::mutex> tl(g_tune_mu);
    tune_load_locked();
    // the nearest bucket of this architecture and precision: closest query
    // bucket first, then closest row bucket (the largest when rows <= 0)
    const std::string head = tune_key(S->arch, S->prec, 0, 0);
    const std::string prefix = head.substr(0, head.size() - 3);  // "arch prec "
    const TuneEntry *best = nullptr;
    int64_t best_d = 0;
    for (const auto &kv : g_tune) {
        if (kv.first.compare(0, prefix.size(), prefix) != 0) continue;
        int eq = 0, er = 0;
        if (std::sscanf(kv.first.c_str() + prefix.size(), "%d %d", &eq, &er) != 2) continue;
        const int64_t d = (int64_t)std::abs(eq - qb) * 4096 + (rb >= 0 ? std::abs(er - rb) : 64 - er);
        if (!best || d < best_d) {
            best = &kv.second;
            best_d = d;
        }
    }
    if (!best) return fail(CM_ENOTFOUND, "no tuned configuration for %s", prefix.c_str());
    *out = best->cfg;
    return CM_OK;
}

}  // extern "C"
