// cm_serve.hip -- the serving loop (include/cm.h): the device side of a server
// (per-session pools of hoisted rows and beams, one persistent step, stream,
// beam buffers and completion event per slot) as the executor of the host
// core in serve_core.h, which holds the sessions, the FIFO admission by arena
// bytes and free slots, the tickets, the statistics and the worker loop.
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "cm_internal.h"
#include "serve_core.h"

namespace {

using cm::fail;

struct SlotDev {
    hipStream_t st = nullptr;
    cm_step *step = nullptr;
    float *d_cost = nullptr;
    // the beams of a micro-batch, query j at word 2 j kb: kb indices, then
    // kb values, written by the step kernel straight into pinned host memory
    uint32_t *h_beam = nullptr;
    uint64_t *h_clk = nullptr;   // pinned: the step kernel's (first start, last end)
    uint32_t *g_beam = nullptr;  // the two, as the device addresses them
    uint64_t *g_clk = nullptr;
    hipEvent_t done = nullptr;
    int32_t kb = 0;
};

}  // namespace

struct cm_server {
    const cm_model *model = nullptr;
    cm_server_cfg cfg{};
    int device = 0;

    // session pools (device): hoisted rows and latest beam of every session
    float *d_U = nullptr;           // [max_sessions][max_stages][32]
    int32_t *d_beam_idx = nullptr;  // [max_sessions][k]
    float *d_beam_val = nullptr;
    // session set-up
    hipStream_t setup = nullptr;
    float *h_pipe = nullptr;        // pinned [max_stages][56]
    float *d_pipe = nullptr;
    int32_t *h_beam_init = nullptr; // pinned: (-1) x k then (+inf) x k
    std::mutex setup_mu;

    SlotDev slot[cm::serve::MAX_SLOTS];

    cm::serve::Executor *exec = nullptr;
    cm::serve::Core *core = nullptr;
    std::thread worker;
};

namespace {

float *session_U(cm_server &V, int32_t s)
{
    return V.d_U + (int64_t)s * V.cfg.max_stages * cm::H;
}

// The device side of the server for the host core: a micro-batch is one
// persistent step (cm_step_run's kernels, hoisted rows from the session pool)
// on the slot's stream, followed by the slot's completion event.  The step
// kernel writes the micro-batch's beams and its clock pair straight into the
// slot's pinned host buffers: a copy would run as a kernel of its own, which
// cannot start while the next micro-batch's step kernel fills every compute
// unit, so the batch would complete only when that one ends.
class HipExecutor final : public cm::serve::Executor {
public:
    explicit HipExecutor(cm_server *V) : V_(V) {}

    bool launch(int si, const std::vector<cm::serve::Work> &batch, int32_t kb,
                std::string *err) override
    {
        SlotDev &sl = V_->slot[si];
        std::vector<cm::StepReq> sr(batch.size());
        int64_t off = 0;
        for (size_t j = 0; j < batch.size(); ++j) {
            const cm::serve::Work &w = batch[j];
            cm::StepReq &q = sr[j];
            q.x = w.x;
            q.t = w.t;
            q.u = session_U(*V_, w.session);
            q.pipe = nullptr;
            q.cost = sl.d_cost + off;
            q.idx = reinterpret_cast<int32_t *>(sl.g_beam + (int64_t)j * 2 * kb);
            q.val = reinterpret_cast<float *>(sl.g_beam + (int64_t)j * 2 * kb + kb);
            q.sidx = V_->d_beam_idx + (int64_t)w.session * V_->cfg.k;
            q.sval = V_->d_beam_val + (int64_t)w.session * V_->cfg.k;
            q.S = w.S;
            q.N = w.N;
            off += w.N;
        }
        sl.kb = kb;
        if (cm::step_launch(sl.step, sr.data(), (int)sr.size(), kb, false, sl.st, sl.g_clk) !=
            CM_OK) {
            *err = cm_last_error();
            return false;
        }
        const hipError_t e = hipEventRecord(sl.done, sl.st);
        if (e != hipSuccess) {
            *err = hipGetErrorString(e);
            return false;
        }
        return true;
    }

    // the slot streams and graphs belong to the server's device: a thread
    // whose current device is another one leaves the launch to the worker
    bool launch_here() override
    {
        int d = -1;
        return hipGetDevice(&d) == hipSuccess && d == V_->device;
    }

    int poll(int si, std::string *err) override
    {
        const hipError_t e = hipEventQuery(V_->slot[si].done);
        if (e == hipSuccess) return 1;
        if (e == hipErrorNotReady) return 0;
        *err = hipGetErrorString(e);
        return -1;
    }

    const uint32_t *beam(int si, size_t j) override
    {
        const SlotDev &sl = V_->slot[si];
        return sl.h_beam + j * 2 * (size_t)sl.kb;
    }

    double kernel_us(int si) override
    {
        const SlotDev &sl = V_->slot[si];
        return (double)(sl.h_clk[1] - sl.h_clk[0]) / cm::CLOCK_MHZ;
    }

    void kernel_clock(int si, double *start_us, double *end_us) override
    {
        const SlotDev &sl = V_->slot[si];
        *start_us = (double)sl.h_clk[0] / cm::CLOCK_MHZ;
        *end_us = (double)sl.h_clk[1] / cm::CLOCK_MHZ;
    }

private:
    cm_server *V_;
};

cm_status query_bytes(int32_t S, int32_t N, cm_precision prec, std::string *err)
{
    const cm_status st = cm::check_query_bytes(0, S, N, prec, false);
    if (st != CM_OK) *err = cm_last_error();
    return st;
}

void free_server(cm_server *V)
{
    delete V->core;
    delete V->exec;
    for (auto &s : V->slot) {
        if (s.step) (void)cm_step_destroy(s.step);
        if (s.st) (void)hipStreamDestroy(s.st);
        if (s.d_cost) (void)hipFree(s.d_cost);
        if (s.h_beam) (void)hipHostFree(s.h_beam);
        if (s.h_clk) (void)hipHostFree(s.h_clk);
        if (s.done) (void)hipEventDestroy(s.done);
    }
    if (V->d_U) (void)hipFree(V->d_U);
    if (V->d_beam_idx) (void)hipFree(V->d_beam_idx);
    if (V->d_beam_val) (void)hipFree(V->d_beam_val);
    if (V->setup) (void)hipStreamDestroy(V->setup);
    if (V->h_pipe) (void)hipHostFree(V->h_pipe);
    if (V->d_pipe) (void)hipFree(V->d_pipe);
    if (V->h_beam_init) (void)hipHostFree(V->h_beam_init);
    delete V;
}

cm_status check_cfg(const cm_server_cfg *c)
{
    if (!c) return fail(CM_EINVAL, "cfg is NULL");
    if (c->precision != CM_BF16 && c->precision != CM_FP8)
        return fail(CM_EUNSUPPORTED, "the server supports CM_BF16 and CM_FP8 only");
    if (c->k < 1 || c->k > CM_MAX_K) return fail(CM_EINVAL, "k outside [1, %d]", CM_MAX_K);
    if (c->max_slots < 1 || c->max_slots > cm::serve::MAX_SLOTS)
        return fail(CM_EINVAL, "max_slots outside [1, %d]", cm::serve::MAX_SLOTS);
    if (c->max_pending < 1 || c->max_sessions < 1 || c->max_stages < 1 ||
        c->max_batch_queries < 1 || c->max_batch_queries > CM_STEP_MAX_QUERIES ||
        c->max_batch_cands < 1 || c->max_batch_cands > INT32_MAX || c->arena_bytes < 1)
        return fail(CM_EINVAL, "bad server capacities");
    if ((int64_t)c->max_sessions * c->max_stages > ((int64_t)1 << 31))
        return fail(CM_EINVAL, "session pool too large");
    return CM_OK;
}

// A status of the core, with its message as the thread's last error.
cm_status from_core(cm_status st, const std::string &msg)
{
    return st == CM_OK ? st : fail(st, "%s", msg.c_str());
}

}  // namespace

extern "C" {

cm_status cm_server_create(const cm_model *model, const cm_server_cfg *cfg, cm_server **out)
{
    using namespace cm;
    if (!model || !out) return fail(CM_EINVAL, "NULL argument");
    *out = nullptr;
    cm_status rc = check_cfg(cfg);
    if (rc != CM_OK) return rc;
    cm_server *V = new (std::nothrow) cm_server;
    if (!V) return fail(CM_ENOMEM, "host allocation failed");
    V->model = model;
    V->cfg = *cfg;
    if (hipGetDevice(&V->device) != hipSuccess || V->device != model->m.device) {
        free_server(V);
        return fail(CM_EINVAL, "the model is not on the current device");
    }
    const cm_server_cfg &c = V->cfg;
    bool ok = true;
    ok = ok && hipMalloc((void **)&V->d_U, (size_t)c.max_sessions * c.max_stages * H * 4) == hipSuccess;
    ok = ok && hipMalloc((void **)&V->d_beam_idx, (size_t)c.max_sessions * c.k * 4) == hipSuccess;
    ok = ok && hipMalloc((void **)&V->d_beam_val, (size_t)c.max_sessions * c.k * 4) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&V->setup, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&V->h_pipe, (size_t)c.max_stages * FP * 4, 0) == hipSuccess;
    ok = ok && hipMalloc((void **)&V->d_pipe, (size_t)c.max_stages * FP * 4) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&V->h_beam_init, (size_t)c.k * 8, 0) == hipSuccess;
    for (int i = 0; ok && i < c.max_slots; ++i) {
        SlotDev &s = V->slot[i];
        const size_t nb = (size_t)c.max_batch_queries * c.k;
        ok = ok && hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipMalloc((void **)&s.d_cost, (size_t)c.max_batch_cands * 4) == hipSuccess;
        ok = ok && hipHostMalloc((void **)&s.h_beam, 2 * nb * 4, hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess;
        ok = ok && hipHostMalloc((void **)&s.h_clk, 16, hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess;
        ok = ok && hipHostGetDevicePointer((void **)&s.g_beam, s.h_beam, 0) == hipSuccess;
        ok = ok && hipHostGetDevicePointer((void **)&s.g_clk, s.h_clk, 0) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&s.done, hipEventDisableTiming) == hipSuccess;
        if (ok) {
            const cm_step_desc sd{c.max_batch_queries, 1, c.max_batch_cands, c.k, 1};
            ok = cm_step_create(model, cfg->precision, &sd, &s.step) == CM_OK;
        }
    }
    if (ok) {
        V->exec = new (std::nothrow) HipExecutor(V);
        V->core = V->exec ? new (std::nothrow) cm::serve::Core(c, V->exec) : nullptr;
        ok = V->core != nullptr;
    }
    if (!ok) {
        (void)hipGetLastError();
        free_server(V);
        return fail(CM_ENOMEM, "server allocation failed");
    }
    V->core->bytes_check = query_bytes;
    // a launch configuration the autotuner picked for micro-batches of this
    // size on this device and precision (tuning cache), if there is one
    cm_step_config tuned;
    if (cm_step_tuned_config(V->slot[0].step, c.max_batch_queries, 0, &tuned) == CM_OK)
        for (int i = 0; i < c.max_slots; ++i) (void)cm_step_set_config(V->slot[i].step, &tuned);
    for (int j = 0; j < c.k; ++j) {
        V->h_beam_init[j] = -1;
        const float inf = __builtin_inff();
        std::memcpy(&V->h_beam_init[c.k + j], &inf, 4);
    }
    try {
        V->worker = std::thread([V] {
            (void)hipSetDevice(V->device);
            V->core->run();
        });
    } catch (...) {
        free_server(V);
        return fail(CM_ENOMEM, "worker thread could not start");
    }
    *out = V;
    return CM_OK;
}

cm_status cm_server_destroy(cm_server *V)
{
    if (!V) return fail(CM_EINVAL, "server is NULL");
    V->core->stop();
    if (V->worker.joinable()) V->worker.join();
    cm_status rc = CM_OK;
    for (int i = 0; i < V->cfg.max_slots; ++i)
        if (V->slot[i].st && hipStreamSynchronize(V->slot[i].st) != hipSuccess)
            rc = fail(CM_EDEVICE, "waiting for the server's streams failed");
    free_server(V);
    return rc;
}

cm_status cm_session_open(cm_server *V, const float *pipe_host, int32_t n_stages,
                          int32_t *session_out)
{
    using namespace cm;
    if (!V || !pipe_host || !session_out) return fail(CM_EINVAL, "NULL argument");
    if (n_stages < 1) return fail(CM_EINVAL, "n_stages %d < 1", n_stages);
    if (n_stages > V->cfg.max_stages)
        return fail(CM_E2BIG, "%d stages, the server holds %d", n_stages, V->cfg.max_stages);
    int32_t sid = -1;
    std::string msg;
    cm_status rc = V->core->session_reserve(n_stages, &sid, &msg);
    if (rc != CM_OK) return from_core(rc, msg);
    {
        std::lock_guard<std::mutex> lk(V->setup_mu);
        std::memcpy(V->h_pipe, pipe_host, (size_t)n_stages * FP * 4);
        const cm_query q{n_stages, 0, 0, 0, 0, 0};
        const cm_batch b{1, &q, V->d_pipe, nullptr, nullptr};
        hipError_t e = hipMemcpyAsync(V->d_pipe, V->h_pipe, (size_t)n_stages * FP * 4,
                                      hipMemcpyHostToDevice, V->setup);
        if (e == hipSuccess)
            e = hipMemcpyAsync(V->d_beam_idx + (int64_t)sid * V->cfg.k, V->h_beam_init,
                               (size_t)V->cfg.k * 4, hipMemcpyHostToDevice, V->setup);
        if (e == hipSuccess)
            e = hipMemcpyAsync(V->d_beam_val + (int64_t)sid * V->cfg.k, V->h_beam_init + V->cfg.k,
                               (size_t)V->cfg.k * 4, hipMemcpyHostToDevice, V->setup);
        if (e != hipSuccess) {
            rc = fail(CM_EDEVICE, "session set-up copy failed: %s", hipGetErrorString(e));
        } else {
            rc = cm_hoist_stages(V->model, V->cfg.precision, &b, session_U(*V, sid), V->setup);
            if (rc == CM_OK && (e = hipStreamSynchronize(V->setup)) != hipSuccess)
                rc = fail(CM_EDEVICE, "session set-up failed: %s", hipGetErrorString(e));
        }
    }
    V->core->session_ready(sid, rc == CM_OK);
    if (rc != CM_OK) return rc;
    *session_out = sid;
    return CM_OK;
}

cm_status cm_session_close(cm_server *V, int32_t sid)
{
    if (!V) return fail(CM_EINVAL, "server is NULL");
    std::string msg;
    return from_core(V->core->session_close(sid, &msg), msg);
}

cm_status cm_session_beam(cm_server *V, int32_t sid, int32_t k, int32_t *idx, float *val)
{
    if (!V || !idx || !val) return fail(CM_EINVAL, "NULL argument");
    if (k < 1 || k > V->cfg.k) return fail(CM_EINVAL, "k=%d outside [1, %d]", k, V->cfg.k);
    std::string msg;
    const cm_status rc = V->core->session_idle(sid, &msg);
    if (rc != CM_OK) return from_core(rc, msg);
    std::lock_guard<std::mutex> lk(V->setup_mu);
    CM_HIP(hipMemcpyAsync(idx, V->d_beam_idx + (int64_t)sid * V->cfg.k, (size_t)k * 4,
                          hipMemcpyDeviceToHost, V->setup));
    CM_HIP(hipMemcpyAsync(val, V->d_beam_val + (int64_t)sid * V->cfg.k, (size_t)k * 4,
                          hipMemcpyDeviceToHost, V->setup));
    CM_HIP(hipStreamSynchronize(V->setup));
    return CM_OK;
}

cm_status cm_serve_submit(cm_server *V, int32_t sid, const cm_request *rq, uint64_t *ticket)
{
    if (!V || !rq || !ticket) return fail(CM_EINVAL, "NULL argument");
    std::string msg;
    return from_core(V->core->submit(sid, rq, ticket, &msg), msg);
}

cm_status cm_serve_submit_batch(cm_server *V, int32_t n, const int32_t *sessions,
                                const cm_request *reqs, uint64_t *tickets)
{
    if (!V || n < 0 || (n > 0 && (!sessions || !reqs || !tickets)))
        return fail(CM_EINVAL, "NULL argument or n < 0");
    std::string msg;
    return from_core(V->core->submit_batch(n, sessions, reqs, tickets, &msg), msg);
}

cm_status cm_serve_poll(cm_server *V, uint64_t ticket, cm_result *out)
{
    if (!V || !out) return fail(CM_EINVAL, "NULL argument");
    std::string msg;
    const cm_status rc = V->core->poll(ticket, out, &msg);
    return rc == CM_EAGAIN ? rc : from_core(rc, msg);
}

cm_status cm_serve_wait(cm_server *V, uint64_t ticket, int32_t timeout_ms, cm_result *out)
{
    if (!V || !out) return fail(CM_EINVAL, "NULL argument");
    if (timeout_ms < 0) return fail(CM_EINVAL, "timeout_ms < 0");
    std::string msg;
    return from_core(V->core->wait(ticket, timeout_ms, out, &msg), msg);
}

cm_status cm_serve_wait_all(cm_server *V, int32_t n, const uint64_t *tickets, int32_t timeout_ms,
                            cm_result *outs)
{
    if (!V || n < 0 || (n > 0 && !tickets)) return fail(CM_EINVAL, "NULL argument or n < 0");
    if (timeout_ms < 0) return fail(CM_EINVAL, "timeout_ms < 0");
    std::string msg;
    return from_core(V->core->wait_all(n, tickets, timeout_ms, outs, &msg), msg);
}

cm_status cm_server_get_stats(cm_server *V, cm_server_stats *o)
{
    if (!V || !o) return fail(CM_EINVAL, "NULL argument");
    V->core->stats(o);
    return CM_OK;
}

cm_status cm_server_reset_stats(cm_server *V)
{
    if (!V) return fail(CM_EINVAL, "server is NULL");
    V->core->reset_stats();
    return CM_OK;
}

cm_status cm_server_fail_next_launch(cm_server *V)
{
    if (!V) return fail(CM_EINVAL, "server is NULL");
    V->core->fail_next_launch();
    return CM_OK;
}

cm_status cm_server_set_step_config(cm_server *V, const cm_step_config *c)
{
    if (!V || !c) return fail(CM_EINVAL, "NULL argument");
    for (int i = 0; i < V->cfg.max_slots; ++i) {
        const cm_status rc = cm_step_set_config(V->slot[i].step, c);
        if (rc != CM_OK) return rc;
    }
    return CM_OK;
}

cm_status cm_server_get_step_config(const cm_server *V, cm_step_config *c)
{
    if (!V || !c) return fail(CM_EINVAL, "NULL argument");
    return cm_step_get_config(V->slot[0].step, c);
}

}  // extern "C"
