// cm_serve.hip -- the serving loop (include/cm.h): sessions with
// device-resident hoisted rows and beams, FIFO admission by arena bytes and
// free slots, micro-batches as persistent steps on per-slot streams, a native
// worker thread, latency statistics.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "cm_internal.h"

namespace {

using cm::fail;
using Clock = std::chrono::steady_clock;

constexpr int MAX_SERVER_SLOTS = 8;

enum class St { Pending, Admitted, Done, Canceled, Failed };

struct Req {
    int32_t session = -1;
    int32_t N = 0, k = 0, S = 0;
    const void *x = nullptr;  // bf16 bits or e4m3 codes, as the server's precision
    const float *t = nullptr;
    int64_t bytes = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    St state = St::Pending;
    std::vector<int32_t> idx;
    std::vector<float> val;
};

struct Session {
    bool used = false;
    bool closing = false;  // closed by the caller, request still in flight
    int32_t S = 0;
    bool busy = false;     // a request of this session is admitted
};

struct SlotState {
    hipStream_t st = nullptr;
    cm_step *step = nullptr;
    float *d_cost = nullptr;
    // the beams of a micro-batch, query j at word 2 j kb: kb indices, then
    // kb values (one copy to the host covers the whole micro-batch)
    uint32_t *d_beam = nullptr;
    uint32_t *h_beam = nullptr;  // pinned
    uint64_t *h_clk = nullptr; // pinned: the step kernel's (first start, last end)
    hipEvent_t done = nullptr;
    bool busy = false;
    int32_t kb = 0;            // beam width of the micro-batch (the server's k)
    std::vector<uint64_t> tickets;
    int64_t bytes = 0, rows = 0, cands = 0;
};

double us_since(Clock::time_point t0)
{
    return std::chrono::duration<double, std::micro>(Clock::now() - t0).count();
}

}  // namespace

struct cm_server {
    const cm_model *model = nullptr;
    cm_server_cfg cfg{};
    int device = 0;
    Clock::time_point t0;

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

    SlotState slot[MAX_SERVER_SLOTS];

    std::mutex mu;                  // everything below
    std::condition_variable cv_work, cv_done;
    std::vector<Session> sessions;
    std::unordered_map<uint64_t, Req> reqs;
    std::deque<uint64_t> pending;
    uint64_t next_ticket = 1;
    int64_t arena_in_use = 0, arena_high = 0;
    int32_t in_flight = 0;
    bool stop = false;
    cm_status fault = CM_OK;
    std::string fault_msg;
    // statistics
    int64_t n_sub = 0, n_done = 0, n_cancel = 0, n_cands = 0, n_rows = 0, n_mb = 0;
    double first_submit = -1, last_done = 0, kernel_us = 0;
    int64_t kernel_bytes = 0;
    std::vector<double> lat;

    std::thread worker;
};

namespace {

// Feature bytes per row: bf16 bits or e4m3 codes.
int64_t feature_bytes(cm_precision prec) { return prec == CM_FP8 ? cm::FS : cm::FS * 2; }

int64_t request_bytes(cm_precision prec, int32_t S, int32_t N, int32_t k)
{
    return (int64_t)S * N * (feature_bytes(prec) + cm::C * 4) + (int64_t)N * 4 + (int64_t)k * 8;
}

void free_server(cm_server *V)
{
    for (auto &s : V->slot) {
        if (s.step) (void)cm_step_destroy(s.step);
        if (s.st) (void)hipStreamDestroy(s.st);
        if (s.d_cost) (void)hipFree(s.d_cost);
        if (s.d_beam) (void)hipFree(s.d_beam);
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

float *session_U(cm_server &V, int32_t s)
{
    return V.d_U + (int64_t)s * V.cfg.max_stages * cm::H;
}

// Fail every queued and admitted request after a device error (mu held).
void set_fault(cm_server &V, const char *what, hipError_t e)
{
    if (V.fault == CM_OK) {
        V.fault = CM_EDEVICE;
        V.fault_msg = std::string(what) + ": " + hipGetErrorString(e);
    }
    for (auto &kv : V.reqs)
        if (kv.second.state == St::Pending || kv.second.state == St::Admitted)
            kv.second.state = St::Failed;
    V.pending.clear();
    V.cv_done.notify_all();
}

// Retire a finished micro-batch (mu held).
void retire(cm_server &V, SlotState &sl)
{
    V.kernel_us += (double)(sl.h_clk[1] - sl.h_clk[0]) / cm::CLOCK_MHZ;
    V.kernel_bytes += sl.rows * (feature_bytes(V.cfg.precision) + cm::C * 4) + sl.cands * 4;
    const double now = us_since(V.t0);
    for (size_t j = 0; j < sl.tickets.size(); ++j) {
        auto it = V.reqs.find(sl.tickets[j]);
        if (it == V.reqs.end()) continue;
        Req &r = it->second;
        Session &ss = V.sessions[r.session];
        ss.busy = false;
        if (ss.closing) {
            ss.closing = false;
            ss.used = false;
        }
        V.arena_in_use -= r.bytes;
        --V.in_flight;
        if (r.state != St::Admitted) continue;
        const uint32_t *b = sl.h_beam + (size_t)j * 2 * sl.kb;
        r.idx.resize(r.k);
        r.val.resize(r.k);
        std::memcpy(r.idx.data(), b, (size_t)r.k * 4);
        std::memcpy(r.val.data(), b + sl.kb, (size_t)r.k * 4);
        r.t_done = now;
        r.state = St::Done;
        ++V.n_done;
        V.n_cands += r.N;
        V.n_rows += (int64_t)r.N * r.S;
        V.lat.push_back(r.t_done - r.t_submit);
        V.last_done = now;
    }
    sl.tickets.clear();
    sl.busy = false;
    V.cv_done.notify_all();
}

// Admit queued requests into one micro-batch on `sl` and launch it (mu held).
// Returns false when nothing could be admitted.
bool admit(cm_server &V, SlotState &sl)
{
    std::vector<uint64_t> take;
    std::vector<int32_t> in_batch;
    int64_t bytes = 0, cands = 0, rows = 0;
    // every micro-batch selects the server's k (a session's beam has k
    // entries); a request's smaller k is a prefix of that sorted beam
    const int32_t kb = V.cfg.k;
    for (auto it = V.pending.begin(); it != V.pending.end(); ++it) {
        Req &r = V.reqs[*it];
        Session &ss = V.sessions[r.session];
        if (ss.busy || std::find(in_batch.begin(), in_batch.end(), r.session) != in_batch.end())
            continue;  // one beam step of a session at a time
        if (V.arena_in_use + bytes + r.bytes > V.cfg.arena_bytes) break;  // FIFO on memory
        if ((int32_t)take.size() == V.cfg.max_batch_queries ||
            cands + r.N > V.cfg.max_batch_cands)
            break;
        take.push_back(*it);
        in_batch.push_back(r.session);
        bytes += r.bytes;
        cands += r.N;
        rows += (int64_t)r.N * r.S;
    }
    if (take.empty()) return false;
    const double now = us_since(V.t0);
    std::vector<cm::StepReq> sr(take.size());
    int64_t off = 0;
    for (size_t j = 0; j < take.size(); ++j) {
        Req &r = V.reqs[take[j]];
        V.pending.erase(std::find(V.pending.begin(), V.pending.end(), take[j]));
        V.sessions[r.session].busy = true;
        r.state = St::Admitted;
        r.t_admit = now;
        cm::StepReq &q = sr[j];
        q.x = r.x;
        q.t = r.t;
        q.u = session_U(V, r.session);
        q.pipe = nullptr;
        q.cost = sl.d_cost + off;
        q.idx = reinterpret_cast<int32_t *>(sl.d_beam + (int64_t)j * 2 * kb);
        q.val = reinterpret_cast<float *>(sl.d_beam + (int64_t)j * 2 * kb + kb);
        q.sidx = V.d_beam_idx + (int64_t)r.session * V.cfg.k;
        q.sval = V.d_beam_val + (int64_t)r.session * V.cfg.k;
        q.S = r.S;
        q.N = r.N;
        off += r.N;
    }
    V.arena_in_use += bytes;
    V.arena_high = std::max(V.arena_high, V.arena_in_use);
    V.in_flight += (int32_t)take.size();
    sl.tickets = take;
    sl.kb = kb;
    sl.bytes = bytes;
    sl.rows = rows;
    sl.cands = cands;
    sl.busy = true;
    ++V.n_mb;
    cm_status rc = cm::step_launch(sl.step, sr.data(), (int)sr.size(), kb, false, sl.st);
    hipError_t e = rc == CM_OK ? hipSuccess : hipErrorLaunchFailure;
    const size_t nb = take.size() * (size_t)kb;
    if (e == hipSuccess)
        e = hipMemcpyAsync(sl.h_beam, sl.d_beam, 2 * nb * sizeof(uint32_t), hipMemcpyDeviceToHost,
                           sl.st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(sl.h_clk, cm::step_clock(sl.step), 2 * sizeof(uint64_t),
                           hipMemcpyDeviceToHost, sl.st);
    if (e == hipSuccess) e = hipEventRecord(sl.done, sl.st);
    if (e != hipSuccess) set_fault(V, "micro-batch launch", e);
    return true;
}

void worker_main(cm_server *Vp)
{
    cm_server &V = *Vp;
    (void)hipSetDevice(V.device);
    std::unique_lock<std::mutex> lk(V.mu);
    for (;;) {
        bool progress = false;
        bool any_busy = false;
        for (int i = 0; i < V.cfg.max_slots; ++i) {
            SlotState &sl = V.slot[i];
            if (!sl.busy) continue;
            const hipError_t e = hipEventQuery(sl.done);
            if (e == hipSuccess) {
                retire(V, sl);
                progress = true;
            } else if (e != hipErrorNotReady) {
                set_fault(V, "micro-batch", e);
                sl.busy = false;
                sl.tickets.clear();
            } else {
                any_busy = true;
            }
        }
        if (V.fault == CM_OK)
            for (int i = 0; i < V.cfg.max_slots && !V.pending.empty(); ++i)
                if (!V.slot[i].busy && admit(V, V.slot[i])) {
                    progress = true;
                    any_busy = true;
                }
        if (V.stop && V.pending.empty() && !any_busy) break;
        if (progress) continue;
        if (!any_busy) {
            V.cv_work.wait(lk);  // nothing on the device: sleep until a submission
        } else {
            // work on the device: look again soon, without holding the lock
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        }
    }
}

cm_status check_cfg(const cm_server_cfg *c)
{
    if (!c) return fail(CM_EINVAL, "cfg is NULL");
    if (c->precision != CM_BF16 && c->precision != CM_FP8)
        return fail(CM_EUNSUPPORTED, "the server supports CM_BF16 and CM_FP8 only");
    if (c->k < 1 || c->k > CM_MAX_K) return fail(CM_EINVAL, "k outside [1, %d]", CM_MAX_K);
    if (c->max_slots < 1 || c->max_slots > MAX_SERVER_SLOTS)
        return fail(CM_EINVAL, "max_slots outside [1, %d]", MAX_SERVER_SLOTS);
    if (c->max_pending < 1 || c->max_sessions < 1 || c->max_stages < 1 ||
        c->max_batch_queries < 1 || c->max_batch_queries > CM_STEP_MAX_QUERIES ||
        c->max_batch_cands < 1 || c->max_batch_cands > INT32_MAX || c->arena_bytes < 1)
        return fail(CM_EINVAL, "bad server capacities");
    if ((int64_t)c->max_sessions * c->max_stages > ((int64_t)1 << 31))
        return fail(CM_EINVAL, "session pool too large");
    return CM_OK;
}

// Checks of a request against the server and its session (mu held).
cm_status check_request(cm_server &V, int32_t sid, const cm_request *rq)
{
    if (!rq) return fail(CM_EINVAL, "request is NULL");
    if (rq->n_cands < 0) return fail(CM_EINVAL, "n_cands < 0");
    if (rq->k < 1 || rq->k > V.cfg.k) return fail(CM_EINVAL, "k=%d outside [1, %d]", rq->k, V.cfg.k);
    if (rq->n_cands > 0) {
        if (!rq->sched || !rq->terms) return fail(CM_EINVAL, "sched or terms is NULL");
        if ((uintptr_t)rq->sched % 16 || (uintptr_t)rq->terms % 16)
            return fail(CM_EINVAL, "sched and terms must be 16-byte aligned");
    }
    if (rq->n_cands > V.cfg.max_batch_cands)
        return fail(CM_E2BIG, "%d candidates, a micro-batch holds %lld", rq->n_cands,
                    (long long)V.cfg.max_batch_cands);
    if (V.fault != CM_OK) return fail(V.fault, "%s", V.fault_msg.c_str());
    if (V.stop) return fail(CM_ECANCELED, "the server is stopping");
    if (sid < 0 || sid >= (int32_t)V.sessions.size() || !V.sessions[sid].used ||
        V.sessions[sid].closing)
        return fail(CM_ENOTFOUND, "no open session %d", sid);
    const cm_status st =
        cm::check_query_bytes(0, V.sessions[sid].S, rq->n_cands, V.cfg.precision, false);
    if (st != CM_OK) return st;
    const int64_t bytes = request_bytes(V.cfg.precision, V.sessions[sid].S, rq->n_cands, rq->k);
    if (bytes > V.cfg.arena_bytes)
        return fail(CM_E2BIG, "request needs %lld arena bytes, the arena has %lld",
                    (long long)bytes, (long long)V.cfg.arena_bytes);
    return CM_OK;
}

// Queue a checked request (mu held); returns its ticket.
uint64_t enqueue(cm_server &V, int32_t sid, const cm_request *rq)
{
    const uint64_t id = V.next_ticket++;
    Req &r = V.reqs[id];
    r.session = sid;
    r.N = rq->n_cands;
    r.k = rq->k;
    r.S = V.sessions[sid].S;
    r.x = rq->sched;
    r.t = rq->terms;
    r.bytes = request_bytes(V.cfg.precision, r.S, r.N, r.k);
    r.t_submit = us_since(V.t0);
    if (V.first_submit < 0) V.first_submit = r.t_submit;
    ++V.n_sub;
    V.pending.push_back(id);
    return id;
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
    V->t0 = Clock::now();
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
        SlotState &s = V->slot[i];
        const size_t nb = (size_t)c.max_batch_queries * c.k;
        ok = ok && hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipMalloc((void **)&s.d_cost, (size_t)c.max_batch_cands * 4) == hipSuccess;
        ok = ok && hipMalloc((void **)&s.d_beam, 2 * nb * 4) == hipSuccess;
        ok = ok && hipHostMalloc((void **)&s.h_beam, 2 * nb * 4, 0) == hipSuccess;
        ok = ok && hipHostMalloc((void **)&s.h_clk, 16, 0) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&s.done, hipEventDisableTiming) == hipSuccess;
        if (ok) {
            const cm_step_desc sd{c.max_batch_queries, 1, c.max_batch_cands, c.k, 1};
            ok = cm_step_create(model, cfg->precision, &sd, &s.step) == CM_OK;
        }
    }
    if (!ok) {
        (void)hipGetLastError();
        free_server(V);
        return fail(CM_ENOMEM, "server allocation failed");
    }
    for (int j = 0; j < c.k; ++j) {
        V->h_beam_init[j] = -1;
        const float inf = __builtin_inff();
        std::memcpy(&V->h_beam_init[c.k + j], &inf, 4);
    }
    V->sessions.resize(c.max_sessions);
    try {
        V->worker = std::thread(worker_main, V);
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
    {
        std::lock_guard<std::mutex> lk(V->mu);
        V->stop = true;
    }
    V->cv_work.notify_all();
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
    {
        std::lock_guard<std::mutex> lk(V->mu);
        if (V->fault != CM_OK) return fail(V->fault, "%s", V->fault_msg.c_str());
        for (int32_t s = 0; s < (int32_t)V->sessions.size(); ++s)
            if (!V->sessions[s].used) {
                sid = s;
                break;
            }
        if (sid < 0) return fail(CM_EAGAIN, "no free session");
        V->sessions[sid] = Session{};
        V->sessions[sid].used = true;
        V->sessions[sid].closing = true;  // not usable until set up
        V->sessions[sid].S = n_stages;
    }
    cm_status rc = CM_OK;
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
    std::lock_guard<std::mutex> lk(V->mu);
    if (rc != CM_OK) {
        V->sessions[sid].used = false;
        V->sessions[sid].closing = false;
        return rc;
    }
    V->sessions[sid].closing = false;
    *session_out = sid;
    return CM_OK;
}

cm_status cm_session_close(cm_server *V, int32_t sid)
{
    if (!V) return fail(CM_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(V->mu);
    if (sid < 0 || sid >= (int32_t)V->sessions.size() || !V->sessions[sid].used ||
        V->sessions[sid].closing)
        return fail(CM_ENOTFOUND, "no open session %d", sid);
    for (auto it = V->pending.begin(); it != V->pending.end();) {
        Req &r = V->reqs[*it];
        if (r.session == sid) {
            r.state = St::Canceled;
            ++V->n_cancel;
            it = V->pending.erase(it);
        } else {
            ++it;
        }
    }
    if (V->sessions[sid].busy) V->sessions[sid].closing = true;  // freed when it retires
    else V->sessions[sid].used = false;
    V->cv_done.notify_all();
    return CM_OK;
}

cm_status cm_session_beam(cm_server *V, int32_t sid, int32_t k, int32_t *idx, float *val)
{
    if (!V || !idx || !val) return fail(CM_EINVAL, "NULL argument");
    if (k < 1 || k > V->cfg.k) return fail(CM_EINVAL, "k=%d outside [1, %d]", k, V->cfg.k);
    {
        std::lock_guard<std::mutex> lk(V->mu);
        if (sid < 0 || sid >= (int32_t)V->sessions.size() || !V->sessions[sid].used ||
            V->sessions[sid].closing)
            return fail(CM_ENOTFOUND, "no open session %d", sid);
        if (V->sessions[sid].busy) return fail(CM_EAGAIN, "a request of session %d is in flight", sid);
    }
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
    std::lock_guard<std::mutex> lk(V->mu);
    cm_status rc = check_request(*V, sid, rq);
    if (rc != CM_OK) return rc;
    if ((int32_t)V->pending.size() >= V->cfg.max_pending)
        return fail(CM_EAGAIN, "queue full (%d requests)", V->cfg.max_pending);
    *ticket = enqueue(*V, sid, rq);
    V->cv_work.notify_one();
    return CM_OK;
}

cm_status cm_serve_submit_batch(cm_server *V, int32_t n, const int32_t *sessions,
                                const cm_request *reqs, uint64_t *tickets)
{
    if (!V || n < 0 || (n > 0 && (!sessions || !reqs || !tickets)))
        return fail(CM_EINVAL, "NULL argument or n < 0");
    std::lock_guard<std::mutex> lk(V->mu);
    for (int32_t j = 0; j < n; ++j) {
        cm_status rc = check_request(*V, sessions[j], &reqs[j]);
        if (rc != CM_OK) return rc;
    }
    if ((int64_t)V->pending.size() + n > V->cfg.max_pending)
        return fail(CM_EAGAIN, "queue full (%d requests)", V->cfg.max_pending);
    for (int32_t j = 0; j < n; ++j) tickets[j] = enqueue(*V, sessions[j], &reqs[j]);
    V->cv_work.notify_one();
    return CM_OK;
}

}  // extern "C"

namespace {

// The ticket's state as a status, copying a finished result (mu held).
cm_status poll_locked(cm_server &V, uint64_t ticket, cm_result *out)
{
    auto it = V.reqs.find(ticket);
    if (it == V.reqs.end()) return fail(CM_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Req &r = it->second;
    switch (r.state) {
    case St::Pending:
    case St::Admitted:
        return CM_EAGAIN;
    case St::Canceled:
        V.reqs.erase(it);
        return fail(CM_ECANCELED, "request %llu was canceled", (unsigned long long)ticket);
    case St::Failed:
        return fail(CM_EDEVICE, "%s", V.fault_msg.c_str());
    case St::Done:
        break;
    }
    if (out->k < r.k || !out->idx || !out->val)
        return fail(CM_EINVAL, "result capacity %d below the request's k %d", out->k, r.k);
    std::memcpy(out->idx, r.idx.data(), (size_t)r.k * 4);
    std::memcpy(out->val, r.val.data(), (size_t)r.k * 4);
    out->n = r.k;
    out->t_submit_us = r.t_submit;
    out->t_admit_us = r.t_admit;
    out->t_done_us = r.t_done;
    V.reqs.erase(it);
    return CM_OK;
}

}  // namespace

extern "C" {

cm_status cm_serve_poll(cm_server *V, uint64_t ticket, cm_result *out)
{
    if (!V || !out) return fail(CM_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(V->mu);
    return poll_locked(*V, ticket, out);
}

cm_status cm_serve_wait(cm_server *V, uint64_t ticket, int32_t timeout_ms, cm_result *out)
{
    if (!V || !out) return fail(CM_EINVAL, "NULL argument");
    if (timeout_ms < 0) return fail(CM_EINVAL, "timeout_ms < 0");
    const auto until = Clock::now() + std::chrono::milliseconds(timeout_ms);
    std::unique_lock<std::mutex> lk(V->mu);
    for (;;) {
        const cm_status rc = poll_locked(*V, ticket, out);
        if (rc != CM_EAGAIN) return rc;
        if (V->cv_done.wait_until(lk, until) == std::cv_status::timeout) {
            const cm_status rc2 = poll_locked(*V, ticket, out);
            return rc2 == CM_EAGAIN ? fail(CM_EAGAIN, "timed out") : rc2;
        }
    }
}

cm_status cm_serve_wait_all(cm_server *V, int32_t n, const uint64_t *tickets, int32_t timeout_ms,
                            cm_result *outs)
{
    if (!V || n < 0 || (n > 0 && !tickets)) return fail(CM_EINVAL, "NULL argument or n < 0");
    if (timeout_ms < 0) return fail(CM_EINVAL, "timeout_ms < 0");
    const auto until = Clock::now() + std::chrono::milliseconds(timeout_ms);
    std::unique_lock<std::mutex> lk(V->mu);
    for (;;) {
        bool all = true;
        for (int32_t j = 0; j < n && all; ++j) {
            auto it = V->reqs.find(tickets[j]);
            if (it == V->reqs.end())
                return fail(CM_ENOTFOUND, "unknown ticket %llu", (unsigned long long)tickets[j]);
            all = it->second.state != St::Pending && it->second.state != St::Admitted;
        }
        if (all) break;
        if (V->cv_done.wait_until(lk, until) == std::cv_status::timeout) {
            bool again = false;
            for (int32_t j = 0; j < n && !again; ++j) {
                auto it = V->reqs.find(tickets[j]);
                again = it != V->reqs.end() &&
                        (it->second.state == St::Pending || it->second.state == St::Admitted);
            }
            if (again) return fail(CM_EAGAIN, "timed out");
            break;
        }
    }
    cm_status first = CM_OK;
    for (int32_t j = 0; j < n; ++j) {
        cm_status rc;
        if (outs) {
            rc = poll_locked(*V, tickets[j], &outs[j]);
        } else {
            auto it = V->reqs.find(tickets[j]);
            if (it == V->reqs.end()) {
                rc = fail(CM_ENOTFOUND, "unknown ticket %llu", (unsigned long long)tickets[j]);
            } else if (it->second.state == St::Done || it->second.state == St::Canceled) {
                rc = it->second.state == St::Done ? CM_OK : CM_ECANCELED;
                V->reqs.erase(it);
            } else {
                rc = fail(CM_EDEVICE, "%s", V->fault_msg.c_str());
            }
        }
        if (rc != CM_OK && first == CM_OK) first = rc;
    }
    return first;
}

cm_status cm_server_get_stats(cm_server *V, cm_server_stats *o)
{
    if (!V || !o) return fail(CM_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(V->mu);
    std::memset(o, 0, sizeof *o);
    o->submitted = V->n_sub;
    o->completed = V->n_done;
    o->canceled = V->n_cancel;
    o->candidates = V->n_cands;
    o->rows = V->n_rows;
    o->micro_batches = V->n_mb;
    o->wall_us = V->first_submit >= 0 ? std::max(0.0, V->last_done - V->first_submit) : 0.0;
    o->cands_per_s = o->wall_us > 0 ? (double)V->n_cands / (o->wall_us * 1e-6) : 0.0;
    if (!V->lat.empty()) {
        std::vector<double> l = V->lat;
        std::sort(l.begin(), l.end());
        auto pct = [&](double p) {
            const size_t i = (size_t)std::min<double>(l.size() - 1, std::ceil(p * l.size()) - 1);
            return l[i];
        };
        o->p50_us = pct(0.50);
        o->p99_us = pct(0.99);
        o->max_us = l.back();
    }
    o->queue_depth = (int32_t)V->pending.size();
    o->in_flight = V->in_flight;
    o->arena_in_use = V->arena_in_use;
    o->arena_high_water = V->arena_high;
    o->kernel_us = V->kernel_us;
    o->kernel_bytes = V->kernel_bytes;
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

cm_status cm_server_reset_stats(cm_server *V)
{
    if (!V) return fail(CM_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(V->mu);
    V->n_sub = V->n_done = V->n_cancel = V->n_cands = V->n_rows = V->n_mb = 0;
    V->first_submit = -1;
    V->last_done = 0;
    V->kernel_us = 0;
    V->kernel_bytes = 0;
    V->arena_high = V->arena_in_use;
    V->lat.clear();
    return CM_OK;
}

}  // extern "C"
