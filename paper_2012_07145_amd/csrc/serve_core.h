// serve_core.h -- the host side of the serving loop (include/cm.h, cm_server_*):
// sessions, the FIFO of queued requests, admission by free slots and arena
// bytes, ticket states, micro-batch retirement, latency statistics and the
// worker loop.  Plain C++17 with no HIP header: the device work sits behind
// the Executor interface (cm_serve.hip implements it with persistent steps on
// HIP streams), so this core also builds and runs on the CPU with a fake
// executor, under the address and thread sanitizers.
//
// Each search session runs the beam search of Sec. 4 over one pipeline and
// submits one query per beam step (Sec. 4.4: the options it selected are
// featurized and evaluated, then added to the beam); a session's steps depend
// on each other, so a session has at most one request admitted at a time.
#pragma once

#include <stdint.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "cm.h"

namespace cm {
namespace serve {

constexpr int MAX_SLOTS = 8;

// One admitted request as the executor sees it.
struct Work {
    uint64_t ticket;
    int32_t session;
    int32_t S, N;        // the session's stages, the request's candidates
    const void *x;       // features (caller's device memory)
    const float *t;      // cost terms (caller's device memory)
};

// The device side: one micro-batch in flight per slot.
class Executor {
public:
    virtual ~Executor() = default;
    // Queue `batch` as one micro-batch on `slot`, each query selecting its kb
    // best.  False (with *err) if it could not be queued.
    virtual bool launch(int slot, const std::vector<Work> &batch, int32_t kb,
                        std::string *err) = 0;
    // 1: the slot's micro-batch has finished; 0: still running; -1: failed
    // (with *err).
    virtual int poll(int slot, std::string *err) = 0;
    // Beam of query j of the slot's finished micro-batch: kb indices, then kb
    // values (as uint32 bits), valid until the slot's next launch.
    virtual const uint32_t *beam(int slot, size_t j) = 0;
    // GPU time (microseconds) of the slot's finished micro-batch's kernel.
    virtual double kernel_us(int slot) = 0;
    // Device clock (microseconds from an arbitrary origin) of that kernel's
    // first wave start and last wave end.
    virtual void kernel_clock(int slot, double *start_us, double *end_us) = 0;
    // Whether launch() may be called from the calling thread as well as from
    // the worker (which always may).
    virtual bool launch_here() { return true; }
};

// Bytes a request takes from the arena while admitted.
int64_t request_bytes(cm_precision prec, int32_t S, int32_t N, int32_t k);

class Core {
public:
    using Clock = std::chrono::steady_clock;

    // cfg must have been validated; ex must outlive the core.
    Core(const cm_server_cfg &cfg, Executor *ex);

    // ---- sessions
    // Reserve a session of S stages (not usable until session_ready).
    cm_status session_reserve(int32_t S, int32_t *sid, std::string *err);
    // Finish a reservation: ok = its device state is in place.
    void session_ready(int32_t sid, bool ok);
    // Close: queued requests are canceled; an admitted one still completes.
    cm_status session_close(int32_t sid, std::string *err);
    // CM_OK when the session is open and idle (its beam may be read).
    cm_status session_idle(int32_t sid, std::string *err);

    // ---- requests
    // Validate and queue (the checks and errors of cm_serve_submit).
    cm_status submit(int32_t sid, const cm_request *rq, uint64_t *ticket, std::string *err);
    cm_status submit_batch(int32_t n, const int32_t *sessions, const cm_request *reqs,
                           uint64_t *tickets, std::string *err);
    cm_status poll(uint64_t ticket, cm_result *out, std::string *err);
    cm_status wait(uint64_t ticket, int32_t timeout_ms, cm_result *out, std::string *err);
    cm_status wait_all(int32_t n, const uint64_t *tickets, int32_t timeout_ms, cm_result *outs,
                       std::string *err);

    // ---- statistics
    void stats(cm_server_stats *out);
    void reset_stats();

    // ---- worker
    // The worker loop: admits queued requests into free slots, retires
    // finished micro-batches; returns after stop() once nothing is queued or
    // in flight (or the server has failed).
    void run();
    void stop();
    // The next micro-batch launch fails as if the device had refused it: the
    // server enters its failed state and every queued or admitted request
    // returns CM_EDEVICE (failure handling, forced from the host).
    void fail_next_launch();

    // Per-request check of the evaluator's size limit, set by the owner
    // (cm_serve.hip: check_query_bytes); CM_OK when unset.
    cm_status (*bytes_check)(int32_t S, int32_t N, cm_precision prec, std::string *err) = nullptr;

private:
    enum class St { Pending, Admitted, Done, Canceled, Failed };
    struct Req {
        int32_t session = -1;
        int32_t N = 0, k = 0, S = 0;
        const void *x = nullptr;
        const float *t = nullptr;
        int64_t bytes = 0;
        double t_submit = 0, t_admit = 0, t_done = 0;
        St state = St::Pending;
        std::vector<int32_t> idx;
        std::vector<float> val;
    };
    struct Session {
        bool used = false;
        bool closing = false;  // closed by the caller (or being set up)
        bool busy = false;     // a request of this session is admitted
        int32_t S = 0;
    };
    struct Slot {
        bool busy = false;
        int32_t kb = 0;
        std::vector<uint64_t> tickets;
        int64_t rows = 0, cands = 0;
    };

    double now_us() const;
    cm_status check_locked(int32_t sid, const cm_request *rq, std::string *err);
    uint64_t enqueue_locked(int32_t sid, const cm_request *rq);
    cm_status poll_locked(uint64_t ticket, cm_result *out, std::string *err);
    void set_fault_locked(const std::string &what);
    void retire_locked(int slot);
    bool admit_locked(int slot);
    void admit_here_locked();

    const cm_server_cfg cfg_;
    Executor *const ex_;
    const Clock::time_point t0_;

    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::vector<Session> sessions_;
    std::unordered_map<uint64_t, Req> reqs_;
    std::deque<uint64_t> pending_;  // queued tickets, submission order
    Slot slot_[MAX_SLOTS];
    uint64_t next_ticket_ = 1;
    int64_t arena_in_use_ = 0, arena_high_ = 0;
    int32_t in_flight_ = 0;
    bool stop_ = false;
    bool fail_next_ = false;
    cm_status fault_ = CM_OK;
    std::string fault_msg_;
    // statistics
    int64_t n_sub_ = 0, n_done_ = 0, n_cancel_ = 0, n_cands_ = 0, n_rows_ = 0, n_mb_ = 0;
    double first_submit_ = -1, last_done_ = 0, kernel_us_ = 0;
    double kclk_first_ = -1, kclk_last_ = 0;  // kernel start / end envelope (device clock)
    // (start, end) of the most recent KRING kernels, in completion order
    static constexpr int KRING = 4096;
    std::vector<std::pair<double, double>> kring_ = std::vector<std::pair<double, double>>(KRING);
    int64_t kring_n_ = 0;
    int64_t kernel_bytes_ = 0;
    std::vector<double> lat_;
};

}  // namespace serve
}  // namespace cm
