// serve_core.cpp -- the serving loop's host core (see serve_core.h).  No HIP.
#include "serve_core.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>

namespace cm {
namespace serve {

namespace {

int64_t feature_bytes(cm_precision prec) { return prec == CM_FP8 ? 40 : 80; }

}  // namespace

int64_t request_bytes(cm_precision prec, int32_t S, int32_t N, int32_t k)
{
    return (int64_t)S * N * (feature_bytes(prec) + 32) + (int64_t)N * 4 + (int64_t)k * 8;
}

Core::Core(const cm_server_cfg &cfg, Executor *ex) : cfg_(cfg), ex_(ex), t0_(Clock::now())
{
    sessions_.resize(cfg.max_sessions);
}

double Core::now_us() const
{
    return std::chrono::duration<double, std::micro>(Clock::now() - t0_).count();
}

// ------------------------------------------------------------ sessions

cm_status Core::session_reserve(int32_t S, int32_t *sid, std::string *err)
{
    std::lock_guard<std::mutex> lk(mu_);
    if (fault_ != CM_OK) {
        *err = fault_msg_;
        return fault_;
    }
    for (int32_t s = 0; s < (int32_t)sessions_.size(); ++s)
        if (!sessions_[s].used) {
            sessions_[s] = Session{};
            sessions_[s].used = true;
            sessions_[s].closing = true;  // not usable until set up
            sessions_[s].S = S;
            *sid = s;
            return CM_OK;
        }
    *err = "no free session";
    return CM_EAGAIN;
}

void Core::session_ready(int32_t sid, bool ok)
{
    std::lock_guard<std::mutex> lk(mu_);
    Session &s = sessions_[sid];
    s.closing = false;
    if (!ok) s.used = false;
}

cm_status Core::session_close(int32_t sid, std::string *err)
{
    std::lock_guard<std::mutex> lk(mu_);
    if (sid < 0 || sid >= (int32_t)sessions_.size() || !sessions_[sid].used ||
        sessions_[sid].closing) {
        *err = "no open session " + std::to_string(sid);
        return CM_ENOTFOUND;
    }
    std::deque<uint64_t> keep;
    for (uint64_t t : pending_) {
        Req &r = reqs_.at(t);
        if (r.session == sid) {
            r.state = St::Canceled;
            ++n_cancel_;
        } else {
            keep.push_back(t);
        }
    }
    pending_.swap(keep);
    if (sessions_[sid].busy) sessions_[sid].closing = true;  // freed when it retires
    else sessions_[sid].used = false;
    cv_done_.notify_all();
    return CM_OK;
}

cm_status Core::session_idle(int32_t sid, std::string *err)
{
    std::lock_guard<std::mutex> lk(mu_);
    if (sid < 0 || sid >= (int32_t)sessions_.size() || !sessions_[sid].used ||
        sessions_[sid].closing) {
        *err = "no open session " + std::to_string(sid);
        return CM_ENOTFOUND;
    }
    if (sessions_[sid].busy) {
        *err = "a request of session " + std::to_string(sid) + " is in flight";
        return CM_EAGAIN;
    }
    return CM_OK;
}

// ------------------------------------------------------------ requests

cm_status Core::check_locked(int32_t sid, const cm_request *rq, std::string *err)
{
    if (!rq) {
        *err = "request is NULL";
        return CM_EINVAL;
    }
    if (rq->n_cands < 0) {
        *err = "n_cands < 0";
        return CM_EINVAL;
    }
    if (rq->k < 1 || rq->k > cfg_.k) {
        *err = "k=" + std::to_string(rq->k) + " outside [1, " + std::to_string(cfg_.k) + "]";
        return CM_EINVAL;
    }
    if (rq->n_cands > 0) {
        if (!rq->sched || !rq->terms) {
            *err = "sched or terms is NULL";
            return CM_EINVAL;
        }
        if ((uintptr_t)rq->sched % 16 || (uintptr_t)rq->terms % 16) {
            *err = "sched and terms must be 16-byte aligned";
            return CM_EINVAL;
        }
    }
    if (rq->n_cands > cfg_.max_batch_cands) {
        *err = std::to_string(rq->n_cands) + " candidates, a micro-batch holds " +
               std::to_string(cfg_.max_batch_cands);
        return CM_E2BIG;
    }
    if (fault_ != CM_OK) {
        *err = fault_msg_;
        return fault_;
    }
    if (stop_) {
        *err = "the server is stopping";
        return CM_ECANCELED;
    }
    if (sid < 0 || sid >= (int32_t)sessions_.size() || !sessions_[sid].used ||
        sessions_[sid].closing) {
        *err = "no open session " + std::to_string(sid);
        return CM_ENOTFOUND;
    }
    const int32_t S = sessions_[sid].S;
    if (bytes_check) {
        const cm_status st = bytes_check(S, rq->n_cands, cfg_.precision, err);
        if (st != CM_OK) return st;
    }
    const int64_t bytes = request_bytes(cfg_.precision, S, rq->n_cands, rq->k);
    if (bytes > cfg_.arena_bytes) {
        *err = "request needs " + std::to_string(bytes) + " arena bytes, the arena has " +
               std::to_string(cfg_.arena_bytes);
        return CM_E2BIG;
    }
    return CM_OK;
}

uint64_t Core::enqueue_locked(int32_t sid, const cm_request *rq)
{
    const uint64_t id = next_ticket_++;
    Req &r = reqs_[id];
    r.session = sid;
    r.N = rq->n_cands;
    r.k = rq->k;
    r.S = sessions_[sid].S;
    r.x = rq->sched;
    r.t = rq->terms;
    r.bytes = request_bytes(cfg_.precision, r.S, r.N, r.k);
    r.t_submit = now_us();
    if (first_submit_ < 0) first_submit_ = r.t_submit;
    ++n_sub_;
    pending_.push_back(id);
    return id;
}

cm_status Core::submit(int32_t sid, const cm_request *rq, uint64_t *ticket, std::string *err)
{
    std::lock_guard<std::mutex> lk(mu_);
    const cm_status st = check_locked(sid, rq, err);
    if (st != CM_OK) return st;
    if ((int64_t)pending_.size() >= cfg_.max_pending) {
        *err = "queue full (" + std::to_string(cfg_.max_pending) + " requests)";
        return CM_EAGAIN;
    }
    *ticket = enqueue_locked(sid, rq);
    admit_here_locked();
    cv_work_.notify_one();
    return CM_OK;
}

cm_status Core::submit_batch(int32_t n, const int32_t *sessions, const cm_request *reqs,
                             uint64_t *tickets, std::string *err)
{
    std::lock_guard<std::mutex> lk(mu_);
    for (int32_t j = 0; j < n; ++j) {
        const cm_status st = check_locked(sessions[j], &reqs[j], err);
        if (st != CM_OK) return st;
    }
    if ((int64_t)pending_.size() + n > cfg_.max_pending) {
        *err = "queue full (" + std::to_string(cfg_.max_pending) + " requests)";
        return CM_EAGAIN;
    }
    for (int32_t j = 0; j < n; ++j) tickets[j] = enqueue_locked(sessions[j], &reqs[j]);
    admit_here_locked();
    cv_work_.notify_one();
    return CM_OK;
}

cm_status Core::poll_locked(uint64_t ticket, cm_result *out, std::string *err)
{
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) {
        *err = "unknown ticket " + std::to_string(ticket);
        return CM_ENOTFOUND;
    }
    Req &r = it->second;
    switch (r.state) {
    case St::Pending:
    case St::Admitted:
        return CM_EAGAIN;
    case St::Canceled:
        reqs_.erase(it);
        *err = "request " + std::to_string(ticket) + " was canceled";
        return CM_ECANCELED;
    case St::Failed:
        *err = fault_msg_;
        return CM_EDEVICE;
    case St::Done:
        break;
    }
    if (out->k < r.k || !out->idx || !out->val) {
        *err = "result capacity " + std::to_string(out->k) + " below the request's k " +
               std::to_string(r.k);
        return CM_EINVAL;
    }
    std::memcpy(out->idx, r.idx.data(), (size_t)r.k * 4);
    std::memcpy(out->val, r.val.data(), (size_t)r.k * 4);
    out->n = r.k;
    out->t_submit_us = r.t_submit;
    out->t_admit_us = r.t_admit;
    out->t_done_us = r.t_done;
    reqs_.erase(it);
    return CM_OK;
}

cm_status Core::poll(uint64_t ticket, cm_result *out, std::string *err)
{
    std::lock_guard<std::mutex> lk(mu_);
    return poll_locked(ticket, out, err);
}

// Deadline of a timed wait.  On the system clock: libstdc++ waits for a
// steady-clock deadline with pthread_cond_clockwait, which the thread
// sanitizer does not intercept (it then reports the condition variable's
// mutex as locked twice); a system-clock deadline waits with
// pthread_cond_timedwait.
static std::chrono::system_clock::time_point deadline(int32_t timeout_ms)
{
    return std::chrono::system_clock::now() + std::chrono::milliseconds(timeout_ms);
}

cm_status Core::wait(uint64_t ticket, int32_t timeout_ms, cm_result *out, std::string *err)
{
    const auto until = deadline(timeout_ms);
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
        const cm_status rc = poll_locked(ticket, out, err);
        if (rc != CM_EAGAIN) return rc;
        if (cv_done_.wait_until(lk, until) == std::cv_status::timeout) {
            const cm_status rc2 = poll_locked(ticket, out, err);
            if (rc2 == CM_EAGAIN) *err = "timed out";
            return rc2;
        }
    }
}

cm_status Core::wait_all(int32_t n, const uint64_t *tickets, int32_t timeout_ms, cm_result *outs,
                         std::string *err)
{
    const auto until = deadline(timeout_ms);
    std::unique_lock<std::mutex> lk(mu_);
    auto unfinished = [&](int32_t j) {
        auto it = reqs_.find(tickets[j]);
        return it != reqs_.end() &&
               (it->second.state == St::Pending || it->second.state == St::Admitted);
    };
    for (;;) {
        bool all = true;
        for (int32_t j = 0; j < n && all; ++j) {
            if (reqs_.find(tickets[j]) == reqs_.end()) {
                *err = "unknown ticket " + std::to_string(tickets[j]);
                return CM_ENOTFOUND;
            }
            all = !unfinished(j);
        }
        if (all) break;
        if (cv_done_.wait_until(lk, until) == std::cv_status::timeout) {
            bool again = false;
            for (int32_t j = 0; j < n && !again; ++j) again = unfinished(j);
            if (again) {
                *err = "timed out";
                return CM_EAGAIN;
            }
            break;
        }
    }
    cm_status first = CM_OK;
    std::string first_err;
    for (int32_t j = 0; j < n; ++j) {
        cm_status rc;
        std::string e;
        if (outs) {
            rc = poll_locked(tickets[j], &outs[j], &e);
        } else {
            auto it = reqs_.find(tickets[j]);
            if (it == reqs_.end()) {
                rc = CM_ENOTFOUND;
                e = "unknown ticket " + std::to_string(tickets[j]);
            } else if (it->second.state == St::Done || it->second.state == St::Canceled) {
                rc = it->second.state == St::Done ? CM_OK : CM_ECANCELED;
                if (rc != CM_OK) e = "request " + std::to_string(tickets[j]) + " was canceled";
                reqs_.erase(it);
            } else {
                rc = CM_EDEVICE;
                e = fault_msg_;
            }
        }
        if (rc != CM_OK && first == CM_OK) {
            first = rc;
            first_err = e;
        }
    }
    if (first != CM_OK) *err = first_err;
    return first;
}

// ------------------------------------------------------------ statistics

void Core::stats(cm_server_stats *o)
{
    std::lock_guard<std::mutex> lk(mu_);
    std::memset(o, 0, sizeof *o);
    o->submitted = n_sub_;
    o->completed = n_done_;
    o->canceled = n_cancel_;
    o->candidates = n_cands_;
    o->rows = n_rows_;
    o->micro_batches = n_mb_;
    o->wall_us = first_submit_ >= 0 ? std::max(0.0, last_done_ - first_submit_) : 0.0;
    o->cands_per_s = o->wall_us > 0 ? (double)n_cands_ / (o->wall_us * 1e-6) : 0.0;
    if (!lat_.empty()) {
        std::vector<double> l = lat_;
        std::sort(l.begin(), l.end());
        auto pct = [&](double p) {
            const size_t i = (size_t)std::min<double>(l.size() - 1, std::ceil(p * l.size()) - 1);
            return l[i];
        };
        o->p50_us = pct(0.50);
        o->p99_us = pct(0.99);
        o->max_us = l.back();
    }
    o->queue_depth = (int32_t)pending_.size();
    o->in_flight = in_flight_;
    o->arena_in_use = arena_in_use_;
    o->arena_high_water = arena_high_;
    o->kernel_us = kernel_us_;
    o->kernel_bytes = kernel_bytes_;
    o->kernel_span_us = kclk_first_ < 0 ? 0.0 : kclk_last_ - kclk_first_;
    // union of the recorded kernels' [start, end] intervals
    const size_t nk = (size_t)std::min<int64_t>(kring_n_, KRING);
    std::vector<std::pair<double, double>> iv(kring_.begin(), kring_.begin() + (ptrdiff_t)nk);
    std::sort(iv.begin(), iv.end());
    double busy = 0, cs = 0, ce = 0;
    for (size_t i = 0; i < iv.size(); ++i) {
        if (i == 0 || iv[i].first > ce) {
            busy += ce - cs;
            cs = iv[i].first;
            ce = iv[i].second;
        } else if (iv[i].second > ce) {
            ce = iv[i].second;
        }
    }
    if (!iv.empty()) busy += ce - cs;
    o->kernel_busy_us = busy;
    o->kernel_busy_launches = (int64_t)nk;
}

void Core::reset_stats()
{
    std::lock_guard<std::mutex> lk(mu_);
    n_sub_ = n_done_ = n_cancel_ = n_cands_ = n_rows_ = n_mb_ = 0;
    first_submit_ = -1;
    last_done_ = 0;
    kernel_us_ = 0;
    kernel_bytes_ = 0;
    kclk_first_ = -1;
    kclk_last_ = 0;
    kring_n_ = 0;
    arena_high_ = arena_in_use_;
    lat_.clear();
}

// ------------------------------------------------------------ worker

// Fail every queued and admitted request (the device, or a launch, failed).
void Core::set_fault_locked(const std::string &what)
{
    if (fault_ == CM_OK) {
        fault_ = CM_EDEVICE;
        fault_msg_ = what;
    }
    for (auto &kv : reqs_)
        if (kv.second.state == St::Pending || kv.second.state == St::Admitted)
            kv.second.state = St::Failed;
    pending_.clear();
    cv_done_.notify_all();
}

// A slot's micro-batch has ended: release its requests' arena bytes and
// sessions and, for the ones still admitted (the batch finished normally),
// copy their beams out of the executor.
void Core::retire_locked(int si)
{
    Slot &sl = slot_[si];
    const bool ok = fault_ == CM_OK;
    if (ok) {
        kernel_us_ += ex_->kernel_us(si);
        kernel_bytes_ += sl.rows * (feature_bytes(cfg_.precision) + 32) + sl.cands * 4;
        double ks = 0, ke = 0;
        ex_->kernel_clock(si, &ks, &ke);
        if (kclk_first_ < 0 || ks < kclk_first_) kclk_first_ = ks;
        if (ke > kclk_last_) kclk_last_ = ke;
        kring_[(size_t)(kring_n_ % KRING)] = {ks, ke};
        ++kring_n_;
    }
    const double now = now_us();
    for (size_t j = 0; j < sl.tickets.size(); ++j) {
        auto it = reqs_.find(sl.tickets[j]);
        if (it == reqs_.end()) continue;
        Req &r = it->second;
        Session &ss = sessions_[r.session];
        ss.busy = false;
        if (ss.closing) {
            ss.closing = false;
            ss.used = false;
        }
        arena_in_use_ -= r.bytes;
        --in_flight_;
        if (r.state != St::Admitted) continue;
        const uint32_t *b = ex_->beam(si, j);
        r.idx.resize(r.k);
        r.val.resize(r.k);
        std::memcpy(r.idx.data(), b, (size_t)r.k * 4);
        std::memcpy(r.val.data(), b + sl.kb, (size_t)r.k * 4);
        r.t_done = now;
        r.state = St::Done;
        ++n_done_;
        n_cands_ += r.N;
        n_rows_ += (int64_t)r.N * r.S;
        lat_.push_back(r.t_done - r.t_submit);
        last_done_ = now;
    }
    sl.tickets.clear();
    sl.busy = false;
    cv_done_.notify_all();
}

// Admit queued requests, in submission order, into one micro-batch on slot
// `si` and launch it.  A request waits while its session has one admitted
// (later requests of other sessions go ahead); admission stops at the first
// request that does not fit the arena or the micro-batch (FIFO on memory).
// False when nothing could be admitted.
bool Core::admit_locked(int si)
{
    Slot &sl = slot_[si];
    std::vector<uint64_t> take;
    std::vector<uint8_t> in_batch(sessions_.size(), 0);
    int64_t bytes = 0, cands = 0, rows = 0;
    for (uint64_t t : pending_) {
        const Req &r = reqs_.at(t);
        if (sessions_[r.session].busy || in_batch[r.session]) continue;
        if (arena_in_use_ + bytes + r.bytes > cfg_.arena_bytes) break;
        if ((int32_t)take.size() == cfg_.max_batch_queries || cands + r.N > cfg_.max_batch_cands)
            break;
        take.push_back(t);
        in_batch[r.session] = 1;
        bytes += r.bytes;
        cands += r.N;
        rows += (int64_t)r.N * r.S;
    }
    if (take.empty()) return false;
    // remove the admitted tickets (a subsequence of the queue) in one pass
    std::deque<uint64_t> rest;
    size_t k = 0;
    for (uint64_t t : pending_) {
        if (k < take.size() && t == take[k]) ++k;
        else rest.push_back(t);
    }
    pending_.swap(rest);
    const double now = now_us();
    std::vector<Work> work(take.size());
    for (size_t j = 0; j < take.size(); ++j) {
        Req &r = reqs_.at(take[j]);
        sessions_[r.session].busy = true;
        r.state = St::Admitted;
        r.t_admit = now;
        work[j] = Work{take[j], r.session, r.S, r.N, r.x, r.t};
    }
    arena_in_use_ += bytes;
    arena_high_ = std::max(arena_high_, arena_in_use_);
    in_flight_ += (int32_t)take.size();
    sl.tickets = take;
    sl.kb = cfg_.k;  // every micro-batch selects the server's k; a request's
                     // smaller k is a prefix of that sorted beam
    sl.rows = rows;
    sl.cands = cands;
    sl.busy = true;
    ++n_mb_;
    std::string err;
    bool ok;
    if (fail_next_) {
        fail_next_ = false;
        ok = false;
        err = "launch failure forced from the host";
    } else {
        ok = ex_->launch(si, work, sl.kb, &err);
    }
    if (!ok) {
        set_fault_locked("micro-batch launch: " + err);
        retire_locked(si);  // nothing of it runs: release its requests
    }
    return true;
}

// At an idle server (no micro-batch on the device, the worker asleep), fill
// the slots from the submitting thread, so that the work is launched without
// waiting for the worker to wake up (the worker then only watches for the
// micro-batches' ends).  The same admission as the worker's, under the same
// lock.  While micro-batches run, the polling worker admits.
void Core::admit_here_locked()
{
    if (fault_ != CM_OK || stop_) return;
    for (int i = 0; i < cfg_.max_slots; ++i)
        if (slot_[i].busy) return;
    if (!ex_->launch_here()) return;
    for (int i = 0; i < cfg_.max_slots && !pending_.empty(); ++i)
        if (!slot_[i].busy) admit_locked(i);
}

void Core::run()
{
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
        bool progress = false;
        bool any_busy = false;
        for (int i = 0; i < cfg_.max_slots; ++i) {
            if (!slot_[i].busy) continue;
            std::string err;
            const int e = ex_->poll(i, &err);
            if (e > 0) {
                retire_locked(i);
                progress = true;
            } else if (e < 0) {
                set_fault_locked("micro-batch: " + err);
                retire_locked(i);
                progress = true;
            } else {
                any_busy = true;
            }
        }
        if (fault_ == CM_OK)
            for (int i = 0; i < cfg_.max_slots && !pending_.empty(); ++i)
                if (!slot_[i].busy && admit_locked(i)) {
                    progress = true;
                    any_busy = any_busy || slot_[i].busy;
                }
        if (stop_ && pending_.empty() && !any_busy) break;
        if (progress) continue;
        if (!any_busy) {
            cv_work_.wait(lk);  // nothing on the device: sleep until a submission
        } else {
            // work on the device: look again soon, without holding the lock (a
            // spin keeps a lone request's latency down; the worker is the
            // server's own thread)
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        }
    }
}

void Core::stop()
{
    {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
    }
    cv_work_.notify_all();
}

void Core::fail_next_launch()
{
    std::lock_guard<std::mutex> lk(mu_);
    fail_next_ = true;
}

}  // namespace serve
}  // namespace cm
