// CPU test of the serving loop's host core (csrc/serve_core.{h,cpp}) with a
// fake executor: admission in submission order, one admitted request per
// session (Sec. 4: a session's beam steps depend on each other), the arena
// and micro-batch limits, ticket states, cancellation, the failed state after
// a forced launch failure or a failed micro-batch, and concurrent clients.
// Built with g++ under the address and the thread sanitizer by
// tests/test_serve_core_cpu.py; exits non-zero on the first failed check.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

#include "serve_core.h"

using cm::serve::Core;
using cm::serve::Executor;
using cm::serve::Work;

#define CHECK(c)                                                                \
    do {                                                                        \
        if (!(c)) {                                                             \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            std::exit(1);                                                       \
        }                                                                       \
    } while (0)

namespace {

// A beam that depends only on the ticket, so a result that reaches the wrong
// ticket shows.
uint32_t beam_idx(uint64_t ticket, int i) { return (uint32_t)((ticket * 7919 + i) % 100003); }
float beam_val(uint64_t ticket, int i) { return (float)ticket + 0.25f * (float)i; }

class FakeExecutor : public Executor {
public:
    int delay = 2;                 // polls before a micro-batch finishes
    std::atomic<bool> hold{false}; // keep every micro-batch running
    int fail_poll_at = -1;         // the n-th launch's micro-batch fails
    std::atomic<bool> here{true};  // launches allowed from a submitting thread
    std::mutex mu;
    std::vector<std::vector<Work>> launches;
    int64_t in_flight_bytes = 0, max_in_flight_bytes = 0;
    cm_precision prec = CM_BF16;
    int32_t k = 8;

    bool launch(int si, const std::vector<Work> &batch, int32_t kb, std::string *) override
    {
        std::lock_guard<std::mutex> lk(mu);
        Slot &s = slot_[si];
        CHECK(!s.busy);
        s.busy = true;
        s.left = delay;
        s.kb = kb;
        s.n = (int)launches.size();
        s.bytes = 0;
        s.beams.assign(batch.size() * 2 * kb, 0);
        for (size_t j = 0; j < batch.size(); ++j) {
            for (int i = 0; i < kb; ++i) {
                s.beams[j * 2 * kb + i] = beam_idx(batch[j].ticket, i);
                const float v = beam_val(batch[j].ticket, i);
                std::memcpy(&s.beams[j * 2 * kb + kb + i], &v, 4);
            }
            s.bytes += cm::serve::request_bytes(prec, batch[j].S, batch[j].N, k);
        }
        in_flight_bytes += s.bytes;
        max_in_flight_bytes = std::max(max_in_flight_bytes, in_flight_bytes);
        launches.push_back(batch);
        return true;
    }
    int poll(int si, std::string *err) override
    {
        std::lock_guard<std::mutex> lk(mu);
        Slot &s = slot_[si];
        CHECK(s.busy);
        if (hold) return 0;
        if (s.n == fail_poll_at) {
            *err = "fake device failure";
            s.busy = false;
            in_flight_bytes -= s.bytes;
            return -1;
        }
        if (--s.left > 0) return 0;
        s.busy = false;
        in_flight_bytes -= s.bytes;
        return 1;
    }
    const uint32_t *beam(int si, size_t j) override { return &slot_[si].beams[j * 2 * slot_[si].kb]; }
    bool launch_here() override { return here; }
    size_t n_launches()
    {
        std::lock_guard<std::mutex> lk(mu);
        return launches.size();
    }
    double kernel_us(int) override { return 1.0; }
    // kernel i (in completion order, from 1) ran at device times
    // [2i, 2i + width]: disjoint for width 1, overlapping its successor for 3
    void kernel_clock(int, double *s, double *e) override
    {
        clk_ += 2.0;
        *s = clk_;
        *e = clk_ + width;
    }
    double clk_ = 0.0, width = 1.0;

private:
    struct Slot {
        bool busy = false;
        int left = 0, kb = 0, n = 0;
        int64_t bytes = 0;
        std::vector<uint32_t> beams;
    };
    Slot slot_[cm::serve::MAX_SLOTS];
};

cm_server_cfg config(int slots, int64_t arena, int pending, int sessions, int batch_q)
{
    cm_server_cfg c{};
    c.precision = CM_BF16;
    c.k = 8;
    c.arena_bytes = arena;
    c.max_slots = slots;
    c.max_pending = pending;
    c.max_sessions = sessions;
    c.max_stages = 64;
    c.max_batch_queries = batch_q;
    c.max_batch_cands = 1 << 16;
    return c;
}

// A request over fake (never dereferenced) 16-byte aligned device addresses.
cm_request request(int32_t n, int32_t k)
{
    return cm_request{n, k, reinterpret_cast<const void *>(0x100000), reinterpret_cast<const float *>(0x200000)};
}

struct Server {
    FakeExecutor ex;
    Core core;
    std::thread worker;
    explicit Server(const cm_server_cfg &c) : core(c, &ex) { worker = std::thread([this] { core.run(); }); }
    ~Server()
    {
        ex.hold = false;
        core.stop();
        worker.join();
    }
    int32_t open(int32_t S)
    {
        int32_t sid = -1;
        std::string e;
        CHECK(core.session_reserve(S, &sid, &e) == CM_OK);
        core.session_ready(sid, true);
        return sid;
    }
};

void check_result(Core &core, uint64_t t, int32_t k)
{
    std::vector<int32_t> idx(8);
    std::vector<float> val(8);
    cm_result r{8, 0, idx.data(), val.data(), 0, 0, 0};
    std::string e;
    CHECK(core.wait(t, 20000, &r, &e) == CM_OK);
    CHECK(r.n == k);
    for (int i = 0; i < k; ++i) {
        CHECK((uint32_t)idx[i] == beam_idx(t, i));
        CHECK(val[i] == beam_val(t, i));
    }
    CHECK(r.t_submit_us <= r.t_admit_us && r.t_admit_us <= r.t_done_us);
}

void test_results_order_and_sessions()
{
    auto sp = std::make_unique<Server>(config(3, 1 << 30, 1024, 8, 4));
    Server &s = *sp;
    std::vector<int32_t> sids;
    for (int i = 0; i < 6; ++i) sids.push_back(s.open(3 + i));
    std::vector<std::pair<uint64_t, int32_t>> tk;
    std::string e;
    for (int r = 0; r < 60; ++r) {
        const int32_t sid = sids[(r * 5) % 6];
        const cm_request q = request(16 + r * 13, 1 + r % 8);
        uint64_t t = 0;
        CHECK(s.core.submit(sid, &q, &t, &e) == CM_OK);
        tk.push_back({t, q.k});
    }
    for (auto &p : tk) check_result(s.core, p.first, p.second);
    cm_server_stats st;
    s.core.stats(&st);
    // the executor's lock is taken only after the core's is released (the
    // worker takes them in the order core, executor)
    std::lock_guard<std::mutex> lk(s.ex.mu);
    std::map<int32_t, uint64_t> last;  // per session, tickets in submission order
    for (auto &b : s.ex.launches) {
        CHECK(b.size() <= 4);
        std::set<int32_t> seen;
        for (auto &w : b) {
            CHECK(seen.insert(w.session).second);  // one request per session and batch
            CHECK(w.ticket > last[w.session]);
            last[w.session] = w.ticket;
        }
    }
    CHECK(st.completed == 60 && st.submitted == 60 && st.in_flight == 0 && st.arena_in_use == 0);
    CHECK(st.micro_batches == (int64_t)s.ex.launches.size());
    // the fake's kernels run at device times [2i, 2i + 1], i = 1 .. micro-batches
    CHECK(st.kernel_us == (double)st.micro_batches);
    CHECK(st.kernel_span_us == 2.0 * (double)(st.micro_batches - 1) + 1.0);
    CHECK(st.kernel_busy_launches == st.micro_batches);
    CHECK(st.kernel_busy_us == (double)st.micro_batches);  // disjoint unit intervals
    CHECK(st.p50_us <= st.p99_us && st.p99_us <= st.max_us);
}

void test_arena_is_fifo_and_never_exceeded()
{
    const int64_t one = cm::serve::request_bytes(CM_BF16, 10, 100, 8);
    auto sp = std::make_unique<Server>(config(4, 2 * one, 1024, 16, 8));
    Server &s = *sp;
    std::vector<int32_t> sids;
    for (int i = 0; i < 12; ++i) sids.push_back(s.open(10));
    std::vector<uint64_t> tk;
    std::string e;
    for (int i = 0; i < 12; ++i) {
        const cm_request q = request(100, 8);
        uint64_t t = 0;
        CHECK(s.core.submit(sids[i], &q, &t, &e) == CM_OK);
        tk.push_back(t);
    }
    for (uint64_t t : tk) check_result(s.core, t, 8);
    cm_server_stats st;
    s.core.stats(&st);
    CHECK(st.arena_high_water <= 2 * one);
    {
        std::lock_guard<std::mutex> lk(s.ex.mu);
        CHECK(s.ex.max_in_flight_bytes <= 2 * one);
        // admission in submission order
        uint64_t prev = 0;
        for (auto &b : s.ex.launches)
            for (auto &w : b) {
                CHECK(w.ticket > prev);
                prev = w.ticket;
            }
    }
    // a request larger than the arena can never be admitted
    const cm_request big = request(201, 8);
    uint64_t t = 0;
    CHECK(s.core.submit(sids[0], &big, &t, &e) == CM_E2BIG);
}

void test_errors_queue_full_and_cancel()
{
    auto sp = std::make_unique<Server>(config(1, 1 << 30, 3, 4, 1));
    Server &s = *sp;
    const int32_t a = s.open(4), b = s.open(4);
    std::string e;
    uint64_t t = 0;
    cm_request q = request(10, 9);  // k above the server's 8
    CHECK(s.core.submit(a, &q, &t, &e) == CM_EINVAL);
    q = request(10, 8);
    CHECK(s.core.submit(77, &q, &t, &e) == CM_ENOTFOUND);
    q = request((1 << 16) + 1, 8);
    CHECK(s.core.submit(a, &q, &t, &e) == CM_E2BIG);
    q = request(10, 8);
    q.sched = reinterpret_cast<const void *>(0x100004);
    CHECK(s.core.submit(a, &q, &t, &e) == CM_EINVAL);
    // hold the device: one request admitted, the queue fills up
    s.ex.hold = true;
    q = request(10, 8);
    uint64_t t0 = 0, t1 = 0, t2 = 0, t3 = 0;
    CHECK(s.core.submit(a, &q, &t0, &e) == CM_OK);
    for (int i = 0; i < 2000; ++i) {  // wait for its admission
        cm_server_stats st;
        s.core.stats(&st);
        if (st.in_flight == 1) break;
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
    CHECK(s.core.submit(a, &q, &t1, &e) == CM_OK);
    CHECK(s.core.submit(b, &q, &t2, &e) == CM_OK);
    CHECK(s.core.submit(b, &q, &t3, &e) == CM_OK);
    uint64_t t4 = 0;
    CHECK(s.core.submit(b, &q, &t4, &e) == CM_EAGAIN);  // queue full
    std::vector<int32_t> idx(8);
    std::vector<float> val(8);
    cm_result r{8, 0, idx.data(), val.data(), 0, 0, 0};
    CHECK(s.core.poll(t1, &r, &e) == CM_EAGAIN);
    CHECK(s.core.poll(999999, &r, &e) == CM_ENOTFOUND);
    CHECK(s.core.wait(t1, 5, &r, &e) == CM_EAGAIN);  // times out
    // closing b cancels its queued requests; a's queued one still completes
    CHECK(s.core.session_close(b, &e) == CM_OK);
    CHECK(s.core.poll(t2, &r, &e) == CM_ECANCELED);
    CHECK(s.core.poll(t3, &r, &e) == CM_ECANCELED);
    CHECK(s.core.poll(t3, &r, &e) == CM_ENOTFOUND);  // released
    CHECK(s.core.session_idle(a, &e) == CM_EAGAIN);   // a request of a is in flight
    s.ex.hold = false;
    check_result(s.core, t0, 8);
    check_result(s.core, t1, 8);
    CHECK(s.core.session_idle(a, &e) == CM_OK);
    cm_result small{4, 0, idx.data(), val.data(), 0, 0, 0};
    uint64_t t5 = 0;
    CHECK(s.core.submit(a, &q, &t5, &e) == CM_OK);
    CHECK(s.core.wait(t5, 20000, &small, &e) == CM_EINVAL);  // capacity below k
    check_result(s.core, t5, 8);
    cm_server_stats st;
    s.core.stats(&st);
    CHECK(st.canceled == 2 && st.completed == 3);
}

void test_forced_launch_failure()
{
    auto sp = std::make_unique<Server>(config(2, 1 << 30, 1024, 8, 2));
    Server &s = *sp;
    std::vector<int32_t> sids;
    for (int i = 0; i < 6; ++i) sids.push_back(s.open(5));
    s.ex.hold = true;  // the first micro-batch stays on the device
    std::string e;
    const cm_request q = request(50, 8);
    uint64_t first = 0;
    CHECK(s.core.submit(sids[0], &q, &first, &e) == CM_OK);
    for (int i = 0; i < 2000 && s.ex.n_launches() == 0; ++i)
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    s.core.fail_next_launch();
    // queued in one call, before the worker can admit any of them
    std::vector<uint64_t> tk(5);
    std::vector<cm_request> qs(5, q);
    CHECK(s.core.submit_batch(5, sids.data() + 1, qs.data(), tk.data(), &e) == CM_OK);
    std::vector<int32_t> idx(8);
    std::vector<float> val(8);
    cm_result r{8, 0, idx.data(), val.data(), 0, 0, 0};
    for (uint64_t t : tk) CHECK(s.core.wait(t, 20000, &r, &e) == CM_EDEVICE);
    s.ex.hold = false;
    CHECK(s.core.wait(first, 20000, &r, &e) == CM_EDEVICE);  // admitted before: failed too
    uint64_t t = 0;
    CHECK(s.core.submit(sids[0], &q, &t, &e) == CM_EDEVICE);
    int32_t sid = 0;
    CHECK(s.core.session_reserve(5, &sid, &e) == CM_EDEVICE);
    CHECK(s.core.wait_all((int32_t)tk.size(), tk.data(), 100, nullptr, &e) == CM_EDEVICE);
    // the micro-batch already on the device still ends and releases its arena
    cm_server_stats st;
    for (int i = 0; i < 20000; ++i) {
        s.core.stats(&st);
        if (st.in_flight == 0) break;
        std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
    CHECK(st.in_flight == 0 && st.arena_in_use == 0 && st.completed == 0);
}

void test_failed_micro_batch()
{
    auto sp = std::make_unique<Server>(config(1, 1 << 30, 1024, 8, 1));
    Server &s = *sp;
    s.ex.fail_poll_at = 1;  // the second micro-batch fails on the device
    std::vector<int32_t> sids;
    for (int i = 0; i < 4; ++i) sids.push_back(s.open(5));
    // queued in one call: submitted one at a time, a later submission could
    // meet the failed state the second micro-batch has already left
    std::vector<uint64_t> tk(4);
    std::vector<cm_request> qs(4, request(20, 8));
    std::string e;
    CHECK(s.core.submit_batch(4, sids.data(), qs.data(), tk.data(), &e) == CM_OK);
    check_result(s.core, tk[0], 8);
    std::vector<int32_t> idx(8);
    std::vector<float> val(8);
    cm_result r{8, 0, idx.data(), val.data(), 0, 0, 0};
    for (int i = 1; i < 4; ++i) CHECK(s.core.wait(tk[i], 20000, &r, &e) == CM_EDEVICE);
    CHECK(e.find("fake device failure") != std::string::npos);
}

void test_concurrent_clients()
{
    auto sp = std::make_unique<Server>(config(4, 1 << 30, 4096, 32, 16));
    Server &s = *sp;
    s.ex.delay = 1;
    std::vector<std::thread> th;
    std::atomic<int> done{0};
    for (int c = 0; c < 8; ++c)
        th.emplace_back([&, c] {
            const int32_t sid = s.open(2 + c);
            std::string e;
            for (int r = 0; r < 150; ++r) {
                const cm_request q = request(1 + (r * 31 + c) % 500, 1 + (r + c) % 8);
                uint64_t t = 0;
                CHECK(s.core.submit(sid, &q, &t, &e) == CM_OK);
                if (r % 3 == 0) {
                    check_result(s.core, t, q.k);
                } else {
                    std::vector<int32_t> idx(8);
                    std::vector<float> val(8);
                    cm_result res{8, 0, idx.data(), val.data(), 0, 0, 0};
                    cm_status st;
                    while ((st = s.core.poll(t, &res, &e)) == CM_EAGAIN) std::this_thread::yield();
                    CHECK(st == CM_OK && (uint32_t)idx[0] == beam_idx(t, 0));
                }
                done.fetch_add(1);
            }
            CHECK(s.core.session_close(sid, &e) == CM_OK);
        });
    for (auto &t : th) t.join();
    CHECK(done.load() == 8 * 150);
    cm_server_stats st;
    s.core.stats(&st);
    CHECK(st.completed == 8 * 150 && st.in_flight == 0 && st.queue_depth == 0);
}

// The busy time is the union of the kernels' intervals: overlapping kernels
// count once, and only the most recent 4096 are kept.
void test_kernel_busy_time()
{
    Server s(config(2, 1 << 30, 64, 4, 8));
    s.ex.width = 3.0;
    const int32_t sid = s.open(4);
    std::string e;
    for (int r = 0; r < 5000; ++r) {
        const cm_request q = request(16, 1);
        uint64_t t = 0;
        CHECK(s.core.submit(sid, &q, &t, &e) == CM_OK);
        check_result(s.core, t, 1);
    }
    cm_server_stats st;
    s.core.stats(&st);
    CHECK(st.micro_batches == 5000);
    CHECK(st.kernel_us == 5000.0);  // the fake reports 1 us per kernel
    CHECK(st.kernel_span_us == 2.0 * 4999 + 3.0);
    CHECK(st.kernel_busy_launches == 4096);
    CHECK(st.kernel_busy_us == 2.0 * 4095 + 3.0);  // [2i, 2i + 3] for the last 4096 i
    s.core.reset_stats();
    s.core.stats(&st);
    CHECK(st.kernel_busy_launches == 0 && st.kernel_busy_us == 0.0 && st.kernel_span_us == 0.0);
}

void test_stop_drains_the_queue()
{
    std::vector<uint64_t> tk;
    auto exp = std::make_unique<FakeExecutor>();
    FakeExecutor &ex = *exp;
    auto corep = std::make_unique<Core>(config(2, 1 << 30, 1024, 8, 4), &ex);
    Core &core = *corep;
    std::string e;
    int32_t sid = 0;
    CHECK(core.session_reserve(3, &sid, &e) == CM_OK);
    core.session_ready(sid, true);
    for (int i = 0; i < 10; ++i) {
        const cm_request q = request(30, 8);
        uint64_t t = 0;
        CHECK(core.submit(sid, &q, &t, &e) == CM_OK);
        tk.push_back(t);
    }
    core.stop();
    core.run();  // returns once everything queued has completed
    for (uint64_t t : tk) check_result(core, t, 8);
    const cm_request q = request(30, 8);
    uint64_t t = 0;
    CHECK(core.submit(sid, &q, &t, &e) == CM_ECANCELED);
}

// A submission to an idle server is launched by the submitting thread
// before the call returns; with that refused, the worker launches it.  Later
// submissions, while a micro-batch runs, are the worker's.
void test_launch_from_submitting_thread()
{
    for (bool here : {true, false}) {
        auto sp = std::make_unique<Server>(config(2, 1 << 30, 1024, 8, 4));
        Server &s = *sp;
        s.ex.here = here;
        s.ex.hold = true;  // nothing finishes until released
        const int32_t sid = s.open(5);
        const int32_t sid2 = s.open(7);
        std::string e;
        const cm_request q = request(40, 8);
        uint64_t t1 = 0;
        CHECK(s.core.submit(sid, &q, &t1, &e) == CM_OK);
        if (here) CHECK(s.ex.n_launches() == 1);
        const int32_t sids[2] = {sid, sid2};
        const cm_request qs[2] = {request(40, 8), request(50, 4)};
        uint64_t tk[2] = {0, 0};
        // sid's second request waits for its first; sid2's goes to the other
        // slot, launched by the worker (a micro-batch is running)
        CHECK(s.core.submit_batch(2, sids, qs, tk, &e) == CM_OK);
        s.ex.hold = false;
        check_result(s.core, t1, 8);
        check_result(s.core, tk[0], 8);
        check_result(s.core, tk[1], 4);
        // (the worker alone may take the first two requests in one batch)
        if (here) CHECK(s.ex.n_launches() == 3);
    }
}

}  // namespace

int main()
{
    test_results_order_and_sessions();
    test_arena_is_fifo_and_never_exceeded();
    test_errors_queue_full_and_cancel();
    test_forced_launch_failure();
    test_failed_micro_batch();
    test_concurrent_clients();
    test_kernel_busy_time();
    test_stop_drains_the_queue();
    test_launch_from_submitting_thread();
    std::printf("serve core: all checks passed\n");
    return 0;
}
