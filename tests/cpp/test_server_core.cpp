// CPU test of the serving core (admission by device-memory budget and
// in-flight limit, arrival order, coalescing per (dtype, predecessors)
// class, completion, waits, pinned results, release, statistics,
// cancellation) with a fake executor whose "device" work completes after a
// simulated delay.  Built with ThreadSanitizer (and separately with
// AddressSanitizer) by tests/test_host_cpp.py; prints "ok" and exits 0 when
// every check holds, else prints the failed check and exits 1.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "apsp_server_core.h"

using namespace apsp::serve;

static std::atomic<int> g_failures{0};
#define CHECK(cond)                                                                    \
    do {                                                                               \
        if (!(cond)) {                                                                 \
            std::fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #cond);    \
            g_failures.fetch_add(1);                                                   \
        }                                                                              \
    } while (0)

// Device work that finishes `delay` after launch; statuses chosen per n.
struct FakeExec : Executor {
    struct Work {
        Req *r;
        Clock::time_point ready;
        apsp_status_t st;
    };
    // every member below is touched only under the core's lock (or, for
    // prepare/unprepare, on a request no other thread can see)
    int64_t budget = 0;
    int64_t device_bytes = 0;  // bytes the fake device holds now
    int64_t peak_bytes = 0;
    std::vector<Work> running;
    std::vector<uint64_t> admitted_order;  // tickets in launch order
    std::vector<size_t> group_sizes;
    std::vector<int> group_classes_mixed;  // 1 if a group mixed (dtype, pred) classes
    std::chrono::microseconds delay{200};
    std::atomic<int> prepared{0}, unprepared{0};
    bool fail_n_77 = true;  // requests with n == 77 fail with a negative cycle

    bool prepare(Req *r, const apsp_request_t &q) override {
        auto *copy = new std::vector<char>((size_t)q.n * (size_t)q.n * 4);
        std::memcpy(copy->data(), q.weights, copy->size());  // the weights are read now, not later
        r->exec = copy;
        prepared.fetch_add(1);
        return true;
    }
    void unprepare(Req *r) override {
        delete (std::vector<char> *)r->exec;
        r->exec = nullptr;
        unprepared.fetch_add(1);
    }
    void hold(int64_t bytes) {
        device_bytes += bytes;
        peak_bytes = std::max(peak_bytes, device_bytes);
    }
    apsp_status_t status_of(const Req *r) const {
        return (fail_n_77 && r->n == 77) ? APSP_ERROR_NEGATIVE_CYCLE : APSP_SUCCESS;
    }
    int64_t launch_group(std::vector<Req *> &batch) override {
        group_sizes.push_back(batch.size());
        int mixed = 0;
        int64_t arena = 0;
        for (Req *r : batch) {
            mixed |= (r->dtype != batch[0]->dtype || r->want_pred != batch[0]->want_pred);
            admitted_order.push_back(r->ticket);
            arena += (int64_t)(r->resident + r->transient);
        }
        group_classes_mixed.push_back(mixed);
        // the group holds its members' bytes as one arena (as the HIP executor does)
        int64_t delta = arena;
        for (Req *r : batch) {
            delta -= (int64_t)(r->resident + r->transient);
            r->resident = r->transient = 0;
        }
        hold(arena);
        auto *g = new int64_t[2]{arena, (int64_t)batch.size()};
        for (Req *r : batch) {
            running.push_back({r, Clock::now() + delay, status_of(r)});
            groups_of[r] = g;
        }
        return delta;
    }
    void launch_large(Req *r) override {
        admitted_order.push_back(r->ticket);
        hold((int64_t)(r->resident + r->transient));
        running.push_back({r, Clock::now() + 4 * delay, status_of(r)});
    }
    int64_t poll(std::vector<std::pair<Req *, apsp_status_t>> &done) override {
        int64_t freed = 0;
        const auto now = Clock::now();
        for (auto it = running.begin(); it != running.end();) {
            if (it->ready <= now) {
                Req *r = it->r;
                freed += (int64_t)r->transient;
                device_bytes -= (int64_t)r->transient;
                r->transient = 0;
                done.push_back({r, it->st});
                it = running.erase(it);
            } else {
                ++it;
            }
        }
        return freed;
    }
    void result(const Req *r, const void **d_dist, const int32_t **d_pred) override {
        *d_dist = ((std::vector<char> *)r->exec)->data();
        if (d_pred) *d_pred = nullptr;
    }
    int64_t release(Req *r) override {
        int64_t extra = 0;
        device_bytes -= (int64_t)(r->resident + r->transient);
        auto it = groups_of.find(r);
        if (it != groups_of.end()) {
            int64_t *g = it->second;
            if (--g[1] == 0) {
                extra = g[0];
                device_bytes -= g[0];
                delete[] g;
            }
            groups_of.erase(it);
        }
        delete (std::vector<char> *)r->exec;
        r->exec = nullptr;
        return extra;
    }
    bool busy() override { return !running.empty(); }

    std::map<const Req *, int64_t *> groups_of;
};

static apsp_request_t make_req(const std::vector<int32_t> &w, int64_t n, apsp_dtype_t dt, bool pred) {
    apsp_request_t q{};
    q.weights = w.data();
    q.n = n;
    q.ld = 0;
    q.dtype = dt;
    q.want_pred = pred ? 1 : 0;
    q.borrow = 0;
    return q;
}

static size_t footprint(int64_t n, bool pred) {
    const size_t mat = ((size_t)(n * n) * 4 + 255) / 256 * 256;
    return mat + (pred ? mat : 0) + 256;
}

// Budget, arrival order and coalescing under concurrent clients.
static void test_concurrent_clients() {
    FakeExec ex;
    CoreConfig cfg;
    cfg.budget = 24 << 20;   // 24 MiB: forces admission waits
    cfg.fixed = 1 << 20;
    cfg.max_inflight = 12;
    cfg.max_queue = 10000;
    cfg.batch_max_n = 200;
    cfg.poll_period = std::chrono::microseconds(20);
    ex.budget = cfg.budget;
    Core core(cfg, &ex);
    core.start([] {});
    const int kThreads = 4, kPer = 60;
    std::vector<int32_t> big((size_t)1000 * 1000, 1);
    std::atomic<int> ok{0}, neg{0};
    std::vector<std::thread> th;
    for (int t = 0; t < kThreads; ++t) {
        th.emplace_back([&, t] {
            std::mt19937 rng(1234 + t);
            for (int i = 0; i < kPer; ++i) {
                int64_t n = (rng() % 3 == 0) ? 300 + rng() % 700 : 16 + rng() % 185;
                if (i % 17 == 5) n = 77;
                const apsp_dtype_t dt = (rng() & 1) ? APSP_INT32 : APSP_FLOAT32;
                const bool pred = (rng() % 3) == 0;
                uint64_t ticket = 0;
                apsp_status_t st = core.submit(make_req(big, n, dt, pred), n > 200 ? (size_t)(n * n) * 4 : 0, &ticket);
                CHECK(st == APSP_SUCCESS);
                if (st != APSP_SUCCESS) continue;
                st = core.wait(ticket, -1);
                if (n == 77) {
                    CHECK(st == APSP_ERROR_NEGATIVE_CYCLE);
                    neg.fetch_add(1);
                } else {
                    CHECK(st == APSP_SUCCESS);
                    // results are readable while pinned, then released
                    const apsp_status_t rs = core.with_result(ticket, [&](int64_t nn, const void *d, const int32_t *) {
                        return (nn == n && d != nullptr) ? APSP_SUCCESS : APSP_ERROR_INVALID_VALUE;
                    });
                    CHECK(rs == APSP_SUCCESS);
                    ok.fetch_add(1);
                }
                CHECK(core.release(ticket) == APSP_SUCCESS);
                CHECK(core.release(ticket) == APSP_ERROR_UNKNOWN_TICKET);
                CHECK(core.poll(ticket) == APSP_ERROR_UNKNOWN_TICKET);
            }
        });
    }
    for (auto &x : th) x.join();
    const apsp_server_stats_t s = core.stats();
    core.stop();
    CHECK(ok.load() + neg.load() == kThreads * kPer);
    CHECK(s.submitted == kThreads * kPer);
    CHECK(s.completed == ok.load());
    CHECK(s.failed == neg.load());
    CHECK(s.queued == 0 && s.inflight == 0);
    CHECK(s.bytes_in_use == cfg.fixed);           // everything released
    CHECK(ex.peak_bytes + cfg.fixed <= cfg.budget);  // the budget was never exceeded
    CHECK(ex.device_bytes == 0);
    CHECK(s.p50_latency_ms > 0 && s.p99_latency_ms >= s.p50_latency_ms);
    // every request was launched exactly once
    std::set<uint64_t> launched(ex.admitted_order.begin(), ex.admitted_order.end());
    CHECK(launched.size() == ex.admitted_order.size() && (int)launched.size() == kThreads * kPer);
    for (int m : ex.group_classes_mixed) CHECK(m == 0);  // a group holds one (dtype, pred) class
    CHECK(ex.prepared.load() == kThreads * kPer);
}

// Requests admitted strictly in arrival order, one at a time (max_inflight 1).
static void test_fifo_order() {
    FakeExec ex;
    CoreConfig cfg;
    cfg.budget = 1 << 30;
    cfg.max_inflight = 1;
    cfg.batch_max_n = 0;  // never coalesce
    cfg.poll_period = std::chrono::microseconds(20);
    Core core(cfg, &ex);
    core.start([] {});
    std::vector<int32_t> w((size_t)64 * 64, 1);
    std::vector<uint64_t> tickets;
    for (int i = 0; i < 40; ++i) {
        uint64_t t = 0;
        CHECK(core.submit(make_req(w, 8 + i, APSP_INT32, false), 1024, &t) == APSP_SUCCESS);
        tickets.push_back(t);
    }
    for (uint64_t t : tickets) {
        CHECK(core.wait(t, -1) == APSP_SUCCESS);
        CHECK(core.release(t) == APSP_SUCCESS);
    }
    core.stop();
    CHECK(ex.admitted_order == tickets);
}

// Submit-time refusals, a full queue, timeouts, cancellation at stop.
static void test_refusals_and_cancellation() {
    FakeExec ex;
    ex.delay = std::chrono::microseconds(200000);  // 0.2 s of "device" work per coalesced request
    CoreConfig cfg;
    cfg.budget = 8 << 20;
    cfg.fixed = 1 << 20;
    cfg.max_inflight = 1;
    cfg.max_queue = 3;
    cfg.batch_max_n = 512;
    cfg.poll_period = std::chrono::microseconds(20);
    Core core(cfg, &ex);
    core.start([] {});
    std::vector<int32_t> w((size_t)2048 * 2048, 1);
    uint64_t t = 0;
    // larger than the whole budget minus the fixed part: refused at submit
    CHECK(core.submit(make_req(w, 2048, APSP_INT32, false), 0, &t) == APSP_ERROR_OUT_OF_MEMORY);
    CHECK(core.submit(make_req(w, 1500, APSP_INT32, true), 0, &t) == APSP_ERROR_OUT_OF_MEMORY);
    uint64_t first = 0;
    CHECK(core.submit(make_req(w, 100, APSP_INT32, false), 0, &first) == APSP_SUCCESS);
    // the first one holds the only in-flight slot; three more fill the queue
    std::vector<uint64_t> queued;
    for (int i = 0; i < 6; ++i) {
        uint64_t q = 0;
        const apsp_status_t st = core.submit(make_req(w, 100 + i, APSP_FLOAT32, false), 0, &q);
        if (st == APSP_SUCCESS)
            queued.push_back(q);
        else
            CHECK(st == APSP_ERROR_QUEUE_FULL);
    }
    CHECK(queued.size() >= 2 && queued.size() <= 3);
    CHECK(core.wait(first, 1000) == APSP_ERROR_TIMEOUT);  // still running
    CHECK(core.release(first) == APSP_ERROR_NOT_READY);
    CHECK(core.poll(987654) == APSP_ERROR_UNKNOWN_TICKET);
    // a waiter blocked while the server stops gets CANCELLED or the result
    std::atomic<int> waited{-1};
    std::thread waiter([&] { waited = (int)core.wait(queued.back(), -1); });
    std::this_thread::sleep_for(std::chrono::milliseconds(20));
    core.stop();
    waiter.join();
    CHECK(waited.load() == APSP_ERROR_CANCELLED || waited.load() == APSP_SUCCESS);
    const apsp_server_stats_t s = core.stats();
    CHECK(s.cancelled >= 2);
    CHECK(s.submitted == (int64_t)(1 + queued.size()));
    CHECK(core.submit(make_req(w, 10, APSP_INT32, false), 0, &t) == APSP_ERROR_CANCELLED);
}

// release racing with readers of the same ticket: release waits for them.
static void test_release_waits_for_readers() {
    FakeExec ex;
    ex.delay = std::chrono::microseconds(50);
    CoreConfig cfg;
    cfg.budget = 1 << 30;
    cfg.batch_max_n = 512;
    cfg.poll_period = std::chrono::microseconds(20);
    Core core(cfg, &ex);
    core.start([] {});
    std::vector<int32_t> w((size_t)300 * 300, 3);
    for (int round = 0; round < 50; ++round) {
        uint64_t t = 0;
        CHECK(core.submit(make_req(w, 300, APSP_INT32, false), 0, &t) == APSP_SUCCESS);
        CHECK(core.wait(t, -1) == APSP_SUCCESS);
        std::atomic<int> reads{0};
        std::thread reader([&] {
            for (int i = 0; i < 20; ++i) {
                const apsp_status_t st = core.with_result(t, [&](int64_t n, const void *d, const int32_t *) {
                    // the buffer stays valid while pinned: read all of it
                    const int32_t *v = (const int32_t *)d;
                    int64_t sum = 0;
                    for (int64_t e = 0; e < n * n; ++e) sum += v[e];
                    return sum == 3 * n * n ? APSP_SUCCESS : APSP_ERROR_INVALID_VALUE;
                });
                if (st == APSP_ERROR_UNKNOWN_TICKET) break;  // released meanwhile
                CHECK(st == APSP_SUCCESS);
                reads.fetch_add(1);
            }
        });
        std::this_thread::sleep_for(std::chrono::microseconds(round * 10));
        CHECK(core.release(t) == APSP_SUCCESS);
        reader.join();
    }
    core.stop();
    CHECK(ex.device_bytes == 0);
}

int main() {
    test_fifo_order();
    test_concurrent_clients();
    test_refusals_and_cancellation();
    test_release_waits_for_readers();
    if (g_failures.load() != 0) {
        std::fprintf(stderr, "%d check(s) failed\n", g_failures.load());
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
