// Host-side core of the serving runtime: the request table, admission by
// device-memory budget and in-flight limit, coalescing of small requests
// per (dtype, predecessors) class, completion bookkeeping, waits and
// latency statistics.  It holds no device code and makes no HIP call: every
// device action goes through an Executor (the HIP one in apsp_server.hip; a
// fake one in the CPU tests, which run this file under ThreadSanitizer).
//
// Threads: client threads call submit / poll / wait / result / release /
// stats; one scheduler thread (run()) polls the executor for finished work
// and admits queued requests.  One mutex guards all state; the executor is
// only ever called with that mutex held, except prepare()/unprepare() on a
// request that is not yet (or no longer) in the table.
#pragma once

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "apsp.h"

namespace apsp {
namespace serve {

using Clock = std::chrono::steady_clock;

enum class RState { Queued, Running, Done, Failed, Cancelled };

struct Req {
    uint64_t ticket = 0;
    int64_t n = 0;
    apsp_dtype_t dtype = APSP_INT32;
    bool want_pred = false;
    bool coalesced = false;  // admitted into a batched launch (n <= batch_max_n)
    size_t resident = 0;     // budget bytes held until release
    size_t transient = 0;    // budget bytes held until completion
    RState state = RState::Queued;
    apsp_status_t result = APSP_SUCCESS;
    int pins = 0;            // callers reading the result (release waits for them)
    bool released = false;   // release has begun (the ticket is gone for every other call)
    Clock::time_point t_submit, t_done;
    void *exec = nullptr;    // the executor's per-request state
};

// Device side of the server.  Called with the core's lock held unless noted.
struct Executor {
    virtual ~Executor() = default;
    // Outside the lock, before the request enters the table: take a copy of
    // the caller's weights (or note borrowed ones).  False: out of memory.
    virtual bool prepare(Req *r, const apsp_request_t &q) = 0;
    // Outside the lock: undo prepare() for a request that never entered.
    virtual void unprepare(Req *r) = 0;
    // Launch requests admitted together (each is Running; one that cannot be
    // launched is reported with its error by the next poll()).  Returns the
    // change of the
    // budget bytes in use (a batched launch may hold its members' bytes in
    // one arena: it then zeroes their resident/transient and returns the
    // arena's size).
    virtual int64_t launch_group(std::vector<Req *> &batch) = 0;
    virtual void launch_large(Req *r) = 0;
    // Appends (request, status) for work that has completed since the last
    // call; drives sliced work.  Returns the budget bytes it freed (a large
    // request's transient work memory).
    virtual int64_t poll(std::vector<std::pair<Req *, apsp_status_t>> &done) = 0;
    // Device pointers of a finished request's results.
    virtual void result(const Req *r, const void **d_dist, const int32_t **d_pred) = 0;
    // Frees a released request's device memory; returns the budget bytes
    // freed beyond r->resident + r->transient (a batched arena whose last
    // member leaves).
    virtual int64_t release(Req *r) = 0;
    // Work still on the device (the scheduler drains it before stopping).
    virtual bool busy() = 0;
};

struct CoreConfig {
    int64_t budget = 0;        // device bytes
    int64_t fixed = 0;         // bytes the executor holds for the server's lifetime
    int32_t max_inflight = 64;
    int32_t max_queue = 4096;
    int32_t batch_max_n = 512;  // 0: never coalesce
    std::chrono::microseconds poll_period{50};
};

class Core {
public:
    Core(const CoreConfig &cfg, Executor *ex) : cfg_(cfg), ex_(ex), bytes_in_use_(cfg.fixed) {}

    // Starts the scheduler thread, which first runs init() (the executor's
    // per-thread set-up, e.g. selecting the device).
    template <class Init>
    void start(Init init) {
        scheduler_ = std::thread([this, init] {
            init();
            run();
        });
    }

    // transient: work memory the request needs while it runs (0 when coalesced).
    apsp_status_t submit(const apsp_request_t &q, size_t transient, uint64_t *ticket) {
        const auto t0 = Clock::now();
        std::unique_ptr<Req> r(new (std::nothrow) Req());
        if (!r) return APSP_ERROR_OUT_OF_MEMORY;
        r->n = q.n;
        r->dtype = q.dtype;
        r->want_pred = q.want_pred != 0;
        r->coalesced = q.n <= cfg_.batch_max_n;
        r->t_submit = t0;
        const size_t mat = (size_t)(q.n * q.n) * 4;
        r->resident = round_up(mat, 256) + (r->want_pred ? round_up(mat, 256) : 0) + 256;
        r->transient = r->coalesced ? 0 : transient;
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (stopping_) return APSP_ERROR_CANCELLED;
            if ((int64_t)(r->resident + r->transient) > cfg_.budget - cfg_.fixed) return APSP_ERROR_OUT_OF_MEMORY;
            if ((int64_t)pending_.size() >= cfg_.max_queue) return APSP_ERROR_QUEUE_FULL;
        }
        if (!ex_->prepare(r.get(), q)) return APSP_ERROR_OUT_OF_MEMORY;
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (stopping_) {
                ex_->unprepare(r.get());
                return APSP_ERROR_CANCELLED;
            }
            r->ticket = next_ticket_++;
            *ticket = r->ticket;
            ++submitted_;
            if (!have_first_) {
                first_submit_ = t0;
                have_first_ = true;
            }
            const uint64_t t = r->ticket;
            pending_.push_back(r.get());
            reqs_[t] = r.release();
        }
        cv_sched_.notify_one();
        return APSP_SUCCESS;
    }

    apsp_status_t poll(uint64_t ticket) {
        std::lock_guard<std::mutex> lk(mu_);
        const Req *r = find(ticket);
        return r ? state_status(r) : APSP_ERROR_UNKNOWN_TICKET;
    }

    apsp_status_t wait(uint64_t ticket, int64_t timeout_us) {
        std::unique_lock<std::mutex> lk(mu_);
        Req *r = find(ticket);
        if (!r) return APSP_ERROR_UNKNOWN_TICKET;
        ++r->pins;  // the request stays in the table while this thread waits on it
        auto ready = [&] { return state_status(r) != APSP_ERROR_NOT_READY || stopping_; };
        ++waiters_;
        bool ok = true;
        if (timeout_us < 0)
            cv_done_.wait(lk, ready);
        else
            ok = cv_done_.wait_until(
                lk, deadline(std::chrono::microseconds(std::min<int64_t>(timeout_us, kMaxTimeoutUs))), ready);
        --waiters_;
        --r->pins;
        apsp_status_t st = state_status(r);
        cv_done_.notify_all();
        if (stopping_ && st == APSP_ERROR_NOT_READY) return APSP_ERROR_CANCELLED;
        if (!ok) return APSP_ERROR_TIMEOUT;
        return st;
    }

    // Device pointers of a finished request (valid until release).
    apsp_status_t result(uint64_t ticket, const void **d_dist, const int32_t **d_pred) {
        std::lock_guard<std::mutex> lk(mu_);
        const Req *r = find(ticket);
        if (!r) return APSP_ERROR_UNKNOWN_TICKET;
        const apsp_status_t st = state_status(r);
        if (st != APSP_SUCCESS) return st;
        ex_->result(r, d_dist, d_pred);
        return APSP_SUCCESS;
    }

    // Runs fn(n, d_dist, d_pred) on a finished request's results outside the
    // lock while the request is pinned: a concurrent release of the same
    // ticket waits until fn has returned.
    template <class Fn>
    apsp_status_t with_result(uint64_t ticket, Fn fn) {
        const void *dd = nullptr;
        const int32_t *pp = nullptr;
        Req *r = nullptr;
        {
            std::lock_guard<std::mutex> lk(mu_);
            r = find(ticket);
            if (!r) return APSP_ERROR_UNKNOWN_TICKET;
            const apsp_status_t st = state_status(r);
            if (st != APSP_SUCCESS) return st;
            ex_->result(r, &dd, &pp);
            ++r->pins;
        }
        const apsp_status_t st = fn(r->n, dd, pp);
        {
            std::lock_guard<std::mutex> lk(mu_);
            --r->pins;
        }
        cv_done_.notify_all();
        return st;
    }

    apsp_status_t release(uint64_t ticket) {
        {
            std::unique_lock<std::mutex> lk(mu_);
            Req *r = find(ticket);
            if (!r) return APSP_ERROR_UNKNOWN_TICKET;
            if (r->state == RState::Queued || r->state == RState::Running) return APSP_ERROR_NOT_READY;
            if (r->released) return APSP_ERROR_UNKNOWN_TICKET;
            r->released = true;  // one release per ticket, even while readers finish
            cv_done_.wait(lk, [&] { return r->pins == 0; });
            const int64_t extra = ex_->release(r);
            bytes_in_use_ -= (int64_t)(r->resident + r->transient) + extra;
            if (r->state != RState::Cancelled) --inflight_;
            reqs_.erase(ticket);
            delete r;
        }
        cv_sched_.notify_one();
        return APSP_SUCCESS;
    }

    apsp_server_stats_t stats() {
        std::lock_guard<std::mutex> lk(mu_);
        apsp_server_stats_t s{};
        s.submitted = submitted_;
        s.completed = completed_;
        s.failed = failed_;
        s.cancelled = cancelled_;
        s.queued = (int64_t)pending_.size();
        s.inflight = inflight_;
        s.bytes_in_use = bytes_in_use_;
        if (!latencies_ms_.empty()) {
            s.p50_latency_ms = percentile(latencies_ms_, 0.50);
            s.p99_latency_ms = percentile(latencies_ms_, 0.99);
            for (int large = 0; large < 2; ++large) {
                std::vector<double> c;
                for (size_t i = 0; i < latencies_ms_.size(); ++i)
                    if (latency_large_[i] == large) c.push_back(latencies_ms_[i]);
                if (c.empty()) continue;
                (large ? s.p50_large_ms : s.p50_small_ms) = percentile(c, 0.50);
                (large ? s.p99_large_ms : s.p99_small_ms) = percentile(c, 0.99);
            }
            const double span = std::chrono::duration<double>(last_done_ - first_submit_).count();
            s.solves_per_s = span > 0 ? (double)completed_ / span : 0.0;
        }
        return s;
    }

    // Cancels queued requests, drains running ones, wakes every waiter and
    // frees every request.  No other call may start once this has begun,
    // except waits already blocked (they return APSP_ERROR_CANCELLED).
    void stop() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stopping_ = true;
            for (Req *r : pending_) {
                r->state = RState::Cancelled;
                ++cancelled_;
            }
            pending_.clear();
        }
        cv_sched_.notify_all();
        if (scheduler_.joinable()) scheduler_.join();  // drains running work
        std::unique_lock<std::mutex> lk(mu_);
        cv_done_.notify_all();
        cv_done_.wait(lk, [&] {
            if (waiters_ != 0) return false;
            for (auto &kv : reqs_)
                if (kv.second->pins != 0) return false;
            return true;
        });
        for (auto &kv : reqs_) {
            ex_->release(kv.second);
            delete kv.second;
        }
        reqs_.clear();
    }

    int64_t bytes_in_use() {
        std::lock_guard<std::mutex> lk(mu_);
        return bytes_in_use_;
    }

private:
    static size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

    // Timed waits take a system-clock deadline: the condition variable then
    // waits with pthread_cond_timedwait, which thread checkers understand
    // (a steady-clock wait goes through pthread_cond_clockwait).  A clock
    // step only lengthens or shortens one poll period or one timed wait.
    static constexpr int64_t kMaxTimeoutUs = (int64_t)1e15;  // ~31 years: the deadline cannot overflow
    static std::chrono::system_clock::time_point deadline(std::chrono::microseconds d) {
        return std::chrono::system_clock::now() + d;
    }

    static double percentile(std::vector<double> v, double q) {
        std::sort(v.begin(), v.end());
        const size_t i = (size_t)std::min<double>((double)v.size() - 1, std::ceil(q * (double)v.size()) - 1);
        return v[i];
    }

    static apsp_status_t state_status(const Req *r) {
        switch (r->state) {
            case RState::Queued:
            case RState::Running: return APSP_ERROR_NOT_READY;
            case RState::Done: return APSP_SUCCESS;
            case RState::Failed: return r->result;
            case RState::Cancelled: return APSP_ERROR_CANCELLED;
        }
        return APSP_ERROR_NOT_READY;
    }

    Req *find(uint64_t ticket) {
        auto it = reqs_.find(ticket);
        if (it == reqs_.end() || it->second->released) return nullptr;
        return it->second;
    }

    void finish_locked(Req *r, apsp_status_t st) {
        r->t_done = Clock::now();
        if (r->state == RState::Cancelled) return;
        r->result = st;
        if (st == APSP_SUCCESS) {
            r->state = RState::Done;
            ++completed_;
        } else {
            r->state = RState::Failed;
            ++failed_;
        }
        latencies_ms_.push_back(std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count());
        latency_large_.push_back(r->coalesced ? 0 : 1);
        last_done_ = r->t_done;
    }

    bool poll_locked() {
        done_.clear();
        bytes_in_use_ -= ex_->poll(done_);
        for (auto &d : done_) finish_locked(d.first, d.second);
        return !done_.empty();
    }

    // Arrival order; a request whose footprint does not fit waits and blocks
    // later ones, so large requests are not starved.
    void admit_locked() {
        std::map<int, std::vector<Req *>> classes;  // dtype * 2 + predecessors -> coalesced requests
        while (!pending_.empty() && inflight_ < cfg_.max_inflight) {
            Req *r = pending_.front();
            const int64_t need = (int64_t)(r->resident + r->transient);
            if (bytes_in_use_ + need > cfg_.budget) break;
            pending_.pop_front();
            bytes_in_use_ += need;
            ++inflight_;
            r->state = RState::Running;
            if (r->coalesced)
                classes[(int)r->dtype * 2 + (r->want_pred ? 1 : 0)].push_back(r);
            else
                ex_->launch_large(r);
        }
        for (auto &kv : classes) bytes_in_use_ += ex_->launch_group(kv.second);
    }

    bool admissible_locked() const {
        return !pending_.empty() && inflight_ < cfg_.max_inflight &&
               bytes_in_use_ + (int64_t)(pending_.front()->resident + pending_.front()->transient) <= cfg_.budget;
    }

    void run() {
        std::unique_lock<std::mutex> lk(mu_);
        while (true) {
            if (poll_locked()) cv_done_.notify_all();
            if (stopping_ && !ex_->busy()) break;
            if (!stopping_) admit_locked();
            if (ex_->busy())
                cv_sched_.wait_until(lk, deadline(cfg_.poll_period));
            else if (!stopping_ && !admissible_locked())
                cv_sched_.wait(lk);
        }
    }

    CoreConfig cfg_;
    Executor *ex_;
    std::mutex mu_;
    std::condition_variable cv_sched_, cv_done_;
    std::thread scheduler_;
    bool stopping_ = false;
    std::deque<Req *> pending_;
    std::map<uint64_t, Req *> reqs_;
    uint64_t next_ticket_ = 1;
    int64_t bytes_in_use_ = 0;
    int inflight_ = 0;
    int waiters_ = 0;
    std::vector<std::pair<Req *, apsp_status_t>> done_;
    int64_t submitted_ = 0, completed_ = 0, failed_ = 0, cancelled_ = 0;
    std::vector<double> latencies_ms_;
    std::vector<char> latency_large_;
    Clock::time_point first_submit_, last_done_;
    bool have_first_ = false;
};

}  // namespace serve
}  // namespace apsp
