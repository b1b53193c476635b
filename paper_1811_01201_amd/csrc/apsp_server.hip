// Serving runtime: a request loop on one GPU with continuous batching.
//
// Client threads submit host weight matrices; a scheduler thread admits
// requests in arrival order while the device-memory budget and the
// in-flight limit allow, and launches them without waiting for earlier
// ones:
//   * requests with n <= batch_max_n that are admitted together are
//     coalesced, per (dtype, predecessors) class, into one batched fused
//     launch on the batch stream (their results live in that launch's packed
//     arena until every member is released);
//   * larger requests get their own buffers and run apsp_solve on one of
//     n_streams streams, so they overlap each other and the batched work;
//     with slice_rounds > 0 their launch sequence goes out slice_rounds
//     rounds at a time (a stepper), the next slice only once the last one
//     has finished, so requests admitted meanwhile are not queued behind a
//     large solve's remaining rounds (round-level preemption).
// Results stay resident in device memory until released; releasing returns
// their bytes to the budget, which admits waiting requests.  Completion is
// observed by polling a per-launch event; latency = completion observed -
// submit.  Every result is the one apsp_solve gives for that request alone
// (exact arithmetic; the kernels' choices depend only on n, dtype and
// predecessors, never on the mix).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "apsp_internal.h"

using namespace apsp;
using Clock = std::chrono::steady_clock;

namespace {

enum class RState { Queued, Running, Done, Failed, Cancelled };

struct Group;

struct Request {
    uint64_t ticket = 0;
    int64_t n = 0;
    apsp_dtype_t dtype = APSP_INT32;
    bool want_pred = false;
    void *h_staging = nullptr;  // pinned copy of the weights until uploaded (owned)
    const void *h_src = nullptr;  // upload source: h_staging or the caller's pinned rows
    int64_t h_ld = 0;             // leading dimension of h_src (elements)
    size_t bytes_dist = 0, bytes_pred = 0;
    size_t resident = 0;   // bytes held until release
    size_t transient = 0;  // bytes held until completion
    RState state = RState::Queued;
    apsp_status_t result = APSP_SUCCESS;
    // large path
    void *d_dist = nullptr;
    int32_t *d_pred = nullptr;
    void *d_work = nullptr;
    int32_t *d_status = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    apsp_stepper_t *stepper = nullptr;  // sliced large path
    hipEvent_t slice_done = nullptr;
    bool all_issued = true;
    apsp_status_t slice_error = APSP_SUCCESS;
    // batched path
    std::shared_ptr<Group> group;
    int64_t group_off = 0;  // element offset in the group's arena
    int group_index = 0;
    Clock::time_point t_submit, t_done;
};

struct Group {
    apsp_dtype_t dtype = APSP_INT32;
    bool want_pred = false;
    void *d_arena = nullptr;  // packed dist | packed pred | status | metadata
    size_t bytes = 0;
    int64_t pred_off_bytes = 0, status_off_bytes = 0;
    void *h_meta = nullptr;   // pinned metadata source of the upload
    hipEvent_t done = nullptr;
    int members = 0;          // unreleased members
    std::vector<Request *> reqs;
};

size_t elem_size(apsp_dtype_t) { return 4; }

}  // namespace

struct apsp_server {
    apsp_server_config_t cfg{};
    int device = 0;
    int cus = 256;
    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::thread scheduler;
    bool stopping = false;
    std::deque<Request *> pending;
    std::map<uint64_t, Request *> reqs;
    std::vector<std::shared_ptr<Group>> running_groups;
    std::vector<Request *> running_large;
    uint64_t next_ticket = 1;
    int64_t bytes_in_use = 0;
    int inflight = 0;  // admitted and not yet released
    int waiters = 0;
    std::vector<hipStream_t> streams;
    int next_stream = 0;
    hipStream_t batch_stream = nullptr;
    void *batch_scratch = nullptr;
    int64_t batch_scratch_elems = 0;
    int32_t *batch_counters = nullptr;
    int batch_grid = 0;
    // statistics
    int64_t submitted = 0, completed = 0, failed = 0, cancelled = 0;
    std::vector<double> latencies_ms;
    std::vector<char> latency_large;  // per latency: a large (not coalesced) request
    Clock::time_point first_submit, last_done;
    bool have_first = false;

    void run();
    void admit_locked();
    void launch_group(std::vector<Request *> &batch);
    void launch_large(Request *r);
    bool poll_locked();
    void finish(Request *r, apsp_status_t st);
    void free_request_device(Request *r);
};

namespace {

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

// Completion of running work (called with the lock held).  Returns true if
// anything finished.
bool apsp_server::poll_locked() {
    bool any = false;
    for (auto it = running_large.begin(); it != running_large.end();) {
        Request *r = *it;
        if (!r->all_issued) {
            // sliced: the next slice once the previous one has finished
            if (hipEventQuery(r->slice_done) == hipSuccess) {
                int32_t last = 0;
                apsp_status_t st = apsp_stepper_step(r->stepper, cfg.slice_rounds, &last);
                hipError_t e = hipSuccess;
                if (st == APSP_SUCCESS) e = hipEventRecord(last ? r->done : r->slice_done, r->stream);
                if (st != APSP_SUCCESS || e != hipSuccess) {
                    // what was issued still runs: let it finish, then fail the request
                    r->slice_error = st != APSP_SUCCESS ? st : APSP_ERROR_HIP;
                    hipStreamSynchronize(r->stream);
                    hipEventRecord(r->done, r->stream);
                    last = 1;
                }
                if (last) r->all_issued = true;
            }
            ++it;
            continue;
        }
        if (hipEventQuery(r->done) == hipSuccess) {
            int32_t st = 0;
            hipMemcpy(&st, r->d_status, sizeof(int32_t), hipMemcpyDeviceToHost);
            if (r->slice_error != APSP_SUCCESS) st = r->slice_error;
            if (r->stepper) stepper_destroy(r->stepper, false);  // its work has completed
            r->stepper = nullptr;
            if (r->slice_done) hipEventDestroy(r->slice_done);
            r->slice_done = nullptr;
            if (r->d_work) hipFreeAsync(r->d_work, r->stream);
            r->d_work = nullptr;
            bytes_in_use -= (int64_t)r->transient;
            r->transient = 0;
            finish(r, (apsp_status_t)st);
            it = running_large.erase(it);
            any = true;
        } else {
            ++it;
        }
    }
    for (auto it = running_groups.begin(); it != running_groups.end();) {
        Group *g = it->get();
        if (hipEventQuery(g->done) == hipSuccess) {
            std::vector<int32_t> st(g->reqs.size(), 0);
            hipMemcpy(st.data(), (char *)g->d_arena + g->status_off_bytes, st.size() * 4,
                      hipMemcpyDeviceToHost);
            hipHostFree(g->h_meta);
            g->h_meta = nullptr;
            for (size_t i = 0; i < g->reqs.size(); ++i) {
                Request *r = g->reqs[i];
                if (r->h_staging) {
                    hipHostFree(r->h_staging);
                    r->h_staging = nullptr;
                }
                finish(r, (apsp_status_t)st[i]);
            }
            it = running_groups.erase(it);
            any = true;
        } else {
            ++it;
        }
    }
    return any;
}

void apsp_server::finish(Request *r, apsp_status_t st) {
    r->t_done = Clock::now();
    if (r->state == RState::Cancelled) return;
    r->result = st;
    if (st == APSP_SUCCESS) {
        r->state = RState::Done;
        ++completed;
    } else {
        r->state = RState::Failed;
        ++failed;
    }
    latencies_ms.push_back(std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count());
    latency_large.push_back(r->group ? 0 : 1);
    last_done = r->t_done;
    if (r->h_staging) {
        hipHostFree(r->h_staging);
        r->h_staging = nullptr;
    }
}

void apsp_server::free_request_device(Request *r) {
    hipStream_t s = r->stream ? r->stream : batch_stream;
    if (r->d_dist) hipFreeAsync(r->d_dist, s);
    if (r->d_pred) hipFreeAsync(r->d_pred, s);
    if (r->d_work) hipFreeAsync(r->d_work, s);
    if (r->d_status) hipFreeAsync(r->d_status, s);
    if (r->done) hipEventDestroy(r->done);
    r->d_dist = r->d_work = nullptr;
    r->d_pred = r->d_status = nullptr;
    r->done = nullptr;
    if (r->group) {
        Group *g = r->group.get();
        if (--g->members == 0) {
            if (g->d_arena) hipFreeAsync(g->d_arena, batch_stream);
            if (g->done) hipEventDestroy(g->done);
            g->d_arena = nullptr;
            g->done = nullptr;
            bytes_in_use -= (int64_t)g->bytes;
        }
        r->group.reset();
    }
}

void apsp_server::launch_large(Request *r) {
    r->stream = streams[next_stream++ % streams.size()];
    hipStream_t s = r->stream;
    apsp_status_t st = APSP_SUCCESS;
    if (hipMallocAsync(&r->d_dist, r->bytes_dist, s) != hipSuccess ||
        (r->want_pred && hipMallocAsync((void **)&r->d_pred, r->bytes_pred, s) != hipSuccess) ||
        hipMallocAsync((void **)&r->d_status, 256, s) != hipSuccess ||
        (r->transient && hipMallocAsync(&r->d_work, r->transient, s) != hipSuccess)) {
        st = APSP_ERROR_OUT_OF_MEMORY;
    }
    if (st == APSP_SUCCESS &&
        hipMemcpy2DAsync(r->d_dist, (size_t)r->n * 4, r->h_src, (size_t)r->h_ld * 4, (size_t)r->n * 4,
                         (size_t)r->n, hipMemcpyHostToDevice, s) != hipSuccess)
        st = APSP_ERROR_HIP;
    apsp_options_t opt{};
    opt.d_status = r->d_status;
    if (st == APSP_SUCCESS && hipEventCreateWithFlags(&r->done, hipEventDisableTiming) != hipSuccess)
        st = APSP_ERROR_HIP;
    if (st == APSP_SUCCESS && cfg.slice_rounds > 0) {
        // sliced: record the solve, issue its first slice
        int32_t last = 0;
        st = stepper_create(r->n, r->dtype, r->want_pred, &opt, true, r->d_work, r->transient, &r->stepper);
        if (st == APSP_SUCCESS && hipEventCreateWithFlags(&r->slice_done, hipEventDisableTiming) != hipSuccess)
            st = APSP_ERROR_HIP;
        if (st == APSP_SUCCESS) st = apsp_stepper_begin(r->stepper, r->d_dist, r->d_pred, s);
        if (st == APSP_SUCCESS) st = apsp_stepper_step(r->stepper, cfg.slice_rounds, &last);
        if (st == APSP_SUCCESS && hipEventRecord(last ? r->done : r->slice_done, s) != hipSuccess)
            st = APSP_ERROR_HIP;
        r->all_issued = last != 0;
    } else if (st == APSP_SUCCESS) {
        st = solve_internal(r->d_dist, r->d_pred, r->n, r->dtype, s, opt, r->d_work, r->transient);
        if (st == APSP_SUCCESS && hipEventRecord(r->done, s) != hipSuccess) st = APSP_ERROR_HIP;
    }
    r->state = RState::Running;
    if (st != APSP_SUCCESS) {
        hipStreamSynchronize(s);
        if (r->stepper) stepper_destroy(r->stepper, false);
        r->stepper = nullptr;
        if (r->slice_done) hipEventDestroy(r->slice_done);
        r->slice_done = nullptr;
        r->all_issued = true;
        bytes_in_use -= (int64_t)r->transient;
        r->transient = 0;
        finish(r, st);
        return;
    }
    running_large.push_back(r);
}

// One batched fused launch for requests of one (dtype, predecessors) class.
void apsp_server::launch_group(std::vector<Request *> &batch) {
    auto g = std::make_shared<Group>();
    g->dtype = batch[0]->dtype;
    g->want_pred = batch[0]->want_pred;
    const int32_t B = (int32_t)batch.size();
    std::vector<int32_t> ns(B);
    std::vector<int64_t> offs(B);
    int64_t total = 0;
    for (int32_t b = 0; b < B; ++b) {
        ns[b] = (int32_t)batch[b]->n;
        offs[b] = total;
        total += (int64_t)round_up((size_t)(batch[b]->n * batch[b]->n), 4);
    }
    const size_t dist_bytes = round_up((size_t)total * 4, 256);
    const size_t pred_bytes = g->want_pred ? dist_bytes : 0;
    const size_t status_bytes = round_up((size_t)B * 4, 256);
    std::vector<char> meta_host;
    int32_t n_team = 0;
    int64_t need_scratch = 0;
    bool lean = false;
    batch_meta(ns.data(), offs.data(), B, g->dtype, g->want_pred, nullptr, meta_host, n_team, need_scratch, lean);
    const size_t meta_bytes = round_up(meta_host.size(), 256);
    g->pred_off_bytes = (int64_t)dist_bytes;
    g->status_off_bytes = (int64_t)(dist_bytes + pred_bytes);
    g->bytes = dist_bytes + pred_bytes + status_bytes + meta_bytes;
    g->members = B;
    g->reqs = batch;
    bytes_in_use += (int64_t)g->bytes;
    for (auto *r : batch) {
        bytes_in_use -= (int64_t)(r->resident + r->transient);  // accounted by the group instead
        r->resident = r->transient = 0;
    }
    apsp_status_t st = need_scratch > batch_scratch_elems ? APSP_ERROR_INVALID_ARGUMENT : APSP_SUCCESS;
    hipStream_t s = batch_stream;
    if (st == APSP_SUCCESS && hipHostMalloc(&g->h_meta, meta_bytes) != hipSuccess) st = APSP_ERROR_OUT_OF_MEMORY;
    if (st == APSP_SUCCESS) {
        std::memcpy(g->h_meta, meta_host.data(), meta_host.size());
        if (hipMallocAsync(&g->d_arena, g->bytes, s) != hipSuccess) st = APSP_ERROR_OUT_OF_MEMORY;
    }
    char *arena = (char *)g->d_arena;
    const void *meta = arena + dist_bytes + pred_bytes + status_bytes;
    if (st == APSP_SUCCESS &&
        hipMemcpyAsync((void *)meta, g->h_meta, meta_host.size(), hipMemcpyHostToDevice, s) != hipSuccess)
        st = APSP_ERROR_HIP;
    for (int32_t b = 0; b < B && st == APSP_SUCCESS; ++b) {
        Request *r = batch[b];
        r->group = g;
        r->group_off = offs[b];
        r->group_index = b;
        if (hipMemcpy2DAsync(arena + offs[b] * 4, (size_t)r->n * 4, r->h_src, (size_t)r->h_ld * 4,
                             (size_t)r->n * 4, (size_t)r->n, hipMemcpyHostToDevice, s) != hipSuccess)
            st = APSP_ERROR_HIP;
    }
    if (st == APSP_SUCCESS) {
        // the scratch holds 2 x CUs work matrices of 8-byte elements, i.e.
        // 4 x CUs of 4-byte ones: room for the lean kernel's workgroups
        const int grid = lean ? std::min(4, batched_blocks_per_cu(g->dtype, true)) * cus : batch_grid;
        BatchLaunch L{meta, B, n_team, batch_scratch_elems, batch_scratch, batch_counters, grid, lean};
        st = batched_launch(L, g->dtype, g->want_pred, arena,
                            g->want_pred ? (int32_t *)(arena + g->pred_off_bytes) : nullptr,
                            (int32_t *)(arena + g->status_off_bytes), s);
    }
    if (st == APSP_SUCCESS && (hipEventCreateWithFlags(&g->done, hipEventDisableTiming) != hipSuccess ||
                               hipEventRecord(g->done, s) != hipSuccess))
        st = APSP_ERROR_HIP;
    for (auto *r : batch) r->state = RState::Running;
    if (st != APSP_SUCCESS) {
        hipStreamSynchronize(s);
        for (auto *r : batch) {
            r->group = g;
            finish(r, st);
        }
        return;
    }
    running_groups.push_back(g);
}

// Admission (lock held): arrival order; a request whose footprint does not
// fit waits (and blocks later ones, so large requests are not starved).
void apsp_server::admit_locked() {
    std::map<int, std::vector<Request *>> classes;  // dtype*2 + pred -> small requests
    while (!pending.empty() && inflight < cfg.max_inflight) {
        Request *r = pending.front();
        const int64_t need = (int64_t)(r->resident + r->transient);
        if (bytes_in_use + need > cfg.hbm_budget_bytes) break;
        pending.pop_front();
        bytes_in_use += need;
        ++inflight;
        if (r->n <= cfg.batch_max_n)
            classes[(int)r->dtype * 2 + (r->want_pred ? 1 : 0)].push_back(r);
        else
            launch_large(r);
    }
    for (auto &kv : classes) launch_group(kv.second);
}

void apsp_server::run() {
    hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
        const bool busy = !running_large.empty() || !running_groups.empty();
        if (stopping && !busy) break;
        if (poll_locked()) cv_done.notify_all();
        if (!stopping) admit_locked();
        if (!running_large.empty() || !running_groups.empty())
            cv_sched.wait_for(lk, std::chrono::microseconds(50));
        else if (!stopping && (pending.empty() || inflight >= cfg.max_inflight ||
                               bytes_in_use + (int64_t)(pending.front()->resident +
                                                        pending.front()->transient) >
                                   cfg.hbm_budget_bytes))
            cv_sched.wait(lk);
    }
}

// ------------------------------------------------------------------ C ABI
extern "C" {

apsp_status_t apsp_server_create(const apsp_server_config_t *config, apsp_server_t **out) {
    if (!out) return APSP_ERROR_INVALID_ARGUMENT;
    *out = nullptr;
    apsp_server_config_t cfg{};
    if (config) cfg = *config;
    if (cfg.hbm_budget_bytes < 0 || cfg.max_inflight < 0 || cfg.n_streams < 0 || cfg.max_queue < 0 ||
        cfg.batch_max_n > 1024 || cfg.slice_rounds < 0)
        return APSP_ERROR_INVALID_ARGUMENT;
    auto *sv = new (std::nothrow) apsp_server();
    if (!sv) return APSP_ERROR_OUT_OF_MEMORY;
    if (hipGetDevice(&sv->device) != hipSuccess) {
        delete sv;
        return APSP_ERROR_HIP;
    }
    hipDeviceGetAttribute(&sv->cus, hipDeviceAttributeMultiprocessorCount, sv->device);
    if (cfg.hbm_budget_bytes == 0) {
        size_t free_b = 0, total_b = 0;
        hipMemGetInfo(&free_b, &total_b);
        cfg.hbm_budget_bytes = (int64_t)(free_b / 2);
    }
    if (cfg.max_inflight == 0) cfg.max_inflight = 64;
    if (cfg.n_streams == 0) cfg.n_streams = 8;
    if (cfg.max_queue == 0) cfg.max_queue = 4096;
    if (cfg.batch_max_n == 0) cfg.batch_max_n = 512;
    if (cfg.batch_max_n < 0) cfg.batch_max_n = 0;  // never coalesce
    sv->cfg = cfg;
    // keep freed device memory in the stream-ordered pool for reuse
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, sv->device) == hipSuccess) {
        uint64_t keep = UINT64_MAX;
        hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    for (int i = 0; i < cfg.n_streams; ++i) {
        hipStream_t s;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            apsp_server_destroy(sv);
            return APSP_ERROR_HIP;
        }
        sv->streams.push_back(s);
    }
    if (hipStreamCreateWithFlags(&sv->batch_stream, hipStreamNonBlocking) != hipSuccess) {
        apsp_server_destroy(sv);
        return APSP_ERROR_HIP;
    }
    if (cfg.batch_max_n > 0) {
        // work matrices of up to 128-padded batch_max_n (every team configuration fits)
        const int64_t ldp = std::max<int64_t>(128, (cfg.batch_max_n + 127) / 128 * 128);
        sv->batch_grid = 2 * sv->cus;
        sv->batch_scratch_elems = ldp * ldp;
        const size_t bytes = (size_t)sv->batch_grid * sv->batch_scratch_elems * 8;
        if ((int64_t)bytes >= cfg.hbm_budget_bytes ||
            hipMalloc(&sv->batch_scratch, bytes) != hipSuccess ||
            hipMalloc((void **)&sv->batch_counters, 32) != hipSuccess ||
            hipMemset(sv->batch_counters, 0, 32) != hipSuccess) {
            apsp_server_destroy(sv);
            return APSP_ERROR_OUT_OF_MEMORY;
        }
        sv->bytes_in_use = (int64_t)bytes;
    }
    sv->scheduler = std::thread([sv] { sv->run(); });
    *out = sv;
    return APSP_SUCCESS;
}

apsp_status_t apsp_server_submit(apsp_server_t *sv, const apsp_request_t *req, uint64_t *ticket) {
    if (!sv || !req || !ticket || !req->weights || req->n < 1 || req->n > kMaxN ||
        (req->dtype != APSP_INT32 && req->dtype != APSP_FLOAT32) ||
        (req->ld != 0 && req->ld < req->n))
        return APSP_ERROR_INVALID_ARGUMENT;
    const auto t0 = Clock::now();
    auto *r = new (std::nothrow) Request();
    if (!r) return APSP_ERROR_OUT_OF_MEMORY;
    r->n = req->n;
    r->dtype = req->dtype;
    r->want_pred = req->want_pred != 0;
    r->t_submit = t0;
    r->bytes_dist = (size_t)(r->n * r->n) * elem_size(r->dtype);
    r->bytes_pred = r->want_pred ? (size_t)(r->n * r->n) * 4 : 0;
    r->resident = round_up(r->bytes_dist, 256) + round_up(r->bytes_pred, 256) + 256;
    r->transient = r->n <= sv->cfg.batch_max_n ? 0 : solve_work_bytes(r->n, r->dtype, r->want_pred);
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->stopping) {
            delete r;
            return APSP_ERROR_CANCELLED;
        }
        const int64_t fixed = sv->batch_scratch ? (int64_t)sv->batch_grid * sv->batch_scratch_elems * 8 : 0;
        if ((int64_t)(r->resident + r->transient) > sv->cfg.hbm_budget_bytes - fixed) {
            delete r;
            return APSP_ERROR_OUT_OF_MEMORY;
        }
        if ((int64_t)sv->pending.size() >= sv->cfg.max_queue) {
            delete r;
            return APSP_ERROR_QUEUE_FULL;
        }
    }
    const int64_t ld = req->ld ? req->ld : req->n;
    if (req->borrow) {
        r->h_src = req->weights;
        r->h_ld = ld;
    } else {
        if (hipHostMalloc(&r->h_staging, std::max<size_t>(r->bytes_dist, 4)) != hipSuccess) {
            delete r;
            return APSP_ERROR_OUT_OF_MEMORY;
        }
        const size_t row = (size_t)r->n * 4;
        for (int64_t i = 0; i < r->n; ++i)
            std::memcpy((char *)r->h_staging + (size_t)i * row,
                        (const char *)req->weights + (size_t)(i * ld) * 4, row);
        r->h_src = r->h_staging;
        r->h_ld = r->n;
    }
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->stopping) {
            hipHostFree(r->h_staging);
            delete r;
            return APSP_ERROR_CANCELLED;
        }
        r->ticket = sv->next_ticket++;
        sv->reqs[r->ticket] = r;
        sv->pending.push_back(r);
        ++sv->submitted;
        if (!sv->have_first) {
            sv->first_submit = t0;
            sv->have_first = true;
        }
        *ticket = r->ticket;
    }
    sv->cv_sched.notify_one();
    return APSP_SUCCESS;
}

static apsp_status_t state_status(const Request *r) {
    switch (r->state) {
        case RState::Queued:
        case RState::Running: return APSP_ERROR_NOT_READY;
        case RState::Done: return APSP_SUCCESS;
        case RState::Failed: return r->result;
        case RState::Cancelled: return APSP_ERROR_CANCELLED;
    }
    return APSP_ERROR_NOT_READY;
}

apsp_status_t apsp_server_poll(apsp_server_t *sv, uint64_t ticket) {
    if (!sv) return APSP_ERROR_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return APSP_ERROR_UNKNOWN_TICKET;
    return state_status(it->second);
}

apsp_status_t apsp_server_wait(apsp_server_t *sv, uint64_t ticket, int64_t timeout_us) {
    if (!sv) return APSP_ERROR_INVALID_ARGUMENT;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return APSP_ERROR_UNKNOWN_TICKET;
    Request *r = it->second;
    auto ready = [&] { return state_status(r) != APSP_ERROR_NOT_READY || sv->stopping; };
    ++sv->waiters;
    bool ok = true;
    if (timeout_us < 0)
        sv->cv_done.wait(lk, ready);
    else
        ok = sv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
    --sv->waiters;
    sv->cv_done.notify_all();
    if (sv->stopping && state_status(r) == APSP_ERROR_NOT_READY) return APSP_ERROR_CANCELLED;
    if (!ok) return APSP_ERROR_TIMEOUT;
    return state_status(r);
}

apsp_status_t apsp_server_result(apsp_server_t *sv, uint64_t ticket, const void **d_dist,
                                 const int32_t **d_pred) {
    if (!sv) return APSP_ERROR_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return APSP_ERROR_UNKNOWN_TICKET;
    Request *r = it->second;
    const apsp_status_t st = state_status(r);
    if (st != APSP_SUCCESS) return st;
    const void *dd = r->d_dist;
    const int32_t *pp = r->d_pred;
    if (r->group) {
        char *arena = (char *)r->group->d_arena;
        dd = arena + r->group_off * 4;
        pp = r->want_pred ? (const int32_t *)(arena + r->group->pred_off_bytes + r->group_off * 4) : nullptr;
    }
    if (d_dist) *d_dist = dd;
    if (d_pred) *d_pred = pp;
    return APSP_SUCCESS;
}

apsp_status_t apsp_server_copy_result(apsp_server_t *sv, uint64_t ticket, void *h_dist,
                                      int32_t *h_pred) {
    const void *dd = nullptr;
    const int32_t *pp = nullptr;
    apsp_status_t st = apsp_server_result(sv, ticket, &dd, &pp);
    if (st != APSP_SUCCESS) return st;
    size_t nbytes = 0;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        Request *r = sv->reqs[ticket];
        nbytes = (size_t)(r->n * r->n) * 4;
    }
    if (h_dist && hipMemcpy(h_dist, dd, nbytes, hipMemcpyDeviceToHost) != hipSuccess) return APSP_ERROR_HIP;
    if (h_pred) {
        if (!pp) return APSP_ERROR_INVALID_ARGUMENT;
        if (hipMemcpy(h_pred, pp, nbytes, hipMemcpyDeviceToHost) != hipSuccess) return APSP_ERROR_HIP;
    }
    return APSP_SUCCESS;
}

apsp_status_t apsp_server_release(apsp_server_t *sv, uint64_t ticket) {
    if (!sv) return APSP_ERROR_INVALID_ARGUMENT;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        auto it = sv->reqs.find(ticket);
        if (it == sv->reqs.end()) return APSP_ERROR_UNKNOWN_TICKET;
        Request *r = it->second;
        if (r->state == RState::Queued || r->state == RState::Running) return APSP_ERROR_NOT_READY;
        sv->free_request_device(r);
        sv->bytes_in_use -= (int64_t)(r->resident + r->transient);
        if (r->state != RState::Cancelled) --sv->inflight;
        if (r->h_staging) hipHostFree(r->h_staging);
        sv->reqs.erase(it);
        delete r;
    }
    sv->cv_sched.notify_one();
    return APSP_SUCCESS;
}

apsp_status_t apsp_server_stats(apsp_server_t *sv, apsp_server_stats_t *out) {
    if (!sv || !out) return APSP_ERROR_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lk(sv->mu);
    apsp_server_stats_t s{};
    s.submitted = sv->submitted;
    s.completed = sv->completed;
    s.failed = sv->failed;
    s.cancelled = sv->cancelled;
    s.queued = (int64_t)sv->pending.size();
    s.inflight = sv->inflight;
    s.bytes_in_use = sv->bytes_in_use;
    if (!sv->latencies_ms.empty()) {
        std::vector<double> v = sv->latencies_ms;
        std::sort(v.begin(), v.end());
        auto pct = [&](double q) {
            size_t i = (size_t)std::min<double>((double)v.size() - 1, std::ceil(q * v.size()) - 1);
            return v[i];
        };
        s.p50_latency_ms = pct(0.50);
        s.p99_latency_ms = pct(0.99);
        for (int large = 0; large < 2; ++large) {
            std::vector<double> c;
            for (size_t i = 0; i < sv->latencies_ms.size(); ++i)
                if (sv->latency_large[i] == large) c.push_back(sv->latencies_ms[i]);
            if (c.empty()) continue;
            std::sort(c.begin(), c.end());
            auto q = [&](double f) { return c[(size_t)std::min<double>((double)c.size() - 1, std::ceil(f * c.size()) - 1)]; };
            (large ? s.p50_large_ms : s.p50_small_ms) = q(0.50);
            (large ? s.p99_large_ms : s.p99_small_ms) = q(0.99);
        }
        const double span = std::chrono::duration<double>(sv->last_done - sv->first_submit).count();
        s.solves_per_s = span > 0 ? (double)sv->completed / span : 0.0;
    }
    *out = s;
    return APSP_SUCCESS;
}

apsp_status_t apsp_server_destroy(apsp_server_t *sv) {
    if (!sv) return APSP_ERROR_INVALID_ARGUMENT;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stopping = true;
        for (Request *r : sv->pending) {
            r->state = RState::Cancelled;
            ++sv->cancelled;
        }
        sv->pending.clear();
    }
    sv->cv_sched.notify_all();
    if (sv->scheduler.joinable()) sv->scheduler.join();  // drains running work
    {
        std::unique_lock<std::mutex> lk(sv->mu);
        sv->cv_done.notify_all();
        sv->cv_done.wait(lk, [&] { return sv->waiters == 0; });
        for (auto &kv : sv->reqs) {
            Request *r = kv.second;
            sv->free_request_device(r);
            if (r->h_staging) hipHostFree(r->h_staging);
            delete r;
        }
        sv->reqs.clear();
    }
    for (auto s : sv->streams) hipStreamSynchronize(s);
    if (sv->batch_stream) hipStreamSynchronize(sv->batch_stream);
    if (sv->batch_scratch) hipFree(sv->batch_scratch);
    if (sv->batch_counters) hipFree(sv->batch_counters);
    for (auto s : sv->streams) hipStreamDestroy(s);
    if (sv->batch_stream) hipStreamDestroy(sv->batch_stream);
    delete sv;
    return APSP_SUCCESS;
}

}  // extern "C"
