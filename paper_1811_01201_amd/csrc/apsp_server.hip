// Serving runtime: a request loop on one GPU with continuous batching.
//
// The scheduling core (request table, admission by device-memory budget,
// coalescing, completion bookkeeping, statistics) is apsp_server_core.h;
// this file is its HIP executor:
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
// Host staging of the weights and the status words read back come from a
// pool of pinned buffers that are reused, so steady-state submissions
// allocate no pinned memory; status words are copied back asynchronously,
// ordered before the completion event, so the scheduler never waits on a
// device copy.  Every result is the one apsp_solve gives for that request
// alone (exact arithmetic; the kernels' choices depend only on n, dtype and
// predecessors, never on the mix).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "apsp_internal.h"
#include "apsp_server_core.h"

using namespace apsp;
using apsp::serve::Req;

namespace {

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Pinned host buffers in power-of-two size classes (256 bytes and up), kept
// for reuse after they are returned; at most `keep` bytes are retained.
class PinnedPool {
public:
    explicit PinnedPool(size_t keep) : keep_(keep) {}
    ~PinnedPool() {
        for (auto &kv : free_)
            for (void *p : kv.second) (void)hipHostFree(p);
    }
    void *get(size_t bytes) {
        const int c = size_class(bytes);
        {
            std::lock_guard<std::mutex> lk(mu_);
            auto &v = free_[c];
            if (!v.empty()) {
                void *p = v.back();
                v.pop_back();
                held_ -= class_bytes(c);
                return p;
            }
        }
        void *p = nullptr;
        if (hipHostMalloc(&p, class_bytes(c)) != hipSuccess) return nullptr;
        return p;
    }
    void put(void *p, size_t bytes) {
        if (!p) return;
        const int c = size_class(bytes);
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (held_ + class_bytes(c) <= keep_) {
                free_[c].push_back(p);
                held_ += class_bytes(c);
                return;
            }
        }
        (void)hipHostFree(p);
    }

private:
    static int size_class(size_t bytes) {
        int c = 8;  // 256 bytes
        while (((size_t)1 << c) < bytes) ++c;
        return c;
    }
    static size_t class_bytes(int c) { return (size_t)1 << c; }
    size_t keep_;
    size_t held_ = 0;
    std::mutex mu_;
    std::map<int, std::vector<void *>> free_;
};

struct Group;

// Executor state of one request.
struct RExec {
    void *h_staging = nullptr;  // pinned copy of the weights until uploaded (pool)
    size_t staging_bytes = 0;
    const void *h_src = nullptr;  // upload source: h_staging or the caller's pinned rows
    int64_t h_ld = 0;             // leading dimension of h_src (elements)
    // large path
    void *d_dist = nullptr;
    int32_t *d_pred = nullptr;
    void *d_work = nullptr;
    int32_t *d_status = nullptr;
    int32_t *h_status = nullptr;  // pinned, written by an async copy before `done`
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    apsp_stepper_t *stepper = nullptr;  // sliced large path
    hipEvent_t slice_done = nullptr;
    bool all_issued = true;
    apsp_status_t slice_error = APSP_SUCCESS;
    // batched path
    std::shared_ptr<Group> group;
    int64_t group_off = 0;  // element offset in the group's arena
};

struct Group {
    apsp_dtype_t dtype = APSP_INT32;
    bool want_pred = false;
    void *d_arena = nullptr;  // packed dist | packed pred | status | metadata
    size_t bytes = 0;
    int64_t pred_off_bytes = 0, status_off_bytes = 0;
    void *h_meta = nullptr;   // pinned: metadata source of the upload, then the status words read back
    size_t h_meta_bytes = 0;
    hipEvent_t done = nullptr;
    int members = 0;          // unreleased members
    std::vector<Req *> reqs;
};

RExec *ex_of(const Req *r) { return (RExec *)r->exec; }

}  // namespace

struct apsp_server {
    apsp_server_config_t cfg{};
    int device = 0;
    int cus = 256;
    std::vector<hipStream_t> streams;
    int next_stream = 0;
    hipStream_t batch_stream = nullptr;
    void *batch_scratch = nullptr;
    int64_t batch_scratch_elems = 0;
    int32_t *batch_counters = nullptr;
    int batch_grid = 0;
    int64_t fixed_bytes = 0;
    PinnedPool pinned{(size_t)1 << 30};
    struct HipExec;
    std::unique_ptr<HipExec> exec;
    std::unique_ptr<serve::Core> core;
};

struct apsp_server::HipExec final : serve::Executor {
    apsp_server *sv;
    std::vector<Req *> running_large;
    std::vector<std::shared_ptr<Group>> running_groups;
    std::vector<std::pair<Req *, apsp_status_t>> failed_at_launch;

    explicit HipExec(apsp_server *s) : sv(s) {}

    bool prepare(Req *r, const apsp_request_t &q) override {
        auto *e = new (std::nothrow) RExec();
        if (!e) return false;
        const int64_t ld = q.ld ? q.ld : q.n;
        if (q.borrow) {
            e->h_src = q.weights;
            e->h_ld = ld;
        } else {
            e->staging_bytes = std::max<size_t>((size_t)(q.n * q.n) * 4, 4);
            e->h_staging = sv->pinned.get(e->staging_bytes);
            if (!e->h_staging) {
                delete e;
                return false;
            }
            const size_t row = (size_t)q.n * 4;
            for (int64_t i = 0; i < q.n; ++i)
                std::memcpy((char *)e->h_staging + (size_t)i * row, (const char *)q.weights + (size_t)(i * ld) * 4,
                            row);
            e->h_src = e->h_staging;
            e->h_ld = q.n;
        }
        r->exec = e;
        return true;
    }

    void drop_staging(RExec *e) {
        if (e->h_staging) sv->pinned.put(e->h_staging, e->staging_bytes);
        e->h_staging = nullptr;
    }

    void unprepare(Req *r) override {
        RExec *e = ex_of(r);
        if (!e) return;
        drop_staging(e);
        delete e;
        r->exec = nullptr;
    }

    void fail_now(Req *r, apsp_status_t st) { failed_at_launch.push_back({r, st}); }

    // After the last kernel of a large request: the status word goes to
    // pinned memory, then the completion event.
    static apsp_status_t finish_issue(RExec *e, hipStream_t s) {
        if (hipMemcpyAsync(e->h_status, e->d_status, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipEventRecord(e->done, s) != hipSuccess)
            return APSP_ERROR_HIP;
        return APSP_SUCCESS;
    }

    void launch_large(Req *r) override {
        RExec *e = ex_of(r);
        e->stream = sv->streams[sv->next_stream++ % sv->streams.size()];
        hipStream_t s = e->stream;
        const size_t mat = (size_t)(r->n * r->n) * 4;
        apsp_status_t st = APSP_SUCCESS;
        e->h_status = (int32_t *)sv->pinned.get(256);
        if (!e->h_status || hipMallocAsync(&e->d_dist, mat, s) != hipSuccess ||
            (r->want_pred && hipMallocAsync((void **)&e->d_pred, mat, s) != hipSuccess) ||
            hipMallocAsync((void **)&e->d_status, 256, s) != hipSuccess ||
            (r->transient && hipMallocAsync(&e->d_work, r->transient, s) != hipSuccess)) {
            st = APSP_ERROR_OUT_OF_MEMORY;
        }
        if (st == APSP_SUCCESS &&
            hipMemcpy2DAsync(e->d_dist, (size_t)r->n * 4, e->h_src, (size_t)e->h_ld * 4, (size_t)r->n * 4,
                             (size_t)r->n, hipMemcpyHostToDevice, s) != hipSuccess)
            st = APSP_ERROR_HIP;
        apsp_options_t opt{};
        opt.d_status = e->d_status;
        if (st == APSP_SUCCESS && hipEventCreateWithFlags(&e->done, hipEventDisableTiming) != hipSuccess)
            st = APSP_ERROR_HIP;
        if (st == APSP_SUCCESS && sv->cfg.slice_rounds > 0) {
            // sliced: record the solve, issue its first slice
            int32_t last = 0;
            st = stepper_create(r->n, r->dtype, r->want_pred, &opt, true, e->d_work, r->transient, &e->stepper);
            if (st == APSP_SUCCESS && hipEventCreateWithFlags(&e->slice_done, hipEventDisableTiming) != hipSuccess)
                st = APSP_ERROR_HIP;
            if (st == APSP_SUCCESS) st = apsp_stepper_begin(e->stepper, e->d_dist, e->d_pred, s);
            if (st == APSP_SUCCESS) st = apsp_stepper_step(e->stepper, sv->cfg.slice_rounds, &last);
            if (st == APSP_SUCCESS) {
                if (last)
                    st = finish_issue(e, s);
                else if (hipEventRecord(e->slice_done, s) != hipSuccess)
                    st = APSP_ERROR_HIP;
            }
            e->all_issued = last != 0;
        } else if (st == APSP_SUCCESS) {
            st = solve_internal(e->d_dist, e->d_pred, r->n, r->dtype, s, opt, e->d_work, r->transient);
            if (st == APSP_SUCCESS) st = finish_issue(e, s);
        }
        if (st != APSP_SUCCESS) {
            (void)hipStreamSynchronize(s);
            if (e->stepper) stepper_destroy(e->stepper, false);
            e->stepper = nullptr;
            if (e->slice_done) (void)hipEventDestroy(e->slice_done);
            e->slice_done = nullptr;
            e->all_issued = true;
            if (e->d_work) (void)hipFreeAsync(e->d_work, s);
            e->d_work = nullptr;
            drop_staging(e);
            fail_now(r, st);
            return;
        }
        running_large.push_back(r);
    }

    int64_t launch_group(std::vector<Req *> &batch) override {
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
        batch_meta(ns.data(), offs.data(), B, g->dtype, g->want_pred, nullptr, meta_host, n_team, need_scratch,
                   lean);
        const size_t meta_bytes = round_up(meta_host.size(), 256);
        g->pred_off_bytes = (int64_t)dist_bytes;
        g->status_off_bytes = (int64_t)(dist_bytes + pred_bytes);
        g->bytes = dist_bytes + pred_bytes + status_bytes + meta_bytes;
        g->members = B;
        g->reqs = batch;
        int64_t delta = (int64_t)g->bytes;
        for (auto *r : batch) {
            delta -= (int64_t)(r->resident + r->transient);  // accounted by the group instead
            r->resident = r->transient = 0;
            ex_of(r)->group = g;
        }
        apsp_status_t st = need_scratch > sv->batch_scratch_elems ? APSP_ERROR_INVALID_ARGUMENT : APSP_SUCCESS;
        hipStream_t s = sv->batch_stream;
        // one pinned buffer: the metadata to upload, later the status words read back
        g->h_meta_bytes = std::max(meta_bytes, status_bytes);
        if (st == APSP_SUCCESS && !(g->h_meta = sv->pinned.get(g->h_meta_bytes))) st = APSP_ERROR_OUT_OF_MEMORY;
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
            Req *r = batch[b];
            RExec *e = ex_of(r);
            e->group_off = offs[b];
            if (hipMemcpy2DAsync(arena + offs[b] * 4, (size_t)r->n * 4, e->h_src, (size_t)e->h_ld * 4,
                                 (size_t)r->n * 4, (size_t)r->n, hipMemcpyHostToDevice, s) != hipSuccess)
                st = APSP_ERROR_HIP;
        }
        if (st == APSP_SUCCESS) {
            // the scratch holds 2 x CUs work matrices of 8-byte elements, i.e.
            // 4 x CUs of 4-byte ones: room for the lean kernel's workgroups
            const int grid = lean ? std::min(4, batched_blocks_per_cu(g->dtype, true)) * sv->cus : sv->batch_grid;
            BatchLaunch L{meta, B, n_team, sv->batch_scratch_elems, sv->batch_scratch, sv->batch_counters, grid, lean};
            st = batched_launch(L, g->dtype, g->want_pred, arena,
                                g->want_pred ? (int32_t *)(arena + g->pred_off_bytes) : nullptr,
                                (int32_t *)(arena + g->status_off_bytes), s);
        }
        // the status words come back into the pinned buffer (stream order puts
        // this after the metadata upload has been consumed), then the event
        if (st == APSP_SUCCESS &&
            (hipMemcpyAsync(g->h_meta, arena + g->status_off_bytes, (size_t)B * 4, hipMemcpyDeviceToHost, s) !=
                 hipSuccess ||
             hipEventCreateWithFlags(&g->done, hipEventDisableTiming) != hipSuccess ||
             hipEventRecord(g->done, s) != hipSuccess))
            st = APSP_ERROR_HIP;
        if (st != APSP_SUCCESS) {
            (void)hipStreamSynchronize(s);
            for (auto *r : batch) {
                drop_staging(ex_of(r));
                fail_now(r, st);
            }
            return delta;
        }
        running_groups.push_back(g);
        return delta;
    }

    int64_t poll(std::vector<std::pair<Req *, apsp_status_t>> &done) override {
        int64_t freed = 0;
        for (auto &f : failed_at_launch) {
            freed += (int64_t)f.first->transient;
            f.first->transient = 0;
            done.push_back(f);
        }
        failed_at_launch.clear();
        for (auto it = running_large.begin(); it != running_large.end();) {
            Req *r = *it;
            RExec *e = ex_of(r);
            if (!e->all_issued) {
                // sliced: the next slice once the previous one has finished
                if (hipEventQuery(e->slice_done) == hipSuccess) {
                    int32_t last = 0;
                    apsp_status_t st = apsp_stepper_step(e->stepper, sv->cfg.slice_rounds, &last);
                    if (st == APSP_SUCCESS) {
                        if (last)
                            st = finish_issue(e, e->stream);
                        else if (hipEventRecord(e->slice_done, e->stream) != hipSuccess)
                            st = APSP_ERROR_HIP;
                    }
                    if (st != APSP_SUCCESS) {
                        // what was issued still runs: let it finish, then fail the request
                        e->slice_error = st;
                        (void)hipStreamSynchronize(e->stream);
                        (void)hipEventRecord(e->done, e->stream);
                        last = 1;
                    }
                    if (last) e->all_issued = true;
                }
                ++it;
                continue;
            }
            if (hipEventQuery(e->done) == hipSuccess) {
                const apsp_status_t st =
                    e->slice_error != APSP_SUCCESS ? e->slice_error : (apsp_status_t)*e->h_status;
                if (e->stepper) stepper_destroy(e->stepper, false);  // its work has completed
                e->stepper = nullptr;
                if (e->slice_done) (void)hipEventDestroy(e->slice_done);
                e->slice_done = nullptr;
                if (e->d_work) (void)hipFreeAsync(e->d_work, e->stream);
                e->d_work = nullptr;
                drop_staging(e);
                freed += (int64_t)r->transient;
                r->transient = 0;
                done.push_back({r, st});
                it = running_large.erase(it);
            } else {
                ++it;
            }
        }
        for (auto it = running_groups.begin(); it != running_groups.end();) {
            Group *g = it->get();
            if (hipEventQuery(g->done) == hipSuccess) {
                const int32_t *status = (const int32_t *)g->h_meta;
                for (size_t i = 0; i < g->reqs.size(); ++i) {
                    Req *r = g->reqs[i];
                    drop_staging(ex_of(r));
                    done.push_back({r, (apsp_status_t)status[i]});
                }
                sv->pinned.put(g->h_meta, g->h_meta_bytes);
                g->h_meta = nullptr;
                it = running_groups.erase(it);
            } else {
                ++it;
            }
        }
        return freed;
    }

    void result(const Req *r, const void **d_dist, const int32_t **d_pred) override {
        const RExec *e = ex_of(r);
        const void *dd = e->d_dist;
        const int32_t *pp = e->d_pred;
        if (e->group) {
            char *arena = (char *)e->group->d_arena;
            dd = arena + e->group_off * 4;
            pp = r->want_pred ? (const int32_t *)(arena + e->group->pred_off_bytes + e->group_off * 4) : nullptr;
        }
        if (d_dist) *d_dist = dd;
        if (d_pred) *d_pred = pp;
    }

    int64_t release(Req *r) override {
        RExec *e = ex_of(r);
        if (!e) return 0;
        int64_t extra = 0;
        hipStream_t s = e->stream ? e->stream : sv->batch_stream;
        if (e->d_dist) (void)hipFreeAsync(e->d_dist, s);
        if (e->d_pred) (void)hipFreeAsync(e->d_pred, s);
        if (e->d_work) (void)hipFreeAsync(e->d_work, s);
        if (e->d_status) (void)hipFreeAsync(e->d_status, s);
        if (e->done) (void)hipEventDestroy(e->done);
        if (e->h_status) sv->pinned.put(e->h_status, 256);
        if (e->group) {
            Group *g = e->group.get();
            if (--g->members == 0) {
                if (g->d_arena) (void)hipFreeAsync(g->d_arena, sv->batch_stream);
                if (g->done) (void)hipEventDestroy(g->done);
                if (g->h_meta) sv->pinned.put(g->h_meta, g->h_meta_bytes);
                g->d_arena = nullptr;
                g->done = nullptr;
                g->h_meta = nullptr;
                extra = (int64_t)g->bytes;
            }
            e->group.reset();
        }
        drop_staging(e);
        delete e;
        r->exec = nullptr;
        return extra;
    }

    bool busy() override { return !running_large.empty() || !running_groups.empty() || !failed_at_launch.empty(); }
};

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
    (void)hipDeviceGetAttribute(&sv->cus, hipDeviceAttributeMultiprocessorCount, sv->device);
    if (cfg.hbm_budget_bytes == 0) {
        size_t free_b = 0, total_b = 0;
        (void)hipMemGetInfo(&free_b, &total_b);
        cfg.hbm_budget_bytes = (int64_t)(free_b / 2);
    }
    if (cfg.max_inflight == 0) cfg.max_inflight = 64;
    if (cfg.n_streams == 0) cfg.n_streams = 8;
    if (cfg.max_queue == 0) cfg.max_queue = 4096;
    if (cfg.batch_max_n == 0) cfg.batch_max_n = 512;
    if (cfg.batch_max_n < 0) cfg.batch_max_n = 0;  // never coalesce
    sv->cfg = cfg;
    auto fail = [&](apsp_status_t st) {
        apsp_server_destroy(sv);
        return st;
    };
    // keep freed device memory in the stream-ordered pool for reuse
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, sv->device) == hipSuccess) {
        uint64_t keep = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    for (int i = 0; i < cfg.n_streams; ++i) {
        hipStream_t s;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return fail(APSP_ERROR_HIP);
        sv->streams.push_back(s);
    }
    if (hipStreamCreateWithFlags(&sv->batch_stream, hipStreamNonBlocking) != hipSuccess) return fail(APSP_ERROR_HIP);
    if (cfg.batch_max_n > 0) {
        // work matrices of up to 128-padded batch_max_n (every team configuration fits)
        const int64_t ldp = std::max<int64_t>(128, (cfg.batch_max_n + 127) / 128 * 128);
        sv->batch_grid = 2 * sv->cus;
        sv->batch_scratch_elems = ldp * ldp;
        const size_t bytes = (size_t)sv->batch_grid * sv->batch_scratch_elems * 8;
        if ((int64_t)bytes >= cfg.hbm_budget_bytes || hipMalloc(&sv->batch_scratch, bytes) != hipSuccess ||
            hipMalloc((void **)&sv->batch_counters, 32) != hipSuccess ||
            hipMemset(sv->batch_counters, 0, 32) != hipSuccess ||
            hipDeviceSynchronize() != hipSuccess)  // the null-stream memset done before any stream uses them
            return fail(APSP_ERROR_OUT_OF_MEMORY);
        sv->fixed_bytes = (int64_t)bytes;
    }
    serve::CoreConfig cc;
    cc.budget = cfg.hbm_budget_bytes;
    cc.fixed = sv->fixed_bytes;
    cc.max_inflight = cfg.max_inflight;
    cc.max_queue = cfg.max_queue;
    cc.batch_max_n = cfg.batch_max_n;
    sv->exec.reset(new (std::nothrow) apsp_server::HipExec(sv));
    if (!sv->exec) return fail(APSP_ERROR_OUT_OF_MEMORY);
    sv->core.reset(new (std::nothrow) serve::Core(cc, sv->exec.get()));
    if (!sv->core) return fail(APSP_ERROR_OUT_OF_MEMORY);
    const int dev = sv->device;
    sv->core->start([dev] { (void)hipSetDevice(dev); });
    *out = sv;
    return APSP_SUCCESS;
}

apsp_status_t apsp_server_submit(apsp_server_t *sv, const apsp_request_t *req, uint64_t *ticket) {
    if (!sv || !req || !ticket || !req->weights || req->n < 1 || req->n > kMaxN ||
        (req->dtype != APSP_INT32 && req->dtype != APSP_FLOAT32) || (req->ld != 0 && req->ld < req->n))
        return APSP_ERROR_INVALID_ARGUMENT;
    const size_t transient =
        req->n <= sv->cfg.batch_max_n ? 0 : solve_work_bytes(req->n, req->dtype, req->want_pred != 0);
    return sv->core->submit(*req, transient, ticket);
}

apsp_status_t apsp_server_poll(apsp_server_t *sv, uint64_t ticket) {
    if (!sv) return APSP_ERROR_INVALID_ARGUMENT;
    return sv->core->poll(ticket);
}

apsp_status_t apsp_server_wait(apsp_server_t *sv, uint64_t ticket, int64_t timeout_us) {
    if (!sv) return APSP_ERROR_INVALID_ARGUMENT;
    return sv->core->wait(ticket, timeout_us);
}

apsp_status_t apsp_server_result(apsp_server_t *sv, uint64_t ticket, const void **d_dist,
                                 const int32_t **d_pred) {
    if (!sv) return APSP_ERROR_INVALID_ARGUMENT;
    return sv->core->result(ticket, d_dist, d_pred);
}

apsp_status_t apsp_server_copy_result(apsp_server_t *sv, uint64_t ticket, void *h_dist, int32_t *h_pred) {
    if (!sv) return APSP_ERROR_INVALID_ARGUMENT;
    // the request stays pinned (a concurrent release waits) while it is copied
    return sv->core->with_result(ticket, [&](int64_t n, const void *dd, const int32_t *pp) -> apsp_status_t {
        const size_t nbytes = (size_t)(n * n) * 4;
        if (h_pred && !pp) return APSP_ERROR_INVALID_ARGUMENT;
        if (h_dist && hipMemcpy(h_dist, dd, nbytes, hipMemcpyDeviceToHost) != hipSuccess) return APSP_ERROR_HIP;
        if (h_pred && hipMemcpy(h_pred, pp, nbytes, hipMemcpyDeviceToHost) != hipSuccess) return APSP_ERROR_HIP;
        return APSP_SUCCESS;
    });
}

apsp_status_t apsp_server_release(apsp_server_t *sv, uint64_t ticket) {
    if (!sv) return APSP_ERROR_INVALID_ARGUMENT;
    return sv->core->release(ticket);
}

apsp_status_t apsp_server_stats(apsp_server_t *sv, apsp_server_stats_t *out) {
    if (!sv || !out) return APSP_ERROR_INVALID_ARGUMENT;
    *out = sv->core->stats();
    return APSP_SUCCESS;
}

apsp_status_t apsp_server_destroy(apsp_server_t *sv) {
    if (!sv) return APSP_ERROR_INVALID_ARGUMENT;
    if (sv->core) sv->core->stop();  // cancels queued requests, drains running ones, frees all
    for (auto s : sv->streams) (void)hipStreamSynchronize(s);
    if (sv->batch_stream) (void)hipStreamSynchronize(sv->batch_stream);
    sv->core.reset();
    sv->exec.reset();
    if (sv->batch_scratch) (void)hipFree(sv->batch_scratch);
    if (sv->batch_counters) (void)hipFree(sv->batch_counters);
    for (auto s : sv->streams) (void)hipStreamDestroy(s);
    if (sv->batch_stream) (void)hipStreamDestroy(sv->batch_stream);
    delete sv;
    return APSP_SUCCESS;
}

}  // extern "C"
