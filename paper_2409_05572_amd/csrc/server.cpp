// Serving runtime: several solves resident on one GPU.
//
// Each slot owns a context (its own stream and grow-only workspace) and a
// host worker thread that runs one solve at a time. Requests wait in a FIFO
// queue; the head request starts on a free slot as soon as the device
// workspace held by all slots, after that slot grows to the request's
// footprint, fits the HBM budget (the slot with the largest workspace that
// needs the least growth is chosen). When it does not fit, the other idle
// slots give their workspace back (each on its own worker thread) and the
// request is tried again; a request never waits on memory that only idle
// slots hold. Different slots run their kernels on different streams, so
// small solves overlap on the GPU; a solve's arithmetic does not depend on
// what else runs, so results match a lone se_solve.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "engine.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    se_ticket id = 0;
    const se_matrix* A = nullptr;
    se_params p{};
    const double* X0 = nullptr;
    double* V = nullptr;
    double* lambda = nullptr;
    uint64_t footprint = 0;
    se_info info{};
    se_status status = SE_OK;
    bool done = false;
    Clock::time_point t_submit, t_start, t_end;
};

struct Slot {
    se_ctx* ctx = nullptr;
    std::thread worker;
    Request* job = nullptr;  // assigned request (nullptr = idle)
    uint64_t held = 0;       // device workspace held by the slot's context
    bool trim = false;       // idle slot asked to release its workspace
};

}  // namespace

struct se_server {
    int device = 0;
    uint64_t budget = 0;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_work;  // a slot may have work
    std::condition_variable cv_done;  // some request finished
    std::deque<Request*> queue;
    std::unordered_map<se_ticket, std::unique_ptr<Request>> reqs;
    se_ticket next = 1;
    bool stop = false;

    uint64_t held_total() const {
        uint64_t s = 0;
        for (const Slot& sl : slots) s += sl.held;
        return s;
    }

    // Assign queued requests to idle slots while the budget allows. When the
    // head request does not fit, the other idle slots are asked to release
    // their workspace; each does so on its own thread and schedules again.
    // Otherwise a running solve's end schedules again. Since a request's
    // footprint is at most the budget, the head request always fits once
    // nothing runs and the idle slots are trimmed. Caller holds mu.
    void schedule() {
        while (!queue.empty()) {
            Request* r = queue.front();
            int best = -1;
            uint64_t best_growth = UINT64_MAX;
            for (int i = 0; i < (int)slots.size(); ++i) {
                if (slots[i].job || slots[i].trim) continue;
                const uint64_t growth = r->footprint > slots[i].held ? r->footprint - slots[i].held : 0;
                if (growth < best_growth || (growth == best_growth && best >= 0 &&
                                             slots[i].held > slots[best].held)) {
                    best = i;
                    best_growth = growth;
                }
            }
            if (best < 0) return;  // no idle slot (or only slots being trimmed)
            if (best_growth > 0 && held_total() + best_growth > budget) {
                bool asked = false;
                for (int i = 0; i < (int)slots.size(); ++i)
                    if (i != best && !slots[i].job && !slots[i].trim && slots[i].held > 0) {
                        slots[i].trim = true;
                        asked = true;
                    }
                if (asked) cv_work.notify_all();
                return;  // wait for trimmed or finishing slots
            }
            slots[best].held += best_growth;
            slots[best].job = r;
            queue.pop_front();
            r->t_start = Clock::now();
            cv_work.notify_all();
        }
    }

    void run_slot(int i) {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            cv_work.wait(lk, [&] { return stop || slots[i].job != nullptr || slots[i].trim; });
            if (slots[i].trim && !slots[i].job) {
                // give the workspace back (the slot's last solve has
                // synchronized its stream), then retry the queue
                lk.unlock();
                (void)hipStreamSynchronize(slots[i].ctx->stream);
                slots[i].ctx->ws.release();
                lk.lock();
                slots[i].held = 0;
                slots[i].trim = false;
                schedule();
                continue;
            }
            Request* r = slots[i].job;
            if (!r) return;  // stop with nothing assigned
            lk.unlock();
            std::memset(&r->info, 0, sizeof(r->info));
            (void)hipGetLastError();  // a stale error of this thread must not fail the solve
            const se_status st = se::solve(slots[i].ctx, r->A, &r->p, r->X0, r->V, r->lambda, &r->info);
            const uint64_t held = slots[i].ctx->ws.device_bytes();
            lk.lock();
            r->status = st;
            r->t_end = Clock::now();
            r->done = true;
            slots[i].job = nullptr;
            slots[i].held = held;
            schedule();
            cv_done.notify_all();
            if (stop && queue.empty()) {
                bool idle = true;
                for (const Slot& sl : slots) idle = idle && !sl.job;
                if (idle) cv_work.notify_all();
            }
        }
    }
};

extern "C" {

uint64_t se_solve_footprint(int64_t n, int64_t nnz, int32_t n_ev, int32_t n_extra, int32_t precision,
                            int32_t solver) {
    if (n < 1 || n_ev < 1 || n_extra < 0) return 0;
    return (uint64_t)se::solve_workspace_bytes(n, nnz, n_ev + n_extra, precision, solver);
}

se_status se_server_create(se_ctx* ctx, uint64_t hbm_budget_bytes, int32_t max_slots, se_server** out) {
    if (!ctx || !out || max_slots < 1 || max_slots > 16 || hbm_budget_bytes == 0) return SE_ERR_INVALID_ARG;
    *out = nullptr;
    if (hipSetDevice(ctx->device) != hipSuccess) return SE_ERR_HIP;
    auto* s = new (std::nothrow) se_server();
    if (!s) return SE_ERR_OOM;
    s->device = ctx->device;
    s->budget = hbm_budget_bytes;
    s->slots.resize(max_slots);
    for (Slot& sl : s->slots) {
        sl.ctx = new (std::nothrow) se_ctx();
        hipStream_t stream = nullptr;
        if (!sl.ctx || hipStreamCreate(&stream) != hipSuccess) {
            delete sl.ctx;
            sl.ctx = nullptr;
            for (Slot& o : s->slots)
                if (o.ctx) {
                    (void)hipStreamDestroy(o.ctx->stream);
                    delete o.ctx;
                }
            delete s;
            return SE_ERR_HIP;
        }
        sl.ctx->device = ctx->device;
        sl.ctx->stream = stream;
    }
    for (int i = 0; i < max_slots; ++i) s->slots[i].worker = std::thread([s, i] { s->run_slot(i); });
    *out = s;
    return SE_OK;
}

se_status se_submit(se_server* srv, const se_matrix* A, const se_params* params, const double* X0,
                    double* V, double* lambda, se_ticket* ticket) {
    if (!srv || !A || !params || !V || !lambda || !ticket) return SE_ERR_INVALID_ARG;
    if (!A->ctx || A->ctx->device != srv->device || A->is_complex) return SE_ERR_INVALID_ARG;
    const se_status v = se::validate_solve(A, params);
    if (v != SE_OK) return v;
    auto r = std::make_unique<Request>();
    r->A = A;
    r->p = *params;
    r->X0 = X0;
    r->V = V;
    r->lambda = lambda;
    r->footprint = se_solve_footprint(A->n, A->nnz, params->n_ev, params->n_extra, params->precision,
                                      params->solver);
    if (r->footprint > srv->budget) return SE_ERR_REJECTED;
    // (a mixed-precision solve makes the matrix's FP32 values on its own slot
    // stream, once per matrix, under the matrix's lock)
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return SE_ERR_REJECTED;
    r->id = srv->next++;
    r->t_submit = Clock::now();
    *ticket = r->id;
    srv->queue.push_back(r.get());
    srv->reqs.emplace(r->id, std::move(r));
    srv->schedule();
    return SE_OK;
}

se_status se_poll(se_server* srv, se_ticket ticket, int32_t* done) {
    if (!srv || !done) return SE_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return SE_ERR_INVALID_ARG;
    *done = it->second->done ? 1 : 0;
    return SE_OK;
}

se_status se_wait(se_server* srv, se_ticket ticket, se_info* info, double* queue_ms, double* run_ms) {
    if (!srv) return SE_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return SE_ERR_INVALID_ARG;
    Request* r = it->second.get();
    srv->cv_done.wait(lk, [&] { return r->done; });
    if (info) *info = r->info;
    if (queue_ms)
        *queue_ms = std::chrono::duration<double, std::milli>(r->t_start - r->t_submit).count();
    if (run_ms) *run_ms = std::chrono::duration<double, std::milli>(r->t_end - r->t_start).count();
    const se_status st = r->status;
    srv->reqs.erase(it);
    return st;
}

void se_server_destroy(se_server* srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        for (Request* r : srv->queue) {
            r->status = SE_ERR_REJECTED;
            r->t_start = r->t_end = Clock::now();
            r->done = true;
        }
        srv->queue.clear();
        srv->cv_work.notify_all();
        srv->cv_done.notify_all();
    }
    for (Slot& sl : srv->slots)
        if (sl.worker.joinable()) sl.worker.join();
    (void)hipSetDevice(srv->device);
    for (Slot& sl : srv->slots) {
        if (!sl.ctx) continue;
        (void)hipStreamSynchronize(sl.ctx->stream);
        sl.ctx->ws.release();
        (void)hipStreamDestroy(sl.ctx->stream);
        delete sl.ctx;
    }
    delete srv;
}

}  // extern "C"
