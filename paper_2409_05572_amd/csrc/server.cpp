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
//
// Batched mode (se_server_create_batched): one engine thread advances all
// resident solves together, one LOBPCG iteration per step, with one launch per
// phase for all of them (batch.hip). A step is a fixed sequence of launches
// (issued directly or replayed from a graph built once); the host uploads the
// step's decisions, runs the step, reads back every solve's residual ratios
// and decides the next step (one synchronization per step for all solves).
// New requests join at step boundaries.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstddef>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batch.h"
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

// A resident solve of the batched engine (host side).
struct BSlot {
    Request* r = nullptr;
    se::DevBuf mem;  // panels, partials and small matrices (grow-only)
    se::Strategy ctl;
    int n_ev = 0, nb = 0, j = 0, n_shr = 0, n_exp = 0;
    bool init = false, have_drop = false;
    // decisions for the next step
    int a = 0, expand = 0, shrink = 0;
    std::vector<int> act;
};

// Sizes of a batched solve of order n and block width nb.
struct BPlan {
    int poff, nch_g, nch_r;
    long long ldw, rows_g, rows_r;
    size_t doubles;
};
BPlan bplan(long long n, int nb) {
    BPlan b;
    b.poff = nb + (nb & 1);
    b.ldw = 2 * (long long)b.poff + 2;
    // Gram chunks: about 64 per solve, at least 256 rows, multiples of 32
    long long rg = (n + 63) / 64;
    rg = std::max(256LL, (rg + 31) / 32 * 32);
    b.rows_g = rg;
    b.nch_g = (int)((n + rg - 1) / rg);
    b.rows_r = 2048;  // as launch_resid_norms (its chunk count is used for the final check too)
    b.nch_r = (int)std::max(1LL, (n + b.rows_r - 1) / b.rows_r);
    b.doubles = 8 * (size_t)n * b.ldw + (size_t)b.nch_g * se::kBMMax * se::kBMMax +
                (size_t)b.nch_r * 2 * se::kBNbMax + se::bsmall_doubles() + 64;
    return b;
}

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

    // batched mode
    bool batched = false;
    bool use_graph = false;
    std::atomic<long long> steps{0};          // steps run by the engine
    std::atomic<long long> graph_steps{0};    // of which replayed from the captured graph
    std::thread engine;
    hipStream_t bst = nullptr;   // lane 0, admission and result copies
    hipStream_t bst2 = nullptr;  // lane 1
    hipEvent_t ev_ctl = nullptr;
    std::vector<BSlot> bslots;
    se::DevBuf d_fix, d_ctl, d_dyn, d_jobs;
    se::HostBuf h_fix, h_ctl, h_dyn, h_out;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int graph_grid = 0;

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

    // ---- batched mode ----
    uint64_t held_batched() const {
        uint64_t h = 0;
        for (const BSlot& b : bslots) h += b.mem.bytes;
        return h;
    }

    // Start queued requests on free slots while the budget allows (idle slots
    // give their memory back when the head request does not fit). Caller
    // holds mu; runs on the engine thread, which owns every slot's memory.
    void admit_batched(std::vector<int>& fresh) {
        while (!queue.empty()) {
            Request* r = queue.front();
            // a free slot of the lane with the least resident work (sum of n),
            // then the one holding the most memory
            long long load[2] = {0, 0};
            for (int l = 0; l < lanes(); ++l)
                for (int i = lane_begin(l); i < lane_end(l); ++i)
                    if (bslots[i].r) load[l] += bslots[i].r->A->n;
            int best = -1, best_lane = 0;
            for (int l = 0; l < lanes(); ++l)
                for (int i = lane_begin(l); i < lane_end(l); ++i) {
                    if (bslots[i].r) continue;
                    if (best < 0 || load[l] < load[best_lane] ||
                        (l == best_lane && bslots[i].mem.bytes > bslots[best].mem.bytes)) {
                        best = i;
                        best_lane = l;
                    }
                }
            if (best < 0) return;
            const uint64_t growth = r->footprint > bslots[best].mem.bytes ? r->footprint - bslots[best].mem.bytes : 0;
            if (growth > 0 && held_batched() + growth > budget) {
                bool freed = false;
                for (int i = 0; i < (int)bslots.size(); ++i)
                    if (i != best && !bslots[i].r && bslots[i].mem.bytes > 0) {
                        bslots[i].mem.release();
                        freed = true;
                    }
                if (!freed || held_batched() + growth > budget) return;  // wait for running solves
            }
            bslots[best].r = r;
            queue.pop_front();
            r->t_start = Clock::now();
            fresh.push_back(best);
        }
    }

    se::BFix* hfix() { return h_fix.as<se::BFix>(); }
    se::BCtl* hctl() { return h_ctl.as<se::BCtl>(); }
    se::BDyn* hdyn() { return h_dyn.as<se::BDyn>(); }
    const double* dev_lam(int s) const {
        return reinterpret_cast<const double*>(d_dyn.as<char>() + sizeof(se::BDyn) * s + offsetof(se::BDyn, lam));
    }

    // Device memory, constants, state and start block of a new solve.
    se_status setup_slot(int s) {
        BSlot& b = bslots[s];
        Request* r = b.r;
        const se_matrix* A = r->A;
        const long long n = A->n;
        b.n_ev = r->p.n_ev;
        b.nb = r->p.n_ev + r->p.n_extra;
        const BPlan pl = bplan(n, b.nb);
        if (b.mem.ensure(sizeof(double) * pl.doubles) != hipSuccess) return SE_ERR_OOM;
        double* q = b.mem.as<double>();
        const size_t panel = (size_t)n * pl.ldw;
        se::BFix F{};
        F.rowptr = A->rowptr;
        F.col = A->col;
        F.val = A->val;
        F.xp[0] = q;
        F.xp[1] = q + panel;
        F.axp[0] = q + 2 * panel;
        F.axp[1] = q + 3 * panel;
        F.xpd = q + 4 * panel;
        F.w[0] = q + 5 * panel;
        F.w[1] = q + 6 * panel;
        F.aw = q + 7 * panel;
        F.part = q + 8 * panel;
        F.rpart = F.part + (size_t)pl.nch_g * se::kBMMax * se::kBMMax;
        F.sm = F.rpart + (size_t)pl.nch_r * 2 * se::kBNbMax;
        F.anorm = A->anorm;
        F.rows_g = pl.rows_g;
        F.rows_r = pl.rows_r;
        F.n = (int)n;
        F.nb = b.nb;
        int n_es = r->p.n_es;
        if (n_es <= 0) n_es = b.n_ev + std::min(5, r->p.n_extra - 1);
        F.n_es = n_es;
        F.ldw = (int)pl.ldw;
        F.poff = pl.poff;
        F.nch_g = pl.nch_g;
        F.nch_r = pl.nch_r;
        hfix()[s] = F;
        se::BDyn& D = hdyn()[s];
        std::memset(&D, 0, sizeof(D));
        D.w = b.nb;
        if (hipMemcpyAsync(d_fix.as<se::BFix>() + s, &hfix()[s], sizeof(se::BFix), hipMemcpyHostToDevice, bst) !=
                hipSuccess ||
            hipMemcpyAsync(d_dyn.as<se::BDyn>() + s, &D, sizeof(se::BDyn), hipMemcpyHostToDevice, bst) != hipSuccess)
            return SE_ERR_HIP;
        hipError_t e;
        if (!r->X0)
            e = se::launch_seeded_block(bst, n, b.nb, (unsigned long long)r->p.seed, F.w[0], pl.ldw, false);
        else if (r->p.ptr_mode == SE_PTR_HOST) {
            e = hipMemcpyAsync(F.w[1], r->X0, sizeof(double) * (size_t)n * b.nb, hipMemcpyHostToDevice, bst);
            if (e == hipSuccess) e = se::launch_colmajor_to_rowmajor(bst, n, b.nb, F.w[1], n, F.w[0], pl.ldw);
        } else {
            e = se::launch_colmajor_to_rowmajor(bst, n, b.nb, r->X0, n, F.w[0], pl.ldw);
        }
        if (e != hipSuccess) return SE_ERR_HIP;
        // the host's copies must not change before the copies above ran
        if (hipStreamSynchronize(bst) != hipSuccess) return SE_ERR_HIP;
        b.ctl = se::Strategy{};
        b.ctl.kind = r->p.strategy;
        b.ctl.j_e = r->p.j_e;
        b.ctl.j_s = r->p.j_s;
        b.ctl.j_p = r->p.j_p;
        b.ctl.j_warm = r->p.j_warm;
        b.ctl.mu = r->p.mu;
        b.ctl.r_warm = r->p.r_warm;
        const bool se_on = b.ctl.enabled() && r->p.n_extra >= 2 && n_es >= b.n_ev && n_es < b.nb;
        if (!se_on) b.ctl.kind = SE_STRAT_NONE;
        b.j = b.n_shr = b.n_exp = 0;
        b.have_drop = false;
        b.init = true;
        b.a = b.expand = b.shrink = 0;
        std::memset(&r->info, 0, sizeof(r->info));
        return SE_OK;
    }

    // Fresh residual of the returned pairs, results to the caller's buffers.
    se_status finish_slot(int s, bool conv) {
        BSlot& b = bslots[s];
        Request* r = b.r;
        const se::BFix& F = hfix()[s];
        const se::BDyn& D = hdyn()[s];
        const long long n = F.n;
        const int k = b.n_ev;
        const double* X = F.xp[D.cur];
        double* out = F.sm + se::BSmall::G;
        hipError_t e = se::launch_spmm(bst, (int)n, F.rowptr, F.col, F.val, X, F.ldw, F.aw, F.ldw, k, nullptr, 0);
        if (e == hipSuccess)
            e = se::launch_resid_norms(bst, n, X, F.aw, F.ldw, k, dev_lam(s), F.rpart, out, nullptr, 0);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h_out.p, out, sizeof(double) * 2 * k, hipMemcpyDeviceToHost, bst);
        if (e == hipSuccess) {
            if (r->p.ptr_mode == SE_PTR_HOST) {
                e = se::launch_rowmajor_to_colmajor(bst, n, k, X, F.ldw, F.w[1], n);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(r->V, F.w[1], sizeof(double) * (size_t)n * k, hipMemcpyDeviceToHost, bst);
            } else {
                e = se::launch_rowmajor_to_colmajor(bst, n, k, X, F.ldw, r->V, n);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(r->lambda, dev_lam(s), sizeof(double) * k, hipMemcpyDeviceToDevice, bst);
            }
        }
        if (e == hipSuccess) e = hipStreamSynchronize(bst);
        if (e != hipSuccess) {
            r->info.hip_error = (int)e;
            return SE_ERR_HIP;
        }
        if (r->p.ptr_mode == SE_PTR_HOST) std::memcpy(r->lambda, D.lam, sizeof(double) * k);
        const double* o = h_out.as<double>();
        double ms = 0.0, mp = 0.0;
        for (int i = 0; i < k; ++i) {
            const double rn = std::sqrt(o[i]), xn = std::sqrt(o[k + i]);
            ms = std::max(ms, rn / (F.anorm * xn));
            mp = std::max(mp, rn / (F.anorm * xn + xn * std::fabs(D.lam[i])));
        }
        se_info& I = r->info;
        I.iterations = b.j;
        I.n_shrinks = b.n_shr;
        I.n_expands = b.n_exp;
        I.max_stop_ratio = ms;
        I.max_paper_ratio = mp;
        I.converged = (conv && ms <= r->p.tol * 1.01) ? 1 : 0;
        I.workspace_bytes = b.mem.bytes;
        return I.converged ? SE_OK : SE_NOT_CONVERGED;
    }

    // Decisions after the residual check of iteration j (as se_solve's LOBPCG
    // loop): returns true when the solve ends here (*conv: all pairs passed).
    bool decide(int s, bool* conv) {
        BSlot& b = bslots[s];
        const Request* r = b.r;
        const se::BDyn& D = hdyn()[s];
        const int j = ++b.j;
        const int k = D.k;
        double rr = 0.0;
        bool all = true;
        for (int i = 0; i < b.n_ev; ++i) {
            rr = std::max(rr, D.paper[i]);
            all = all && D.stop[i] <= r->p.tol;
        }
        b.ctl.observe(j, rr);
        *conv = all;
        if (all || j >= r->p.max_iter) return true;
        if (r->p.time_limit_s > 0 &&
            std::chrono::duration<double>(Clock::now() - r->t_start).count() > r->p.time_limit_s)
            return true;
        b.act.clear();
        for (int i = 0; i < k; ++i) {
            const bool locked = r->p.soft_lock && i < b.n_ev && D.stop[i] <= r->p.tol;
            if (!locked) b.act.push_back(i);
        }
        b.a = (int)b.act.size();
        const bool want = b.ctl.ifexpand(j);
        b.expand = 0;
        if (want && b.have_drop) {
            b.expand = 1;
            b.have_drop = false;
            b.ctl.did_expand(j);
            ++b.n_exp;
        }
        b.shrink = 0;
        if (b.ctl.ifshrink(j)) {
            b.shrink = 1;
            b.have_drop = true;
            b.ctl.did_shrink(j);
            ++b.n_shr;
        }
        return false;
    }

    // Slots are split into two lanes, each with its own stream and graph, so
    // that one lane's small dense phase overlaps the other lane's products
    // over n.
    int nlanes = 2;
    int lanes() const { return bslots.size() >= 2 ? nlanes : 1; }
    int lane_begin(int l) const { return l == 0 ? 0 : ((int)bslots.size() + 1) / 2; }
    int lane_end(int l) const { return l + 1 == lanes() ? (int)bslots.size() : lane_begin(l + 1); }
    hipStream_t lane_stream(int l) const { return l == 0 ? bst : bst2; }
    static size_t jobs_stride() { return (se::batch_jobs_bytes() + 255) / 256 * 256; }

    void drop_graphs() {
        for (int l = 0; l < 2; ++l) {
            if (gexec[l]) (void)hipGraphExecDestroy(gexec[l]);
            if (graph[l]) (void)hipGraphDestroy(graph[l]);
            gexec[l] = nullptr;
            graph[l] = nullptr;
        }
    }

    // One step: the decisions go up, every lane runs its launches (a graph
    // replay, or direct launches), the lanes' states come back.
    hipError_t run_step(int grid) {
        const int ns = (int)bslots.size();
        auto step = [&](se::Launcher& L, int l) {
            const int s0 = lane_begin(l), n = lane_end(l) - s0;
            return se::launch_batch_step(L, n, d_fix.as<se::BFix>() + s0, d_ctl.as<se::BCtl>() + s0,
                                         d_dyn.as<se::BDyn>() + s0, d_jobs.as<char>() + jobs_stride() * l, grid);
        };
        if (use_graph && (!gexec[0] || grid > graph_grid)) {
            // (re)build the lanes' graphs node by node (no stream capture)
            drop_graphs();
            hipError_t e = hipSuccess;
            for (int l = 0; l < lanes() && e == hipSuccess; ++l) {
                e = hipGraphCreate(&graph[l], 0);
                if (e == hipSuccess) {
                    se::Launcher G;
                    G.graph = graph[l];
                    e = step(G, l);
                }
                if (e == hipSuccess) e = hipGraphInstantiate(&gexec[l], graph[l], nullptr, nullptr, 0);
            }
            if (e != hipSuccess) {
                // no graph: the same launches, issued directly from now on
                (void)hipGetLastError();
                drop_graphs();
                use_graph = false;
            } else {
                graph_grid = grid;
            }
        }
        hipError_t e = hipMemcpyAsync(d_ctl.p, h_ctl.p, sizeof(se::BCtl) * ns, hipMemcpyHostToDevice, bst);
        if (e == hipSuccess && lanes() > 1) e = hipEventRecord(ev_ctl, bst);
        if (e == hipSuccess && lanes() > 1) e = hipStreamWaitEvent(bst2, ev_ctl, 0);
        for (int l = 0; l < lanes() && e == hipSuccess; ++l) {
            hipStream_t st = lane_stream(l);
            if (use_graph) {
                e = hipGraphLaunch(gexec[l], st);
            } else {
                se::Launcher D;
                D.st = st;
                e = step(D, l);
            }
            const int s0 = lane_begin(l), n = lane_end(l) - s0;
            if (e == hipSuccess)
                e = hipMemcpyAsync(hdyn() + s0, d_dyn.as<se::BDyn>() + s0, sizeof(se::BDyn) * n,
                                   hipMemcpyDeviceToHost, st);
        }
        for (int l = 0; l < lanes() && e == hipSuccess; ++l) e = hipStreamSynchronize(lane_stream(l));
        if (e == hipSuccess && use_graph) ++graph_steps;
        return e;
    }

    void run_batched() {
        (void)hipSetDevice(device);
        const int ns = (int)bslots.size();
        std::vector<int> fresh;
        std::vector<std::pair<int, se_status>> ended;
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            fresh.clear();
            admit_batched(fresh);
            bool any = false;
            for (const BSlot& b : bslots) any = any || b.r;
            if (!any) {
                if (stop && queue.empty()) return;
                cv_work.wait(lk);
                continue;
            }
            lk.unlock();
            ended.clear();
            for (int s : fresh) {
                const se_status st = setup_slot(s);
                if (st != SE_OK) ended.emplace_back(s, st);
            }
            // a failed setup leaves its slot idle for this step
            auto is_ended = [&](int s) {
                for (auto& e : ended)
                    if (e.first == s) return true;
                return false;
            };
            long long grid = 0;
            for (int s = 0; s < ns; ++s) {
                se::BCtl& C = hctl()[s];
                BSlot& b = bslots[s];
                C.mode = se::BMODE_IDLE;
                if (!b.r || is_ended(s)) continue;
                grid += 2 * ((hfix()[s].n + 63) / 64);
                if (b.init) {
                    C.mode = se::BMODE_INIT;
                    C.a = C.expand = C.shrink = 0;
                } else {
                    C.mode = se::BMODE_ITER;
                    C.a = b.a;
                    C.expand = b.expand;
                    C.shrink = b.shrink;
                    for (int i = 0; i < b.a; ++i) C.act[i] = b.act[i];
                }
            }
            bool stepped = false;
            if (grid > 0) {
                int g = 256;
                while (g < grid) g *= 2;
                const hipError_t e = run_step(g);
                ++steps;
                if (e != hipSuccess) {
                    // every resident solve fails; the engine goes on with new requests
                    (void)hipGetLastError();
                    for (int s = 0; s < ns; ++s)
                        if (bslots[s].r && !is_ended(s)) {
                            bslots[s].r->info.hip_error = (int)e;
                            ended.emplace_back(s, SE_ERR_HIP);
                        }
                } else {
                    stepped = true;
                }
            }
            if (stepped) {
                for (int s = 0; s < ns; ++s) {
                    BSlot& b = bslots[s];
                    if (!b.r || is_ended(s)) continue;
                    b.init = false;
                    if (hdyn()[s].k < b.n_ev) {
                        ended.emplace_back(s, SE_ERR_BREAKDOWN);
                        continue;
                    }
                    bool conv = false;
                    if (decide(s, &conv)) ended.emplace_back(s, finish_slot(s, conv));
                }
            }
            lk.lock();
            for (auto& e : ended) {
                Request* r = bslots[e.first].r;
                r->status = e.second;
                r->t_end = Clock::now();
                r->info.time_ms = std::chrono::duration<double, std::milli>(r->t_end - r->t_start).count();
                r->done = true;
                bslots[e.first].r = nullptr;
            }
            if (!ended.empty()) cv_done.notify_all();
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

se_status se_server_create_batched(se_ctx* ctx, uint64_t hbm_budget_bytes, int32_t max_slots, se_server** out) {
    if (!ctx || !out || max_slots < 1 || max_slots > se::kMaxBatch || hbm_budget_bytes == 0)
        return SE_ERR_INVALID_ARG;
    *out = nullptr;
    if (hipSetDevice(ctx->device) != hipSuccess) return SE_ERR_HIP;
    auto* s = new (std::nothrow) se_server();
    if (!s) return SE_ERR_OOM;
    s->device = ctx->device;
    s->budget = hbm_budget_bytes;
    s->batched = true;
    // Direct launches by default (measured faster than graph replays of the
    // same step on MI355X: each graph node adds about 10 us); SE_BATCH_GRAPH=1
    // replays a graph built once per server.
    const char* gr = std::getenv("SE_BATCH_GRAPH");
    s->use_graph = gr && gr[0] == '1';
    const char* nl = std::getenv("SE_BATCH_LANES");
    s->nlanes = (nl && nl[0] == '1') ? 1 : 2;
    s->bslots.resize(max_slots);
    const size_t ns = (size_t)max_slots;
    // Non-blocking: legacy null-stream work of other threads (a matrix being
    // created while a step is captured) must not synchronize with this stream.
    bool ok = hipStreamCreateWithFlags(&s->bst, hipStreamNonBlocking) == hipSuccess &&
              hipStreamCreateWithFlags(&s->bst2, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&s->ev_ctl, hipEventDisableTiming) == hipSuccess;
    ok = ok && s->d_fix.ensure(sizeof(se::BFix) * ns) == hipSuccess;
    ok = ok && s->d_ctl.ensure(sizeof(se::BCtl) * ns) == hipSuccess;
    ok = ok && s->d_dyn.ensure(sizeof(se::BDyn) * ns) == hipSuccess;
    ok = ok && s->d_jobs.ensure(se_server::jobs_stride() * 2) == hipSuccess;
    ok = ok && s->h_fix.ensure(sizeof(se::BFix) * ns) == hipSuccess;
    ok = ok && s->h_ctl.ensure(sizeof(se::BCtl) * ns) == hipSuccess;
    ok = ok && s->h_dyn.ensure(sizeof(se::BDyn) * ns) == hipSuccess;
    ok = ok && s->h_out.ensure(sizeof(double) * 2 * se::kBNbMax) == hipSuccess;
    if (ok) {
        std::memset(s->h_fix.p, 0, sizeof(se::BFix) * ns);
        std::memset(s->h_dyn.p, 0, sizeof(se::BDyn) * ns);
        ok = hipMemcpy(s->d_fix.p, s->h_fix.p, sizeof(se::BFix) * ns, hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(s->d_dyn.p, s->h_dyn.p, sizeof(se::BDyn) * ns, hipMemcpyHostToDevice) == hipSuccess;
    }
    if (!ok) {
        s->d_fix.release();
        s->d_ctl.release();
        s->d_dyn.release();
        s->d_jobs.release();
        s->h_fix.release();
        s->h_ctl.release();
        s->h_dyn.release();
        s->h_out.release();
        if (s->bst) (void)hipStreamDestroy(s->bst);
        if (s->bst2) (void)hipStreamDestroy(s->bst2);
        if (s->ev_ctl) (void)hipEventDestroy(s->ev_ctl);
        delete s;
        return SE_ERR_HIP;
    }
    s->engine = std::thread([s] { s->run_batched(); });
    *out = s;
    return SE_OK;
}

se_status se_server_batch_stats(se_server* srv, int64_t* steps, int64_t* graph_steps) {
    if (!srv || !srv->batched) return SE_ERR_INVALID_ARG;
    if (steps) *steps = srv->steps.load();
    if (graph_steps) *graph_steps = srv->graph_steps.load();
    return SE_OK;
}

uint64_t se_batched_footprint(int64_t n, int32_t n_ev, int32_t n_extra) {
    if (n < 1 || n_ev < 1 || n_extra < 0) return 0;
    return sizeof(double) * (uint64_t)bplan(n, n_ev + n_extra).doubles;
}

se_status se_submit(se_server* srv, const se_matrix* A, const se_params* params, const double* X0,
                    double* V, double* lambda, se_ticket* ticket) {
    if (!srv || !A || !params || !V || !lambda || !ticket) return SE_ERR_INVALID_ARG;
    if (!A->ctx || A->ctx->device != srv->device || A->is_complex) return SE_ERR_INVALID_ARG;
    const se_status v = se::validate_solve(A, params);
    if (v != SE_OK) return v;
    if (srv->batched) {
        const int nb = params->n_ev + params->n_extra;
        if (params->solver != SE_LOBPCG || params->precision != SE_FP64 || params->precond != SE_PRECOND_NONE ||
            params->expand_vectors != SE_EXPAND_XDROP || nb > se::kBNbMax || A->n_heavy > 0 ||
            A->n > (int64_t)INT32_MAX / 2)
            return SE_ERR_UNSUPPORTED;
    }
    auto r = std::make_unique<Request>();
    r->A = A;
    r->p = *params;
    r->X0 = X0;
    r->V = V;
    r->lambda = lambda;
    r->footprint = srv->batched ? se_batched_footprint(A->n, params->n_ev, params->n_extra)
                                : se_solve_footprint(A->n, A->nnz, params->n_ev, params->n_extra,
                                                     params->precision, params->solver);
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
    if (srv->batched)
        srv->cv_work.notify_all();
    else
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
    if (srv->engine.joinable()) srv->engine.join();
    (void)hipSetDevice(srv->device);
    if (srv->batched) {
        (void)hipStreamSynchronize(srv->bst);
        (void)hipStreamSynchronize(srv->bst2);
        srv->drop_graphs();
        for (BSlot& b : srv->bslots) b.mem.release();
        srv->d_fix.release();
        srv->d_ctl.release();
        srv->d_dyn.release();
        srv->d_jobs.release();
        srv->h_fix.release();
        srv->h_ctl.release();
        srv->h_dyn.release();
        srv->h_out.release();
        (void)hipStreamDestroy(srv->bst);
        (void)hipStreamDestroy(srv->bst2);
        (void)hipEventDestroy(srv->ev_ctl);
    }
    (void)hipGetLastError();  // nothing reported here may linger for a later launch check
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
