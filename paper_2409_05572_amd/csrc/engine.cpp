// Solver drivers: LOBPCG (Algorithm 3) and subspace iteration (Algorithm 1)
// with shrink-and-expand (Algorithm 5) on the GPU.
//
// All n-length data lives in "panels" (n x ld row-major FP64 buffers). X, P,
// W and their images AX, AP, AW are separate panels; S = [X, P, W] is a list
// of panel pointers, never a copy. Updates write into spare panels and the
// pointers are swapped, so no kernel reads and writes the same panel.
// The host decides locking, shrink and expansion from a few scalars read back
// per iteration; every n-length operation runs in the HIP kernels.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <utility>

#include "engine.h"

namespace se {

// ---------------------------------------------------------------- strategy --
void Strategy::observe(int j, double r) {
    if ((int)logr.size() <= j) {
        logr.resize(j + 1, 0.0);
        have.resize(j + 1, 0);
    }
    logr[j] = (r > 0.0) ? std::log10(r) : -INFINITY;
    have[j] = 1;
}

bool Strategy::slope(int j, double* c) const {
    auto ok = [&](int i) { return i >= 0 && i < (int)have.size() && have[i]; };
    if (kind == SE_STRAT_SLOPE) {  // eq. (ckslope)
        if (!ok(j - 1) || !ok(j)) return false;
        *c = logr[j - 1] - logr[j];
        return true;
    }
    if (kind == SE_STRAT_SLOPEK) {  // eq. (ckslopek)
        if (j < j_p || !ok(j - j_p) || !ok(j)) return false;
        *c = (logr[j - j_p] - logr[j]) / j_p;
        return true;
    }
    return false;
}

bool Strategy::ifexpand(int j) {
    if (!enabled() || !shrunk) return false;
    if (kind == SE_STRAT_FIX) return j % j_e == 0;  // Algorithm 6
    double c;
    if (!slope(j, &c) || !std::isfinite(c)) return false;
    c_max = std::max(c_max, c);
    return mu * c < c_max;  // Algorithm 7
}

bool Strategy::ifshrink(int j) const {
    if (!enabled() || shrunk) return false;
    if (!warm_done)  // warm-up rule, end of Section 3.2
        return j >= j_warm && j < (int)have.size() && have[j] && logr[j] <= std::log10(r_warm);
    if (kind == SE_STRAT_FIX) return (j - j_s) % j_e == 0;
    return j - j_last_expand == j_s;
}

namespace {

inline long long round_up(long long a, long long b) { return (a + b - 1) / b * b; }

se_status hip_status(hipError_t e) {
    if (e == hipSuccess) return SE_OK;
    if (e == hipErrorOutOfMemory) return SE_ERR_OOM;
    return SE_ERR_HIP;
}

struct Solver {
    se_ctx* ctx;
    const se_matrix* A;
    se_params p;
    hipStream_t st;
    Workspace& ws;
    long long n;
    int ld = 0, nb = 0, n_ev = 0, n_es = 0;
    bool se_on = false;
    hipError_t herr = hipSuccess;

    double *X = nullptr, *P = nullptr, *W = nullptr, *AX = nullptr, *AP = nullptr, *AW = nullptr;
    double *Xn = nullptr, *Pn = nullptr, *AXn = nullptr, *APn = nullptr;
    double *Sd = nullptr, *ASd = nullptr, *T1 = nullptr, *T2 = nullptr;

    int iters = 0, n_shr = 0, n_exp = 0, hist_len = 0;
    bool converged = false;
    double last_r = INFINITY, last_stop = INFINITY;
    Strategy ctl;
    std::chrono::steady_clock::time_point t0;

    // Per-launch timing (params.profile): events recorded around launches on
    // the solver stream, summed per kernel class at the end of the solve.
    struct ProfRec {
        int cls;
        hipEvent_t a, b;
        double bytes, flops;
    };
    std::vector<ProfRec> prof;
    size_t ev_next = 0;
    hipEvent_t open_ev = nullptr;

    Solver(se_ctx* c, const se_matrix* a, const se_params& prm)
        : ctx(c), A(a), p(prm), st(c->stream), ws(c->ws), n(a->n) {}

#define HC(expr)                                   \
    do {                                           \
        hipError_t _e = (expr);                    \
        if (_e != hipSuccess) {                    \
            herr = _e;                             \
            return hip_status(_e);                 \
        }                                          \
    } while (0)
#define ST(expr)                   \
    do {                           \
        se_status _s = (expr);     \
        if (_s < 0) return _s;     \
    } while (0)

    Segs seg1(const double* a, int wa) const {
        Segs s = make_segs(ld);
        push_seg(s, a, wa);
        return s;
    }
    Segs seg3(const double* a, int wa, const double* b, int wb, const double* c, int wc) const {
        Segs s = make_segs(ld);
        push_seg(s, a, wa);
        push_seg(s, b, wb);
        push_seg(s, c, wc);
        return s;
    }

    se_status alloc_panels(int count) {
        const size_t bytes = sizeof(double) * (size_t)n * ld;
        for (int i = 0; i < count; ++i) HC(ws.panel[i].ensure(bytes));
        double** slots[] = {&X, &P, &W, &AX, &AP, &AW, &Xn, &Pn, &AXn, &APn, &Sd, &ASd, &T1, &T2};
        for (int i = 0; i < count; ++i) *slots[i] = ws.panel[i].as<double>();
        return SE_OK;
    }

    se_status alloc_small(int mmax) {
        const size_t mm = (size_t)mmax * mmax;
        HC(ws.G.ensure(sizeof(double) * mm));
        HC(ws.T.ensure(sizeof(double) * mm));
        HC(ws.Z.ensure(sizeof(double) * mm));
        HC(ws.C.ensure(sizeof(double) * mm));
        HC(ws.theta.ensure(sizeof(double) * (mmax + 8)));
        HC(ws.small_work.ensure(sizeof(double) * (2 * mm + 8 * (size_t)mmax + 64)));
        HC(ws.syev_work.ensure(sizeof(double) * syev_work_doubles(mmax)));
        HC(ws.gram_part.ensure(sizeof(double) * std::max(gram_scratch_doubles(n, mmax, mmax),
                                                         (size_t)4096 * 2 * mmax)));
        HC(ws.hlB.ensure(sizeof(double) * mm));
        HC(ws.hlY.ensure(sizeof(double) * mm));
        HC(ws.hlG.ensure(sizeof(double) * mm));
        HC(ws.hlQ.ensure(sizeof(double) * mm));
        HC(ws.act.ensure(sizeof(int) * (mmax + 8)));
        HC(ws.act_hl.ensure(sizeof(int) * (mmax + 8)));
        HC(ws.norms.ensure(sizeof(double) * (2 * mmax + 8)));
        HC(ws.info.ensure(sizeof(double) * (mmax + 16)));
        HC(ws.h_norms.ensure(sizeof(double) * (2 * mmax + 8)));
        HC(ws.h_theta.ensure(sizeof(double) * (mmax + 8)));
        HC(ws.h_info.ensure(sizeof(double) * (mmax + 16)));
        HC(ws.h_act.ensure(sizeof(int) * (mmax + 8)));
        HC(ws.h_act_hl.ensure(sizeof(int) * (mmax + 8)));
        return SE_OK;
    }

    se_status sync() {
        HC(hipStreamSynchronize(st));
        return SE_OK;
    }

    hipEvent_t next_event() {
        if (ev_next == ws.events.size()) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            ws.events.push_back(e);
        }
        return ws.events[ev_next++];
    }
    se_status tic() {
        if (!p.profile) return SE_OK;
        open_ev = next_event();
        if (open_ev) HC(hipEventRecord(open_ev, st));
        return SE_OK;
    }
    se_status toc(int cls, double bytes, double flops) {
        if (!p.profile || !open_ev) return SE_OK;
        hipEvent_t b = next_event();
        if (!b) return SE_OK;
        HC(hipEventRecord(b, st));
        prof.push_back({cls, open_ev, b, bytes, flops});
        open_ev = nullptr;
        return SE_OK;
    }
    void summarize(se_info* info) {
        if (!info || !p.profile) return;
        (void)hipStreamSynchronize(st);
        for (const ProfRec& r : prof) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) continue;
            info->kern_ms[r.cls] += ms;
            info->kern_bytes[r.cls] += r.bytes;
            info->kern_flops[r.cls] += r.flops;
            info->kern_calls[r.cls] += 1;
        }
    }

    // ------------------------------------------------------------ kernels --
    se_status spmm(const double* Xs, double* Ys, int w) {
        ST(tic());
        HC(launch_spmm(st, (int)n, A->rowptr, A->col, A->val, Xs, ld, Ys, ld, w));
        return toc(SE_K_SPMM, 12.0 * A->nnz + 4.0 * (n + 1) + 16.0 * n * w, 2.0 * A->nnz * w);
    }
    se_status gram(const Segs& U, const Segs& V, int sym, double* C) {
        const size_t need = sizeof(double) * gram_scratch_doubles(n, segs_width(U), segs_width(V));
        if (need > ws.gram_part.bytes) {
            ST(sync());  // the old scratch may still be in use by queued kernels
            HC(ws.gram_part.ensure(need));
        }
        ST(tic());
        HC(launch_gram(st, n, U, V, sym, ws.gram_part.as<double>(), C));
        const double mu = segs_width(U), mv = segs_width(V);
        const double fl = (sym && mu == mv) ? n * mu * (mu + 1.0) : 2.0 * n * mu * mv;
        const bool same = sym && U.nseg == 1 && V.nseg == 1 && U.p[0] == V.p[0];
        return toc(SE_K_GRAM, 8.0 * n * (same ? mu : mu + mv), fl);
    }
    se_status update(const Segs& U, const double* C, int N, const Segs& O, double alpha, double beta) {
        ST(tic());
        HC(launch_update(st, n, U, C, N, O, alpha, beta));
        const double K = segs_width(U);
        return toc(SE_K_UPDATE, 8.0 * n * (K + N * (beta != 0.0 ? 2.0 : 1.0)), 2.0 * n * K * N);
    }

    // Products on small row counts (coefficient space of the Rayleigh-Ritz
    // basis); each Segs carries its own leading dimension.
    static Segs segx(const double* p_, int w, long long ldx) {
        Segs s = make_segs(ldx);
        push_seg(s, p_, w);
        return s;
    }
    se_status gram_rows(long long rows, const Segs& U, const Segs& V, int sym, double* C) {
        HC(launch_gram(st, rows, U, V, sym, ws.gram_part.as<double>(), C));
        return SE_OK;
    }
    se_status update_rows(long long rows, const Segs& U, const double* C, int N, const Segs& O,
                          double alpha, double beta) {
        HC(launch_update(st, rows, U, C, N, O, alpha, beta));
        return SE_OK;
    }

    // Coefficients C = [Z1 | C_P] (m x (k + r), leading dimension k + r) of the
    // Hetmaniuk-Lehoucq basis: C_P is an orthonormal basis of the part of the
    // unlocked old X columns (unit vectors E) orthogonal to Z1, i.e. of
    // (I - Z1 Z1^T) E, which equals Z2 Z2^T E. The projection is applied twice
    // before and once after the first Cholesky-QR, so C_P is orthogonal to Z1
    // to working precision. Both Cholesky-QR passes may drop columns: a
    // column kept by the first pass with a pivot near the threshold is mostly
    // amplified rounding, and the reprojection can leave it dependent on the
    // others, which a pass without drop would turn into a non-orthonormal
    // C_P. Returns the final rank through rP.
    se_status hl_coefficients(int m, int k, int a, int& rP) {
        const double* Z1 = ws.Z.as<double>();
        double* B = ws.hlB.as<double>();
        double* Y = ws.hlY.as<double>();
        double* G2 = ws.hlG.as<double>();
        double* Q = ws.hlQ.as<double>();
        double* C = ws.C.as<double>();
        rP = 0;
        if (a > 0) {
            HC(launch_hl_init(st, m, k, Z1, ws.act_hl.as<int>(), a, B, Y));
            const Segs Zs = segx(Z1, k, k);
            ST(update_rows(m, Zs, Y, a, segx(B, a, a), -1.0, 1.0));
            ST(gram_rows(m, Zs, segx(B, a, a), 0, G2));
            ST(update_rows(m, Zs, G2, a, segx(B, a, a), -1.0, 1.0));
            ST(gram_rows(m, segx(B, a, a), segx(B, a, a), 1, ws.G.as<double>()));
            int* info_i = ws.info.as<int>();
            double* info_d = ws.info.as<double>() + (a + 8) / 2 + 4;
            HC(launch_chol_drop(st, a, ws.G.as<double>(), ws.T.as<double>(), ws.small_work.as<double>(),
                                info_i, info_d, 1e-13));
            HC(hipMemcpyAsync(ws.h_info.p, ws.info.p, sizeof(int) * 4, hipMemcpyDeviceToHost, st));
            ST(sync());
            const int r = ws.h_info.as<int>()[0];
            int r2 = 0;
            if (r > 0) {
                ST(update_rows(m, segx(B, a, a), ws.T.as<double>(), r, segx(Q, r, r), 1.0, 0.0));
                ST(gram_rows(m, Zs, segx(Q, r, r), 0, G2));
                ST(update_rows(m, Zs, G2, r, segx(Q, r, r), -1.0, 1.0));
                ST(gram_rows(m, segx(Q, r, r), segx(Q, r, r), 1, ws.G.as<double>()));
                // second pass: a Newton-Schulz step if Q is orthonormal to
                // 1e-8, else Cholesky-QR with drop (decided on the device)
                HC(launch_chol_drop(st, r, ws.G.as<double>(), ws.T.as<double>(), ws.small_work.as<double>(),
                                    info_i, info_d, 1e-13, 1e-8));
                HC(hipMemcpyAsync(ws.h_info.p, ws.info.p, sizeof(int) * 4, hipMemcpyDeviceToHost, st));
                ST(sync());
                r2 = ws.h_info.as<int>()[0];
                if (r2 > 0)
                    ST(update_rows(m, segx(Q, r, r), ws.T.as<double>(), r2, segx(C + k, r2, k + r2), 1.0,
                                   0.0));
            }
            rP = r2;
        }
        HC(launch_copy_cols(st, m, Z1, k, 0, C, k + rP, 0, k));
        return SE_OK;
    }

    // Cholesky-QR applied twice (a third time after a tiny pivot) with column
    // drop. The panel pointer `w_panel` (and `companion`, which receives the
    // same transform) is swapped with a spare. kept_out: original indices of
    // the surviving columns. A pass that follows one whose smallest scaled
    // pivot was >= 1e-8 and that dropped nothing cannot drop a column either;
    // it runs without a read-back and takes a Newton-Schulz step when the
    // block is already orthonormal to 1e-8 (decided on the device).
    // `against` (with images `against_img` for the companion): blocks the
    // panel was made orthogonal to; after a pass with a pivot below 1e-8 the
    // kept columns carry amplified rounding along them, so the projection is
    // repeated before the next pass.
    se_status cholqr(double*& w_panel, int& w, double** companion, std::vector<int>* kept_out,
                     const Segs* against = nullptr, const Segs* against_img = nullptr) {
        std::vector<int> map(w);
        for (int i = 0; i < w; ++i) map[i] = i;
        int passes = 2;
        bool full_rank = false;  // the previous pass kept every column with a healthy pivot
        for (int pass = 0; pass < passes && w > 0; ++pass) {
            const Segs Ws = seg1(w_panel, w);
            ST(gram(Ws, Ws, 1, ws.G.as<double>()));
            int* info_i = ws.info.as<int>();
            double* info_d = ws.info.as<double>() + (w + 8) / 2 + 4;
            if (full_rank) {
                ST(tic());
                HC(launch_chol_drop(st, w, ws.G.as<double>(), ws.T.as<double>(), ws.small_work.as<double>(),
                                    info_i, info_d, -1.0, 1e-8));
                ST(toc(SE_K_SMALL, 16.0 * w * w, w * w * (double)w));
                ST(update(Ws, ws.T.as<double>(), w, seg1(T1, w), 1.0, 0.0));
                std::swap(w_panel, T1);
                if (companion) {
                    ST(update(seg1(*companion, w), ws.T.as<double>(), w, seg1(T2, w), 1.0, 0.0));
                    std::swap(*companion, T2);
                }
                continue;
            }
            ST(tic());
            HC(launch_chol_drop(st, w, ws.G.as<double>(), ws.T.as<double>(), ws.small_work.as<double>(),
                                info_i, info_d, 1e-13));
            ST(toc(SE_K_SMALL, 16.0 * w * w, w * w * (double)w));
            HC(hipMemcpyAsync(ws.h_info.p, ws.info.p, sizeof(double) * (w + 16), hipMemcpyDeviceToHost,
                              st));
            ST(sync());
            const int* hi = ws.h_info.as<int>();
            const double minpiv = ws.h_info.as<double>()[(w + 8) / 2 + 4];
            const int r = hi[0];
            if (r <= 0) {
                w = 0;
                break;
            }
            std::vector<int> nm(r);
            for (int q = 0; q < r; ++q) nm[q] = map[hi[1 + q]];
            map.swap(nm);
            ST(update(Ws, ws.T.as<double>(), r, seg1(T1, r), 1.0, 0.0));
            std::swap(w_panel, T1);
            if (companion) {
                ST(update(seg1(*companion, w), ws.T.as<double>(), r, seg1(T2, r), 1.0, 0.0));
                std::swap(*companion, T2);
            }
            if (pass == 0 && (minpiv < 1e-8 || r < w)) passes = 3;
            full_rank = minpiv >= 1e-8 && r == w;
            w = r;
            if (against && minpiv < 1e-8 && pass + 1 < passes) {
                ST(gram(*against, seg1(w_panel, w), 0, ws.G.as<double>()));
                ST(update(*against, ws.G.as<double>(), w, seg1(w_panel, w), -1.0, 1.0));
                if (companion && against_img)
                    ST(update(*against_img, ws.G.as<double>(), w, seg1(*companion, w), -1.0, 1.0));
            }
        }
        if (kept_out) *kept_out = map;
        return SE_OK;
    }

    // Rayleigh-Ritz on the k columns of X (with AX): X <- X Z, AX <- AX Z.
    se_status rr_plain(int k) {
        ST(gram(seg1(X, k), seg1(AX, k), 1, ws.G.as<double>()));
        ST(tic());
        HC(launch_syev(st, k, ws.G.as<double>(), ws.theta.as<double>(), ws.Z.as<double>(),
                       ws.syev_work.as<double>()));
        ST(toc(SE_K_EIG, 16.0 * k * k, 4.0 * k * k * (double)k));
        ST(update(seg1(X, k), ws.Z.as<double>(), k, seg1(Xn, k), 1.0, 0.0));
        ST(update(seg1(AX, k), ws.Z.as<double>(), k, seg1(AXn, k), 1.0, 0.0));
        std::swap(X, Xn);
        std::swap(AX, AXn);
        return SE_OK;
    }

    se_status load_x0(const double* X0) {
        if (p.ptr_mode == SE_PTR_HOST) {
            // T1 holds n * ld >= n * nb doubles
            HC(hipMemcpyAsync(T1, X0, sizeof(double) * (size_t)n * nb, hipMemcpyHostToDevice, st));
            HC(launch_colmajor_to_rowmajor(st, n, nb, T1, n, X, ld));
        } else {
            HC(launch_colmajor_to_rowmajor(st, n, nb, X0, n, X, ld));
        }
        return SE_OK;
    }

    // Residual check of the current (X, AX, theta) for k columns: per-column
    // ratios of the stopping test and of eq. (rk).
    se_status check(const double* Xp, const double* AXp, int k, std::vector<double>& stop,
                    std::vector<double>& paper, std::vector<double>& lam) {
        ST(tic());
        HC(launch_resid_norms(st, n, Xp, AXp, ld, k, ws.theta.as<double>(), ws.gram_part.as<double>(),
                              ws.norms.as<double>()));
        ST(toc(SE_K_RESID, 16.0 * n * k, 5.0 * n * k));
        HC(hipMemcpyAsync(ws.h_norms.p, ws.norms.p, sizeof(double) * 2 * k, hipMemcpyDeviceToHost, st));
        HC(hipMemcpyAsync(ws.h_theta.p, ws.theta.p, sizeof(double) * k, hipMemcpyDeviceToHost, st));
        ST(sync());
        const double* nr = ws.h_norms.as<double>();
        const double* th = ws.h_theta.as<double>();
        stop.resize(k);
        paper.resize(k);
        lam.assign(th, th + k);
        for (int i = 0; i < k; ++i) {
            const double rn = std::sqrt(std::max(nr[i], 0.0));
            const double xn = std::sqrt(std::max(nr[k + i], 0.0));
            stop[i] = rn / (A->anorm * xn);
            paper[i] = rn / (A->anorm * xn + xn * std::fabs(th[i]));
        }
        return SE_OK;
    }

    void record(int j, double r, double mstop, int k, int pw, int a, int locked, int flags) {
        if (!p.history || hist_len >= p.history_cap) return;
        double* h = p.history + (size_t)hist_len * SE_HISTORY_FIELDS;
        h[0] = j;
        h[1] = r;
        h[2] = mstop;
        h[3] = k;
        h[4] = pw;
        h[5] = a;
        h[6] = locked;
        h[7] = flags;
        ++hist_len;
    }
    void amend_flags(int flags) {
        if (!p.history || hist_len == 0 || hist_len > p.history_cap) return;
        p.history[(size_t)(hist_len - 1) * SE_HISTORY_FIELDS + 7] = flags;
    }

    bool out_of_time() const {
        if (p.time_limit_s <= 0) return false;
        const double el =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return el > p.time_limit_s;
    }

    // ------------------------------------------------------------- LOBPCG --
    se_status lobpcg(const double* X0) {
        ST(alloc_panels(14));
        ST(alloc_small(3 * nb));
        ST(load_x0(X0));
        int k = nb;
        ST(cholqr(X, k, nullptr, nullptr));
        if (k < n_ev) return SE_ERR_BREAKDOWN;
        ST(spmm(X, AX, k));
        ST(rr_plain(k));
        int pw = 0;  // width of P
        bool have_drop = false;
        int dx = 0, dp = 0;
        std::vector<double> stop, paper, lam;
        std::vector<int> act, act_hl, kept;

        for (int j = 1; j <= p.max_iter; ++j) {
            ST(check(X, AX, k, stop, paper, lam));
            double r = 0.0, ms = 0.0;
            bool all = true;
            for (int i = 0; i < n_ev; ++i) {
                r = std::max(r, paper[i]);
                ms = std::max(ms, stop[i]);
                all = all && (stop[i] <= p.tol);
            }
            iters = j;
            last_r = r;
            last_stop = ms;
            ctl.observe(j, r);
            act.clear();
            for (int i = 0; i < k; ++i) {
                const bool locked = p.soft_lock && i < n_ev && stop[i] <= p.tol;
                if (!locked) act.push_back(i);
            }
            record(j, r, ms, k, pw, (int)act.size(), k - (int)act.size(), 0);
            if (all) {
                converged = true;
                break;
            }
            if (out_of_time()) break;
            const bool want_expand = ctl.ifexpand(j);
            int flags = 0;

            // W <- R(:, active) (T = I), orthogonalized against [X, P] twice.
            int a = (int)act.size();
            std::memcpy(ws.h_act.p, act.data(), sizeof(int) * a);
            HC(hipMemcpyAsync(ws.act.p, ws.h_act.p, sizeof(int) * a, hipMemcpyHostToDevice, st));
            ST(tic());
            HC(launch_form_w(st, n, X, AX, ld, ws.theta.as<double>(), ws.act.as<int>(), a, W, ld));
            ST(toc(SE_K_RESID, 24.0 * n * a, 2.0 * n * a));
            const Segs XP = seg3(X, k, P, pw, nullptr, 0);
            for (int pass = 0; pass < 2; ++pass) {
                ST(gram(XP, seg1(W, a), 0, ws.G.as<double>()));
                ST(update(XP, ws.G.as<double>(), a, seg1(W, a), -1.0, 1.0));
            }
            ST(cholqr(W, a, nullptr, nullptr, &XP));
            if (a > 0) ST(spmm(W, AW, a));

            act_hl = act;
            if (want_expand && have_drop) {
                // S_drop <- S_drop - S (S^T S_drop), twice; orthonormalize; the
                // stored images A S_drop receive the same transforms.
                int d0 = dx + dp;
                for (int pass = 0; pass < 2; ++pass) {
                    const Segs S = seg3(X, k, P, pw, W, a);
                    const Segs AS = seg3(AX, k, AP, pw, AW, a);
                    ST(gram(S, seg1(Sd, d0), 0, ws.G.as<double>()));
                    ST(update(S, ws.G.as<double>(), d0, seg1(Sd, d0), -1.0, 1.0));
                    ST(update(AS, ws.G.as<double>(), d0, seg1(ASd, d0), -1.0, 1.0));
                }
                const Segs S = seg3(X, k, P, pw, W, a);
                const Segs AS = seg3(AX, k, AP, pw, AW, a);
                ST(cholqr(Sd, d0, &ASd, &kept, &S, &AS));
                int dxk = 0;
                for (int v : kept) dxk += (v < dx);
                const int dpk = d0 - dxk;
                HC(launch_copy_cols(st, n, Sd, ld, 0, X, ld, k, dxk));
                HC(launch_copy_cols(st, n, ASd, ld, 0, AX, ld, k, dxk));
                HC(launch_copy_cols(st, n, Sd, ld, dxk, P, ld, pw, dpk));
                HC(launch_copy_cols(st, n, ASd, ld, dxk, AP, ld, pw, dpk));
                for (int q = 0; q < dxk; ++q) act_hl.push_back(k + q);
                k += dxk;
                pw += dpk;
                ctl.did_expand(j);
                have_drop = false;
                ++n_exp;
                flags |= 1;
            }

            // Rayleigh-Ritz on S = [X, P, W].
            const int m = k + pw + a;
            const Segs S = seg3(X, k, P, pw, W, a);
            const Segs AS = seg3(AX, k, AP, pw, AW, a);
            ST(gram(S, AS, 1, ws.G.as<double>()));
            ST(tic());
            HC(launch_syev_lowest(st, m, k, ws.G.as<double>(), ws.theta.as<double>(), ws.Z.as<double>(),
                                  ws.syev_work.as<double>()));
            ST(toc(SE_K_EIG, 8.0 * m * m, 4.0 * m * m * (double)m / 3.0));
            const int ahl = (int)act_hl.size();
            std::memcpy(ws.h_act_hl.p, act_hl.data(), sizeof(int) * ahl);
            HC(hipMemcpyAsync(ws.act_hl.p, ws.h_act_hl.p, sizeof(int) * ahl, hipMemcpyHostToDevice, st));
            int rPv = 0;
            ST(tic());
            ST(hl_coefficients(m, k, ahl, rPv));
            ST(toc(SE_K_SMALL, 16.0 * m * (k + ahl), 8.0 * m * (double)k * ahl));
            const int rP = rPv;
            Segs O = make_segs(ld);
            push_seg(O, Xn, k);
            push_seg(O, Pn, rP);
            ST(update(S, ws.C.as<double>(), k + rP, O, 1.0, 0.0));
            Segs AO = make_segs(ld);
            push_seg(AO, AXn, k);
            push_seg(AO, APn, rP);
            ST(update(AS, ws.C.as<double>(), k + rP, AO, 1.0, 0.0));
            std::swap(X, Xn);
            std::swap(P, Pn);
            std::swap(AX, AXn);
            std::swap(AP, APn);
            pw = rP;

            if (ctl.ifshrink(j)) {
                dx = k - n_es;
                dp = std::max(0, pw - n_es);
                dp = std::min(dp, ld - dx);  // S_drop must fit one panel
                HC(launch_copy_cols(st, n, X, ld, n_es, Sd, ld, 0, dx));
                HC(launch_copy_cols(st, n, AX, ld, n_es, ASd, ld, 0, dx));
                HC(launch_copy_cols(st, n, P, ld, n_es, Sd, ld, dx, dp));
                HC(launch_copy_cols(st, n, AP, ld, n_es, ASd, ld, dx, dp));
                k = n_es;
                pw = std::min(pw, n_es);
                have_drop = true;
                ctl.did_shrink(j);
                ++n_shr;
                flags |= 2;
            }
            amend_flags(flags);
        }
        return SE_OK;
    }

    // ------------------------------------------------- subspace iteration --
    se_status si(const double* X0) {
        ST(alloc_panels(14));
        ST(alloc_small(nb));
        ST(load_x0(X0));
        const double sigma = (p.sigma > 0.0) ? p.sigma : A->anorm;
        int k = nb;
        ST(cholqr(X, k, nullptr, nullptr));
        if (k < n_ev) return SE_ERR_BREAKDOWN;
        ST(spmm(X, AX, k));
        ST(rr_plain(k));
        bool have_drop = false;
        int dx = 0;
        std::vector<double> stop, paper, lam;
        for (int j = 1; j <= p.max_iter; ++j) {
            ST(check(X, AX, k, stop, paper, lam));
            double r = 0.0, ms = 0.0;
            bool all = true;
            for (int i = 0; i < n_ev; ++i) {
                r = std::max(r, paper[i]);
                ms = std::max(ms, stop[i]);
                all = all && (stop[i] <= p.tol);
            }
            iters = j;
            last_r = r;
            last_stop = ms;
            ctl.observe(j, r);
            record(j, r, ms, k, 0, k, 0, 0);
            if (all) {
                converged = true;
                break;
            }
            if (out_of_time()) break;
            int flags = 0;
            const bool want_expand = ctl.ifexpand(j);
            // Y <- sigma X - A X (AX is current), then append X_drop.
            ST(tic());
            HC(launch_shift_sub(st, n, X, AX, ld, k, sigma));
            ST(toc(SE_K_RESID, 24.0 * n * k, 2.0 * n * k));
            if (want_expand && have_drop) {
                HC(launch_copy_cols(st, n, Sd, ld, 0, X, ld, k, dx));
                k += dx;
                have_drop = false;
                ctl.did_expand(j);
                ++n_exp;
                flags |= 1;
            }
            ST(cholqr(X, k, nullptr, nullptr));
            if (k < n_ev) return SE_ERR_BREAKDOWN;
            ST(spmm(X, AX, k));
            ST(rr_plain(k));
            if (ctl.ifshrink(j)) {
                dx = k - n_es;
                HC(launch_copy_cols(st, n, X, ld, n_es, Sd, ld, 0, dx));
                k = n_es;
                have_drop = true;
                ctl.did_shrink(j);
                ++n_shr;
                flags |= 2;
            }
            amend_flags(flags);
        }
        return SE_OK;
    }

    // Fresh residual of the returned pairs, then write V and lambda.
    se_status finish(double* V, double* lambda, se_info* info) {
        ST(spmm(X, T2, n_ev));
        std::vector<double> stop, paper, lam;
        ST(check(X, T2, n_ev, stop, paper, lam));
        double ms = 0.0, mp = 0.0;
        for (int i = 0; i < n_ev; ++i) {
            ms = std::max(ms, stop[i]);
            mp = std::max(mp, paper[i]);
        }
        if (p.ptr_mode == SE_PTR_HOST) {
            HC(launch_rowmajor_to_colmajor(st, n, n_ev, X, ld, T1, n));
            HC(hipMemcpyAsync(V, T1, sizeof(double) * (size_t)n * n_ev, hipMemcpyDeviceToHost, st));
            ST(sync());
            std::memcpy(lambda, lam.data(), sizeof(double) * n_ev);
        } else {
            HC(launch_rowmajor_to_colmajor(st, n, n_ev, X, ld, V, n));
            HC(hipMemcpyAsync(lambda, ws.theta.p, sizeof(double) * n_ev, hipMemcpyDeviceToDevice, st));
            ST(sync());
        }
        if (info) {
            info->max_stop_ratio = ms;
            info->max_paper_ratio = mp;
        }
        // Ritz vectors that only met the test through the carried images: the
        // fresh product decides.
        if (converged && !(ms <= p.tol * 1.01)) converged = false;
        return SE_OK;
    }
#undef HC
#undef ST
};

}  // namespace

se_status solve(se_ctx* ctx, const se_matrix* A, const se_params* prm, const double* X0, double* V,
                double* lambda, se_info* info) {
    Solver s(ctx, A, *prm);
    s.t0 = std::chrono::steady_clock::now();
    s.nb = prm->n_ev + prm->n_extra;
    s.n_ev = prm->n_ev;
    s.ld = (int)round_up(s.nb, 8);
    int n_es = prm->n_es;
    if (n_es <= 0) n_es = prm->n_ev + std::min(5, prm->n_extra - 1);
    s.n_es = n_es;
    s.ctl.kind = prm->strategy;
    s.ctl.j_e = prm->j_e;
    s.ctl.j_s = prm->j_s;
    s.ctl.j_p = prm->j_p;
    s.ctl.j_warm = prm->j_warm;
    s.ctl.mu = prm->mu;
    s.ctl.r_warm = prm->r_warm;
    s.se_on = s.ctl.enabled() && prm->n_extra >= 2 && n_es >= prm->n_ev && n_es < s.nb;
    if (!s.se_on) s.ctl.kind = SE_STRAT_NONE;

    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    (void)hipEventRecord(e0, ctx->stream);
    se_status st = (prm->solver == SE_SI) ? s.si(X0) : s.lobpcg(X0);
    if (st >= 0) st = s.finish(V, lambda, info);
    s.summarize(info);
    (void)hipEventRecord(e1, ctx->stream);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s.herr != hipSuccess) ctx->last_hip_error = (int)s.herr;
    if (info) {
        info->iterations = s.iters;
        info->converged = s.converged ? 1 : 0;
        info->n_shrinks = s.n_shr;
        info->n_expands = s.n_exp;
        info->time_ms = ms;
        info->workspace_bytes = ctx->ws.device_bytes();
        info->hip_error = (int)s.herr;
        info->history_len = s.hist_len;
        if (st < 0) {
            info->max_stop_ratio = s.last_stop;
            info->max_paper_ratio = s.last_r;
        }
    }
    if (st < 0) return st;
    return s.converged ? SE_OK : SE_NOT_CONVERGED;
}

}  // namespace se
