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

    int iters = 0, n_shr = 0, n_exp = 0, hist_len = 0, n_reproj = 0, n_implicit = 0;
    bool no_p = false;  // steepest descent: the LOBPCG iteration without P
    int j_off = 0;       // iterations of an earlier (low-precision) phase
    int lp_iters = 0;    // iterations of the low-precision phase
    bool lp_done = false;  // the low-precision phase met the stopping test itself
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
        {
            DevBuf* cb[] = {&ws.apc, &ws.axp, &ws.axq, &ws.gw, &ws.wfold, &ws.cfold};
            for (DevBuf* b : cb) HC(b->ensure(sizeof(double) * mm));
            HC(ws.idx.ensure(sizeof(int) * (mmax + 8)));
        }
        {
            DevBuf* lpb[] = {&ws.lpM, &ws.lpT, &ws.lpQ, &ws.lpB, &ws.lpE, &ws.lpC};
            for (DevBuf* b : lpb) HC(b->ensure(sizeof(double) * mm));
        }
        HC(ws.act.ensure(sizeof(int) * (mmax + 8)));
        HC(ws.act_hl.ensure(sizeof(int) * (mmax + 8)));
        HC(ws.norms.ensure(sizeof(double) * (2 * mmax + 8)));
        HC(ws.info.ensure(sizeof(double) * (mmax + 16)));
        HC(ws.h_norms.ensure(sizeof(double) * (2 * mmax + 8)));
        HC(ws.h_theta.ensure(sizeof(double) * (mmax + 8)));
        HC(ws.h_info.ensure(sizeof(double) * (mmax + 16)));
        HC(ws.h_act.ensure(sizeof(int) * (mmax + 8)));
        HC(ws.h_act_hl.ensure(sizeof(int) * (mmax + 8)));
        HC(ws.h_diag.ensure(sizeof(double) * (mmax + 8)));
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
        HC(launch_spmm(st, (int)n, A->rowptr, A->col, A->val, Xs, ld, Ys, ld, w, A->heavy, A->n_heavy));
        return toc(SE_K_SPMM, 12.0 * A->nnz + 4.0 * (n + 1) + 16.0 * n * w, 2.0 * A->nnz * w);
    }
    // AX = A X and, in the same pass, W = AX - X Theta with the residual and
    // column norms in ws.norms (the next residual check reads them). Falls
    // back to the plain product plus the residual kernel for matrices with
    // heavy rows or widths above 128.
    se_status spmm_residual(int k) {
        if (A->n_heavy > 0 || k > 128) {
            ST(spmm(X, AX, k));
            ST(tic());
            HC(launch_resid_norms(st, n, X, AX, ld, k, ws.theta.as<double>(), ws.gram_part.as<double>(),
                                  ws.norms.as<double>(), W, ld));
            return toc(SE_K_RESID, 24.0 * n * k, 5.0 * n * k);
        }
        const size_t need = sizeof(double) * 2 * (size_t)k * (size_t)spmm_resid_chunks(n);
        if (need > ws.gram_part.bytes) {
            ST(sync());  // the old scratch may still be in use by queued kernels
            HC(ws.gram_part.ensure(need));
        }
        ST(tic());
        HC(launch_spmm_resid(st, (int)n, A->rowptr, A->col, A->val, X, ld, AX, ld, k, A->heavy, A->n_heavy,
                             ws.theta.as<double>(), W, ld, ws.gram_part.as<double>(), ws.norms.as<double>()));
        return toc(SE_K_SPMM, 12.0 * A->nnz + 4.0 * (n + 1) + 24.0 * n * k, 2.0 * A->nnz * k + 5.0 * n * k);
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

    // With the W block held as W T (T = ws.wfold, a x a; S = [X, P, W] has
    // m = q + a columns): gw (m x a, the Gram S^T (A W)) becomes
    // diag(I_q, T^T) gw T, the Gram of the orthonormal basis.
    se_status fold_gram(int m, int q, int a) {
        double* gw = ws.gw.as<double>();
        double* tmp = ws.axq.as<double>();  // free until the carried A_p is formed
        const double* T = ws.wfold.as<double>();
        ST(update_rows(m, segx(gw, a, a), T, a, segx(tmp, a, a), 1.0, 0.0));
        HC(launch_copy_cols(st, q, tmp, a, 0, gw, a, 0, a));
        ST(gram_rows(a, segx(T, a, a), segx(tmp + (size_t)q * a, a, a), 0, gw + (size_t)q * a));
        return SE_OK;
    }
    // ws.cfold = diag(I_q, T) ws.C (m x N, leading dimension N): the update
    // coefficients for S = [X, P, W] when the orthonormal block is W T.
    se_status fold_coefficients(int m, int q, int a, int N) {
        const double* C = ws.C.as<double>();
        double* CF = ws.cfold.as<double>();
        HC(launch_copy_cols(st, q, C, N, 0, CF, N, 0, N));
        ST(update_rows(a, segx(ws.wfold.as<double>(), a, a), C + (size_t)q * N, N,
                       segx(CF + (size_t)q * N, N, N), 1.0, 0.0));
        (void)m;
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
        if (a > 0)
            HC(launch_hl_init(st, m, k, ws.Z.as<double>(), ws.act_hl.as<int>(), a, ws.hlB.as<double>(),
                              ws.hlY.as<double>()));
        return hl_tail(m, k, a, ws.Z.as<double>(), ws.hlB.as<double>(), ws.hlY.as<double>(),
                       ws.C.as<double>(), rP);
    }

    // The HL basis from an explicit start block: B (m x a) holds E and Y
    // (k x a) holds Z1^T E; writes C = [Z1 | C_P] (leading dimension k + rP).
    // Uses ws.G, ws.T, ws.hlG and ws.hlQ.
    se_status hl_tail(int m, int k, int a, const double* Z1, double* B, const double* Y, double* C,
                      int& rP) {
        double* G2 = ws.hlG.as<double>();
        double* Q = ws.hlQ.as<double>();
        rP = 0;
        if (a > 0) {
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
    // `ref_norm2` (with `reproject`): squared column norms of the panel before
    // its one projection against `against`. If a column kept less than half of
    // its squared norm, one projection is not enough (the criterion of Kahan
    // and Parlett for classical Gram-Schmidt): *reproject is set and the call
    // returns with the panel untouched, for the caller to project again.
    // `fold_T` (with `folded`): when the last pass keeps every column, its
    // transform T (w x w) is written there instead of being applied, so the
    // orthonormal block is panel * T; the caller carries T in coefficient
    // space. Not with a companion.
    se_status cholqr(double*& w_panel, int& w, double** companion, std::vector<int>* kept_out,
                     const Segs* against = nullptr, const Segs* against_img = nullptr,
                     const double* ref_norm2 = nullptr, bool* reproject = nullptr, double* fold_T = nullptr,
                     bool* folded = nullptr) {
        if (reproject) *reproject = false;
        if (folded) *folded = false;
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
                const bool fold = fold_T && folded && !companion && pass == passes - 1;
                double* Tp = fold ? fold_T : ws.T.as<double>();
                ST(tic());
                HC(launch_chol_drop(st, w, ws.G.as<double>(), Tp, ws.small_work.as<double>(), info_i, info_d,
                                    -1.0, 1e-8));
                ST(toc(SE_K_SMALL, 16.0 * w * w, w * w * (double)w));
                if (fold) {
                    *folded = true;
                    continue;
                }
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
            const bool test_norms = ref_norm2 && reproject && pass == 0;
            if (test_norms)
                HC(hipMemcpy2DAsync(ws.h_diag.p, sizeof(double), ws.G.as<double>(), sizeof(double) * (w + 1),
                                    sizeof(double), w, hipMemcpyDeviceToHost, st));
            ST(sync());
            if (test_norms) {
                const double* dg = ws.h_diag.as<double>();
                for (int q = 0; q < w; ++q)
                    if (dg[q] < 0.5 * ref_norm2[q]) {
                        *reproject = true;
                        return SE_OK;
                    }
            }
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
        if (!X0) {
            HC(launch_seeded_block(st, n, nb, (unsigned long long)p.seed, X, ld, false));
            return SE_OK;
        }
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
    // ratios of the stopping test and of eq. (rk). With R != nullptr the
    // residual block AX - X Theta is written there (leading dimension ld) in
    // the same pass over X and AX.
    se_status check(const double* Xp, const double* AXp, int k, std::vector<double>& stop,
                    std::vector<double>& paper, std::vector<double>& lam, double* R = nullptr) {
        ST(tic());
        HC(launch_resid_norms(st, n, Xp, AXp, ld, k, ws.theta.as<double>(), ws.gram_part.as<double>(),
                              ws.norms.as<double>(), R, ld));
        ST(toc(SE_K_RESID, (R ? 24.0 : 16.0) * n * k, 5.0 * n * k));
        return check_host(k, stop, paper, lam);
    }

    // Reads back the norms and Ritz values of a residual check and forms the
    // per-column ratios.
    se_status check_host(int k, std::vector<double>& stop, std::vector<double>& paper,
                         std::vector<double>& lam) {
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
        h[0] = j + j_off;
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
    // Every kAxpRefresh iterations the whole of A_p is recomputed over n, so
    // rounding in the carried [X, P] block cannot accumulate.
    static constexpr int kAxpRefresh = 10;
    // Default smallest scaled Schur-complement pivot for the implicit
    // orthonormalization of W (se_params.implicit_pivot).
    static constexpr double kImplicitPiv = 1e-2;
    // X0: FP64 column-major start block; k0 >= 0: the X panel already holds
    // k0 start columns (row-major), e.g. from the low-precision phase.
    // p0 > 0: the P panel holds p0 search directions to continue with (they
    // are orthogonalized against the new X and multiplied by A here).
    se_status lobpcg(const double* X0, int k0 = -1, int p0 = 0) {
        ST(alloc_panels(14));
        ST(alloc_small(3 * nb));
        if (p.precond == SE_PRECOND_JACOBI) {
            HC(ws.pc.ensure(sizeof(double) * (size_t)n));
            HC(launch_jacobi(st, (int)n, A->rowptr, A->col, A->val, ws.pc.as<double>()));
        }
        if (k0 < 0) ST(load_x0(X0));
        int k = k0 < 0 ? nb : k0;
        ST(cholqr(X, k, nullptr, nullptr));
        if (k < n_ev) return SE_ERR_BREAKDOWN;
        ST(spmm(X, AX, k));
        ST(rr_plain(k));
        int pw = 0;            // width of P
        int axp_q = -1;        // order of the carried [X, P]^T A [X, P] (ws.axp), -1 = none
        bool ap_valid = true;  // AP = A P for the current P
        if (p0 > 0) {
            const Segs Xs = seg1(X, k);
            for (int pass = 0; pass < 2; ++pass) {
                ST(gram(Xs, seg1(P, p0), 0, ws.G.as<double>()));
                ST(update(Xs, ws.G.as<double>(), p0, seg1(P, p0), -1.0, 1.0));
            }
            ST(cholqr(P, p0, nullptr, nullptr, &Xs));
            if (p0 > 0) ST(spmm(P, AP, p0));
            pw = p0;
        }
        bool have_drop = false;
        int dx = 0, dp = 0;
        std::vector<double> stop, paper, lam;
        std::vector<int> act, act_hl, kept;

        int resid_k = -1;  // > 0: W and the norms already hold the residual of (X, AX, theta), width resid_k
        for (int j = 1; j <= p.max_iter; ++j) {
            // W (dead since the last basis update) receives R = AX - X Theta,
            // unless the product that formed AX wrote it already.
            if (resid_k == k)
                ST(check_host(k, stop, paper, lam));
            else
                ST(check(X, AX, k, stop, paper, lam, W));
            resid_k = -1;
            double r = 0.0, ms = 0.0;
            bool all = true;
            for (int i = 0; i < n_ev; ++i) {
                r = std::max(r, paper[i]);
                ms = std::max(ms, stop[i]);
                all = all && (stop[i] <= p.tol);
            }
            iters = j + j_off;
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

            // W <- T R(:, active): R is already in W; locked columns are
            // gathered out, then the rows are scaled by T (Jacobi).
            int a = (int)act.size();
            if (a < k) {
                std::memcpy(ws.h_act.p, act.data(), sizeof(int) * a);
                HC(hipMemcpyAsync(ws.act.p, ws.h_act.p, sizeof(int) * a, hipMemcpyHostToDevice, st));
                ST(tic());
                HC(launch_gather_cols(st, n, W, ld, ws.act.as<int>(), a, T1, ld));
                ST(toc(SE_K_RESID, 16.0 * n * a, 0.0));
                std::swap(W, T1);
            }
            const bool precond = p.precond == SE_PRECOND_JACOBI;
            if (precond && a > 0) {
                ST(tic());
                HC(launch_row_scale(st, n, a, ws.pc.as<double>(), W, ld));
                ST(toc(SE_K_RESID, 16.0 * n * a + 8.0 * n, 1.0 * n * a));
            }
            // By the Galerkin condition of the last Rayleigh-Ritz step R is
            // orthogonal to [X, P] up to rounding, so one projection usually
            // suffices; a second one runs when a column lost more than half of
            // its squared norm (its squared norm is the residual norm above).
            const Segs XP = seg3(X, k, P, pw, nullptr, 0);
            const bool expand_now = want_expand && have_drop;
            // Implicit orthonormalization of W (iterations without an
            // expansion): with G = [X, P]^T W and H = W^T W, the Gram matrix of
            // S = [X, P, W] is M = [[I, G], [G^T, H]]; its whitening
            // T_M = [[I, -G R^-1], [0, R^-1]] (R from the Schur complement
            // H - G^T G) makes S T_M orthonormal, and the Rayleigh-Ritz step
            // runs on T_M^T A_p T_M. W is neither projected nor
            // orthonormalized over n. It is taken only when the smallest
            // scaled pivot of the Schur complement is at least kImplicitPiv
            // (one Cholesky pass then leaves an error of order u / pivot);
            // otherwise W is projected and orthonormalized explicitly.
            bool implicit = false;
            int r_w = 0;
            const int q0 = k + pw;
            double* GH = ws.apc.as<double>();  // (q0 + a) x a: G on top of H (apc is free here)
            if (!expand_now && a > 0) {
                const int m0 = q0 + a;
                ST(gram(XP, seg1(W, a), 0, GH));
                ST(gram(seg1(W, a), seg1(W, a), 1, GH + (size_t)q0 * a));
                double* I0 = ws.axq.as<double>();
                HC(launch_fill(st, q0, q0, I0, q0, 0.0));
                HC(launch_add_diag(st, q0, I0, q0, 1.0));
                HC(launch_assemble_ap(st, m0, q0, I0, GH, ws.lpM.as<double>()));
                double minpiv = 0.0;
                ST(tic());
                ST(whiten(m0, q0, 1e-13, r_w, &minpiv));
                ST(toc(SE_K_SMALL, 16.0 * m0 * m0, 2.0 * m0 * m0 * (double)a));
                const double piv_min = p.implicit_pivot > 0.0 ? p.implicit_pivot : kImplicitPiv;
                implicit = piv_min <= 1.0 && minpiv >= piv_min && r_w >= n_ev;
                if (implicit) {
                    ++n_implicit;
                    flags |= 8;
                }
            }
            bool folded = false;
            if (!implicit) {
                if (!expand_now && a > 0) {
                    // G is in hand: W <- W - [X, P] G
                    ST(update(XP, GH, a, seg1(W, a), -1.0, 1.0));
                } else {
                    ST(gram(XP, seg1(W, a), 0, ws.G.as<double>()));
                    ST(update(XP, ws.G.as<double>(), a, seg1(W, a), -1.0, 1.0));
                }
                // In iterations that take the carried-A_p path (no expansion,
                // no refresh), the last Cholesky-QR transform T of W is not
                // applied: the orthonormal block is W T, and T enters the Gram
                // S^T (A W) and the coefficients of the basis update instead.
                const bool carried_path = axp_q == k + pw && !expand_now && j % kAxpRefresh != 0;
                double* fold_T = carried_path ? ws.wfold.as<double>() : nullptr;
                const double* nr = ws.h_norms.as<double>();
                std::vector<double> wn2(a);
                for (int q = 0; q < a; ++q) wn2[q] = nr[act[q]];
                bool again = false;
                if (precond) {
                    // T R is not orthogonal to [X, P]: project a second time
                    // (the residual norms are not those of T R)
                    ST(gram(XP, seg1(W, a), 0, ws.G.as<double>()));
                    ST(update(XP, ws.G.as<double>(), a, seg1(W, a), -1.0, 1.0));
                }
                ST(cholqr(W, a, nullptr, nullptr, &XP, nullptr, precond ? nullptr : wn2.data(),
                          precond ? nullptr : &again, fold_T, &folded));
                if (again) {
                    ++n_reproj;
                    ST(gram(XP, seg1(W, a), 0, ws.G.as<double>()));
                    ST(update(XP, ws.G.as<double>(), a, seg1(W, a), -1.0, 1.0));
                    ST(cholqr(W, a, nullptr, nullptr, &XP, nullptr, nullptr, nullptr, fold_T, &folded));
                }
            }
            if (a > 0) ST(spmm(W, AW, a));

            // steepest descent keeps no P: no HL columns
            if (no_p)
                act_hl.clear();
            else
                act_hl = act;
            if (expand_now) {
                // S_drop <- S_drop - S (S^T S_drop), twice; orthonormalize;
                // then its images A S_drop by one SpMM. Random expansion
                // vectors take the place of [X_drop, P_drop].
                int d0 = dx + dp;
                if (p.expand_vectors == SE_EXPAND_RANDOM)
                    HC(launch_gaussian_cols(st, n, d0, nb, n_exp + 1, (unsigned long long)p.seed, Sd, ld, 0));
                const Segs S = seg3(X, k, P, pw, W, a);
                for (int pass = 0; pass < 2; ++pass) {
                    ST(gram(S, seg1(Sd, d0), 0, ws.G.as<double>()));
                    ST(update(S, ws.G.as<double>(), d0, seg1(Sd, d0), -1.0, 1.0));
                }
                ST(cholqr(Sd, d0, nullptr, &kept, &S));
                int dxk = 0;
                for (int v : kept) dxk += (v < dx);
                const int dpk = d0 - dxk;
                if (d0 > 0) ST(spmm(Sd, ASd, d0));
                if (!ap_valid && pw > 0) ST(spmm(P, AP, pw));
                ap_valid = true;
                HC(launch_copy_cols(st, n, Sd, ld, 0, X, ld, k, dxk));
                HC(launch_copy_cols(st, n, ASd, ld, 0, AX, ld, k, dxk));
                HC(launch_copy_cols(st, n, Sd, ld, dxk, P, ld, pw, dpk));
                HC(launch_copy_cols(st, n, ASd, ld, dxk, AP, ld, pw, dpk));
                if (!no_p)
                    for (int q = 0; q < dxk; ++q) act_hl.push_back(k + q);
                k += dxk;
                pw += dpk;
                ctl.did_expand(j);
                have_drop = false;
                ++n_exp;
                flags |= 1;
            }

            // Rayleigh-Ritz on S = [X, P, W]. Outside expansions the
            // [X, P] block of A_p is the carried C^T A_p C of the previous
            // step (Axp), so only S^T (A W) is a product over n.
            const int m = k + pw + a;
            const Segs S = seg3(X, k, P, pw, W, a);
            const Segs AS = seg3(AX, k, AP, pw, AW, a);
            if (axp_q == k + pw && !(flags & 1) && a > 0 && j % kAxpRefresh != 0) {
                ST(gram(S, seg1(AW, a), 0, ws.gw.as<double>()));
                if (folded) ST(fold_gram(m, k + pw, a));
                HC(launch_assemble_ap(st, m, axp_q, ws.axp.as<double>(), ws.gw.as<double>(),
                                      ws.G.as<double>()));
            } else {
                if (!ap_valid && pw > 0) ST(spmm(P, AP, pw));
                ap_valid = true;
                ST(gram(S, AS, 1, ws.G.as<double>()));
            }
            const int ahl = (int)act_hl.size();
            std::memcpy(ws.h_act_hl.p, act_hl.data(), sizeof(int) * ahl);
            HC(hipMemcpyAsync(ws.act_hl.p, ws.h_act_hl.p, sizeof(int) * ahl, hipMemcpyHostToDevice, st));
            int rPv = 0;
            int mr = m;  // order of the (whitened) Rayleigh-Ritz matrix kept in apc
            const double* Cupd = ws.C.as<double>();
            if (implicit) {
                // generalized Rayleigh-Ritz in the whitened basis S T_M; the
                // update coefficients T_M [Z1 | C_P] are in ws.lpC
                ST(grr(m, k + pw, k, ahl, 1e-13, rPv, r_w, ws.apc.as<double>()));
                mr = r_w;
                Cupd = ws.lpC.as<double>();
            } else {
                HC(launch_copy_cols(st, m, ws.G.as<double>(), m, 0, ws.apc.as<double>(), m, 0, m));
                ST(tic());
                HC(launch_syev_lowest(st, m, k, ws.G.as<double>(), ws.theta.as<double>(), ws.Z.as<double>(),
                                      ws.syev_work.as<double>()));
                ST(toc(SE_K_EIG, 8.0 * m * m, 4.0 * m * m * (double)m / 3.0));
                ST(tic());
                ST(hl_coefficients(m, k, ahl, rPv));
                ST(toc(SE_K_SMALL, 16.0 * m * (k + ahl), 8.0 * m * (double)k * ahl));
                if (folded) {
                    ST(fold_coefficients(m, k + pw, a, k + rPv));
                    Cupd = ws.cfold.as<double>();
                }
            }
            const int rP = rPv;
            // New basis over n; its image A X by one SpMM (no carried images:
            // as cheap as updating them for sparse A, and exact each step).
            // A P is formed only when a whole A_p or an expansion needs it.
            Segs O = make_segs(ld);
            push_seg(O, Xn, k);
            push_seg(O, Pn, rP);
            ST(update(S, Cupd, k + rP, O, 1.0, 0.0));
            std::swap(X, Xn);
            std::swap(P, Pn);
            pw = rP;
            ST(spmm_residual(k));
            resid_k = k;
            ap_valid = false;
            // carried [X, P]^T A [X, P] = C^T A_p C (small products in the
            // orthonormal, possibly whitened, basis of order mr)
            {
                const int q = k + rP;
                ST(update_rows(mr, segx(ws.apc.as<double>(), mr, mr), ws.C.as<double>(), q,
                               segx(ws.axq.as<double>(), q, q), 1.0, 0.0));
                ST(gram_rows(mr, segx(ws.C.as<double>(), q, q), segx(ws.axq.as<double>(), q, q), 1,
                             ws.axp.as<double>()));
                axp_q = q;
            }

            if (ctl.ifshrink(j)) {
                dx = k - n_es;
                dp = std::max(0, pw - n_es);
                dp = std::min(dp, ld - dx);  // S_drop must fit one panel
                if (p.expand_vectors == SE_EXPAND_XDROP) {
                    HC(launch_copy_cols(st, n, X, ld, n_es, Sd, ld, 0, dx));
                    HC(launch_copy_cols(st, n, P, ld, n_es, Sd, ld, dx, dp));
                }
                // keep the rows and columns of X(:, 0:n_es) and P(:, 0:pw') in Axp
                const int pk = std::min(pw, n_es);
                std::vector<int> keep;
                for (int i = 0; i < n_es; ++i) keep.push_back(i);
                for (int i = 0; i < pk; ++i) keep.push_back(k + i);
                const int q = (int)keep.size();
                std::memcpy(ws.h_act.p, keep.data(), sizeof(int) * q);
                HC(hipMemcpyAsync(ws.idx.p, ws.h_act.p, sizeof(int) * q, hipMemcpyHostToDevice, st));
                HC(launch_gather_sym(st, q, ws.idx.as<int>(), ws.axp.as<double>(), axp_q,
                                     ws.axq.as<double>()));
                HC(launch_copy_cols(st, q, ws.axq.as<double>(), q, 0, ws.axp.as<double>(), q, 0, q));
                axp_q = q;
                k = n_es;
                pw = pk;
                have_drop = true;
                ctl.did_shrink(j);
                ++n_shr;
                flags |= 2;
            }
            amend_flags(flags);
        }
        return SE_OK;
    }

    // Chebyshev filter of degree p.filter_degree on the w columns of Y: damps
    // [cut, up] and is one at `lower`, by the scaled three-term recurrence
    // Y_1 = (s_1 / e) (A - cI) Y_0, Y_i = (2 s_i / e) (A - cI) Y_{i-1} -
    // s_{i-1} s_i Y_{i-2}, s_1 = e / (lower - c), s_i = 1 / (2 / s_1 - s_{i-1})
    // (c, e the centre and half-width of [cut, up]), which keeps the block of
    // order one. AY0 = A Y when known (else one more product into tmp). Y and
    // Yalt are two panels that rotate; on return Y holds the filtered block.
    // Without heavy rows each later step is one fused product-and-step pass.
    se_status cheb_filter(double*& Y, double*& Yalt, const double* AY0, double* tmp, int w, double lower,
                          double cut, double up) {
        const double c = 0.5 * (up + cut), e = 0.5 * (up - cut);
        double s = e / (lower - c);
        const double tau = 2.0 / s;
        if (!AY0) {
            ST(spmm(Y, tmp, w));
            AY0 = tmp;
        }
        double alpha = s / e;
        ST(tic());
        HC(launch_cheb_step(st, n, w, alpha, AY0, -c * alpha, Y, 0.0, Yalt, ld));
        ST(toc(SE_K_RESID, 24.0 * n * w, 3.0 * n * w));
        double* prev = Y;
        double* cur = Yalt;
        for (int i = 2; i <= p.filter_degree; ++i) {
            const double s_new = 1.0 / (tau - s);
            alpha = 2.0 * s_new / e;
            if (A->n_heavy == 0) {
                // product and step in one pass: A Y never goes to memory
                ST(tic());
                HC(launch_spmm_cheb(st, (int)n, A->rowptr, A->col, A->val, cur, prev, ld, w, 0, alpha, -c * alpha,
                                    -s * s_new));
                ST(toc(SE_K_SPMM, 12.0 * A->nnz + 4.0 * (n + 1) + 32.0 * n * w, 2.0 * A->nnz * w + 5.0 * n * w));
            } else {
                ST(spmm(cur, tmp, w));
                ST(tic());
                HC(launch_cheb_step(st, n, w, alpha, tmp, -c * alpha, cur, -s * s_new, prev, ld));
                ST(toc(SE_K_RESID, 32.0 * n * w, 5.0 * n * w));
            }
            s = s_new;
            std::swap(prev, cur);
        }
        Y = cur;
        Yalt = prev;
        return SE_OK;
    }

    // ------------------------------------------------- subspace iteration --
    se_status si(const double* X0, int k0 = -1) {
        ST(alloc_panels(14));
        ST(alloc_small(nb));
        if (k0 < 0) ST(load_x0(X0));
        const double sigma = (p.sigma > 0.0) ? p.sigma : A->anorm;
        int k = k0 < 0 ? nb : k0;
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
            iters = j + j_off;
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
            // Y <- sigma X - A X, or the Chebyshev filter on [theta_k, sigma]
            // (AX is current), then append X_drop.
            const bool filt = p.filter_degree > 0 && sigma > lam[k - 1];
            if (filt) {
                ST(cheb_filter(X, Xn, AX, AW, k, lam[0], lam[k - 1], sigma));
            } else {
                ST(tic());
                HC(launch_shift_sub(st, n, X, AX, ld, k, sigma));
                ST(toc(SE_K_RESID, 24.0 * n * k, 2.0 * n * k));
            }
            if (have_drop && p.expand_vectors == SE_EXPAND_POWERED) {
                // one power step on the held X_drop, without orthogonalization:
                // the same filter, or the shifted step divided by
                // sigma - theta_1 to keep it of order one
                if (filt) {
                    ST(cheb_filter(Sd, T1, nullptr, ASd, dx, lam[0], lam[k - 1], sigma));
                } else {
                    ST(spmm(Sd, ASd, dx));
                    const double gap = sigma - lam[0];
                    ST(tic());
                    HC(launch_shift_sub(st, n, Sd, ASd, ld, dx, sigma, gap > 0.0 ? 1.0 / gap : 1.0));
                    ST(toc(SE_K_RESID, 24.0 * n * dx, 3.0 * n * dx));
                }
            }
            if (want_expand && have_drop) {
                if (p.expand_vectors == SE_EXPAND_RANDOM)
                    HC(launch_gaussian_cols(st, n, dx, nb, n_exp + 1, (unsigned long long)p.seed, X, ld, k));
                else
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
                if (p.expand_vectors != SE_EXPAND_RANDOM)
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

    // ------------------------------------------------------------ TraceMIN --
    // Algorithm 4: R = AX - X Theta; D from p.cg_steps conjugate-gradient
    // steps on P A P D = P R (P = I - X X^T, every column at once with its own
    // step lengths, from D = 0); X <- X - D; [X, X_drop] at an expansion;
    // Cholesky-QR; Rayleigh-Ritz; shrink. Panels: R in W, D in P, the CG
    // direction in Pn, its image (A d, then projected) in AW.
    se_status tracemin(const double* X0) {
        ST(alloc_panels(14));
        ST(alloc_small(nb));
        HC(ws.cg.ensure(sizeof(double) * (3 * (size_t)nb + 8)));
        ST(load_x0(X0));
        const int steps = p.cg_steps > 0 ? p.cg_steps : 5;
        int k = nb;
        ST(cholqr(X, k, nullptr, nullptr));
        if (k < n_ev) return SE_ERR_BREAKDOWN;
        ST(spmm(X, AX, k));
        ST(rr_plain(k));
        double* rr = ws.cg.as<double>();
        double* rr_new = rr + nb;
        double* dq = rr + 2 * nb;
        double* part = ws.gram_part.as<double>();
        bool have_drop = false;
        int dx = 0;
        std::vector<double> stop, paper, lam;
        for (int j = 1; j <= p.max_iter; ++j) {
            ST(check(X, AX, k, stop, paper, lam, W));  // W = R = AX - X Theta
            double r = 0.0, ms = 0.0;
            bool all = true;
            for (int i = 0; i < n_ev; ++i) {
                r = std::max(r, paper[i]);
                ms = std::max(ms, stop[i]);
                all = all && (stop[i] <= p.tol);
            }
            iters = j + j_off;
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

            // projected CG from D = 0: r = P R, d = r
            const Segs Xs = seg1(X, k);
            ST(gram(Xs, seg1(W, k), 0, ws.G.as<double>()));
            ST(update(Xs, ws.G.as<double>(), k, seg1(W, k), -1.0, 1.0));
            HC(launch_copy_cols(st, n, W, ld, 0, Pn, ld, 0, k));
            ST(tic());
            HC(launch_col_dots(st, n, k, W, W, ld, part, rr));
            ST(toc(SE_K_RESID, 8.0 * n * k, 2.0 * n * k));
            for (int s = 0; s < steps; ++s) {
                ST(spmm(Pn, AW, k));  // q = A d
                ST(gram(Xs, seg1(AW, k), 0, ws.G.as<double>()));
                ST(update(Xs, ws.G.as<double>(), k, seg1(AW, k), -1.0, 1.0));  // q = P q
                ST(tic());
                HC(launch_col_dots(st, n, k, Pn, AW, ld, part, dq));
                HC(launch_cg_step(st, n, k, rr, dq, Pn, AW, P, W, ld, s == 0, part, rr_new));
                ST(toc(SE_K_RESID, 56.0 * n * k, 8.0 * n * k));
                if (s + 1 < steps) {
                    ST(tic());
                    HC(launch_cg_dir(st, n, k, rr_new, rr, W, Pn, ld));
                    ST(toc(SE_K_RESID, 24.0 * n * k, 2.0 * n * k));
                }
                std::swap(rr, rr_new);
            }
            // X <- X - D
            ST(tic());
            HC(launch_cheb_step(st, n, k, -1.0, P, 0.0, P, 1.0, X, ld));
            ST(toc(SE_K_RESID, 24.0 * n * k, 2.0 * n * k));
            if (ctl.ifexpand(j) && have_drop) {
                if (p.expand_vectors == SE_EXPAND_RANDOM)
                    HC(launch_gaussian_cols(st, n, dx, nb, n_exp + 1, (unsigned long long)p.seed, X, ld, k));
                else
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
                if (p.expand_vectors != SE_EXPAND_RANDOM)
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

    // ----------------------------------------------------- mixed precision --
    // The low-precision phase keeps every n-length block in FP32 or BF16
    // panels and does its arithmetic in FP32 with FP64 reductions; all small
    // dense work stays FP64. Its basis is orthonormal only to the storage
    // precision, so the Rayleigh-Ritz step solves A_p z = theta M z with
    // M = S^T S (grr). Once r(j) <= r_switch, or - with the best r(j) within
    // 100 r_switch - r(j) rises above ten times its best value (the
    // low-precision iteration has reached its floor) or has not improved for
    // kStall iterations, the current X (with X_drop when shrunk) and P are
    // widened to FP64 and the FP64 solver continues.
    static constexpr int kStall = 15;
    void* lp[kNumLpPanels] = {};

    template <class T>
    SegsT<T> lseg1(const T* a, int wa) const {
        SegsT<T> s = make_segs_t<T>(ld);
        push_seg_t(s, a, wa);
        return s;
    }
    template <class T>
    SegsT<T> lseg3(const T* a, int wa, const T* b, int wb, const T* c, int wc) const {
        SegsT<T> s = make_segs_t<T>(ld);
        push_seg_t(s, a, wa);
        push_seg_t(s, b, wb);
        push_seg_t(s, c, wc);
        return s;
    }
    // Unit roundoff of the storage format.
    template <class T>
    static double unit_roundoff() {
        return sizeof(T) == 4 ? 5.9604644775390625e-8 : 3.90625e-3;
    }
    // Drop threshold of the whitening (scaled Cholesky pivots of M or of its
    // Schur complement). The Gram matrices of the stored panels are exact
    // products rounded only by FP32 accumulation (u32 = 2^-24; BF16 products
    // are exact in FP32), and a pivot delta^2 carries a relative error of
    // about u32 / delta^2, so pivots below 450 u32 are dropped: the FP64
    // path's ratio (1e-13 ~ 450 u64).
    static constexpr double kLpDrop2 = 450.0 * 5.9604644775390625e-8;

    template <class T>
    se_status lp_alloc() {
        const size_t bytes = sizeof(T) * (size_t)n * ld;
        for (int i = 0; i < kNumLpPanels; ++i) {
            HC(ws.lp_panel[i].ensure(bytes));
            lp[i] = ws.lp_panel[i].p;
        }
        HC(make_val32(st, A));
        const size_t mm = (size_t)3 * nb * 3 * nb;  // largest K x N of an update
        HC(ws.c32.ensure(sizeof(float) * mm));
        return SE_OK;
    }
    template <class T>
    se_status lp_spmm(const T* Xs, T* Ys, int w) {
        ST(tic());
        HC(launch_spmm_lp<T>(st, (int)n, A->rowptr, A->col, A->val32, Xs, ld, Ys, ld, w, A->heavy, A->n_heavy));
        return toc(SE_K_SPMM, 8.0 * A->nnz + 4.0 * (n + 1) + 2.0 * sizeof(T) * n * w, 2.0 * A->nnz * w);
    }
    template <class T>
    se_status lp_gram(const SegsT<T>& U, const SegsT<T>& V, int sym, double* C) {
        const size_t need = sizeof(double) * gram_scratch_doubles(n, segs_width(U), segs_width(V));
        if (need > ws.gram_part.bytes) {
            ST(sync());
            HC(ws.gram_part.ensure(need));
        }
        ST(tic());
        HC(launch_gram_lp<T>(st, n, U, V, sym, ws.gram_part.as<double>(), C));
        const double mu = segs_width(U), mv = segs_width(V);
        const double fl = (sym && mu == mv) ? n * mu * (mu + 1.0) : 2.0 * n * mu * mv;
        const bool same = sym && U.nseg == V.nseg && U.p[0] == V.p[0];
        return toc(SE_K_GRAM, (double)sizeof(T) * n * (same ? mu : mu + mv), fl);
    }
    template <class T>
    se_status lp_update(const SegsT<T>& U, const double* C, int N, const SegsT<T>& O, double alpha,
                        double beta) {
        ST(tic());
        HC(launch_update_lp<T>(st, n, U, C, N, O, alpha, beta, ws.c32.as<float>()));
        const double K = segs_width(U);
        return toc(SE_K_UPDATE, (double)sizeof(T) * n * (K + N * (beta != 0.0 ? 2.0 : 1.0)),
                   2.0 * n * K * N);
    }
    template <class T>
    se_status lp_check(const T* Xp, const T* AXp, int k, std::vector<double>& stop,
                       std::vector<double>& paper, std::vector<double>& lam) {
        ST(tic());
        HC(launch_resid_norms_lp<T>(st, n, Xp, AXp, ld, k, ws.theta.as<double>(), ws.gram_part.as<double>(),
                                    ws.norms.as<double>()));
        ST(toc(SE_K_RESID, 2.0 * sizeof(T) * n * k, 5.0 * n * k));
        return check_host(k, stop, paper, lam);
    }

    // Whitening of the basis for the generalized Rayleigh-Ritz step: writes
    // T_M (m x r, ws.lpT, leading dimension r) with T_M^T M T_M = I for
    // M = ws.lpM, dropping dependent columns (scaled pivots below drop2).
    // When the first q columns are orthonormal up to E = M11 - I with
    // ||E||_F <= 1e-2 (the X and P columns that leave every Rayleigh-Ritz
    // step whitened, rounded to the storage format), only the Schur
    // complement of the other a2 = m - q columns is factorized:
    //   B = -M11^{-1} M12 (Neumann series to E^3), S22 = M22 + M12^T B,
    //   S22 = R^T R (scaled, with drop) -> T22 = R^{-1},
    //   T11 = M11^{-1/2} = I - E/2 + 3E^2/8 - 5E^3/16,
    //   T_M = [[T11, B T22], [0, T22]].
    // Otherwise (or when the check fails) the whole of M is factorized.
    se_status whiten(int m, int q, double drop2, int& r, double* minpiv = nullptr) {
        if (minpiv) *minpiv = 0.0;
        double* M = ws.lpM.as<double>();
        double* TM = ws.lpT.as<double>();
        int* info_i = ws.info.as<int>();
        const int doff = (m + 8) / 2 + 4;
        double* info_d = ws.info.as<double>() + doff;
        const size_t rb = sizeof(double) * (doff + 2);
        const int a2 = m - q;
        if (q > 0 && a2 > 0) {
            double* E = ws.hlB.as<double>();    // q x q
            double* M12 = ws.hlY.as<double>();  // q x a2
            double* Fa = ws.hlG.as<double>();   // q x a2
            double* Fb = ws.hlQ.as<double>();   // q x a2
            double* S22 = ws.lpQ.as<double>();  // a2 x a2
            double* G22 = ws.lpB.as<double>();  // a2 x a2
            double* H = ws.lpE.as<double>();    // q x q
            double* T11 = ws.lpC.as<double>();  // q x q
            double* BT = ws.C.as<double>();     // q x r2
            double* T22 = ws.T.as<double>();    // a2 x r2
            const long long qq = (long long)q * q;
            const Segs Es = segx(E, q, q);
            HC(launch_copy_cols(st, q, M, m, 0, E, q, 0, q));
            HC(launch_add_diag(st, q, E, q, -1.0));
            HC(launch_sumsq(st, qq, E, info_d + 1));
            HC(launch_copy_cols(st, q, M, m, q, M12, a2, 0, a2));
            // F = M12 - E (M12 - E (M12 - E M12)) = M11^{-1} M12 + O(E^4)
            HC(launch_copy_cols(st, q, M12, a2, 0, Fa, a2, 0, a2));
            ST(update_rows(q, Es, M12, a2, segx(Fa, a2, a2), -1.0, 1.0));
            HC(launch_copy_cols(st, q, M12, a2, 0, Fb, a2, 0, a2));
            ST(update_rows(q, Es, Fa, a2, segx(Fb, a2, a2), -1.0, 1.0));
            HC(launch_copy_cols(st, q, M12, a2, 0, Fa, a2, 0, a2));
            ST(update_rows(q, Es, Fb, a2, segx(Fa, a2, a2), -1.0, 1.0));
            HC(launch_axpby(st, (long long)q * a2, 0.0, Fa, -1.0, Fa));  // B = -F
            HC(launch_copy_cols(st, a2, M + (size_t)q * m, m, q, S22, a2, 0, a2));
            ST(gram_rows(q, segx(M12, a2, a2), segx(Fa, a2, a2), 0, G22));
            HC(launch_axpby(st, (long long)a2 * a2, 1.0, G22, 1.0, S22));
            HC(launch_chol_drop(st, a2, S22, T22, ws.small_work.as<double>(), info_i, info_d, drop2));
            // T11 = I + E (-1/2 I + E (3/8 I - 5/16 E))
            HC(launch_copy_cols(st, q, E, q, 0, H, q, 0, q));
            HC(launch_axpby(st, qq, 0.0, E, -5.0 / 16.0, H));
            HC(launch_add_diag(st, q, H, q, 3.0 / 8.0));
            ST(update_rows(q, Es, H, q, segx(T11, q, q), 1.0, 0.0));
            HC(launch_add_diag(st, q, T11, q, -0.5));
            ST(update_rows(q, Es, T11, q, segx(H, q, q), 1.0, 0.0));
            HC(launch_add_diag(st, q, H, q, 1.0));
            HC(hipMemcpyAsync(ws.h_info.p, ws.info.p, rb, hipMemcpyDeviceToHost, st));
            ST(sync());
            const int r2 = ws.h_info.as<int>()[0];
            const double e2 = ws.h_info.as<double>()[doff + 1];
            if (minpiv) *minpiv = ws.h_info.as<double>()[doff];
            if (e2 <= 1e-4) {
                r = q + r2;
                if (r2 > 0) ST(update_rows(q, segx(Fa, a2, a2), T22, r2, segx(BT, r2, r2), 1.0, 0.0));
                HC(launch_copy_cols(st, q, H, q, 0, TM, r, 0, q));
                HC(launch_copy_cols(st, q, BT, r2, 0, TM, r, q, r2));
                HC(launch_fill(st, a2, q, TM + (size_t)q * r, r, 0.0));
                HC(launch_copy_cols(st, a2, T22, r2, 0, TM + (size_t)q * r, r, q, r2));
                return SE_OK;
            }
        }
        HC(launch_chol_drop(st, m, M, TM, ws.small_work.as<double>(), info_i, info_d, drop2));
        HC(hipMemcpyAsync(ws.h_info.p, ws.info.p, sizeof(int) * 4, hipMemcpyDeviceToHost, st));
        ST(sync());
        r = ws.h_info.as<int>()[0];
        return SE_OK;
    }

    // Generalized Rayleigh-Ritz on m basis columns: M = ws.lpM and
    // A_p = ws.G (both FP64, m x m); the first q columns are the whitened X
    // and P of the previous step (see whiten). With T_M from whiten, the k
    // lowest pairs of T_M^T A_p T_M give theta and Y (r x k). With ahl > 0
    // the HL basis is built in the whitened coordinates from the old X columns
    // act_hl (indices into S), whose coordinates there are E' = T_M^T M E.
    // Output: the coefficients C = T_M [Y | C_P'] in ws.lpC (m x (k + rP));
    // k is lowered to r if fewer columns survive.
    // r_given >= 0: T_M is already in ws.lpT with r columns (whiten was
    // called by the caller). ap_copy: receives T_M^T A_p T_M (r x r) before
    // the eigensolver overwrites it.
    se_status grr(int m, int q, int& k, int ahl, double drop2, int& rP, int r_given = -1,
                  double* ap_copy = nullptr) {
        double* M = ws.lpM.as<double>();
        double* TM = ws.lpT.as<double>();
        double* Q = ws.lpQ.as<double>();
        double* Ar = ws.lpB.as<double>();
        ST(tic());
        int r = r_given;
        if (r < 0) ST(whiten(m, q, drop2, r));
        if (r < n_ev) return SE_ERR_BREAKDOWN;
        k = std::min(k, r);
        ST(update_rows(m, segx(ws.G.as<double>(), m, m), TM, r, segx(Q, r, r), 1.0, 0.0));
        ST(gram_rows(m, segx(TM, r, r), segx(Q, r, r), 1, Ar));
        if (ap_copy) HC(launch_copy_cols(st, r, Ar, r, 0, ap_copy, r, 0, r));
        HC(launch_syev_lowest(st, r, k, Ar, ws.theta.as<double>(), ws.Z.as<double>(),
                              ws.syev_work.as<double>()));
        double* Cr = ws.C.as<double>();
        rP = 0;
        if (ahl > 0) {
            // E' (r x a): rows act_hl of M T_M, transposed; then Y^T E'.
            ST(update_rows(m, segx(M, m, m), TM, r, segx(Q, r, r), 1.0, 0.0));
            HC(launch_hl_init(st, m, r, Q, ws.act_hl.as<int>(), ahl, ws.hlQ.as<double>(),
                              ws.lpE.as<double>()));
            ST(gram_rows(r, segx(ws.Z.as<double>(), k, k), segx(ws.lpE.as<double>(), ahl, ahl), 0,
                         ws.hlY.as<double>()));
            ST(hl_tail(r, k, ahl, ws.Z.as<double>(), ws.lpE.as<double>(), ws.hlY.as<double>(), Cr, rP));
        } else {
            HC(launch_copy_cols(st, r, ws.Z.as<double>(), k, 0, Cr, k, 0, k));
        }
        ST(update_rows(m, segx(TM, r, r), Cr, k + rP, segx(ws.lpC.as<double>(), k + rP, k + rP), 1.0, 0.0));
        return toc(SE_K_EIG, 8.0 * m * m, 4.0 * m * m * (double)m);
    }

    double r_switch_value(double u) const {
        if (p.r_switch > 0.0) return p.r_switch;
        // Defaults: a few times above the lowest r(j) a block stored with
        // unit roundoff u resolves (FP32: 1e-5; BF16: 4e-2, about ten times
        // its machine epsilon 2^-8).
        return u < 1e-6 ? 1e-5 : 4e-2;
    }

    // Widens the low-precision X (and X_drop) into the FP64 X panel and the
    // search directions P into the FP64 P panel; returns the column counts.
    template <class T>
    se_status lp_to_f64(const T* Xl, int k, const T* Sdl, int dx, const T* Pl, int pw, int& k0, int& p0) {
        ST(alloc_panels(14));
        HC(launch_rows_lp_to_f64<T>(st, n, k, Xl, ld, X, ld));
        if (dx > 0) HC(launch_rows_lp_to_f64<T>(st, n, dx, Sdl, ld, X + k, ld));
        if (pw > 0) HC(launch_rows_lp_to_f64<T>(st, n, pw, Pl, ld, P, ld));
        k0 = k + dx;
        p0 = pw;
        return SE_OK;
    }

    // LOBPCG (Algorithm 3) with shrink-and-expand on low-precision panels.
    // No soft locking (the low-precision residuals stop above tol); W is
    // R(:, all) and is not orthogonalized separately: the Cholesky factor of
    // M removes its dependence on [X, P] and scales it.
    template <class T>
    se_status lobpcg_lp(const double* X0, int& k0, int& p0) {
        ST(alloc_panels(14));
        ST(alloc_small(3 * nb));
        ST(lp_alloc<T>());
        T* L[kNumLpPanels];
        for (int i = 0; i < kNumLpPanels; ++i) L[i] = static_cast<T*>(lp[i]);
        T *Xl = L[0], *Pl = L[1], *Wl = L[2], *AXl = L[3], *APl = L[4], *AWl = L[5];
        T *Xnl = L[6], *Pnl = L[7], *AXnl = L[8], *APnl = L[9], *Sdl = L[10], *ASdl = L[11];
        const double u = unit_roundoff<T>();
        const double drop2 = kLpDrop2;
        const double rsw = r_switch_value(u);
        if (!X0) {
            HC(launch_seeded_block(st, n, nb, (unsigned long long)p.seed, T1, n, true));
            HC(launch_colmajor_to_rows_lp<T>(st, n, nb, T1, n, Xl, ld));
        } else if (p.ptr_mode == SE_PTR_HOST) {
            HC(hipMemcpyAsync(T1, X0, sizeof(double) * (size_t)n * nb, hipMemcpyHostToDevice, st));
            HC(launch_colmajor_to_rows_lp<T>(st, n, nb, T1, n, Xl, ld));
        } else {
            HC(launch_colmajor_to_rows_lp<T>(st, n, nb, X0, n, Xl, ld));
        }
        int k = nb;
        ST(lp_spmm(Xl, AXl, k));
        {
            const SegsT<T> Xs = lseg1(Xl, k);
            ST(lp_gram(Xs, Xs, 1, ws.lpM.as<double>()));
            ST(lp_gram(Xs, lseg1(AXl, k), 1, ws.G.as<double>()));
            int kk = k, rP = 0;
            ST(grr(k, 0, kk, 0, drop2, rP));
            ST(lp_update(Xs, ws.lpC.as<double>(), kk, lseg1(Xnl, kk), 1.0, 0.0));
            ST(lp_update(lseg1(AXl, k), ws.lpC.as<double>(), kk, lseg1(AXnl, kk), 1.0, 0.0));
            std::swap(Xl, Xnl);
            std::swap(AXl, AXnl);
            k = kk;
        }
        int pw = 0, dx = 0, dp = 0;
        bool have_drop = false;
        double best = INFINITY;
        int j_best = 0;
        std::vector<double> stop, paper, lam;
        std::vector<int> act, act_hl;
        for (int j = 1; j <= p.max_iter; ++j) {
            ST(lp_check(Xl, AXl, k, stop, paper, lam));
            double r = 0.0, ms = 0.0;
            bool all = true;
            for (int i = 0; i < n_ev; ++i) {
                r = std::max(r, paper[i]);
                ms = std::max(ms, stop[i]);
                all = all && (stop[i] <= p.tol);
            }
            iters = j;
            lp_iters = j;
            last_r = r;
            last_stop = ms;
            ctl.observe(j, r);
            record(j, r, ms, k, pw, k, 0, 4);
            if (r < best) {
                best = r;
                j_best = j;
            }
            if (all) {
                lp_done = true;
                break;
            }
            const bool near_floor = best <= 100.0 * rsw;  // early iterations may rise and stall
            if (r <= rsw || (near_floor && (r > 10.0 * best || j - j_best >= kStall)) || out_of_time())
                break;
            const bool want_expand = ctl.ifexpand(j);
            int flags = 4;

            const int a = k;
            act.resize(a);
            for (int i = 0; i < a; ++i) act[i] = i;
            std::memcpy(ws.h_act.p, act.data(), sizeof(int) * a);
            HC(hipMemcpyAsync(ws.act.p, ws.h_act.p, sizeof(int) * a, hipMemcpyHostToDevice, st));
            ST(tic());
            HC(launch_form_w_lp<T>(st, n, Xl, AXl, ld, ws.theta.as<double>(), ws.act.as<int>(), a, Wl, ld));
            ST(toc(SE_K_RESID, 3.0 * sizeof(T) * n * a, 2.0 * n * a));
            ST(lp_spmm(Wl, AWl, a));
            // S = [X, P, S_drop (at an expansion), W]: X and P leave the
            // previous step whitened, so they lead (q columns); S_drop joins
            // the block that is factorized, and its X part is kept with X.
            if (no_p)
                act_hl.clear();
            else
                act_hl = act;
            const bool expand = want_expand && have_drop;
            const int dd = expand ? dx + dp : 0;
            if (expand) {
                if (!no_p)
                    for (int q = 0; q < dx; ++q) act_hl.push_back(k + pw + q);
                ctl.did_expand(j);
                have_drop = false;
                ++n_exp;
                flags |= 1;
            }
            const int q = k + pw;
            const int m = q + dd + a;
            SegsT<T> S = make_segs_t<T>(ld), AS = make_segs_t<T>(ld);
            push_seg_t(S, (const T*)Xl, k);
            push_seg_t(S, (const T*)Pl, pw);
            push_seg_t(S, (const T*)Sdl, dd);
            push_seg_t(S, (const T*)Wl, a);
            push_seg_t(AS, (const T*)AXl, k);
            push_seg_t(AS, (const T*)APl, pw);
            push_seg_t(AS, (const T*)ASdl, dd);
            push_seg_t(AS, (const T*)AWl, a);
            ST(lp_gram(S, S, 1, ws.lpM.as<double>()));
            ST(lp_gram(S, AS, 1, ws.G.as<double>()));
            const int ahl = (int)act_hl.size();
            std::memcpy(ws.h_act_hl.p, act_hl.data(), sizeof(int) * ahl);
            HC(hipMemcpyAsync(ws.act_hl.p, ws.h_act_hl.p, sizeof(int) * ahl, hipMemcpyHostToDevice, st));
            int kk = k + (expand ? dx : 0), rP = 0;
            ST(grr(m, q, kk, ahl, drop2, rP));
            SegsT<T> O = make_segs_t<T>(ld);
            push_seg_t(O, (const T*)Xnl, kk);
            push_seg_t(O, (const T*)Pnl, rP);
            ST(lp_update(S, ws.lpC.as<double>(), kk + rP, O, 1.0, 0.0));
            std::swap(Xl, Xnl);
            std::swap(Pl, Pnl);
            k = kk;
            pw = rP;
            // images of the new X and P by SpMM (cheaper than updating them
            // with the m-column coefficient matrix for sparse A)
            ST(lp_spmm(Xl, AXl, k));
            if (pw > 0) ST(lp_spmm(Pl, APl, pw));
            if (ctl.ifshrink(j) && k > n_es) {
                dx = k - n_es;
                dp = std::max(0, pw - n_es);
                dp = std::min(dp, ld - dx);
                HC(launch_copy_cols_lp<T>(st, n, Xl, ld, n_es, Sdl, ld, 0, dx));
                HC(launch_copy_cols_lp<T>(st, n, AXl, ld, n_es, ASdl, ld, 0, dx));
                HC(launch_copy_cols_lp<T>(st, n, Pl, ld, n_es, Sdl, ld, dx, dp));
                HC(launch_copy_cols_lp<T>(st, n, APl, ld, n_es, ASdl, ld, dx, dp));
                k = n_es;
                pw = std::min(pw, n_es);
                have_drop = true;
                ctl.did_shrink(j);
                ++n_shr;
                flags |= 2;
            }
            amend_flags(flags);
        }
        if (lp_done)  // X leaves in FP64 with its Ritz values (finish re-checks)
            return lp_to_f64(Xl, k, Sdl, 0, Pl, 0, k0, p0);
        const int dxk = have_drop ? std::min(dx, nb - k) : 0;
        return lp_to_f64(Xl, k, Sdl, dxk, Pl, std::min(pw, ld), k0, p0);
    }

    // Subspace iteration (Algorithm 1) with shrink-and-expand on
    // low-precision panels: Y = sigma X - A X (plus X_drop at an expansion),
    // then the generalized Rayleigh-Ritz step on span(Y).
    // The Chebyshev filter of cheb_filter on low-precision blocks: each step's
    // product A Y is stored, and the step is formed in FP64 and rounded once.
    template <class T>
    se_status cheb_filter_lp(T*& Y, T*& Yalt, const T* AY0, T* tmp, int w, double lower, double cut,
                             double up) {
        const double c = 0.5 * (up + cut), e = 0.5 * (up - cut);
        double s = e / (lower - c);
        const double tau = 2.0 / s;
        if (!AY0) {
            ST(lp_spmm(Y, tmp, w));
            AY0 = tmp;
        }
        double alpha = s / e;
        ST(tic());
        HC(launch_cheb_step_lp<T>(st, n, w, alpha, AY0, -c * alpha, Y, 0.0, Yalt, ld));
        ST(toc(SE_K_RESID, 3.0 * sizeof(T) * n * w, 3.0 * n * w));
        T* prev = Y;
        T* cur = Yalt;
        for (int i = 2; i <= p.filter_degree; ++i) {
            const double s_new = 1.0 / (tau - s);
            alpha = 2.0 * s_new / e;
            if (A->n_heavy == 0) {
                ST(tic());
                HC(launch_spmm_cheb_lp<T>(st, (int)n, A->rowptr, A->col, A->val32, cur, prev, ld, w, 0, alpha,
                                          -c * alpha, -s * s_new));
                ST(toc(SE_K_SPMM, 8.0 * A->nnz + 4.0 * (n + 1) + 4.0 * sizeof(T) * n * w,
                       2.0 * A->nnz * w + 5.0 * n * w));
            } else {
                ST(lp_spmm(cur, tmp, w));
                ST(tic());
                HC(launch_cheb_step_lp<T>(st, n, w, alpha, tmp, -c * alpha, cur, -s * s_new, prev, ld));
                ST(toc(SE_K_RESID, 4.0 * sizeof(T) * n * w, 5.0 * n * w));
            }
            s = s_new;
            std::swap(prev, cur);
        }
        Y = cur;
        Yalt = prev;
        return SE_OK;
    }

    template <class T>
    se_status si_lp(const double* X0, int& k0) {
        int p0 = 0;
        ST(alloc_panels(14));
        ST(alloc_small(nb));
        ST(lp_alloc<T>());
        T* Xl = static_cast<T*>(lp[0]);
        T* AXl = static_cast<T*>(lp[3]);
        T* Xnl = static_cast<T*>(lp[6]);
        T* AXnl = static_cast<T*>(lp[8]);
        T* Sdl = static_cast<T*>(lp[10]);
        T* T1l = static_cast<T*>(lp[1]);  // filter products
        T* T2l = static_cast<T*>(lp[2]);  // rotation panel of the powered X_drop
        const double u = unit_roundoff<T>();
        const double drop2 = kLpDrop2;
        const double rsw = r_switch_value(u);
        const double sigma = (p.sigma > 0.0) ? p.sigma : A->anorm;
        if (!X0) {
            HC(launch_seeded_block(st, n, nb, (unsigned long long)p.seed, T1, n, true));
            HC(launch_colmajor_to_rows_lp<T>(st, n, nb, T1, n, Xl, ld));
        } else if (p.ptr_mode == SE_PTR_HOST) {
            HC(hipMemcpyAsync(T1, X0, sizeof(double) * (size_t)n * nb, hipMemcpyHostToDevice, st));
            HC(launch_colmajor_to_rows_lp<T>(st, n, nb, T1, n, Xl, ld));
        } else {
            HC(launch_colmajor_to_rows_lp<T>(st, n, nb, X0, n, Xl, ld));
        }
        int k = nb, dx = 0;
        bool have_drop = false;
        double best = INFINITY;
        int j_best = 0;
        std::vector<double> stop, paper, lam;
        // Rayleigh-Ritz on span(X): AX, M, A_p, grr, X <- X C, AX <- AX C.
        auto rr = [&]() -> se_status {
            ST(lp_spmm(Xl, AXl, k));
            const SegsT<T> Xs = lseg1(Xl, k);
            ST(lp_gram(Xs, Xs, 1, ws.lpM.as<double>()));
            ST(lp_gram(Xs, lseg1(AXl, k), 1, ws.G.as<double>()));
            int kk = k, rP = 0;
            ST(grr(k, 0, kk, 0, drop2, rP));
            ST(lp_update(Xs, ws.lpC.as<double>(), kk, lseg1(Xnl, kk), 1.0, 0.0));
            ST(lp_update(lseg1(AXl, k), ws.lpC.as<double>(), kk, lseg1(AXnl, kk), 1.0, 0.0));
            std::swap(Xl, Xnl);
            std::swap(AXl, AXnl);
            k = kk;
            return SE_OK;
        };
        ST(rr());
        for (int j = 1; j <= p.max_iter; ++j) {
            ST(lp_check(Xl, AXl, k, stop, paper, lam));
            double r = 0.0, ms = 0.0;
            bool all = true;
            for (int i = 0; i < n_ev; ++i) {
                r = std::max(r, paper[i]);
                ms = std::max(ms, stop[i]);
                all = all && (stop[i] <= p.tol);
            }
            iters = j;
            lp_iters = j;
            last_r = r;
            last_stop = ms;
            ctl.observe(j, r);
            record(j, r, ms, k, 0, k, 0, 4);
            if (r < best) {
                best = r;
                j_best = j;
            }
            if (all) {
                lp_done = true;
                break;
            }
            const bool near_floor = best <= 100.0 * rsw;  // early iterations may rise and stall
            if (r <= rsw || (near_floor && (r > 10.0 * best || j - j_best >= kStall)) || out_of_time())
                break;
            int flags = 4;
            const bool want_expand = ctl.ifexpand(j);
            // Y <- sigma X - A X or the Chebyshev filter; a powered X_drop
            // takes the same step
            const bool filt = p.filter_degree > 0 && sigma > lam[k - 1];
            if (filt) {
                ST(cheb_filter_lp<T>(Xl, Xnl, AXl, T1l, k, lam[0], lam[k - 1], sigma));
            } else {
                ST(tic());
                HC(launch_shift_sub_lp<T>(st, n, Xl, AXl, ld, k, sigma));
                ST(toc(SE_K_RESID, 3.0 * sizeof(T) * n * k, 2.0 * n * k));
            }
            if (have_drop && p.expand_vectors == SE_EXPAND_POWERED) {
                if (filt) {
                    ST(cheb_filter_lp<T>(Sdl, T2l, nullptr, T1l, dx, lam[0], lam[k - 1], sigma));
                } else {
                    ST(lp_spmm(Sdl, T1l, dx));
                    const double gap = sigma - lam[0];
                    ST(tic());
                    HC(launch_shift_sub_lp<T>(st, n, Sdl, T1l, ld, dx, sigma, gap > 0.0 ? 1.0 / gap : 1.0));
                    ST(toc(SE_K_RESID, 3.0 * sizeof(T) * n * dx, 3.0 * n * dx));
                }
            }
            if (want_expand && have_drop) {
                HC(launch_copy_cols_lp<T>(st, n, Sdl, ld, 0, Xl, ld, k, dx));
                k += dx;
                have_drop = false;
                ctl.did_expand(j);
                ++n_exp;
                flags |= 1;
            }
            ST(rr());
            if (ctl.ifshrink(j) && k > n_es) {
                dx = k - n_es;
                HC(launch_copy_cols_lp<T>(st, n, Xl, ld, n_es, Sdl, ld, 0, dx));
                k = n_es;
                have_drop = true;
                ctl.did_shrink(j);
                ++n_shr;
                flags |= 2;
            }
            amend_flags(flags);
        }
        if (lp_done) return lp_to_f64(Xl, k, Sdl, 0, Xl, 0, k0, p0);
        return lp_to_f64(Xl, k, Sdl, have_drop ? std::min(dx, nb - k) : 0, Xl, 0, k0, p0);
    }

    // Mixed precision: the low-precision phase, then the FP64 solver from its
    // X (a fresh shrink-and-expand controller, history rows continuing).
    template <class T>
    se_status mixed(const double* X0) {
        const Strategy ctl0 = ctl;
        int k0 = 0, p0 = 0;
        ST(p.solver == SE_SI ? si_lp<T>(X0, k0) : lobpcg_lp<T>(X0, k0, p0));
        if (lp_done) {
            converged = true;
            return SE_OK;
        }
        if (k0 < n_ev) return SE_ERR_BREAKDOWN;
        ctl = ctl0;
        j_off = lp_iters;
        return p.solver == SE_SI ? si(nullptr, k0) : lobpcg(nullptr, k0, p0);
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

// Device workspace a solve of this shape allocates (the sizes of
// Solver::alloc_panels, alloc_small and lp_alloc), plus the FP32 copy of the
// matrix values for mixed precision.
// The copy is made under the matrix's lock and published only once the
// conversion on `st` has finished, so solves on other streams (serving slots)
// that find it can use it at once.
hipError_t make_val32(hipStream_t st, const se_matrix* A) {
    std::lock_guard<std::mutex> lk(A->val32_mu);
    if (A->val32) return hipSuccess;
    float* v = nullptr;
    hipError_t e = hipMalloc(&v, sizeof(float) * ((size_t)A->nnz + kCsrPad));
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(v + A->nnz, 0, sizeof(float) * kCsrPad, st);
    if (e == hipSuccess) e = launch_f64_to_f32(st, A->nnz, A->val, v);
    const hipError_t es = hipStreamSynchronize(st);
    if (e == hipSuccess) e = es;
    if (e != hipSuccess) {
        (void)hipFree(v);
        return e;
    }
    A->val32 = v;
    return hipSuccess;
}

size_t solve_workspace_bytes(long long n, long long nnz, int nb, int precision, int solver) {
    const long long ld = round_up(nb, 8);
    const int mmax = (solver == SE_SI || solver == SE_TRACEMIN) ? nb : 3 * nb;
    const size_t mm = (size_t)mmax * mmax;
    size_t bytes = sizeof(double) * (size_t)kNumPanels * n * ld;
    size_t small = 4 * mm + (mmax + 8) + (2 * mm + 8 * (size_t)mmax + 64) + syev_work_doubles(mmax) +
                   std::max(gram_scratch_doubles(n, mmax, mmax), (size_t)4096 * 2 * mmax) + 4 * mm +
                   3 * (2 * (size_t)mmax + 16) + 6 * mm + (size_t)mmax + 8 + 6 * mm +
                   (solver == SE_TRACEMIN ? 3 * (size_t)mmax + 8 : 0) +
                   (solver == SE_LOBPCG || solver == SE_SD ? (size_t)n : 0);  // Jacobi diagonal
    if (precision != SE_FP64) {
        const size_t es = precision == SE_FP32_MIXED ? 4 : 2;
        bytes += es * (size_t)kNumLpPanels * n * ld + sizeof(float) * ((size_t)nnz + kCsrPad) +
                 sizeof(float) * (size_t)9 * nb * nb;
    }
    return bytes + sizeof(double) * small;
}

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
    s.no_p = prm->solver == SE_SD;
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
    se_status st;
    if (prm->precision == SE_FP32_MIXED)
        st = s.mixed<float>(X0);
    else if (prm->precision == SE_BF16_MIXED)
        st = s.mixed<bf16_t>(X0);
    else
        st = (prm->solver == SE_SI) ? s.si(X0) : (prm->solver == SE_TRACEMIN) ? s.tracemin(X0) : s.lobpcg(X0);
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
        info->lp_iterations = s.lp_iters;
        info->n_reprojections = s.n_reproj;
        if (st < 0) {
            info->max_stop_ratio = s.last_stop;
            info->max_paper_ratio = s.last_r;
        }
    }
    if (st < 0) return st;
    return s.converged ? SE_OK : SE_NOT_CONVERGED;
}

}  // namespace se
