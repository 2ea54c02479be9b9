// Complex Hermitian solver drivers: LOBPCG (Algorithm 3) and subspace
// iteration (Algorithm 1) with shrink-and-expand (Algorithm 5), FP64.
//
// The paper states the problem for Hermitian A in C^{n x n} (Section 1); every
// transpose of the algorithms is a conjugate transpose. Complex n-length
// blocks are panels of n x ldc complex entries (interleaved), which the
// matrix-core Gram and update kernels of the real path process through their
// real view (see complex.hip): S^H (A S) is a combined real Gram product and
// S C a real update by the embedding of C. The iteration is the plain form of
// Algorithm 3: W = R(:, active) is projected against [X, P] twice and
// orthonormalized by Cholesky-QR twice (columns dropped below a scaled pivot
// of 1e-13), A_p = S^H (A S) is formed over n at every iteration, and the
// images AX, AP follow the basis updates as in Algorithm 3 (AW by the CSR
// product). Locking, the HL basis and the shrink-and-expand decisions are as
// in the real drivers.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <utility>
#include <vector>

#include "engine.h"

namespace se {

namespace {

inline long long zround_up(long long a, long long b) { return (a + b - 1) / b * b; }

se_status zhip_status(hipError_t e) {
    if (e == hipSuccess) return SE_OK;
    if (e == hipErrorOutOfMemory) return SE_ERR_OOM;
    return SE_ERR_HIP;
}

constexpr double kZDrop = 1e-13;  // scaled Cholesky pivot below which a column is dropped

struct SolverZ {
    se_ctx* ctx;
    const se_matrix* A;
    se_params p;
    hipStream_t st;
    Workspace& ws;
    long long n;
    int ldc = 0, nb = 0, n_ev = 0, n_es = 0;
    bool se_on = false;
    hipError_t herr = hipSuccess;

    // complex panels (n x ldc complex entries)
    double *X = nullptr, *P = nullptr, *W = nullptr, *AX = nullptr, *AP = nullptr, *AW = nullptr;
    double *Xn = nullptr, *Pn = nullptr, *AXn = nullptr, *APn = nullptr;
    double *Xd = nullptr, *Pd = nullptr, *T1 = nullptr, *T2 = nullptr;

    int iters = 0, n_shr = 0, n_exp = 0, hist_len = 0;
    bool converged = false;
    double last_r = INFINITY, last_stop = INFINITY;
    Strategy ctl;
    std::chrono::steady_clock::time_point t0;
    std::vector<double> theta;  // current Ritz values (host)

    struct ProfRec {
        int cls;
        hipEvent_t a, b;
        double bytes, flops;
    };
    std::vector<ProfRec> prof;
    size_t ev_next = 0;
    hipEvent_t open_ev = nullptr;

    SolverZ(se_ctx* c, const se_matrix* a, const se_params& prm)
        : ctx(c), A(a), p(prm), st(c->stream), ws(c->ws), n(a->n) {}

#define HC(expr)                                   \
    do {                                           \
        hipError_t _e = (expr);                    \
        if (_e != hipSuccess) {                    \
            herr = _e;                             \
            return zhip_status(_e);                \
        }                                          \
    } while (0)
#define ST(expr)                   \
    do {                           \
        se_status _s = (expr);     \
        if (_s < 0) return _s;     \
    } while (0)

    // Real view of complex panels: columns [2 c, 2 c + 2) hold column c.
    Segs zs(const double* a, int wa) const {
        Segs s = make_segs(2LL * ldc);
        push_seg(s, a, 2 * wa);
        return s;
    }
    Segs zs3(const double* a, int wa, const double* b, int wb, const double* c, int wc) const {
        Segs s = make_segs(2LL * ldc);
        push_seg(s, a, 2 * wa);
        push_seg(s, b, 2 * wb);
        push_seg(s, c, 2 * wc);
        return s;
    }
    static Segs zrows(const double* a, int wa, long long ldz) {  // m-row complex blocks
        Segs s = make_segs(2LL * ldz);
        push_seg(s, a, 2 * wa);
        return s;
    }

    se_status alloc(int mmax) {
        const size_t bytes = sizeof(double) * 2 * (size_t)n * ldc;
        for (int i = 0; i < 14; ++i) HC(ws.panel[i].ensure(bytes));
        double** slots[] = {&X, &P, &W, &AX, &AP, &AW, &Xn, &Pn, &AXn, &APn, &Xd, &Pd, &T1, &T2};
        for (int i = 0; i < 14; ++i) *slots[i] = ws.panel[i].as<double>();
        const size_t mm = (size_t)mmax * mmax;
        HC(ws.G.ensure(sizeof(double) * 2 * mm));       // complex Gram results
        HC(ws.T.ensure(sizeof(double) * 2 * mm));       // complex Cholesky-QR transform
        HC(ws.Z.ensure(sizeof(double) * 2 * mm));       // complex Ritz vectors
        HC(ws.C.ensure(sizeof(double) * 2 * mm));       // complex update coefficients
        HC(ws.lpM.ensure(sizeof(double) * 4 * mm));     // real Gram of the views (2m x 2m)
        HC(ws.lpT.ensure(sizeof(double) * 4 * mm));     // real embedding of coefficients
        HC(ws.hlB.ensure(sizeof(double) * 2 * mm));
        HC(ws.hlY.ensure(sizeof(double) * 2 * mm));
        HC(ws.hlG.ensure(sizeof(double) * 2 * mm));
        HC(ws.theta.ensure(sizeof(double) * (mmax + 8)));
        HC(ws.lpE.ensure(sizeof(double) * (2 * mmax + 8)));  // Ritz values duplicated per real column
        HC(ws.small_work.ensure(sizeof(double) * (2 * mm + 8 * (size_t)mmax + 64)));
        HC(ws.syev_work.ensure(sizeof(double) * heev_z_work_doubles(mmax)));
        HC(ws.gram_part.ensure(sizeof(double) * std::max(gram_scratch_doubles(n, 2 * mmax, 2 * mmax),
                                                         (size_t)4096 * 4 * mmax)));
        HC(ws.act.ensure(sizeof(int) * (2 * mmax + 8)));
        HC(ws.act_hl.ensure(sizeof(int) * (mmax + 8)));
        HC(ws.idx.ensure(sizeof(int) * (2 * mmax + 8)));
        HC(ws.norms.ensure(sizeof(double) * (4 * mmax + 8)));
        HC(ws.info.ensure(sizeof(double) * (mmax + 16)));
        HC(ws.h_norms.ensure(sizeof(double) * (4 * mmax + 8)));
        HC(ws.h_theta.ensure(sizeof(double) * (mmax + 8)));
        HC(ws.h_info.ensure(sizeof(double) * (mmax + 16)));
        HC(ws.h_act.ensure(sizeof(int) * (2 * mmax + 8)));
        HC(ws.h_act_hl.ensure(sizeof(int) * (mmax + 8)));
        // idx = 0, 0, 1, 1, ...: duplicates each Ritz value for the two real
        // columns of its complex column
        std::vector<int> dup(2 * mmax);
        for (int i = 0; i < 2 * mmax; ++i) dup[i] = i / 2;
        std::memcpy(ws.h_act.p, dup.data(), sizeof(int) * dup.size());
        HC(hipMemcpyAsync(ws.idx.p, ws.h_act.p, sizeof(int) * dup.size(), hipMemcpyHostToDevice, st));
        return sync();
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

    // ------------------------------------------------------------ products --
    se_status spmm(const double* Xs, double* Ys, int w) {
        ST(tic());
        HC(launch_spmm_z(st, (int)n, A->rowptr, A->col, A->val, Xs, ldc, Ys, ldc, w));
        return toc(SE_K_SPMM, 20.0 * A->nnz + 4.0 * (n + 1) + 32.0 * n * w, 8.0 * A->nnz * w);
    }
    // C (mu x mv complex) = U^H V over `rows` rows of the real views U, V.
    se_status zgram(long long rows, const Segs& U, const Segs& V, double* C) {
        const int mu2 = segs_width(U), mv2 = segs_width(V);
        const size_t need = sizeof(double) * gram_scratch_doubles(rows, mu2, mv2);
        if (need > ws.gram_part.bytes) {
            ST(sync());
            HC(ws.gram_part.ensure(need));
        }
        const bool same = U.nseg == 1 && V.nseg == 1 && U.p[0] == V.p[0] && U.ld == V.ld && mu2 == mv2;
        if (rows == n) ST(tic());
        HC(launch_gram(st, rows, U, V, same ? 1 : 0, ws.gram_part.as<double>(), ws.lpM.as<double>()));
        HC(launch_zgram_combine(st, mu2 / 2, mv2 / 2, ws.lpM.as<double>(), C));
        if (rows == n) {
            const double mu = mu2, mv = mv2;
            return toc(SE_K_GRAM, 8.0 * n * (same ? mu : mu + mv), same ? n * mu * (mu + 1.0) : 2.0 * n * mu * mv);
        }
        return SE_OK;
    }
    // O = beta O + alpha U C over `rows` rows (C: K x N complex, views U of
    // width 2K and O of width 2N).
    se_status zupdate(long long rows, const Segs& U, const double* C, int N, const Segs& O, double alpha,
                      double beta) {
        const int K = segs_width(U) / 2;
        HC(launch_zembed(st, K, N, C, ws.lpT.as<double>()));
        if (rows == n) ST(tic());
        HC(launch_update(st, rows, U, ws.lpT.as<double>(), 2 * N, O, alpha, beta));
        if (rows == n)
            return toc(SE_K_UPDATE, 16.0 * n * (K + N * (beta != 0.0 ? 2.0 : 1.0)), 8.0 * n * K * N);
        return SE_OK;
    }

    // Cholesky-QR of the w columns of panel Wp (with drop in the first pass,
    // none in the second), through tmp; returns the kept count and, through
    // kept (if given), the input columns kept by the first pass.
    se_status cholqr(double* Wp, int& w, double* tmp, std::vector<int>* kept) {
        for (int pass = 0; pass < 2 && w > 0; ++pass) {
            ST(zgram(n, zs(Wp, w), zs(Wp, w), ws.G.as<double>()));
            int* info_i = ws.info.as<int>();
            double* info_d = ws.info.as<double>() + (w + 8) / 2 + 4;
            ST(tic());
            HC(launch_cholz(st, w, ws.G.as<double>(), ws.T.as<double>(), ws.small_work.as<double>(), info_i, info_d,
                            pass == 0 ? kZDrop : -1.0));
            ST(toc(SE_K_SMALL, 0.0, 0.0));
            HC(hipMemcpyAsync(ws.h_info.p, ws.info.p, sizeof(double) * (w + 16), hipMemcpyDeviceToHost, st));
            ST(sync());
            const int* hi = ws.h_info.as<int>();
            const int r = hi[0];
            if (pass == 0 && kept) kept->assign(hi + 1, hi + 1 + r);
            if (r <= 0) {
                w = 0;
                break;
            }
            ST(zupdate(n, zs(Wp, w), ws.T.as<double>(), r, zs(tmp, r), 1.0, 0.0));
            ST(tic());
            HC(launch_copy_cols(st, n, tmp, 2LL * ldc, 0, Wp, 2LL * ldc, 0, 2 * r));
            ST(toc(SE_K_COPY, 32.0 * n * r, 0.0));
            w = r;
        }
        return SE_OK;
    }

    // Rayleigh-Ritz on the m columns of S (segments) with images AS: A_p =
    // S^H (A S), the k lowest pairs into theta (host and ws.theta) and ws.Z
    // (m x k complex).
    se_status ritz(const Segs& S, const Segs& AS, int m, int k) {
        double* Ap = ws.hlG.as<double>();
        ST(zgram(n, S, AS, Ap));
        ST(tic());
        HC(launch_zherm(st, m, Ap));
        HC(launch_heev_lowest_z(st, m, k, Ap, ws.theta.as<double>(), ws.Z.as<double>(), ws.syev_work.as<double>()));
        ST(toc(SE_K_EIG, 0.0, 0.0));
        HC(hipMemcpyAsync(ws.h_theta.p, ws.theta.p, sizeof(double) * k, hipMemcpyDeviceToHost, st));
        ST(sync());
        theta.assign(ws.h_theta.as<double>(), ws.h_theta.as<double>() + k);
        return SE_OK;
    }

    // R = AX - X Theta over k columns into Rp (may be null) and the stopping
    // measures of every column (host).
    se_status residual(int k, double* Rp, std::vector<double>& stop, std::vector<double>& paper) {
        ST(tic());
        HC(launch_gather_cols(st, 1, ws.theta.as<double>(), k, ws.idx.as<int>(), 2 * k, ws.lpE.as<double>(), 2 * k));
        HC(launch_resid_norms(st, n, X, AX, 2LL * ldc, 2 * k, ws.lpE.as<double>(), ws.gram_part.as<double>(),
                              ws.norms.as<double>(), Rp, 2LL * ldc));
        ST(toc(SE_K_RESID, (Rp ? 48.0 : 32.0) * n * k, 10.0 * n * k));
        HC(hipMemcpyAsync(ws.h_norms.p, ws.norms.p, sizeof(double) * 4 * k, hipMemcpyDeviceToHost, st));
        ST(sync());
        const double* nr = ws.h_norms.as<double>();
        stop.resize(k);
        paper.resize(k);
        for (int i = 0; i < k; ++i) {
            const double rn = std::sqrt(std::max(nr[2 * i] + nr[2 * i + 1], 0.0));
            const double xn = std::sqrt(std::max(nr[2 * k + 2 * i] + nr[2 * k + 2 * i + 1], 0.0));
            stop[i] = rn / (A->anorm * xn);
            paper[i] = rn / (A->anorm * xn + xn * std::fabs(theta[i]));
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
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > p.time_limit_s;
    }

    se_status load_x0(const double* X0) {
        if (!X0) {
            HC(launch_seeded_block(st, n, nb, (unsigned long long)p.seed, T1, n, true));
            HC(launch_rcol_to_zrows(st, n, nb, T1, X, ldc));
        } else if (p.ptr_mode == SE_PTR_HOST) {
            HC(hipMemcpyAsync(T1, X0, sizeof(double) * 2 * (size_t)n * nb, hipMemcpyHostToDevice, st));
            HC(launch_zcol_to_rows(st, n, nb, T1, X, ldc));
        } else {
            HC(launch_zcol_to_rows(st, n, nb, X0, X, ldc));
        }
        return SE_OK;
    }

    // Start: X <- orth(X0), A X, Rayleigh-Ritz (Algorithm 3 / Algorithm 1
    // initial step); returns the width.
    se_status start(const double* X0, int& k) {
        ST(load_x0(X0));
        k = nb;
        ST(cholqr(X, k, T1, nullptr));
        if (k < n_ev) return SE_ERR_BREAKDOWN;
        ST(spmm(X, AX, k));
        ST(ritz(zs(X, k), zs(AX, k), k, k));
        ST(zupdate(n, zs(X, k), ws.Z.as<double>(), k, zs(Xn, k), 1.0, 0.0));
        ST(zupdate(n, zs(AX, k), ws.Z.as<double>(), k, zs(AXn, k), 1.0, 0.0));
        std::swap(X, Xn);
        std::swap(AX, AXn);
        return SE_OK;
    }

    // Orthogonalize the w columns of panel B against the segments S twice
    // (B <- B - S (S^H B)).
    se_status project(const Segs& S, double* B, int w) {
        if (segs_width(S) == 0 || w == 0) return SE_OK;
        const int m = segs_width(S) / 2;
        for (int pass = 0; pass < 2; ++pass) {
            ST(zgram(n, S, zs(B, w), ws.G.as<double>()));
            ST(zupdate(n, S, ws.G.as<double>(), w, zs(B, w), -1.0, 1.0));
        }
        (void)m;
        return SE_OK;
    }

    // HL coefficients [Z1 | C_P] into ws.C (m x (k + r) complex), C_P an
    // orthonormal basis of (I - Z1 Z1^H) E for the unit vectors E at the
    // positions of the unlocked old X columns.
    se_status hl(int m, int k, const std::vector<int>& act, int& r) {
        const int a = (int)act.size();
        double* Z1 = ws.Z.as<double>();
        double* B = ws.hlB.as<double>();
        double* Y = ws.hlY.as<double>();
        double* B2 = ws.hlG.as<double>();
        r = 0;
        if (a > 0) {
            std::memcpy(ws.h_act_hl.p, act.data(), sizeof(int) * a);
            HC(hipMemcpyAsync(ws.act_hl.p, ws.h_act_hl.p, sizeof(int) * a, hipMemcpyHostToDevice, st));
            ST(tic());
            HC(launch_hl_init_z(st, m, k, Z1, ws.act_hl.as<int>(), a, B, Y));
            // B <- E - Z1 (Z1^H E), then once more B <- B - Z1 (Z1^H B)
            ST(zupdate(m, zrows(Z1, k, k), Y, a, zrows(B, a, a), -1.0, 1.0));
            ST(zgram(m, zrows(Z1, k, k), zrows(B, a, a), Y));
            ST(zupdate(m, zrows(Z1, k, k), Y, a, zrows(B, a, a), -1.0, 1.0));
            int w = a;
            for (int pass = 0; pass < 2 && w > 0; ++pass) {
                ST(zgram(m, zrows(B, w, w), zrows(B, w, w), ws.G.as<double>()));
                int* info_i = ws.info.as<int>();
                double* info_d = ws.info.as<double>() + (w + 8) / 2 + 4;
                HC(launch_cholz(st, w, ws.G.as<double>(), ws.T.as<double>(), ws.small_work.as<double>(), info_i,
                                info_d, kZDrop));
                HC(hipMemcpyAsync(ws.h_info.p, ws.info.p, sizeof(int) * 2, hipMemcpyDeviceToHost, st));
                ST(sync());
                const int rr = ws.h_info.as<int>()[0];
                if (rr <= 0) {
                    w = 0;
                    break;
                }
                ST(zupdate(m, zrows(B, w, w), ws.T.as<double>(), rr, zrows(B2, rr, rr), 1.0, 0.0));
                if (pass == 0) {  // reproject once: C_P stays orthogonal to Z1 to working precision
                    ST(zgram(m, zrows(Z1, k, k), zrows(B2, rr, rr), Y));
                    ST(zupdate(m, zrows(Z1, k, k), Y, rr, zrows(B2, rr, rr), -1.0, 1.0));
                }
                HC(launch_copy_cols(st, m, B2, 2LL * rr, 0, B, 2LL * rr, 0, 2 * rr));
                w = rr;
            }
            r = w;
            ST(toc(SE_K_SMALL, 0.0, 0.0));
        }
        // ws.C = [Z1 | B] (m x (k + r))
        double* Cc = ws.C.as<double>();
        HC(launch_copy_cols(st, m, Z1, 2LL * k, 0, Cc, 2LL * (k + r), 0, 2 * k));
        if (r > 0) HC(launch_copy_cols(st, m, B, 2LL * r, 0, Cc, 2LL * (k + r), 2 * k, 2 * r));
        return SE_OK;
    }

    // ------------------------------------------------------------- LOBPCG --
    se_status lobpcg(const double* X0) {
        ST(alloc(3 * nb));
        int k = 0;
        ST(start(X0, k));
        int pw = 0;
        int dx = 0, dp = 0;
        bool have_drop = false;
        std::vector<double> stop, paper;
        for (int j = 1; j <= p.max_iter; ++j) {
            ST(residual(k, T1, stop, paper));
            double r = 0.0, ms = 0.0;
            bool all = true;
            for (int i = 0; i < n_ev; ++i) {
                r = std::max(r, paper[i]);
                ms = std::max(ms, stop[i]);
                all = all && stop[i] <= p.tol;
            }
            iters = j;
            last_r = r;
            last_stop = ms;
            ctl.observe(j, r);
            std::vector<int> act;
            int locked = 0;
            for (int i = 0; i < k; ++i) {
                const bool lock = p.soft_lock && i < n_ev && stop[i] <= p.tol;
                if (lock)
                    ++locked;
                else
                    act.push_back(i);
            }
            record(j, r, ms, k, pw, (int)act.size(), locked, 0);
            if (all) {
                converged = true;
                break;
            }
            if (out_of_time()) break;
            int flags = 0;
            const bool want_expand = ctl.ifexpand(j);

            // W <- R(:, active), projected against [X, P] twice, orthonormalized
            int a = (int)act.size();
            {
                std::vector<int> idx2(2 * a);
                for (int q = 0; q < a; ++q) {
                    idx2[2 * q] = 2 * act[q];
                    idx2[2 * q + 1] = 2 * act[q] + 1;
                }
                std::memcpy(ws.h_act.p, idx2.data(), sizeof(int) * 2 * a);
                HC(hipMemcpyAsync(ws.act.p, ws.h_act.p, sizeof(int) * 2 * a, hipMemcpyHostToDevice, st));
                ST(tic());
                HC(launch_gather_cols(st, n, T1, 2LL * ldc, ws.act.as<int>(), 2 * a, W, 2LL * ldc));
                ST(toc(SE_K_COPY, 32.0 * n * a, 0.0));
                ST(sync());  // h_act is reused below
            }
            {
                Segs XP = make_segs(2LL * ldc);
                push_seg(XP, X, 2 * k);
                push_seg(XP, P, 2 * pw);
                ST(project(XP, W, a));
            }
            ST(cholqr(W, a, T2, nullptr));

            // expansion: [X_drop, P_drop] against S = [X, P, W], orthonormalized;
            // columns from X_drop join X, the rest P
            std::vector<int> act_hl = act;
            if (want_expand && have_drop && k + dx <= nb) {
                ST(tic());
                HC(launch_copy_cols(st, n, Xd, 2LL * ldc, 0, T2, 2LL * ldc, 0, 2 * dx));
                if (dp > 0) HC(launch_copy_cols(st, n, Pd, 2LL * ldc, 0, T2, 2LL * ldc, 2 * dx, 2 * dp));
                ST(toc(SE_K_COPY, 32.0 * n * (dx + dp), 0.0));
                int ws_w = dx + dp;
                ST(project(zs3(X, k, P, pw, W, a), T2, ws_w));
                std::vector<int> kept;
                ST(cholqr(T2, ws_w, T1, &kept));
                int kx = 0;
                for (int c : kept) kx += c < dx ? 1 : 0;
                kx = std::min(kx, ws_w);
                const int kp = ws_w - kx;
                // images of the new columns
                ST(spmm(T2, T1, ws_w));
                ST(tic());
                HC(launch_copy_cols(st, n, T2, 2LL * ldc, 0, X, 2LL * ldc, 2 * k, 2 * kx));
                HC(launch_copy_cols(st, n, T1, 2LL * ldc, 0, AX, 2LL * ldc, 2 * k, 2 * kx));
                if (kp > 0) {
                    HC(launch_copy_cols(st, n, T2, 2LL * ldc, 2 * kx, P, 2LL * ldc, 2 * pw, 2 * kp));
                    HC(launch_copy_cols(st, n, T1, 2LL * ldc, 2 * kx, AP, 2LL * ldc, 2 * pw, 2 * kp));
                }
                ST(toc(SE_K_COPY, 64.0 * n * ws_w, 0.0));
                for (int q = 0; q < kx; ++q) act_hl.push_back(k + q);
                k += kx;
                pw += kp;
                have_drop = false;
                ctl.did_expand(j);
                ++n_exp;
                flags |= 1;
            }

            // A_p = S^H (A S) with S = [X, P, W]; the k lowest pairs
            const int m = k + pw + a;
            ST(spmm(W, AW, a));
            ST(ritz(zs3(X, k, P, pw, W, a), zs3(AX, k, AP, pw, AW, a), m, k));
            int r_p = 0;
            ST(hl(m, k, act_hl, r_p));
            // [X, P] <- S [Z1 | C_P], [AX, AP] <- AS [Z1 | C_P]
            {
                Segs O = make_segs(2LL * ldc);
                push_seg(O, Xn, 2 * k);
                push_seg(O, Pn, 2 * r_p);
                ST(zupdate(n, zs3(X, k, P, pw, W, a), ws.C.as<double>(), k + r_p, O, 1.0, 0.0));
                Segs OA = make_segs(2LL * ldc);
                push_seg(OA, AXn, 2 * k);
                push_seg(OA, APn, 2 * r_p);
                ST(zupdate(n, zs3(AX, k, AP, pw, AW, a), ws.C.as<double>(), k + r_p, OA, 1.0, 0.0));
            }
            std::swap(X, Xn);
            std::swap(P, Pn);
            std::swap(AX, AXn);
            std::swap(AP, APn);
            pw = r_p;

            if (se_on && ctl.ifshrink(j) && k > n_es) {
                dx = k - n_es;
                dp = std::max(0, pw - n_es);
                ST(tic());
                HC(launch_copy_cols(st, n, X, 2LL * ldc, 2 * n_es, Xd, 2LL * ldc, 0, 2 * dx));
                if (dp > 0) HC(launch_copy_cols(st, n, P, 2LL * ldc, 2 * n_es, Pd, 2LL * ldc, 0, 2 * dp));
                ST(toc(SE_K_COPY, 32.0 * n * (dx + dp), 0.0));
                k = n_es;
                pw = std::min(pw, n_es);
                theta.resize(k);
                have_drop = true;
                ctl.did_shrink(j);
                ++n_shr;
                flags |= 2;
            }
            amend_flags(flags);
        }
        return SE_OK;
    }

    // ----------------------------------------------- subspace iteration --
    se_status si(const double* X0) {
        ST(alloc(nb));
        int k = 0;
        ST(start(X0, k));
        const double sigma = p.sigma > 0.0 ? p.sigma : A->anorm;
        int dx = 0;
        bool have_drop = false;
        std::vector<double> stop, paper;
        for (int j = 1; j <= p.max_iter; ++j) {
            ST(residual(k, nullptr, stop, paper));
            double r = 0.0, ms = 0.0;
            bool all = true;
            for (int i = 0; i < n_ev; ++i) {
                r = std::max(r, paper[i]);
                ms = std::max(ms, stop[i]);
                all = all && stop[i] <= p.tol;
            }
            iters = j;
            last_r = r;
            last_stop = ms;
            ctl.observe(j, r);
            record(j, r, ms, k, 0, 0, 0, 0);
            if (all) {
                converged = true;
                break;
            }
            if (out_of_time()) break;
            int flags = 0;
            // Y = sigma X - A X (the shifted power step), then X_drop appended
            ST(tic());
            HC(launch_shift_sub(st, n, X, AX, 2LL * ldc, 2 * k, sigma, 1.0));
            ST(toc(SE_K_RESID, 48.0 * n * k, 4.0 * n * k));
            int w = k;
            if (ctl.ifexpand(j) && have_drop && k + dx <= nb) {
                ST(tic());
                HC(launch_copy_cols(st, n, Xd, 2LL * ldc, 0, X, 2LL * ldc, 2 * k, 2 * dx));
                ST(toc(SE_K_COPY, 32.0 * n * dx, 0.0));
                w = k + dx;
                have_drop = false;
                ctl.did_expand(j);
                ++n_exp;
                flags |= 1;
            }
            ST(cholqr(X, w, T1, nullptr));
            if (w < n_ev) return SE_ERR_BREAKDOWN;
            ST(spmm(X, AX, w));
            ST(ritz(zs(X, w), zs(AX, w), w, w));
            ST(zupdate(n, zs(X, w), ws.Z.as<double>(), w, zs(Xn, w), 1.0, 0.0));
            ST(zupdate(n, zs(AX, w), ws.Z.as<double>(), w, zs(AXn, w), 1.0, 0.0));
            std::swap(X, Xn);
            std::swap(AX, AXn);
            k = w;
            if (se_on && ctl.ifshrink(j) && k > n_es) {
                dx = k - n_es;
                ST(tic());
                HC(launch_copy_cols(st, n, X, 2LL * ldc, 2 * n_es, Xd, 2LL * ldc, 0, 2 * dx));
                ST(toc(SE_K_COPY, 32.0 * n * dx, 0.0));
                k = n_es;
                theta.resize(k);
                have_drop = true;
                ctl.did_shrink(j);
                ++n_shr;
                flags |= 2;
            }
            amend_flags(flags);
        }
        return SE_OK;
    }

    // V = X(:, 1:n_ev) (complex column-major), lambda = theta(1:n_ev); the
    // stopping test is taken again from a fresh product.
    se_status finish(double* V, double* lambda, se_info* info) {
        ST(spmm(X, AX, n_ev));
        std::vector<double> stop, paper;
        ST(residual(n_ev, nullptr, stop, paper));
        double ms = 0.0, mp = 0.0;
        for (int i = 0; i < n_ev; ++i) {
            ms = std::max(ms, stop[i]);
            mp = std::max(mp, paper[i]);
        }
        if (p.ptr_mode == SE_PTR_HOST) {
            HC(launch_zrows_to_col(st, n, n_ev, X, ldc, T1));
            HC(hipMemcpyAsync(V, T1, sizeof(double) * 2 * (size_t)n * n_ev, hipMemcpyDeviceToHost, st));
            ST(sync());
            std::memcpy(lambda, theta.data(), sizeof(double) * n_ev);
        } else {
            HC(launch_zrows_to_col(st, n, n_ev, X, ldc, V));
            HC(hipMemcpyAsync(lambda, ws.theta.p, sizeof(double) * n_ev, hipMemcpyDeviceToDevice, st));
            ST(sync());
        }
        if (info) {
            info->max_stop_ratio = ms;
            info->max_paper_ratio = mp;
        }
        if (converged && !(ms <= p.tol * 1.01)) converged = false;
        return SE_OK;
    }
#undef HC
#undef ST
};

}  // namespace

se_status solve_z(se_ctx* ctx, const se_matrix* A, const se_params* prm, const double* X0, double* V,
                  double* lambda, se_info* info) {
    SolverZ s(ctx, A, *prm);
    s.t0 = std::chrono::steady_clock::now();
    s.nb = prm->n_ev + prm->n_extra;
    s.n_ev = prm->n_ev;
    s.ldc = (int)zround_up(s.nb, 4);
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
