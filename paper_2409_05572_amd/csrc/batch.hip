// Batched serving engine, device side: one macro-step advances every resident
// solve by one LOBPCG iteration (Algorithm 3: soft locking, the improved
// Hetmaniuk-Lehoucq basis of Section 2.3, shrink-and-expand of Section 3).
//
// Each phase is one launch over the work items of all resident solves (the
// batched products of bulk.hip and small.hip). Sizes that the arithmetic
// decides (columns dropped by Cholesky-QR, the rank of the HL block) never go
// back to the host: small planning kernels read them on the device and write
// the job lists of the following phases. The sequence of launches is fixed, so
// it can be captured once in a graph and replayed while the widths change.
// The host takes its decisions (locking, expansion, shrink, convergence) once
// per step from the residual norms of the step before.
#include "batch.h"

namespace se {

size_t bsmall_doubles() { return BSmall::EIG + syev_work_doubles(kBMMax); }

namespace {

constexpr int kT = 256;
constexpr double kDrop = 1e-13;  // scaled Cholesky pivot below which a column is dropped
constexpr double kNs = 1e-8;     // orthonormal to this level: a Newton-Schulz step instead

struct BJobs {
    BGramJob gproj[kMaxBatch], gch[kMaxBatch], grr[kMaxBatch];
    BUpdJob uproj[kMaxBatch], uch[kMaxBatch], us[kMaxBatch], uas[kMaxBatch];
    CholJob cch[kMaxBatch], chl[kMaxBatch];
    SmallMMJob mzt[kMaxBatch], mzu[kMaxBatch], mg[kMaxBatch], mu[kMaxBatch];
    BSpmmJob sp[kMaxBatch];
    EigJob eig[kMaxBatch];
    BResidJob rs[kMaxBatch];
    alignas(16) unsigned char eigspace[sizeof(SmallMMJob) * 6 * kMaxBatch + sizeof(CholJob) * 3 * kMaxBatch];
};

__device__ __forceinline__ int* info_i(const BFix& F) { return reinterpret_cast<int*>(F.sm + BSmall::INFO); }
__device__ __forceinline__ double* info_d(const BFix& F) { return F.sm + BSmall::INFO + kBWMax / 2 + 8; }

__device__ __forceinline__ Segs dsegs(long long ld) {
    Segs s{};
    s.nseg = 0;
    s.ld = ld;
    s.off[0] = 0;
    return s;
}
__device__ __forceinline__ void dpush(Segs& s, const double* p, int w) {
    if (w <= 0) return;
    s.p[s.nseg] = p;
    s.w[s.nseg] = w;
    s.off[s.nseg + 1] = s.off[s.nseg] + w;
    s.nseg++;
}

enum Stage { ST_GATHERED, ST_REPROJ, ST_CHOL1, ST_CHOL2, ST_EIG, ST_HL1, ST_HL2, ST_HL3, ST_UPD };

// Job lists of the phases up to the next planning point, one thread per slot.
__global__ void bplan_kernel(int stage, int ns, const BFix* __restrict__ fix, const BCtl* __restrict__ ctl,
                             BDyn* __restrict__ dyn, BJobs* __restrict__ J) {
    const int s = threadIdx.x;
    if (s >= ns) return;
    const BFix& F = fix[s];
    const BCtl& C = ctl[s];
    BDyn& D = dyn[s];
    const bool on = C.mode != BMODE_IDLE;
    const long long n = on ? F.n : 0;
    const long long ld = F.ldw;
    double* sm = F.sm;
    double* X = F.xp[D.cur];
    double* P = X + F.poff;
    double* AX = F.axp[D.cur];
    double* AP = AX + F.poff;
    int* ii = info_i(F);

    // W <- W - [X, P] ([X, P]^T W) (go = false: an empty job)
    auto plan_proj = [&](bool want) {
        const double* W = F.w[D.wcur];
        Segs Q = dsegs(ld);
        dpush(Q, X, D.k);
        dpush(Q, P, D.p);
        Segs Ws = dsegs(ld);
        dpush(Ws, W, D.w);
        const int q = D.k + D.p;
        const bool go = want && on && q > 0 && D.w > 0;
        J->gproj[s] = BGramJob{Q, Ws, go ? n : 0, F.rows_g, q, D.w, 0, F.nch_g, F.part, sm + BSmall::G};
        J->uproj[s] = BUpdJob{Q, Ws, go ? n : 0, q, go ? D.w : 0, sm + BSmall::G, -1.0, 1.0};
    };
    // W^T W, and its Cholesky-QR transform with column drop
    auto plan_gram = [&](bool want) {
        const double* W = F.w[D.wcur];
        Segs Ws = dsegs(ld);
        dpush(Ws, W, D.w);
        const bool go = want && on && D.w > 0;
        J->gch[s] = BGramJob{Ws, Ws, go ? n : 0, F.rows_g, D.w, D.w, 1, F.nch_g, F.part, sm + BSmall::GW};
    };
    auto plan_chol = [&](double ns_tol) {
        const bool go = on && D.w > 0;
        J->cch[s] = CholJob{sm + BSmall::GW, sm + BSmall::T, sm + BSmall::CW, ii, info_d(F), kDrop, ns_tol,
                            go ? D.w : 0};
    };
    // W2 = W T over the kept columns; the kept columns' sources are composed
    // into map (kept positions are increasing, so the update is in place).
    auto plan_apply = [&]() {
        const int r = (on && D.w > 0) ? ii[0] : 0;
        Segs Ws = dsegs(ld);
        dpush(Ws, F.w[D.wcur], D.w);
        Segs Os = dsegs(ld);
        dpush(Os, F.w[D.wcur ^ 1], r);
        J->uch[s] = BUpdJob{Ws, Os, r > 0 ? n : 0, D.w, r, sm + BSmall::T, 1.0, 0.0};
        for (int i = 0; i < r; ++i) D.map[i] = D.map[ii[1 + i]];
        D.wcur ^= 1;
        D.w = r;
    };

    switch (stage) {
        case ST_GATHERED: {
            if (C.mode == BMODE_ITER) {
                D.wcur ^= 1;  // the gather wrote the other W buffer
                D.wa = C.a;
                D.w = C.a + (C.expand ? D.dx + D.dp : 0);
            } else if (C.mode == BMODE_INIT) {
                D.wa = D.w;  // the start block (k = p = 0)
            }
            for (int i = 0; i < D.w; ++i) D.map[i] = i;
            plan_proj(true);
            plan_gram(true);
            break;
        }
        case ST_REPROJ: {
            // One projection suffices unless a column kept less than half of
            // its squared norm (the criterion of Kahan and Parlett for
            // classical Gram-Schmidt); the norms before it are the residual
            // norms of the last check. Appended dropped columns always take
            // the second projection.
            bool again = C.mode == BMODE_ITER && C.expand && D.w > D.wa;
            if (C.mode == BMODE_ITER && D.k + D.p > 0) {
                const double* GW = sm + BSmall::GW;
                for (int i = 0; i < D.wa && !again; ++i)
                    again = GW[(size_t)i * D.w + i] < 0.5 * D.sums[C.act[i]];
            }
            plan_proj(again);
            plan_gram(again);
            plan_chol(0.0);
            break;
        }
        case ST_CHOL1: {
            // after a pass with a pivot below 1e-8 the kept columns carry
            // amplified rounding along [X, P]: project once more
            const bool low = on && D.w > 0 && (info_d(F)[0] < 1e-8 || ii[0] < D.w);
            plan_apply();
            plan_proj(low);
            plan_gram(true);
            plan_chol(kNs);
            break;
        }
        case ST_CHOL2: {
            plan_apply();
            // the kept block is [W (cw) | X_drop (cx) | P_drop (cp)], in this order
            const int dxe = (C.mode == BMODE_ITER && C.expand) ? D.dx : 0;
            int cw = 0, cx = 0;
            for (int i = 0; i < D.w; ++i) {
                cw += D.map[i] < D.wa;
                cx += D.map[i] >= D.wa && D.map[i] < D.wa + dxe;
            }
            D.cx = cx;
            D.m = on ? D.k + D.p + D.w : 0;
            D.kk = C.mode == BMODE_INIT ? D.w : D.k + cx;
            // HL positions in S = [X, P, W]: unlocked X columns, then the kept X_drop columns
            int h = 0;
            if (C.mode == BMODE_ITER) {
                for (int i = 0; i < C.a; ++i) D.hlpos[h++] = C.act[i];
                for (int i = 0; i < cx; ++i) D.hlpos[h++] = D.k + D.p + cw + i;
            }
            D.nhl = h;
            double* W = F.w[D.wcur];
            double* AW = F.aw;
            J->sp[s] = BSpmmJob{F.rowptr, F.col, F.val, W, AW, ld, ld, (int)n, D.w};
            Segs S = dsegs(ld), AS = dsegs(ld);
            dpush(S, X, D.k);
            dpush(S, P, D.p);
            dpush(S, W, D.w);
            dpush(AS, AX, D.k);
            dpush(AS, AP, D.p);
            dpush(AS, AW, D.w);
            J->grr[s] = BGramJob{S, AS, D.m > 0 ? n : 0, F.rows_g, D.m, D.m, 0, F.nch_g, F.part, sm + BSmall::G};
            J->eig[s] = EigJob{sm + BSmall::G, D.theta, sm + BSmall::Z, sm + BSmall::EIG, D.kk > 0 ? D.m : 0,
                               D.kk};
            break;
        }
        case ST_EIG: {
            // B = (I - Z1 Z1^T) E is formed by bhl_kernel; project it against
            // Z1 once more, then its Gram matrix and Cholesky-QR transform
            const int m = D.m, kk = D.kk, h = D.nhl;
            double* Z = sm + BSmall::Z;
            double* B = sm + BSmall::B;
            double* TB = sm + BSmall::TB;
            const int rows = (on && h > 0) ? m : 0;
            const int hh = rows > 0 ? h : 0;
            J->mzt[s] = SmallMMJob{Z, B, TB, 1.0, 0.0, rows, kk, hh, kk, h, h, 1};
            J->mzu[s] = SmallMMJob{Z, TB, B, -1.0, 1.0, rows, kk, hh, kk, h, h, 0};
            J->mg[s] = SmallMMJob{B, B, sm + BSmall::GB, 1.0, 0.0, rows, h, hh, h, h, h, 1};
            J->chl[s] = CholJob{sm + BSmall::GB, TB, sm + BSmall::CW, ii, info_d(F), kDrop, 0.0, hh};
            break;
        }
        case ST_HL1: {
            const int m = D.m, kk = D.kk, h = D.nhl;
            const int r1 = (on && h > 0) ? ii[0] : 0;
            double* Z = sm + BSmall::Z;
            double* B = sm + BSmall::B;
            double* B2 = sm + BSmall::B2;
            double* TB = sm + BSmall::TB;
            const int rows = r1 > 0 ? m : 0;
            J->mu[s] = SmallMMJob{B, TB, B2, 1.0, 0.0, rows, h, r1, h, r1, r1, 0};
            J->mzt[s] = SmallMMJob{Z, B2, TB, 1.0, 0.0, rows, kk, r1, kk, r1, r1, 1};
            J->mzu[s] = SmallMMJob{Z, TB, B2, -1.0, 1.0, rows, kk, r1, kk, r1, r1, 0};
            J->mg[s] = SmallMMJob{B2, B2, sm + BSmall::GB, 1.0, 0.0, rows, r1, r1, r1, r1, r1, 1};
            J->chl[s] = CholJob{sm + BSmall::GB, TB, sm + BSmall::CW, ii, info_d(F), kDrop, kNs, r1};
            D.nhl = r1;
            break;
        }
        case ST_HL2: {
            const int r1 = D.nhl;
            const int r2 = (on && r1 > 0) ? ii[0] : 0;
            // C_P = B2 T (m x r2) into B
            J->mu[s] = SmallMMJob{sm + BSmall::B2, sm + BSmall::TB, sm + BSmall::B, 1.0, 0.0, r2 > 0 ? D.m : 0, r1,
                                  r2, r1, r2, r2, 0};
            D.pp = on ? r2 : 0;
            break;
        }
        case ST_HL3: {
            // [X', P'] = S [Z1 | C_P], [AX', AP'] = AS [Z1 | C_P]; at a shrink
            // the columns past n_es go to the dropped blocks
            const int kk = D.kk, pp = D.pp, N = kk + pp;
            double* W = F.w[D.wcur];
            Segs S = dsegs(ld), AS = dsegs(ld);
            dpush(S, X, D.k);
            dpush(S, P, D.p);
            dpush(S, W, D.w);
            dpush(AS, AX, D.k);
            dpush(AS, AP, D.p);
            dpush(AS, F.aw, D.w);
            double* Xn = F.xp[D.cur ^ 1];
            double* AXn = F.axp[D.cur ^ 1];
            Segs O = dsegs(ld), AO = dsegs(ld);
            if (C.shrink) {
                const int kx = min(kk, F.n_es), kp = min(pp, F.n_es);
                dpush(O, Xn, kx);
                dpush(O, F.xpd, kk - kx);
                dpush(O, Xn + F.poff, kp);
                dpush(O, F.xpd + F.poff, pp - kp);
            } else {
                dpush(O, Xn, kk);
                dpush(O, Xn + F.poff, pp);
            }
            dpush(AO, AXn, kk);
            dpush(AO, AXn + F.poff, pp);
            const long long nn = (on && D.m > 0 && N > 0) ? n : 0;
            J->us[s] = BUpdJob{S, O, nn, D.m, N, sm + BSmall::C, 1.0, 0.0};
            J->uas[s] = BUpdJob{AS, AO, nn, D.m, N, sm + BSmall::C, 1.0, 0.0};
            break;
        }
        case ST_UPD: {
            if (on) {
                const int kk = D.kk, pp = D.pp;
                int k = kk, p = pp;
                if (C.expand) D.dx = D.dp = 0;  // the dropped blocks went back into the basis
                if (C.shrink) {
                    k = min(kk, F.n_es);
                    p = min(pp, F.n_es);
                    D.dx = kk - k;
                    D.dp = pp - p;
                }
                for (int i = 0; i < k; ++i) D.lam[i] = D.theta[i];
                D.cur ^= 1;
                D.k = k;
                D.p = p;
            }
            J->rs[s] = BResidJob{F.xp[D.cur], F.axp[D.cur], D.lam, F.w[D.wcur], F.rpart, D.sums, on ? n : 0, ld,
                                 ld, F.rows_r, on ? D.k : 0, F.nch_r};
            break;
        }
    }
}

// W block of an iteration: the unlocked residual columns, then (at an
// expansion) the dropped columns, gathered into the other W buffer.
// Work items: (slot, 64 rows).
__global__ __launch_bounds__(kT) void bgather_kernel(int ns, const BFix* __restrict__ fix,
                                                     const BCtl* __restrict__ ctl, const BDyn* __restrict__ dyn) {
    __shared__ int s_start[kMaxBatch + 1];
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int s = 0; s < ns; ++s) {
            s_start[s] = acc;
            acc += ctl[s].mode == BMODE_ITER ? (fix[s].n + 63) / 64 : 0;
        }
        s_start[ns] = acc;
    }
    __syncthreads();
    const int total = s_start[ns];
    for (int it = blockIdx.x; it < total; it += gridDim.x) {
        int s = 0;
        while (s + 1 < ns && it >= s_start[s + 1]) ++s;
        s = __builtin_amdgcn_readfirstlane(s);
        const BFix& F = fix[s];
        const BCtl& C = ctl[s];
        const BDyn& D = dyn[s];
        const long long ld = F.ldw;
        const double* src = F.w[D.wcur];
        double* dst = F.w[D.wcur ^ 1];
        const int a = C.a, dx = C.expand ? D.dx : 0, dp = C.expand ? D.dp : 0;
        const int wt = a + dx + dp;
        const long long r0 = (long long)(it - s_start[s]) * 64;
        const int nr = (int)min(64LL, (long long)F.n - r0);
        for (int e = threadIdx.x; e < nr * wt; e += kT) {
            const long long r = r0 + e / wt;
            const int c = e % wt;
            double v;
            if (c < a)
                v = src[r * ld + C.act[c]];
            else if (c < a + dx)
                v = F.xpd[r * ld + (c - a)];
            else
                v = F.xpd[r * ld + F.poff + (c - a - dx)];
            dst[r * ld + c] = v;
        }
    }
}

// Symmetric part of the Rayleigh-Ritz matrix, 0.5 (G + G^T), in place.
__global__ __launch_bounds__(kT) void bsym_kernel(const BFix* __restrict__ fix, const BDyn* __restrict__ dyn) {
    const BDyn& D = dyn[blockIdx.x];
    const int m = D.m;
    double* G = fix[blockIdx.x].sm + BSmall::G;
    for (int e = threadIdx.x; e < m * m; e += kT) {
        const int i = e / m, j = e % m;
        if (i < j) {
            const double v = 0.5 * (G[i * m + j] + G[j * m + i]);
            G[i * m + j] = v;
            G[j * m + i] = v;
        }
    }
}

// HL start block B = (I - Z1 Z1^T) E, E the unit columns at the HL positions.
__global__ __launch_bounds__(kT) void bhl_kernel(const BFix* __restrict__ fix, const BCtl* __restrict__ ctl,
                                                 const BDyn* __restrict__ dyn) {
    const BDyn& D = dyn[blockIdx.y];
    if (ctl[blockIdx.y].mode == BMODE_IDLE) return;
    const int m = D.m, kk = D.kk, h = D.nhl;
    const double* Z = fix[blockIdx.y].sm + BSmall::Z;
    double* B = fix[blockIdx.y].sm + BSmall::B;
    for (int e = blockIdx.x * kT + threadIdx.x; e < m * h; e += gridDim.x * kT) {
        const int r = e / h, c = e % h;
        const int q = D.hlpos[c];
        double s = 0.0;
        for (int i = 0; i < kk; ++i) s = fma(Z[r * kk + i], Z[q * kk + i], s);
        B[e] = (r == q ? 1.0 : 0.0) - s;
    }
}

// Coefficients [Z1 | C_P] (m x (kk + pp)).
__global__ __launch_bounds__(kT) void bassemble_kernel(const BFix* __restrict__ fix, const BCtl* __restrict__ ctl,
                                                       const BDyn* __restrict__ dyn) {
    const BDyn& D = dyn[blockIdx.x];
    if (ctl[blockIdx.x].mode == BMODE_IDLE) return;
    const int m = D.m, kk = D.kk, pp = D.pp, N = kk + pp;
    const double* sm = fix[blockIdx.x].sm;
    const double* Z = sm + BSmall::Z;
    const double* CP = sm + BSmall::B;
    double* C = const_cast<double*>(sm) + BSmall::C;
    for (int e = threadIdx.x; e < m * N; e += kT) {
        const int r = e / N, c = e % N;
        C[e] = c < kk ? Z[r * kk + c] : CP[r * pp + (c - kk)];
    }
}

// Per-column ratios of the stopping test and of eq. (rk) from the residual sums.
__global__ __launch_bounds__(kT) void bratio_kernel(const BFix* __restrict__ fix, const BCtl* __restrict__ ctl,
                                                    BDyn* __restrict__ dyn) {
    BDyn& D = dyn[blockIdx.x];
    if (ctl[blockIdx.x].mode == BMODE_IDLE) return;
    const double anorm = fix[blockIdx.x].anorm;
    const int k = D.k;
    for (int c = threadIdx.x; c < k; c += kT) {
        const double rn = sqrt(D.sums[c]), xn = sqrt(D.sums[k + c]);
        D.stop[c] = rn / (anorm * xn);
        D.paper[c] = rn / (anorm * xn + xn * fabs(D.lam[c]));
    }
}

}  // namespace

size_t batch_jobs_bytes() { return sizeof(BJobs); }

hipError_t launch_batch_step(Launcher& L, int ns, const BFix* fix, const BCtl* ctl, BDyn* dyn, void* jobs,
                             int upd_grid) {
    if (ns <= 0 || ns > kMaxBatch || upd_grid <= 0) return hipErrorInvalidValue;
    if (syev_batched_jobspace_bytes() != sizeof(BJobs::eigspace)) return hipErrorInvalidValue;
    BJobs* J = static_cast<BJobs*>(jobs);
    auto plan = [&](Stage s) { L(bplan_kernel, dim3(1), dim3(64), 0, (int)s, ns, fix, ctl, dyn, J); };
    constexpr int G = kBGridBulk;
    // W block, projected twice against [X, P], Cholesky-QR with drop
    L(bgather_kernel, dim3(G), dim3(kT), 0, ns, fix, ctl, dyn);
    plan(ST_GATHERED);
    launch_gram_batched(L, J->gproj, ns, G);
    launch_update_batched(L, J->uproj, ns, upd_grid);
    launch_gram_batched(L, J->gch, ns, G);
    plan(ST_REPROJ);  // a second projection only where needed
    launch_gram_batched(L, J->gproj, ns, G);
    launch_update_batched(L, J->uproj, ns, upd_grid);
    launch_gram_batched(L, J->gch, ns, G);
    launch_chol_batched(L, J->cch, ns);
    plan(ST_CHOL1);
    // second pass: apply, project again after a low pivot, Cholesky-QR (or Newton-Schulz)
    launch_update_batched(L, J->uch, ns, upd_grid);
    launch_gram_batched(L, J->gproj, ns, G);
    launch_update_batched(L, J->uproj, ns, upd_grid);
    launch_gram_batched(L, J->gch, ns, G);
    launch_chol_batched(L, J->cch, ns);
    plan(ST_CHOL2);
    launch_update_batched(L, J->uch, ns, upd_grid);
    // A W, Rayleigh-Ritz on S = [X, P, W]
    launch_spmm_batched(L, J->sp, ns, G);
    launch_gram_batched(L, J->grr, ns, G);
    L(bsym_kernel, dim3(ns), dim3(kT), 0, fix, dyn);
    launch_syev_lowest_batched(L, J->eig, ns, J->eigspace);
    // HL basis: two Cholesky-QR passes, each after a projection against Z1
    plan(ST_EIG);
    L(bhl_kernel, dim3(16, ns), dim3(kT), 0, fix, ctl, dyn);
    launch_small_mm_batched(L, J->mzt, ns);
    launch_small_mm_batched(L, J->mzu, ns);
    launch_small_mm_batched(L, J->mg, ns);
    launch_chol_batched(L, J->chl, ns);
    plan(ST_HL1);
    launch_small_mm_batched(L, J->mu, ns);
    launch_small_mm_batched(L, J->mzt, ns);
    launch_small_mm_batched(L, J->mzu, ns);
    launch_small_mm_batched(L, J->mg, ns);
    launch_chol_batched(L, J->chl, ns);
    plan(ST_HL2);
    launch_small_mm_batched(L, J->mu, ns);
    plan(ST_HL3);
    L(bassemble_kernel, dim3(ns), dim3(kT), 0, fix, ctl, dyn);
    launch_update_batched(L, J->us, ns, upd_grid);
    launch_update_batched(L, J->uas, ns, upd_grid);
    // next iteration's residual and its ratios
    plan(ST_UPD);
    launch_resid_batched(L, J->rs, ns, G);
    L(bratio_kernel, dim3(ns), dim3(kT), 0, fix, ctl, dyn);
    return L.err;
}

}  // namespace se
