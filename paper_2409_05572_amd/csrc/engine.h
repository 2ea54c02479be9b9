// Host-side engine: context, matrix, workspace and the solver drivers.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <vector>

#include "../../include/se.h"
#include "common.h"

namespace se {

// Grow-only device buffer.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t want) {
        if (want <= bytes) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        hipError_t e = hipMalloc(&p, want < 256 ? 256 : want);
        if (e == hipSuccess) bytes = want;
        return e;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T>
    T* as() const {
        return static_cast<T*>(p);
    }
};

// Grow-only pinned host buffer.
struct HostBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t want) {
        if (want <= bytes) return hipSuccess;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
        hipError_t e = hipHostMalloc(&p, want < 256 ? 256 : want, hipHostMallocDefault);
        if (e == hipSuccess) bytes = want;
        return e;
    }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T>
    T* as() const {
        return static_cast<T*>(p);
    }
};

constexpr int kNumPanels = 14;
constexpr int kNumLpPanels = 12;

struct Workspace {
    DevBuf panel[kNumPanels];       // n x ld FP64 blocks
    DevBuf lp_panel[kNumLpPanels];  // n x ld FP32 / BF16 blocks (mixed precision)
    DevBuf gram_part, G, T, Z, theta, C, small_work, syev_work, lam, act, act_hl, norms, info;
    DevBuf hlB, hlY, hlG, hlQ;
    DevBuf lpM, lpT, lpQ, lpB, lpE, lpC;  // generalized Rayleigh-Ritz (m x m each)
    DevBuf apc, axp, axq, gw, idx;        // carried [X, P]^T A [X, P] (m x m each; idx ints)
    DevBuf wfold, cfold;                  // last Cholesky-QR transform of W, folded coefficients
    DevBuf cg;                            // TraceMIN inner CG: per-column rr, rr_new, d^T q
    DevBuf pc;                            // Jacobi preconditioner diag(1 / |a_ii|) (n doubles)
    DevBuf c32;                           // coefficients of a low-precision update rounded to FP32
    HostBuf h_norms, h_info, h_act, h_act_hl, h_theta, h_diag;
    std::vector<hipEvent_t> events;  // pool for per-launch timing
    size_t device_bytes() const {
        size_t s = 0;
        for (const auto& b : panel) s += b.bytes;
        for (const auto& b : lp_panel) s += b.bytes;
        const DevBuf* all[] = {&gram_part, &G, &T, &Z, &theta, &C, &small_work, &syev_work,
                               &lam, &act, &act_hl, &norms, &info, &hlB, &hlY, &hlG, &hlQ,
                               &lpM, &lpT, &lpQ, &lpB, &lpE, &lpC, &apc, &axp, &axq, &gw, &idx,
                               &wfold, &cfold, &cg, &pc, &c32};
        for (auto* b : all) s += b->bytes;
        return s;
    }
    void release() {
        for (auto& b : panel) b.release();
        for (auto& b : lp_panel) b.release();
        DevBuf* all[] = {&gram_part, &G, &T, &Z, &theta, &C, &small_work, &syev_work,
                         &lam, &act, &act_hl, &norms, &info, &hlB, &hlY, &hlG, &hlQ,
                         &lpM, &lpT, &lpQ, &lpB, &lpE, &lpC, &apc, &axp, &axq, &gw, &idx,
                         &wfold, &cfold, &cg, &pc, &c32};
        for (auto* b : all) b->release();
        h_norms.release();
        h_info.release();
        h_act.release();
        h_act_hl.release();
        h_theta.release();
        h_diag.release();
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        events.clear();
    }
};

// Shrink-and-expand controller (Section 3.2): fix / slope / slopek with the
// warm-up rule. Readings: Algorithm 7's shrink test uses j_s (iterations
// since the last expansion); its expansion test c_max / c > mu is taken as
// mu * c < c_max so that it also fires when the residual grows; c_max is the
// largest slope since the last shrink, current iteration included.
struct Strategy {
    int kind = SE_STRAT_NONE;
    int j_e = 12, j_s = 2, j_p = 10, j_warm = 5;
    double mu = 1.1, r_warm = 1e-4;
    bool shrunk = false, warm_done = false;
    int j_last_expand = -1000000000;
    double c_max = -INFINITY;
    std::vector<double> logr;     // logr[j] = log10 r(j)
    std::vector<char> have;       // have[j] = r(j) recorded

    bool enabled() const {
        return kind == SE_STRAT_FIX || kind == SE_STRAT_SLOPE || kind == SE_STRAT_SLOPEK;
    }
    void observe(int j, double r);
    bool slope(int j, double* c) const;
    bool ifexpand(int j);
    bool ifshrink(int j) const;
    void did_expand(int j) {
        shrunk = false;
        j_last_expand = j;
    }
    void did_shrink(int) {
        shrunk = true;
        warm_done = true;
        c_max = -INFINITY;
    }
};

}  // namespace se

struct se_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    se::Workspace ws;
    int last_hip_error = 0;
};

struct se_matrix {
    se_ctx* ctx = nullptr;  // identity only: never dereferenced after creation
    int device = 0;         // the creating context's device (destroy does not need the context)
    int64_t n = 0, nnz = 0;
    int* rowptr = nullptr;  // int32 offsets on the device
    int* col = nullptr;
    double* val = nullptr;
    mutable float* val32 = nullptr;  // FP32 copy for the mixed-precision phase, made on first use
    mutable std::mutex val32_mu;     // guards the first-use creation of val32
    int is_complex = 0;  // Hermitian with complex values: val holds 2 (nnz + kCsrPad) interleaved doubles
    int* heavy = nullptr;  // rows with more than kHeavyRow nonzeros (one workgroup each in SpMM)
    int n_heavy = 0;
    double anorm = 0.0;
};

namespace se {
se_status solve(se_ctx* ctx, const se_matrix* A, const se_params* p, const double* X0, double* V,
                double* lambda, se_info* info);
size_t solve_workspace_bytes(long long n, long long nnz, int nb, int precision, int solver);
// FP32 copy of the matrix values (A->val32, with kCsrPad zero entries after
// the last), made once per matrix, ordered on `st`.
hipError_t make_val32(hipStream_t st, const se_matrix* A);
se_status validate_solve(const se_matrix* A, const se_params* p);
// Complex Hermitian A (A->is_complex): LOBPCG or SI, FP64; X0, V complex
// column-major interleaved.
se_status solve_z(se_ctx* ctx, const se_matrix* A, const se_params* p, const double* X0, double* V,
                  double* lambda, se_info* info);
}
