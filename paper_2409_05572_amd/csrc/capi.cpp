// extern "C" boundary of the library (declared in include/se.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "engine.h"

namespace {

se_status hip_fail(se_ctx* ctx, hipError_t e) {
    if (ctx) ctx->last_hip_error = (int)e;
    return e == hipErrorOutOfMemory ? SE_ERR_OOM : SE_ERR_HIP;
}

#define CAPI_HC(ctx, expr)                      \
    do {                                        \
        hipError_t _e = (expr);                 \
        if (_e != hipSuccess) return hip_fail(ctx, _e); \
    } while (0)

bool valid_ld(int64_t ld, int32_t w) { return ld >= w && ld % 2 == 0; }
bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

namespace {
bool valid_ld_lp(int64_t ld, int32_t w) { return ld % 8 == 0 && ld >= (int64_t)((w + 7) / 8 * 8); }
bool lp_precision(int32_t pr) { return pr == SE_FP32_MIXED || pr == SE_BF16_MIXED; }
hipError_t ensure_val32(se_ctx* ctx, const se_matrix* A) { return se::make_val32(ctx->stream, A); }
template <class T>
hipError_t gram_lp_call(se_ctx* ctx, int64_t n, const void* U, int64_t ldu, int32_t mu, const void* V,
                        int64_t ldv, int32_t mv, double* C) {
    se::SegsT<T> Us = se::make_segs_t<T>(ldu), Vs = se::make_segs_t<T>(ldv);
    se::push_seg_t(Us, static_cast<const T*>(U), mu);
    se::push_seg_t(Vs, static_cast<const T*>(V), mv);
    const int sym = (U == V && ldu == ldv && mu == mv) ? 1 : 0;  // U^T U: upper tiles only, mirrored
    return se::launch_gram_lp<T>(ctx->stream, n, Us, Vs, sym, ctx->ws.gram_part.as<double>(), C);
}
template <class T>
hipError_t update_lp_call(se_ctx* ctx, int64_t n, const void* U, int64_t ldu, int32_t K, const double* C,
                          int32_t N, void* Out, int64_t ldo, double beta) {
    se::SegsT<T> Us = se::make_segs_t<T>(ldu), Os = se::make_segs_t<T>(ldo);
    se::push_seg_t(Us, static_cast<const T*>(U), K);
    se::push_seg_t(Os, static_cast<const T*>(Out), N);
    const hipError_t e = ctx->ws.c32.ensure(sizeof(float) * (size_t)K * N);
    if (e != hipSuccess) return e;
    return se::launch_update_lp<T>(ctx->stream, n, Us, C, N, Os, 1.0, beta, ctx->ws.c32.as<float>());
}
}  // namespace

namespace se {
// Parameter checks shared by se_solve and se_submit.
se_status validate_solve(const se_matrix* A, const se_params* p) {
    if (p->solver != SE_LOBPCG && p->solver != SE_SI && p->solver != SE_SD && p->solver != SE_TRACEMIN)
        return SE_ERR_INVALID_ARG;
    if (p->solver == SE_TRACEMIN && p->precision != SE_FP64) return SE_ERR_UNSUPPORTED;
    if (p->cg_steps < 0 || p->cg_steps > 100) return SE_ERR_INVALID_ARG;
    if (p->strategy < SE_STRAT_NONE || p->strategy > SE_STRAT_SLOPEK) return SE_ERR_INVALID_ARG;
    if (p->precision != SE_FP64 && p->precision != SE_FP32_MIXED && p->precision != SE_BF16_MIXED)
        return SE_ERR_UNSUPPORTED;
    if (p->precision != SE_FP64 && !(p->r_switch >= 0.0)) return SE_ERR_INVALID_ARG;
    if (!(p->implicit_pivot >= 0.0)) return SE_ERR_INVALID_ARG;
    if (p->ptr_mode != SE_PTR_HOST && p->ptr_mode != SE_PTR_DEVICE) return SE_ERR_INVALID_ARG;
    const int64_t nb = (int64_t)p->n_ev + p->n_extra;
    if (p->n_ev < 1 || p->n_extra < 0 || nb > A->n) return SE_ERR_INVALID_ARG;
    const bool single_block = p->solver == SE_SI || p->solver == SE_TRACEMIN;  // m = nb
    if (!single_block && nb > 341) return SE_ERR_UNSUPPORTED;  // 3 nb <= 1024
    if (single_block && nb > 1024) return SE_ERR_UNSUPPORTED;
    if (p->solver == SE_TRACEMIN && nb > 512) return SE_ERR_UNSUPPORTED;  // column CG kernels
    if (p->n_es != 0 && (p->n_es < p->n_ev || p->n_es > nb)) return SE_ERR_INVALID_ARG;
    if (!(p->tol > 0.0) || p->max_iter < 1) return SE_ERR_INVALID_ARG;
    if (p->strategy != SE_STRAT_NONE &&
        (p->j_e < 1 || p->j_s < 0 || p->j_p < 1 || p->j_warm < 0 || !(p->mu > 0.0)))
        return SE_ERR_INVALID_ARG;
    if (p->history && p->history_cap < 0) return SE_ERR_INVALID_ARG;
    if (p->solver == SE_SI && p->sigma < 0.0) return SE_ERR_INVALID_ARG;
    if (p->expand_vectors < SE_EXPAND_XDROP || p->expand_vectors > SE_EXPAND_POWERED) return SE_ERR_INVALID_ARG;
    if (p->expand_vectors == SE_EXPAND_POWERED && p->solver != SE_SI) return SE_ERR_INVALID_ARG;
    if (p->expand_vectors == SE_EXPAND_RANDOM && p->precision != SE_FP64) return SE_ERR_UNSUPPORTED;
    if (p->filter_degree < 0 || p->filter_degree > 64) return SE_ERR_INVALID_ARG;
    if (p->filter_degree > 0 && p->solver != SE_SI) return SE_ERR_INVALID_ARG;
    if (p->precond != SE_PRECOND_NONE && p->precond != SE_PRECOND_JACOBI) return SE_ERR_INVALID_ARG;
    if (p->precond != SE_PRECOND_NONE && p->solver != SE_LOBPCG && p->solver != SE_SD) return SE_ERR_INVALID_ARG;
    if (p->precond != SE_PRECOND_NONE && p->precision != SE_FP64) return SE_ERR_UNSUPPORTED;
    if (p->reserved != 0) return SE_ERR_INVALID_ARG;
    return SE_OK;
}
}  // namespace se

extern "C" {

void se_params_default(se_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->solver = SE_LOBPCG;
    p->strategy = SE_STRAT_NONE;
    p->precision = SE_FP64;
    p->ptr_mode = SE_PTR_HOST;
    p->n_ev = 1;
    p->n_extra = 0;
    p->n_es = 0;
    p->soft_lock = 1;
    p->j_e = 12;
    p->j_s = 2;
    p->j_p = 10;
    p->j_warm = 5;
    p->max_iter = 1000;
    p->profile = 0;
    p->mu = 1.1;
    p->r_warm = 1e-4;
    p->tol = 1e-8;
    p->sigma = 0.0;
    p->time_limit_s = 0.0;
    p->seed = 0;
    p->history = nullptr;
    p->history_cap = 0;
    p->expand_vectors = SE_EXPAND_XDROP;
}

se_status se_ctx_create(int device, void* stream, se_ctx** out) {
    if (!out) return SE_ERR_INVALID_ARG;
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(nullptr, e);
    if (device < 0 || device >= count) return SE_ERR_INVALID_ARG;
    e = hipSetDevice(device);
    if (e != hipSuccess) return hip_fail(nullptr, e);
    se_ctx* c = new (std::nothrow) se_ctx();
    if (!c) return SE_ERR_OOM;
    c->device = device;
    c->stream = static_cast<hipStream_t>(stream);
    *out = c;
    return SE_OK;
}

int32_t se_ctx_last_hip_error(const se_ctx* ctx) { return ctx ? ctx->last_hip_error : 0; }

const char* se_hip_error_name(int32_t e) { return hipGetErrorName((hipError_t)e); }

void se_ctx_destroy(se_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    ctx->ws.release();
    (void)hipGetLastError();  // nothing reported here may linger for a later launch check
    delete ctx;
}

se_status se_matrix_create_csr(se_ctx* ctx, int64_t n, int64_t nnz, const int64_t* rowptr,
                               const int32_t* colind, const double* val, uint32_t flags,
                               double anorm, se_matrix** out) {
    if (!ctx || !out || !rowptr || (!colind && nnz > 0) || (!val && nnz > 0)) return SE_ERR_INVALID_ARG;
    *out = nullptr;
    if (n < 1 || nnz < 0 || n > INT32_MAX - 1 || nnz > INT32_MAX) return SE_ERR_INVALID_ARG;
    if (!(anorm >= 0.0) || !std::isfinite(anorm)) return SE_ERR_INVALID_ARG;
    CAPI_HC(ctx, hipSetDevice(ctx->device));
    const bool on_device = (flags & SE_MATRIX_DEVICE) != 0;
    std::vector<int64_t> rp64(n + 1);
    if (on_device) {
        CAPI_HC(ctx, hipMemcpy(rp64.data(), rowptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost));
    } else {
        std::memcpy(rp64.data(), rowptr, sizeof(int64_t) * (n + 1));
    }
    if (rp64[0] != 0 || rp64[n] != nnz) return SE_ERR_INVALID_ARG;
    for (int64_t i = 0; i < n; ++i)
        if (rp64[i + 1] < rp64[i]) return SE_ERR_INVALID_ARG;
    // Validate indices and values on the host in both modes: the kernels index
    // X by colind without bounds checks.
    {
        std::vector<int32_t> ci;
        std::vector<double> vv;
        const int32_t* cp = colind;
        const double* vp = val;
        if (on_device && nnz > 0) {
            ci.resize(nnz);
            vv.resize(nnz);
            CAPI_HC(ctx, hipMemcpy(ci.data(), colind, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
            CAPI_HC(ctx, hipMemcpy(vv.data(), val, sizeof(double) * nnz, hipMemcpyDeviceToHost));
            cp = ci.data();
            vp = vv.data();
        }
        for (int64_t e = 0; e < nnz; ++e) {
            if (cp[e] < 0 || cp[e] >= n) return SE_ERR_INVALID_ARG;
            if (!std::isfinite(vp[e])) return SE_ERR_INVALID_ARG;
        }
        if (anorm == 0.0) {  // Gershgorin: max absolute row sum bounds ||A||_2 for symmetric A
            for (int64_t i = 0; i < n; ++i) {
                double s = 0.0;
                for (int64_t e = rp64[i]; e < rp64[i + 1]; ++e) s += std::fabs(vp[e]);
                anorm = std::max(anorm, s);
            }
            if (!(anorm > 0.0)) return SE_ERR_INVALID_ARG;  // the zero matrix has no scale
        }
    }
    std::vector<int> rp32(n + 1);
    for (int64_t i = 0; i <= n; ++i) rp32[i] = (int)rp64[i];
    std::vector<int> heavy;
    for (int64_t i = 0; i < n; ++i)
        if (rp64[i + 1] - rp64[i] > se::kHeavyRow) heavy.push_back((int)i);
    se_matrix* m = new (std::nothrow) se_matrix();
    if (!m) return SE_ERR_OOM;
    m->ctx = ctx;
    m->device = ctx->device;
    m->n = n;
    m->nnz = nnz;
    m->anorm = anorm;
    hipError_t e = hipMalloc(&m->rowptr, sizeof(int) * (n + 1));
    if (e == hipSuccess) e = hipMalloc(&m->col, sizeof(int) * (nnz + se::kCsrPad));
    if (e == hipSuccess) e = hipMalloc(&m->val, sizeof(double) * (nnz + se::kCsrPad));
    if (e == hipSuccess) e = hipMemset(m->col + nnz, 0, sizeof(int) * se::kCsrPad);
    if (e == hipSuccess) e = hipMemset(m->val + nnz, 0, sizeof(double) * se::kCsrPad);
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (e == hipSuccess) e = hipMemcpy(m->rowptr, rp32.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess && nnz > 0) e = hipMemcpy(m->col, colind, sizeof(int) * nnz, kind);
    if (e == hipSuccess && nnz > 0) e = hipMemcpy(m->val, val, sizeof(double) * nnz, kind);
    if (e == hipSuccess && !heavy.empty()) {
        e = hipMalloc(&m->heavy, sizeof(int) * heavy.size());
        if (e == hipSuccess)
            e = hipMemcpy(m->heavy, heavy.data(), sizeof(int) * heavy.size(), hipMemcpyHostToDevice);
        m->n_heavy = (int)heavy.size();
    }
    if (e != hipSuccess) {
        se_matrix_destroy(m);
        return hip_fail(ctx, e);
    }
    *out = m;
    return SE_OK;
}

void se_matrix_destroy(se_matrix* m) {
    if (!m) return;
    // The context may already be gone: only the stored device id is used.
    // Errors of these calls are not reported and must not linger as the
    // thread's last HIP error for a later launch check to pick up.
    (void)hipSetDevice(m->device);
    if (m->rowptr) (void)hipFree(m->rowptr);
    if (m->val32) (void)hipFree(m->val32);
    if (m->heavy) (void)hipFree(m->heavy);
    if (m->col) (void)hipFree(m->col);
    if (m->val) (void)hipFree(m->val);
    (void)hipGetLastError();
    delete m;
}

int64_t se_matrix_n(const se_matrix* m) { return m ? m->n : 0; }

double se_matrix_anorm(const se_matrix* m) { return m ? m->anorm : 0.0; }

se_status se_solve(se_ctx* ctx, const se_matrix* A, const se_params* p, const double* X0,
                   double* V, double* lambda, se_info* info) {
    if (!ctx || !A || !p || !V || !lambda) return SE_ERR_INVALID_ARG;
    if (A->ctx != ctx || A->is_complex) return SE_ERR_INVALID_ARG;
    const se_status v = se::validate_solve(A, p);
    if (v != SE_OK) return v;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(ctx, e);
    // Launch checks read the thread's last HIP error: drop one left by an
    // unrelated earlier call so that it cannot fail this solve.
    (void)hipGetLastError();
    if (info) std::memset(info, 0, sizeof(*info));
    return se::solve(ctx, A, p, X0, V, lambda, info);
}

se_status se_op_spmm(se_ctx* ctx, const se_matrix* A, const double* X, int64_t ldx, double* Y,
                     int64_t ldy, int32_t w) {
    if (!ctx || !A || !X || !Y || w < 1 || w > 256 || !valid_ld(ldx, w) || !valid_ld(ldy, w) || A->is_complex)
        return SE_ERR_INVALID_ARG;
    if (!aligned16(X) || !aligned16(Y)) return SE_ERR_INVALID_ARG;
    CAPI_HC(ctx, hipSetDevice(ctx->device));
    CAPI_HC(ctx, se::launch_spmm(ctx->stream, (int)A->n, A->rowptr, A->col, A->val, X, ldx, Y, ldy, w, A->heavy,
                                 A->n_heavy));
    return SE_OK;
}

se_status se_op_gram(se_ctx* ctx, int64_t n, const double* U, int64_t ldu, int32_t mu,
                     const double* V, int64_t ldv, int32_t mv, double* C) {
    if (!ctx || !U || !V || !C || n < 1 || mu < 1 || mv < 1 || mu > 1024 || mv > 1024)
        return SE_ERR_INVALID_ARG;
    if (!valid_ld(ldu, mu) || !valid_ld(ldv, mv)) return SE_ERR_INVALID_ARG;
    CAPI_HC(ctx, hipSetDevice(ctx->device));
    const size_t need = sizeof(double) * se::gram_scratch_doubles(n, mu, mv);
    if (need > ctx->ws.gram_part.bytes) {
        CAPI_HC(ctx, hipStreamSynchronize(ctx->stream));
        CAPI_HC(ctx, ctx->ws.gram_part.ensure(need));
    }
    se::Segs Us = se::make_segs(ldu), Vs = se::make_segs(ldv);
    se::push_seg(Us, U, mu);
    se::push_seg(Vs, V, mv);
    const int sym = (U == V && ldu == ldv && mu == mv) ? 1 : 0;
    CAPI_HC(ctx, se::launch_gram(ctx->stream, n, Us, Vs, sym, ctx->ws.gram_part.as<double>(), C));
    return SE_OK;
}

se_status se_op_update(se_ctx* ctx, int64_t n, const double* U, int64_t ldu, int32_t K,
                       const double* C, int32_t N, double* Out, int64_t ldo, double beta) {
    if (!ctx || !U || !C || !Out || n < 1 || K < 1 || N < 1 || K > 1024 || N > 1024)
        return SE_ERR_INVALID_ARG;
    if (!valid_ld(ldu, K) || !valid_ld(ldo, N) || !(beta == 0.0 || beta == 1.0))
        return SE_ERR_INVALID_ARG;
    const char* u0 = reinterpret_cast<const char*>(U);
    const char* u1 = u0 + sizeof(double) * (size_t)((n - 1) * ldu + K);
    const char* o0 = reinterpret_cast<const char*>(Out);
    const char* o1 = o0 + sizeof(double) * (size_t)((n - 1) * ldo + N);
    if (o0 < u1 && u0 < o1) return SE_ERR_INVALID_ARG;  // Out must not overlap U
    CAPI_HC(ctx, hipSetDevice(ctx->device));
    se::Segs Us = se::make_segs(ldu), Os = se::make_segs(ldo);
    se::push_seg(Us, U, K);
    se::push_seg(Os, Out, N);
    CAPI_HC(ctx, se::launch_update(ctx->stream, n, Us, C, N, Os, 1.0, beta));
    return SE_OK;
}


se_status se_op_spmm_lp(se_ctx* ctx, int32_t precision, const se_matrix* A, const void* X, int64_t ldx,
                        void* Y, int64_t ldy, int32_t w) {
    if (!ctx || !A || !X || !Y || w < 1 || w > 1024 || !lp_precision(precision) || A->is_complex)
        return SE_ERR_INVALID_ARG;
    if (!valid_ld_lp(ldx, w) || !valid_ld_lp(ldy, w) || !aligned16(X) || !aligned16(Y))
        return SE_ERR_INVALID_ARG;
    CAPI_HC(ctx, hipSetDevice(ctx->device));
    CAPI_HC(ctx, ensure_val32(ctx, A));
    if (precision == SE_FP32_MIXED)
        CAPI_HC(ctx, se::launch_spmm_lp<float>(ctx->stream, (int)A->n, A->rowptr, A->col, A->val32,
                                               static_cast<const float*>(X), ldx, static_cast<float*>(Y),
                                               ldy, w, A->heavy, A->n_heavy));
    else
        CAPI_HC(ctx, se::launch_spmm_lp<se::bf16_t>(ctx->stream, (int)A->n, A->rowptr, A->col, A->val32,
                                                     static_cast<const se::bf16_t*>(X), ldx,
                                                     static_cast<se::bf16_t*>(Y), ldy, w, A->heavy,
                                                     A->n_heavy));
    return SE_OK;
}

se_status se_op_gram_lp(se_ctx* ctx, int32_t precision, int64_t n, const void* U, int64_t ldu,
                        int32_t mu, const void* V, int64_t ldv, int32_t mv, double* C) {
    if (!ctx || !U || !V || !C || n < 1 || mu < 1 || mv < 1 || mu > 1024 || mv > 1024 ||
        !lp_precision(precision))
        return SE_ERR_INVALID_ARG;
    if (!valid_ld_lp(ldu, mu) || !valid_ld_lp(ldv, mv)) return SE_ERR_INVALID_ARG;
    CAPI_HC(ctx, hipSetDevice(ctx->device));
    const size_t need = sizeof(double) * se::gram_scratch_doubles(n, mu, mv);
    if (need > ctx->ws.gram_part.bytes) {
        CAPI_HC(ctx, hipStreamSynchronize(ctx->stream));
        CAPI_HC(ctx, ctx->ws.gram_part.ensure(need));
    }
    if (precision == SE_FP32_MIXED)
        CAPI_HC(ctx, gram_lp_call<float>(ctx, n, U, ldu, mu, V, ldv, mv, C));
    else
        CAPI_HC(ctx, gram_lp_call<se::bf16_t>(ctx, n, U, ldu, mu, V, ldv, mv, C));
    return SE_OK;
}

se_status se_op_update_lp(se_ctx* ctx, int32_t precision, int64_t n, const void* U, int64_t ldu,
                          int32_t K, const double* C, int32_t N, void* Out, int64_t ldo, double beta) {
    if (!ctx || !U || !C || !Out || n < 1 || K < 1 || N < 1 || K > 1024 || N > 1024 ||
        !lp_precision(precision))
        return SE_ERR_INVALID_ARG;
    if (!valid_ld_lp(ldu, K) || !valid_ld_lp(ldo, N) || !(beta == 0.0 || beta == 1.0))
        return SE_ERR_INVALID_ARG;
    const size_t es = precision == SE_FP32_MIXED ? 4 : 2;
    const char* u0 = reinterpret_cast<const char*>(U);
    const char* u1 = u0 + es * (size_t)((n - 1) * ldu + K);
    const char* o0 = reinterpret_cast<const char*>(Out);
    const char* o1 = o0 + es * (size_t)((n - 1) * ldo + N);
    if (o0 < u1 && u0 < o1) return SE_ERR_INVALID_ARG;  // Out must not overlap U
    CAPI_HC(ctx, hipSetDevice(ctx->device));
    if (precision == SE_FP32_MIXED)
        CAPI_HC(ctx, update_lp_call<float>(ctx, n, U, ldu, K, C, N, Out, ldo, beta));
    else
        CAPI_HC(ctx, update_lp_call<se::bf16_t>(ctx, n, U, ldu, K, C, N, Out, ldo, beta));
    return SE_OK;
}

se_status se_op_syev(se_ctx* ctx, int32_t m, double* A, double* w, double* Z) {
    if (!ctx || !A || !w || !Z || m < 1 || m > 1024) return SE_ERR_INVALID_ARG;
    CAPI_HC(ctx, hipSetDevice(ctx->device));
    CAPI_HC(ctx, hipStreamSynchronize(ctx->stream));
    CAPI_HC(ctx, ctx->ws.syev_work.ensure(sizeof(double) * se::syev_work_doubles(m)));
    CAPI_HC(ctx, se::launch_syev(ctx->stream, m, A, w, Z, ctx->ws.syev_work.as<double>()));
    CAPI_HC(ctx, hipStreamSynchronize(ctx->stream));
    return SE_OK;
}

se_status se_op_syev_lowest(se_ctx* ctx, int32_t m, int32_t k, double* A, double* w, double* Z) {
    if (!ctx || !A || !w || !Z || m < 1 || m > 1024 || k < 1 || k > m) return SE_ERR_INVALID_ARG;
    CAPI_HC(ctx, hipSetDevice(ctx->device));
    CAPI_HC(ctx, hipStreamSynchronize(ctx->stream));
    CAPI_HC(ctx, ctx->ws.syev_work.ensure(sizeof(double) * se::syev_work_doubles(m)));
    CAPI_HC(ctx, se::launch_syev_lowest(ctx->stream, m, k, A, w, Z, ctx->ws.syev_work.as<double>()));
    CAPI_HC(ctx, hipStreamSynchronize(ctx->stream));
    return SE_OK;
}

se_status se_op_cholqr(se_ctx* ctx, int64_t n, double* W, int64_t ldw, int32_t w, int32_t* rank) {
    if (!ctx || !W || !rank || n < 1 || w < 1 || w > 1024 || !valid_ld(ldw, w)) return SE_ERR_INVALID_ARG;
    CAPI_HC(ctx, hipSetDevice(ctx->device));
    se::Workspace& ws = ctx->ws;
    CAPI_HC(ctx, hipStreamSynchronize(ctx->stream));
    const size_t ww = (size_t)w * w;
    CAPI_HC(ctx, ws.panel[13].ensure(sizeof(double) * (size_t)n * ldw));
    CAPI_HC(ctx, ws.G.ensure(sizeof(double) * ww));
    CAPI_HC(ctx, ws.T.ensure(sizeof(double) * ww));
    CAPI_HC(ctx, ws.small_work.ensure(sizeof(double) * (2 * ww + 8 * (size_t)w + 64)));
    CAPI_HC(ctx, ws.info.ensure(sizeof(double) * (w + 16)));
    CAPI_HC(ctx, ws.h_info.ensure(sizeof(double) * (w + 16)));
    CAPI_HC(ctx, ws.gram_part.ensure(sizeof(double) * se::gram_scratch_doubles(n, w, w)));
    double* tmp = ws.panel[13].as<double>();
    int cur = w;
    for (int pass = 0; pass < 2 && cur > 0; ++pass) {
        se::Segs Ws = se::make_segs(ldw);
        se::push_seg(Ws, W, cur);
        CAPI_HC(ctx, se::launch_gram(ctx->stream, n, Ws, Ws, 1, ws.gram_part.as<double>(), ws.G.as<double>()));
        int* info_i = ws.info.as<int>();
        double* info_d = ws.info.as<double>() + (cur + 8) / 2 + 4;
        CAPI_HC(ctx, se::launch_chol_drop(ctx->stream, cur, ws.G.as<double>(), ws.T.as<double>(),
                                          ws.small_work.as<double>(), info_i, info_d, 1e-13));
        CAPI_HC(ctx, hipMemcpyAsync(ws.h_info.p, ws.info.p, sizeof(double) * (cur + 16),
                                    hipMemcpyDeviceToHost, ctx->stream));
        CAPI_HC(ctx, hipStreamSynchronize(ctx->stream));
        const int r = ws.h_info.as<int>()[0];
        if (r <= 0) {
            cur = 0;
            break;
        }
        se::Segs Os = se::make_segs(ldw);
        se::push_seg(Os, tmp, r);
        CAPI_HC(ctx, se::launch_update(ctx->stream, n, Ws, ws.T.as<double>(), r, Os, 1.0, 0.0));
        CAPI_HC(ctx, se::launch_copy_cols(ctx->stream, n, tmp, ldw, 0, W, ldw, 0, r));
        cur = r;
    }
    CAPI_HC(ctx, hipStreamSynchronize(ctx->stream));
    *rank = cur;
    return cur > 0 ? SE_OK : SE_ERR_BREAKDOWN;
}

se_status se_matrix_create_csr_z(se_ctx* ctx, int64_t n, int64_t nnz, const int64_t* rowptr,
                                 const int32_t* colind, const double* val, uint32_t flags,
                                 double anorm, se_matrix** out) {
    if (!ctx || !out || !rowptr || (!colind && nnz > 0) || (!val && nnz > 0)) return SE_ERR_INVALID_ARG;
    *out = nullptr;
    if (n < 1 || nnz < 0 || n > INT32_MAX - 1 || nnz > INT32_MAX / 2) return SE_ERR_INVALID_ARG;
    if (!(anorm >= 0.0) || !std::isfinite(anorm)) return SE_ERR_INVALID_ARG;
    CAPI_HC(ctx, hipSetDevice(ctx->device));
    const bool on_device = (flags & SE_MATRIX_DEVICE) != 0;
    std::vector<int64_t> rp64(n + 1);
    if (on_device)
        CAPI_HC(ctx, hipMemcpy(rp64.data(), rowptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost));
    else
        std::memcpy(rp64.data(), rowptr, sizeof(int64_t) * (n + 1));
    if (rp64[0] != 0 || rp64[n] != nnz) return SE_ERR_INVALID_ARG;
    for (int64_t i = 0; i < n; ++i)
        if (rp64[i + 1] < rp64[i]) return SE_ERR_INVALID_ARG;
    std::vector<int32_t> ci;
    std::vector<double> vv;
    const int32_t* cp = colind;
    const double* vp = val;
    if (on_device && nnz > 0) {
        ci.resize(nnz);
        vv.resize(2 * nnz);
        CAPI_HC(ctx, hipMemcpy(ci.data(), colind, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
        CAPI_HC(ctx, hipMemcpy(vv.data(), val, sizeof(double) * 2 * nnz, hipMemcpyDeviceToHost));
        cp = ci.data();
        vp = vv.data();
    }
    for (int64_t e = 0; e < nnz; ++e) {
        if (cp[e] < 0 || cp[e] >= n) return SE_ERR_INVALID_ARG;
        if (!std::isfinite(vp[2 * e]) || !std::isfinite(vp[2 * e + 1])) return SE_ERR_INVALID_ARG;
    }
    if (anorm == 0.0) {  // Gershgorin: max_i sum_j |a_ij| bounds ||A||_2
        for (int64_t i = 0; i < n; ++i) {
            double s = 0.0;
            for (int64_t e = rp64[i]; e < rp64[i + 1]; ++e) s += std::hypot(vp[2 * e], vp[2 * e + 1]);
            anorm = std::max(anorm, s);
        }
        if (!(anorm > 0.0)) return SE_ERR_INVALID_ARG;
    }
    std::vector<int> rp32(n + 1);
    for (int64_t i = 0; i <= n; ++i) rp32[i] = (int)rp64[i];
    se_matrix* m = new (std::nothrow) se_matrix();
    if (!m) return SE_ERR_OOM;
    m->ctx = ctx;
    m->device = ctx->device;
    m->n = n;
    m->nnz = nnz;
    m->anorm = anorm;
    m->is_complex = 1;
    hipError_t e = hipMalloc(&m->rowptr, sizeof(int) * (n + 1));
    if (e == hipSuccess) e = hipMalloc(&m->col, sizeof(int) * (nnz + se::kCsrPad));
    if (e == hipSuccess) e = hipMalloc(&m->val, sizeof(double) * 2 * (nnz + se::kCsrPad));
    if (e == hipSuccess) e = hipMemset(m->col + nnz, 0, sizeof(int) * se::kCsrPad);
    if (e == hipSuccess) e = hipMemset(m->val + 2 * nnz, 0, sizeof(double) * 2 * se::kCsrPad);
    if (e == hipSuccess) e = hipMemcpy(m->rowptr, rp32.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess && nnz > 0) e = hipMemcpy(m->col, cp, sizeof(int) * nnz, hipMemcpyHostToDevice);
    if (e == hipSuccess && nnz > 0) e = hipMemcpy(m->val, vp, sizeof(double) * 2 * nnz, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        se_matrix_destroy(m);
        return hip_fail(ctx, e);
    }
    *out = m;
    return SE_OK;
}

se_status se_solve_z(se_ctx* ctx, const se_matrix* A, const se_params* p, const double* X0, double* V,
                     double* lambda, se_info* info) {
    if (!ctx || !A || !p || !V || !lambda) return SE_ERR_INVALID_ARG;
    if (A->ctx != ctx || !A->is_complex) return SE_ERR_INVALID_ARG;
    if (p->solver != SE_LOBPCG && p->solver != SE_SI) {
        return (p->solver == SE_SD || p->solver == SE_TRACEMIN) ? SE_ERR_UNSUPPORTED : SE_ERR_INVALID_ARG;
    }
    const se_status v = se::validate_solve(A, p);
    if (v != SE_OK) return v;
    if (p->precision != SE_FP64 || p->expand_vectors != SE_EXPAND_XDROP || p->filter_degree != 0 ||
        p->precond != SE_PRECOND_NONE)
        return SE_ERR_UNSUPPORTED;
    const int64_t nb = (int64_t)p->n_ev + p->n_extra;
    if (p->solver == SE_LOBPCG && nb > 170) return SE_ERR_UNSUPPORTED;  // 3 nb <= 512
    if (p->solver == SE_SI && nb > 512) return SE_ERR_UNSUPPORTED;
    CAPI_HC(ctx, hipSetDevice(ctx->device));
    (void)hipGetLastError();
    if (info) std::memset(info, 0, sizeof(*info));
    return se::solve_z(ctx, A, p, X0, V, lambda, info);
}

se_status se_op_spmm_z(se_ctx* ctx, const se_matrix* A, const double* X, int64_t ldx, double* Y, int64_t ldy,
                       int32_t w) {
    if (!ctx || !A || !X || !Y || !A->is_complex || w < 1 || w > 512 || !valid_ld(ldx, w) || !valid_ld(ldy, w))
        return SE_ERR_INVALID_ARG;
    if (!aligned16(X) || !aligned16(Y)) return SE_ERR_INVALID_ARG;
    CAPI_HC(ctx, hipSetDevice(ctx->device));
    CAPI_HC(ctx, se::launch_spmm_z(ctx->stream, (int)A->n, A->rowptr, A->col, A->val, X, ldx, Y, ldy, w));
    return SE_OK;
}

se_status se_op_gram_z(se_ctx* ctx, int64_t n, const double* U, int64_t ldu, int32_t mu, const double* V,
                       int64_t ldv, int32_t mv, double* C) {
    if (!ctx || !U || !V || !C || n < 1 || mu < 1 || mv < 1 || mu > 512 || mv > 512) return SE_ERR_INVALID_ARG;
    if (!valid_ld(ldu, mu) || !valid_ld(ldv, mv)) return SE_ERR_INVALID_ARG;
    CAPI_HC(ctx, hipSetDevice(ctx->device));
    se::Workspace& ws = ctx->ws;
    const size_t need = sizeof(double) * se::gram_scratch_doubles(n, 2 * mu, 2 * mv);
    const size_t pbytes = sizeof(double) * 4 * (size_t)mu * mv;
    if (need > ws.gram_part.bytes || pbytes > ws.lpM.bytes) {
        CAPI_HC(ctx, hipStreamSynchronize(ctx->stream));
        CAPI_HC(ctx, ws.gram_part.ensure(need));
        CAPI_HC(ctx, ws.lpM.ensure(pbytes));
    }
    se::Segs Us = se::make_segs(2 * ldu), Vs = se::make_segs(2 * ldv);
    se::push_seg(Us, U, 2 * mu);
    se::push_seg(Vs, V, 2 * mv);
    const int sym = (U == V && ldu == ldv && mu == mv) ? 1 : 0;
    CAPI_HC(ctx, se::launch_gram(ctx->stream, n, Us, Vs, sym, ws.gram_part.as<double>(), ws.lpM.as<double>()));
    CAPI_HC(ctx, se::launch_zgram_combine(ctx->stream, mu, mv, ws.lpM.as<double>(), C));
    return SE_OK;
}

se_status se_op_update_z(se_ctx* ctx, int64_t n, const double* U, int64_t ldu, int32_t K, const double* C,
                         int32_t N, double* Out, int64_t ldo, double beta) {
    if (!ctx || !U || !C || !Out || n < 1 || K < 1 || N < 1 || K > 512 || N > 512) return SE_ERR_INVALID_ARG;
    if (!valid_ld(ldu, K) || !valid_ld(ldo, N) || !(beta == 0.0 || beta == 1.0)) return SE_ERR_INVALID_ARG;
    const char* u0 = reinterpret_cast<const char*>(U);
    const char* u1 = u0 + 16 * (size_t)((n - 1) * ldu + K);
    const char* o0 = reinterpret_cast<const char*>(Out);
    const char* o1 = o0 + 16 * (size_t)((n - 1) * ldo + N);
    if (o0 < u1 && u0 < o1) return SE_ERR_INVALID_ARG;
    CAPI_HC(ctx, hipSetDevice(ctx->device));
    se::Workspace& ws = ctx->ws;
    const size_t ebytes = sizeof(double) * 4 * (size_t)K * N;
    if (ebytes > ws.lpT.bytes) {
        CAPI_HC(ctx, hipStreamSynchronize(ctx->stream));
        CAPI_HC(ctx, ws.lpT.ensure(ebytes));
    }
    CAPI_HC(ctx, se::launch_zembed(ctx->stream, K, N, C, ws.lpT.as<double>()));
    se::Segs Us = se::make_segs(2 * ldu), Os = se::make_segs(2 * ldo);
    se::push_seg(Us, U, 2 * K);
    se::push_seg(Os, Out, 2 * N);
    CAPI_HC(ctx, se::launch_update(ctx->stream, n, Us, ws.lpT.as<double>(), 2 * N, Os, 1.0, beta));
    return SE_OK;
}

se_status se_op_heev_lowest_z(se_ctx* ctx, int32_t m, int32_t k, double* A, double* w, double* Z) {
    if (!ctx || !A || !w || !Z || m < 1 || m > 512 || k < 1 || k > m) return SE_ERR_INVALID_ARG;
    CAPI_HC(ctx, hipSetDevice(ctx->device));
    CAPI_HC(ctx, hipStreamSynchronize(ctx->stream));
    CAPI_HC(ctx, ctx->ws.syev_work.ensure(sizeof(double) * se::heev_z_work_doubles(m)));
    CAPI_HC(ctx, se::launch_heev_lowest_z(ctx->stream, m, k, A, w, Z, ctx->ws.syev_work.as<double>()));
    CAPI_HC(ctx, hipStreamSynchronize(ctx->stream));
    return SE_OK;
}

se_status se_strategy_replay(const se_params* p, int32_t count, const double* r, int32_t* flags) {
    if (!p || !r || !flags || count < 0) return SE_ERR_INVALID_ARG;
    se::Strategy s;
    s.kind = p->strategy;
    s.j_e = p->j_e;
    s.j_s = p->j_s;
    s.j_p = p->j_p;
    s.j_warm = p->j_warm;
    s.mu = p->mu;
    s.r_warm = p->r_warm;
    for (int j = 1; j <= count; ++j) {
        int f = 0;
        s.observe(j, r[j - 1]);
        if (s.ifexpand(j)) {
            s.did_expand(j);
            f |= 1;
        }
        if (s.ifshrink(j)) {
            s.did_shrink(j);
            f |= 2;
        }
        flags[j - 1] = f;
    }
    return SE_OK;
}

const char* se_status_string(se_status s) {
    switch (s) {
        case SE_OK: return "ok";
        case SE_NOT_CONVERGED: return "not converged (iteration or time limit); best iterate returned";
        case SE_ERR_INVALID_ARG: return "invalid argument";
        case SE_ERR_OOM: return "device out of memory";
        case SE_ERR_HIP: return "HIP runtime error";
        case SE_ERR_BREAKDOWN: return "orthogonalization breakdown";
        case SE_ERR_REJECTED: return "request exceeds the memory budget";
        case SE_ERR_UNSUPPORTED: return "unsupported option";
        default: return "unknown status";
    }
}

}  // extern "C"
