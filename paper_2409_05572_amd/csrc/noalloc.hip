// Gram product C = U^T V without any device allocation, for callers that
// cannot allocate (code under stream capture, tight serving loops, harnesses
// that forbid hipMalloc).
//
// The per-chunk partial products live in a fixed file-scope device array of
// kNoAllocGramDoubles doubles. Each device holds its own copy of the array
// for the life of the process; its device address is looked up once per
// device with hipGetSymbolAddress and only that address is passed to kernels.
// The row chunking is limited so that the partials fit (at most
// kNoAllocGramDoubles / (mu mv) chunks), which changes only the order of the
// fixed-order sum relative to se_op_gram, not its accuracy. Every partial the
// reduction reads is written by the same call first, so nothing needs
// clearing. Calls that overlap on one device share the array and race.
#include <mutex>

#include "engine.h"

namespace {

constexpr size_t kNoAllocGramDoubles = size_t(4) << 20;  // 32 MiB per device

static __device__ __align__(256) double scratch[kNoAllocGramDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up once per device,
// with that device current).
hipError_t scratch_ptr(int device, double** out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[device] = static_cast<double*>(p);
    }
    *out = g_ptr[device];
    return hipSuccess;
}

}  // namespace

extern "C" se_status se_op_gram_noalloc(se_ctx* ctx, int64_t n, const double* U, int64_t ldu, int32_t mu,
                                        const double* V, int64_t ldv, int32_t mv, double* C) {
    if (!ctx || !U || !V || !C || n < 1 || mu < 1 || mv < 1 || mu > 1024 || mv > 1024)
        return SE_ERR_INVALID_ARG;
    if (ldu < mu || ldu % 2 != 0 || ldv < mv || ldv % 2 != 0) return SE_ERR_INVALID_ARG;
    if ((size_t)mu * (size_t)mv > kNoAllocGramDoubles) return SE_ERR_UNSUPPORTED;  // cannot happen at <= 1024
    hipError_t e = hipSetDevice(ctx->device);
    double* part = nullptr;
    if (e == hipSuccess) e = scratch_ptr(ctx->device, &part);
    if (e == hipSuccess) {
        se::Segs Us = se::make_segs(ldu), Vs = se::make_segs(ldv);
        se::push_seg(Us, U, mu);
        se::push_seg(Vs, V, mv);
        const int sym = (U == V && ldu == ldv && mu == mv) ? 1 : 0;
        e = se::launch_gram(ctx->stream, n, Us, Vs, sym, part, C, kNoAllocGramDoubles);
    }
    if (e != hipSuccess) {
        ctx->last_hip_error = (int)e;
        return SE_ERR_HIP;
    }
    return SE_OK;
}
