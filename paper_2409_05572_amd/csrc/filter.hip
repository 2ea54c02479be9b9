// One step of the Chebyshev filter recurrence for subspace iteration, FP64,
// gfx950: Z <- alpha U + beta V + gamma Z over the first k columns of
// row-major n-row panels (U the product A V of the previous step, V the
// previous filtered block, Z the block before it, overwritten in place).
//
// The step is a pure stream (three reads, one write per element), so it is
// bound by HBM: TPR lanes share one row and move 16-byte pairs of columns,
// RPB = 256 / TPR rows per workgroup, no index division. The row length of
// the panels is even, so every row starts 16-byte aligned.
#include "common.h"

namespace se {
namespace {

constexpr int kFilterThreads = 256;

template <int TPR>
__global__ __launch_bounds__(kFilterThreads) void cheb_step_kernel(long long n, int k, double alpha,
                                                                   const double* __restrict__ U, double beta,
                                                                   const double* __restrict__ V, double gamma,
                                                                   double* __restrict__ Z, long long ld) {
    constexpr int RPB = kFilterThreads / TPR;
    const long long r = (long long)blockIdx.x * RPB + threadIdx.x / TPR;
    if (r >= n) return;
    const int lane = threadIdx.x % TPR;
    const long long o = r * ld;
    const bool with_z = gamma != 0.0;  // Z is not read when gamma = 0 (it may hold anything)
    for (int c = 2 * lane; c < k; c += 2 * TPR) {
        if (c + 1 < k) {
            const double2 u = *reinterpret_cast<const double2*>(U + o + c);
            const double2 v = *reinterpret_cast<const double2*>(V + o + c);
            double2 z = make_double2(0.0, 0.0);
            if (with_z) z = *reinterpret_cast<const double2*>(Z + o + c);
            *reinterpret_cast<double2*>(Z + o + c) =
                make_double2(alpha * u.x + beta * v.x + gamma * z.x, alpha * u.y + beta * v.y + gamma * z.y);
        } else {
            const double z = with_z ? Z[o + c] : 0.0;
            Z[o + c] = alpha * U[o + c] + beta * V[o + c] + gamma * z;
        }
    }
}

template <int TPR>
hipError_t cheb_step_launch(hipStream_t st, long long n, int k, double alpha, const double* U, double beta,
                            const double* V, double gamma, double* Z, long long ld) {
    constexpr int RPB = kFilterThreads / TPR;
    const long long grid = (n + RPB - 1) / RPB;
    hipLaunchKernelGGL(cheb_step_kernel<TPR>, dim3((unsigned)grid), dim3(kFilterThreads), 0, st, n, k, alpha, U,
                       beta, V, gamma, Z, ld);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_cheb_step(hipStream_t st, long long n, int k, double alpha, const double* U, double beta,
                            const double* V, double gamma, double* Z, long long ld) {
    if (n <= 0 || k <= 0) return hipSuccess;
    if ((ld & 1) || ld < k) return hipErrorInvalidValue;
    const int pairs = (k + 1) / 2;
    if (pairs <= 8) return cheb_step_launch<8>(st, n, k, alpha, U, beta, V, gamma, Z, ld);
    if (pairs <= 16) return cheb_step_launch<16>(st, n, k, alpha, U, beta, V, gamma, Z, ld);
    if (pairs <= 32) return cheb_step_launch<32>(st, n, k, alpha, U, beta, V, gamma, Z, ld);
    return cheb_step_launch<64>(st, n, k, alpha, U, beta, V, gamma, Z, ld);
}

}  // namespace se
