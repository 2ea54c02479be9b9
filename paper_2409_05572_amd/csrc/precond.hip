// Diagonal (Jacobi) preconditioner T = diag(1 / |a_ii|) for the W <- T R step
// of LOBPCG and steepest descent (Algorithms 2 and 3), FP64, gfx950.
#include "common.h"

namespace se {
namespace {

constexpr int kPcThreads = 256;

// dinv[r] = 1 / |a_rr| (1 when row r stores no diagonal entry or a zero one).
__global__ __launch_bounds__(kPcThreads) void jacobi_kernel(int n, const int* __restrict__ rowptr,
                                                            const int* __restrict__ col,
                                                            const double* __restrict__ val,
                                                            double* __restrict__ dinv) {
    const int r = blockIdx.x * kPcThreads + threadIdx.x;
    if (r >= n) return;
    double d = 0.0;
    for (int p = rowptr[r]; p < rowptr[r + 1]; ++p)
        if (col[p] == r) d += val[p];
    dinv[r] = d != 0.0 ? 1.0 / fabs(d) : 1.0;
}

// W[r, c] *= dinv[r] for c < a: TPR lanes per row, 16-byte column pairs.
template <int TPR>
__global__ __launch_bounds__(kPcThreads) void row_scale_kernel(long long n, int a, const double* __restrict__ dinv,
                                                               double* __restrict__ W, long long ld) {
    constexpr int RPB = kPcThreads / TPR;
    const long long r = (long long)blockIdx.x * RPB + threadIdx.x / TPR;
    if (r >= n) return;
    const int lane = threadIdx.x % TPR;
    const double s = dinv[r];
    double* w = W + r * ld;
    for (int c = 2 * lane; c < a; c += 2 * TPR) {
        if (c + 1 < a) {
            double2 v = *reinterpret_cast<const double2*>(w + c);
            v.x *= s;
            v.y *= s;
            *reinterpret_cast<double2*>(w + c) = v;
        } else {
            w[c] *= s;
        }
    }
}

template <int TPR>
hipError_t row_scale_launch(hipStream_t st, long long n, int a, const double* dinv, double* W, long long ld) {
    constexpr int RPB = kPcThreads / TPR;
    const long long grid = (n + RPB - 1) / RPB;
    hipLaunchKernelGGL(row_scale_kernel<TPR>, dim3((unsigned)grid), dim3(kPcThreads), 0, st, n, a, dinv, W, ld);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_jacobi(hipStream_t st, int n, const int* rowptr, const int* col, const double* val, double* dinv) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(jacobi_kernel, dim3((n + kPcThreads - 1) / kPcThreads), dim3(kPcThreads), 0, st, n, rowptr,
                       col, val, dinv);
    return hipGetLastError();
}

hipError_t launch_row_scale(hipStream_t st, long long n, int a, const double* dinv, double* W, long long ld) {
    if (n <= 0 || a <= 0) return hipSuccess;
    if ((ld & 1) || ld < a) return hipErrorInvalidValue;
    const int pairs = (a + 1) / 2;
    if (pairs <= 8) return row_scale_launch<8>(st, n, a, dinv, W, ld);
    if (pairs <= 16) return row_scale_launch<16>(st, n, a, dinv, W, ld);
    if (pairs <= 32) return row_scale_launch<32>(st, n, a, dinv, W, ld);
    return row_scale_launch<64>(st, n, a, dinv, W, ld);
}

}  // namespace se
