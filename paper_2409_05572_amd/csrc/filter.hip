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

// The sparse product fused with one step of the recurrence, for matrices
// without rows longer than 64 nonzeros: Z[r, c] <- alpha (A Y)[r, c] +
// beta Y[r, c] + gamma Z[r, c] for c < w (Z is not read when gamma = 0). It
// walks the CSR rows like the streaming SpMM: one wave per run of kRun
// consecutive rows takes the run's nonzeros NB at a time, with wave-uniform
// column indices and values (the CSR arrays are padded past their end), issues
// all NB row gathers of Y (16 bytes per lane) before using any, and hands the
// accumulator to the next row at each row boundary. At a row's end the lane
// combines its two sums with the row's own Y and Z entries and stores Z, so
// the product A Y never goes to memory. Lane l owns columns cb + 2l, cb + 2l + 1
// of each 128-column block (an odd width reads the padding column of Y).
constexpr int kRun = 32;

template <int NB>
__global__ __launch_bounds__(kFilterThreads) void spmm_cheb_kernel(int n, const int* __restrict__ rowptr,
                                                                   const int* __restrict__ col,
                                                                   const double* __restrict__ val,
                                                                   const double* __restrict__ Y,
                                                                   double* __restrict__ Z, long long ld, int w,
                                                                   double alpha, double beta, double gamma) {
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane((int)blockIdx.x * (kFilterThreads / 64) + (int)(threadIdx.x >> 6));
    if ((long long)wid * kRun >= n) return;
    const int r0 = wid * kRun;
    const int r1 = min(n, r0 + kRun);
    const int rp = rowptr[min(r0 + lane, r1)];  // lane q: offset of row r0 + q, q <= r1 - r0
    const int pbeg = __builtin_amdgcn_readlane(rp, 0);
    const int pend = __builtin_amdgcn_readlane(rp, r1 - r0);
    const bool with_z = gamma != 0.0;
    for (int cb = 0; cb < w; cb += 128) {
        const int c0 = cb + 2 * lane;
        const bool has0 = c0 < w, has1 = c0 + 1 < w;
        const long long cc = has0 ? c0 : cb;  // lanes without columns read a valid address
        int r = r0;
        int rend = __builtin_amdgcn_readlane(rp, 1);
        double a0 = 0.0, a1 = 0.0;
        auto flush = [&]() {
            const long long o = (long long)r * ld + c0;
            if (has1) {
                const double2 y = *reinterpret_cast<const double2*>(Y + o);
                double2 z = make_double2(0.0, 0.0);
                if (with_z) z = *reinterpret_cast<const double2*>(Z + o);
                *reinterpret_cast<double2*>(Z + o) =
                    make_double2(alpha * a0 + beta * y.x + gamma * z.x, alpha * a1 + beta * y.y + gamma * z.y);
            } else if (has0) {
                const double z = with_z ? Z[o] : 0.0;
                Z[o] = alpha * a0 + beta * Y[o] + gamma * z;
            }
            a0 = 0.0;
            a1 = 0.0;
            ++r;
            if (r < r1) rend = __builtin_amdgcn_readlane(rp, r - r0 + 1);
        };
        for (int p = pbeg; p < pend; p += NB) {
            int j[NB];
            double v[NB];
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                j[u] = col[p + u];
                v[u] = val[p + u];
            }
            double2 x[NB];
#pragma unroll
            for (int u = 0; u < NB; ++u) x[u] = *reinterpret_cast<const double2*>(Y + (long long)j[u] * ld + cc);
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                if (p + u < pend) {
                    while (p + u >= rend) flush();
                    a0 = fma(v[u], x[u].x, a0);
                    a1 = fma(v[u], x[u].y, a1);
                }
            }
        }
        while (r < r1) flush();
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

hipError_t launch_spmm_cheb(hipStream_t st, int n, const int* rowptr, const int* col, const double* val,
                            const double* Y, double* Z, long long ld, int w, int n_heavy, double alpha, double beta,
                            double gamma) {
    if (n <= 0 || w <= 0) return hipSuccess;
    if (n_heavy > 0 || (ld & 1) || ld < w + (w & 1)) return hipErrorInvalidValue;
    const long long waves = ((long long)n + kRun - 1) / kRun;
    const int grid = (int)((waves + kFilterThreads / 64 - 1) / (kFilterThreads / 64));
    hipLaunchKernelGGL(spmm_cheb_kernel<16>, dim3(grid), dim3(kFilterThreads), 0, st, n, rowptr, col, val, Y, Z, ld,
                       w, alpha, beta, gamma);
    return hipGetLastError();
}

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
