// Column-wise conjugate-gradient kernels for TraceMIN's inexact inner solve
// (Algorithm 4: P A P D = P R, a few CG steps on every column at once), FP64,
// gfx950. Every column c carries its own scalars (step length alpha_c, the
// next direction's beta_c), read from device arrays, so a CG step needs no
// host round trip.
//
// Reductions over n follow the residual-norm pattern of the bulk kernels:
// each workgroup sums a chunk of rows (thread t takes column t % k of every
// (256 / k)-th row, so a row's k columns are read by consecutive threads) and
// writes a partial per column; a second kernel adds the partials in a fixed
// order (bitwise reproducible).
#include "common.h"

namespace se {
namespace {

constexpr int kCgThreads = 256;

// part[chunk * k + c] = sum over the chunk's rows of U[r, c] V[r, c].
__global__ __launch_bounds__(kCgThreads) void col_dots_kernel(long long n, int k, const double* __restrict__ U,
                                                              const double* __restrict__ V, long long ld,
                                                              long long rows_per_chunk, double* __restrict__ part) {
    __shared__ double sh[kCgThreads];
    const long long r0 = (long long)blockIdx.x * rows_per_chunk;
    const long long r1 = min(n, r0 + rows_per_chunk);
    const int t = threadIdx.x;
    double* out = part + (long long)blockIdx.x * k;
    if (k <= kCgThreads) {
        const int ngrp = kCgThreads / k;
        const int c = t % k, g = t / k;
        double acc = 0.0;
        if (g < ngrp)
            for (long long r = r0 + g; r < r1; r += ngrp) acc = fma(U[r * ld + c], V[r * ld + c], acc);
        sh[t] = acc;
        __syncthreads();
        if (t < k) {
            double s = 0.0;
            for (int q = 0; q < ngrp; ++q) s += sh[q * k + t];
            out[t] = s;
        }
    } else {
        for (int c = t; c < k; c += kCgThreads) {
            double acc = 0.0;
            for (long long r = r0; r < r1; ++r) acc = fma(U[r * ld + c], V[r * ld + c], acc);
            out[c] = acc;
        }
    }
}

__device__ __forceinline__ double cg_alpha(double rr, double dq) { return (dq > 0.0 && rr > 0.0) ? rr / dq : 0.0; }

// One CG step on every column: alpha_c = rr_c / dq_c (0 once the column's
// residual vanished or its curvature is not positive), D += alpha d (D = alpha
// d when first), R -= alpha Q, and the partial sums of the new R[:, c]^2.
__global__ __launch_bounds__(kCgThreads) void cg_step_kernel(long long n, int k, const double* __restrict__ rr,
                                                             const double* __restrict__ dq,
                                                             const double* __restrict__ Dir,
                                                             const double* __restrict__ Q, double* __restrict__ D,
                                                             double* __restrict__ R, long long ld, int first,
                                                             long long rows_per_chunk, double* __restrict__ part) {
    __shared__ double sh[kCgThreads];
    const long long r0 = (long long)blockIdx.x * rows_per_chunk;
    const long long r1 = min(n, r0 + rows_per_chunk);
    const int t = threadIdx.x;
    double* out = part + (long long)blockIdx.x * k;
    if (k <= kCgThreads) {
        const int ngrp = kCgThreads / k;
        const int c = t % k, g = t / k;
        double acc = 0.0;
        if (g < ngrp) {
            const double a = cg_alpha(rr[c], dq[c]);
            for (long long r = r0 + g; r < r1; r += ngrp) {
                const long long o = r * ld + c;
                D[o] = first ? a * Dir[o] : fma(a, Dir[o], D[o]);
                const double x = fma(-a, Q[o], R[o]);
                R[o] = x;
                acc = fma(x, x, acc);
            }
        }
        sh[t] = acc;
        __syncthreads();
        if (t < k) {
            double s = 0.0;
            for (int q = 0; q < ngrp; ++q) s += sh[q * k + t];
            out[t] = s;
        }
    } else {
        for (int c = t; c < k; c += kCgThreads) {
            const double a = cg_alpha(rr[c], dq[c]);
            double acc = 0.0;
            for (long long r = r0; r < r1; ++r) {
                const long long o = r * ld + c;
                D[o] = first ? a * Dir[o] : fma(a, Dir[o], D[o]);
                const double x = fma(-a, Q[o], R[o]);
                R[o] = x;
                acc = fma(x, x, acc);
            }
            out[c] = acc;
        }
    }
}

// Next direction: Dir[:, c] = R[:, c] + beta_c Dir[:, c], beta_c = rr_new_c / rr_c
// (0 when rr_c = 0).
__global__ __launch_bounds__(kCgThreads) void cg_dir_kernel(long long n, int k, const double* __restrict__ rr_new,
                                                            const double* __restrict__ rr,
                                                            const double* __restrict__ R, double* __restrict__ Dir,
                                                            long long ld, long long rows_per_chunk) {
    const long long r0 = (long long)blockIdx.x * rows_per_chunk;
    const long long r1 = min(n, r0 + rows_per_chunk);
    const int t = threadIdx.x;
    if (k <= kCgThreads) {
        const int ngrp = kCgThreads / k;
        const int c = t % k, g = t / k;
        if (g >= ngrp) return;
        const double b = rr[c] > 0.0 ? rr_new[c] / rr[c] : 0.0;
        for (long long r = r0 + g; r < r1; r += ngrp) {
            const long long o = r * ld + c;
            Dir[o] = fma(b, Dir[o], R[o]);
        }
    } else {
        for (int c = t; c < k; c += kCgThreads) {
            const double b = rr[c] > 0.0 ? rr_new[c] / rr[c] : 0.0;
            for (long long r = r0; r < r1; ++r) {
                const long long o = r * ld + c;
                Dir[o] = fma(b, Dir[o], R[o]);
            }
        }
    }
}

void cg_chunks(long long n, long long& rows, long long& nchunks) {
    rows = 2048;
    nchunks = (n + rows - 1) / rows;
    if (nchunks > 4096) {
        nchunks = 4096;
        rows = (n + nchunks - 1) / nchunks;
        nchunks = (n + rows - 1) / rows;
    }
    if (nchunks < 1) nchunks = 1;
}

}  // namespace

hipError_t launch_col_dots(hipStream_t st, long long n, int k, const double* U, const double* V, long long ld,
                           double* part, double* out) {
    if (n <= 0 || k <= 0) return hipSuccess;
    long long rows, nchunks;
    cg_chunks(n, rows, nchunks);
    hipLaunchKernelGGL(col_dots_kernel, dim3((unsigned)nchunks), dim3(kCgThreads), 0, st, n, k, U, V, ld, rows,
                       part);
    return launch_sum_partials(st, k, (int)nchunks, part, out);
}

hipError_t launch_cg_step(hipStream_t st, long long n, int k, const double* rr, const double* dq, const double* Dir,
                          const double* Q, double* D, double* R, long long ld, bool first, double* part,
                          double* rr_new) {
    if (n <= 0 || k <= 0) return hipSuccess;
    long long rows, nchunks;
    cg_chunks(n, rows, nchunks);
    hipLaunchKernelGGL(cg_step_kernel, dim3((unsigned)nchunks), dim3(kCgThreads), 0, st, n, k, rr, dq, Dir, Q, D,
                       R, ld, first ? 1 : 0, rows, part);
    return launch_sum_partials(st, k, (int)nchunks, part, rr_new);
}

hipError_t launch_cg_dir(hipStream_t st, long long n, int k, const double* rr_new, const double* rr, const double* R,
                         double* Dir, long long ld) {
    if (n <= 0 || k <= 0) return hipSuccess;
    long long rows, nchunks;
    cg_chunks(n, rows, nchunks);
    hipLaunchKernelGGL(cg_dir_kernel, dim3((unsigned)nchunks), dim3(kCgThreads), 0, st, n, k, rr_new, rr, R, Dir,
                       ld, rows);
    return hipGetLastError();
}

}  // namespace se
