// Column-wise conjugate-gradient kernels for TraceMIN's inexact inner solve
// (Algorithm 4: P A P D = P R, a few CG steps on every column at once), FP64,
// gfx950. Every column c carries its own scalars (step length alpha_c, the
// next direction's beta_c), read from device arrays, so a CG step needs no
// host round trip.
//
// Reductions over n: each workgroup sums a chunk of rows and writes a partial
// per column; a second kernel adds the partials in a fixed order (bitwise
// reproducible).
#include "common.h"

namespace se {
namespace {

constexpr int kCgThreads = 256;

// Thread layout of the three kernels: thread t of a workgroup owns the column
// pair cp = t % P (columns 2 cp and 2 cp + 1, P = ceil(k / 2) pairs, 16-byte
// loads; rows start 16-byte aligned since ld is even) and rows r0 + g,
// r0 + g + G, ... of the chunk (g = t / P, G = 256 / P groups); the row loop
// is unrolled four times so that four rows' loads are in flight. k <= 512.
struct PairMap {
    int P, G, cp, g;
    bool active;
    __device__ PairMap(int k) {
        P = (k + 1) / 2;
        G = kCgThreads / P;
        cp = threadIdx.x % P;
        g = threadIdx.x / P;
        active = g < G;
    }
};

__device__ __forceinline__ double2 ld2(const double* p, bool pair) {
    return pair ? *reinterpret_cast<const double2*>(p) : make_double2(p[0], 0.0);
}
__device__ __forceinline__ void st2(double* p, double2 v, bool pair) {
    if (pair)
        *reinterpret_cast<double2*>(p) = v;
    else
        p[0] = v.x;
}

// Sums the per-thread pair accumulators of a workgroup over its row groups
// and writes the chunk's partial for columns 2 cp, 2 cp + 1.
__device__ __forceinline__ void reduce_pairs(const PairMap& m, int k, double2 acc, double2* sh, double* out) {
    sh[threadIdx.x] = m.active ? acc : make_double2(0.0, 0.0);
    __syncthreads();
    if (threadIdx.x < m.P) {
        double2 s = make_double2(0.0, 0.0);
        for (int q = 0; q < m.G; ++q) {
            const double2 v = sh[q * m.P + threadIdx.x];
            s.x += v.x;
            s.y += v.y;
        }
        out[2 * threadIdx.x] = s.x;
        if (2 * threadIdx.x + 1 < k) out[2 * threadIdx.x + 1] = s.y;
    }
}

// part[chunk * k + c] = sum over the chunk's rows of U[r, c] V[r, c].
__global__ __launch_bounds__(kCgThreads) void col_dots_kernel(long long n, int k, const double* __restrict__ U,
                                                              const double* __restrict__ V, long long ld,
                                                              long long rows_per_chunk, double* __restrict__ part) {
    __shared__ double2 sh[kCgThreads];
    const long long r0 = (long long)blockIdx.x * rows_per_chunk;
    const long long r1 = min(n, r0 + rows_per_chunk);
    const PairMap m(k);
    double* out = part + (long long)blockIdx.x * k;
    {
        const int c = 2 * m.cp;
        const bool pair = c + 1 < k;
        double2 acc = make_double2(0.0, 0.0);
        if (m.active) {
#pragma unroll 4
            for (long long r = r0 + m.g; r < r1; r += m.G) {
                const double2 u = ld2(U + r * ld + c, pair), v = ld2(V + r * ld + c, pair);
                acc.x = fma(u.x, v.x, acc.x);
                acc.y = fma(u.y, v.y, acc.y);
            }
        }
        reduce_pairs(m, k, acc, sh, out);
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
    __shared__ double2 sh[kCgThreads];
    const long long r0 = (long long)blockIdx.x * rows_per_chunk;
    const long long r1 = min(n, r0 + rows_per_chunk);
    const PairMap m(k);
    double* out = part + (long long)blockIdx.x * k;
    {
        const int c = 2 * m.cp;
        const bool pair = c + 1 < k;
        double2 acc = make_double2(0.0, 0.0);
        if (m.active) {
            const double ax = cg_alpha(rr[c], dq[c]);
            const double ay = pair ? cg_alpha(rr[c + 1], dq[c + 1]) : 0.0;
#pragma unroll 4
            for (long long r = r0 + m.g; r < r1; r += m.G) {
                const long long o = r * ld + c;
                const double2 d = ld2(Dir + o, pair), q = ld2(Q + o, pair), x = ld2(R + o, pair);
                double2 dd;
                if (first) {
                    dd = make_double2(ax * d.x, ay * d.y);
                } else {
                    const double2 d0 = ld2(D + o, pair);
                    dd = make_double2(fma(ax, d.x, d0.x), fma(ay, d.y, d0.y));
                }
                const double2 rn = make_double2(fma(-ax, q.x, x.x), fma(-ay, q.y, x.y));
                st2(D + o, dd, pair);
                st2(R + o, rn, pair);
                acc.x = fma(rn.x, rn.x, acc.x);
                acc.y = fma(rn.y, rn.y, acc.y);
            }
        }
        reduce_pairs(m, k, acc, sh, out);
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
    const PairMap m(k);
    if (!m.active) return;
    {
        const int c = 2 * m.cp;
        const bool pair = c + 1 < k;
        const double bx = rr[c] > 0.0 ? rr_new[c] / rr[c] : 0.0;
        const double by = (pair && rr[c + 1] > 0.0) ? rr_new[c + 1] / rr[c + 1] : 0.0;
#pragma unroll 4
        for (long long r = r0 + m.g; r < r1; r += m.G) {
            const long long o = r * ld + c;
            const double2 x = ld2(R + o, pair), d = ld2(Dir + o, pair);
            st2(Dir + o, make_double2(fma(bx, d.x, x.x), fma(by, d.y, x.y)), pair);
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
    if (k > 2 * kCgThreads || (ld & 1) || ld < k) return hipErrorInvalidValue;
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
    if (k > 2 * kCgThreads || (ld & 1) || ld < k) return hipErrorInvalidValue;
    long long rows, nchunks;
    cg_chunks(n, rows, nchunks);
    hipLaunchKernelGGL(cg_step_kernel, dim3((unsigned)nchunks), dim3(kCgThreads), 0, st, n, k, rr, dq, Dir, Q, D,
                       R, ld, first ? 1 : 0, rows, part);
    return launch_sum_partials(st, k, (int)nchunks, part, rr_new);
}

hipError_t launch_cg_dir(hipStream_t st, long long n, int k, const double* rr_new, const double* rr, const double* R,
                         double* Dir, long long ld) {
    if (n <= 0 || k <= 0) return hipSuccess;
    if (k > 2 * kCgThreads || (ld & 1) || ld < k) return hipErrorInvalidValue;
    long long rows, nchunks;
    cg_chunks(n, rows, nchunks);
    hipLaunchKernelGGL(cg_dir_kernel, dim3((unsigned)nchunks), dim3(kCgThreads), 0, st, n, k, rr_new, rr, R, Dir,
                       ld, rows);
    return hipGetLastError();
}

}  // namespace se
