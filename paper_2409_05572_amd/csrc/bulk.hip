// n-length (bulk) kernels of the Rayleigh-Ritz step, FP64, gfx950.
//
// Every n x w block is row-major with an even leading dimension, so that a
// row of a block is one contiguous run of memory:
//  * the CSR product gathers whole rows of X per nonzero (coalesced),
//  * the Gram product and the basis update stream contiguous row chunks,
//  * reductions over rows are split into per-workgroup partials that a second
//    kernel sums in a fixed order (bitwise deterministic results).
// Work is mapped to workgroups so that consecutive row ranges run on the same
// XCD (the hardware deals workgroups to the 8 XCDs round-robin), which keeps
// neighbouring rows of the stencil and the column tiles of a row chunk in one
// L2.
#include <algorithm>

#include "common.h"

namespace se {

namespace {

constexpr int kThreads = 256;

// Inverse of the round-robin workgroup-to-XCD dealing: returns a logical index
// such that each XCD receives one contiguous range of logical indices.
__device__ __forceinline__ int xcd_remap(int bid, int G) {
    constexpr int NX = 8;
    const int q = G / NX, r = G % NX;
    const int x = bid % NX, i = bid / NX;
    return x * q + min(x, r) + i;
}

__device__ __forceinline__ const double* seg_addr(const Segs& S, long long row, int c) {
    const double* p = S.p[0];
    int o = 0;
    if (S.nseg > 1 && c >= S.off[1]) { p = S.p[1]; o = S.off[1]; }
    if (S.nseg > 2 && c >= S.off[2]) { p = S.p[2]; o = S.off[2]; }
    if (S.nseg > 3 && c >= S.off[3]) { p = S.p[3]; o = S.off[3]; }
    return p + row * S.ld + (c - o);
}

inline int grid_for(long long work, int per_block, int cap = 1 << 20) {
    long long g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return static_cast<int>(g);
}

// ---------------------------------------------------------------------------
// CSR x block. LPR lanes cooperate on one matrix row; each lane owns two
// adjacent columns (one 16-byte load per gathered row of X).
template <int LPR>
__global__ __launch_bounds__(kThreads) void spmm_kernel(int n, const int* __restrict__ rowptr,
                                                        const int* __restrict__ col,
                                                        const double* __restrict__ val,
                                                        const double* __restrict__ X, long long ldx,
                                                        double* __restrict__ Y, long long ldy,
                                                        int w) {
    constexpr int RPB = kThreads / LPR;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int sub = threadIdx.x / LPR;
    const int lane = threadIdx.x % LPR;
    const int row = blk * RPB + sub;
    if (row >= n) return;
    const int beg = rowptr[row];
    const int end = rowptr[row + 1];
    for (int c0 = 2 * lane; c0 < w; c0 += 2 * LPR) {
        double a0 = 0.0, a1 = 0.0;
        if (c0 + 1 < w) {
            int e = beg;
            for (; e + 2 <= end; e += 2) {
                const int j0 = col[e], j1 = col[e + 1];
                const double v0 = val[e], v1 = val[e + 1];
                const double2 x0 = *reinterpret_cast<const double2*>(X + (long long)j0 * ldx + c0);
                const double2 x1 = *reinterpret_cast<const double2*>(X + (long long)j1 * ldx + c0);
                a0 = fma(v0, x0.x, a0);
                a1 = fma(v0, x0.y, a1);
                a0 = fma(v1, x1.x, a0);
                a1 = fma(v1, x1.y, a1);
            }
            if (e < end) {
                const int j0 = col[e];
                const double v0 = val[e];
                const double2 x0 = *reinterpret_cast<const double2*>(X + (long long)j0 * ldx + c0);
                a0 = fma(v0, x0.x, a0);
                a1 = fma(v0, x0.y, a1);
            }
            *reinterpret_cast<double2*>(Y + (long long)row * ldy + c0) = make_double2(a0, a1);
        } else {
            for (int e = beg; e < end; ++e) a0 = fma(val[e], X[(long long)col[e] * ldx + c0], a0);
            Y[(long long)row * ldy + c0] = a0;
        }
    }
}

template <int LPR>
hipError_t spmm_launch(hipStream_t st, int n, const int* rowptr, const int* col, const double* val,
                       const double* X, long long ldx, double* Y, long long ldy, int w) {
    constexpr int RPB = kThreads / LPR;
    const int grid = (n + RPB - 1) / RPB;
    hipLaunchKernelGGL(spmm_kernel<LPR>, dim3(grid), dim3(kThreads), 0, st, n, rowptr, col, val, X,
                       ldx, Y, ldy, w);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed-order sum of per-chunk partial vectors: out[i] = sum_c part[c * L + i].
__global__ __launch_bounds__(kThreads) void sum_partials_kernel(int L, int nchunks,
                                                                const double* __restrict__ part,
                                                                double* __restrict__ out) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= L) return;
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += part[(long long)c * L + i];
    out[i] = s;
}

// Residual and column norms: per chunk of rows, sum (ax - lam x)^2 and x^2.
__global__ __launch_bounds__(kThreads) void resid_norms_kernel(long long n, const double* __restrict__ X,
                                                               const double* __restrict__ AX,
                                                               long long ld, int k,
                                                               const double* __restrict__ lam,
                                                               long long rows_per_chunk,
                                                               double* __restrict__ part) {
    __shared__ double sr[kThreads];
    __shared__ double sx[kThreads];
    const int chunk = blockIdx.x;
    const long long r0 = (long long)chunk * rows_per_chunk;
    const long long r1 = min(n, r0 + rows_per_chunk);
    const int t = threadIdx.x;
    double* out = part + (long long)chunk * 2 * k;
    if (k <= kThreads) {
        const int ngrp = kThreads / k;
        const int c = t % k, g = t / k;
        double ar = 0.0, axx = 0.0;
        if (g < ngrp) {
            const double l = lam[c];
            for (long long r = r0 + g; r < r1; r += ngrp) {
                const double x = X[r * ld + c];
                const double y = AX[r * ld + c] - l * x;
                ar = fma(y, y, ar);
                axx = fma(x, x, axx);
            }
        }
        sr[t] = ar;
        sx[t] = axx;
        __syncthreads();
        if (t < k) {
            double s1 = 0.0, s2 = 0.0;
            for (int q = 0; q < ngrp; ++q) {
                s1 += sr[q * k + t];
                s2 += sx[q * k + t];
            }
            out[t] = s1;
            out[k + t] = s2;
        }
    } else {
        for (int c = t; c < k; c += kThreads) {
            const double l = lam[c];
            double ar = 0.0, axx = 0.0;
            for (long long r = r0; r < r1; ++r) {
                const double x = X[r * ld + c];
                const double y = AX[r * ld + c] - l * x;
                ar = fma(y, y, ar);
                axx = fma(x, x, axx);
            }
            out[c] = ar;
            out[k + c] = axx;
        }
    }
}

__global__ __launch_bounds__(kThreads) void form_w_kernel(long long n, const double* __restrict__ X,
                                                          const double* __restrict__ AX, long long ld,
                                                          const double* __restrict__ lam,
                                                          const int* __restrict__ act, int a,
                                                          double* __restrict__ W, long long ldw) {
    const long long total = n * a;
    for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < total;
         e += (long long)gridDim.x * kThreads) {
        const long long r = e / a;
        const int jj = (int)(e - r * a);
        const int c = act[jj];
        W[r * ldw + jj] = AX[r * ld + c] - lam[c] * X[r * ld + c];
    }
}

__global__ __launch_bounds__(kThreads) void shift_sub_kernel(long long n, double* __restrict__ X,
                                                             const double* __restrict__ AX,
                                                             long long ld, int k, double sigma) {
    const long long total = n * k;
    for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < total;
         e += (long long)gridDim.x * kThreads) {
        const long long r = e / k;
        const int c = (int)(e - r * k);
        X[r * ld + c] = sigma * X[r * ld + c] - AX[r * ld + c];
    }
}

__global__ __launch_bounds__(kThreads) void copy_cols_kernel(long long n, const double* __restrict__ src,
                                                             long long lds, int sc,
                                                             double* __restrict__ dst, long long ldd,
                                                             int dc, int w) {
    const long long total = n * w;
    for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < total;
         e += (long long)gridDim.x * kThreads) {
        const long long r = e / w;
        const int c = (int)(e - r * w);
        dst[r * ldd + dc + c] = src[r * lds + sc + c];
    }
}

// 32 x 32 tiles through LDS; blockDim = (32, 8).
__global__ void c2r_kernel(long long n, int w, const double* __restrict__ src, long long ldc,
                           double* __restrict__ dst, long long ldr) {
    __shared__ double tile[32][33];
    const long long r0 = (long long)blockIdx.x * 32;
    const int c0 = blockIdx.y * 32;
    for (int q = threadIdx.y; q < 32; q += 8) {
        const int c = c0 + q;
        const long long r = r0 + threadIdx.x;
        tile[q][threadIdx.x] = (c < w && r < n) ? src[(long long)c * ldc + r] : 0.0;
    }
    __syncthreads();
    for (int q = threadIdx.y; q < 32; q += 8) {
        const long long r = r0 + q;
        const int c = c0 + threadIdx.x;
        if (r < n && c < w) dst[r * ldr + c] = tile[threadIdx.x][q];
    }
}

__global__ void r2c_kernel(long long n, int w, const double* __restrict__ src, long long ldr,
                           double* __restrict__ dst, long long ldc) {
    __shared__ double tile[32][33];
    const long long r0 = (long long)blockIdx.x * 32;
    const int c0 = blockIdx.y * 32;
    for (int q = threadIdx.y; q < 32; q += 8) {
        const long long r = r0 + q;
        const int c = c0 + threadIdx.x;
        tile[q][threadIdx.x] = (r < n && c < w) ? src[r * ldr + c] : 0.0;
    }
    __syncthreads();
    for (int q = threadIdx.y; q < 32; q += 8) {
        const int c = c0 + q;
        const long long r = r0 + threadIdx.x;
        if (c < w && r < n) dst[(long long)c * ldc + r] = tile[threadIdx.x][q];
    }
}

// ---------------------------------------------------------------------------
// Gram product C = U^T V. Workgroup = (row chunk, 96 x 96 output tile); each
// thread keeps a 6 x 6 register tile; 16 rows of U and V are staged in LDS
// per step. Partials per chunk are reduced by gram_reduce_kernel.
constexpr int GT = 96;
constexpr int GK = 16;

__device__ __forceinline__ void tile_decode(int t, int nt_v, int sym, int& ti, int& tj) {
    if (!sym) {
        ti = t / nt_v;
        tj = t % nt_v;
        return;
    }
    int i = 0;
    while (t >= nt_v - i) {
        t -= nt_v - i;
        ++i;
    }
    ti = i;
    tj = i + t;
}

__global__ __launch_bounds__(kThreads) void gram_kernel(long long n, Segs U, Segs V, int mu, int mv,
                                                        int nt_v, int sym, int ntiles,
                                                        long long rows_per_chunk,
                                                        double* __restrict__ part) {
    __shared__ double Us[GK][GT + 2];
    __shared__ double Vs[GK][GT + 2];
    const int lin = xcd_remap(blockIdx.x, gridDim.x);
    const int chunk = lin / ntiles;
    const int tile = lin % ntiles;
    int ti, tj;
    tile_decode(tile, nt_v, sym, ti, tj);
    const long long r0 = (long long)chunk * rows_per_chunk;
    const long long r1 = min(n, r0 + rows_per_chunk);
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int cu0 = ti * GT, cv0 = tj * GT;
    double acc[6][6];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < 6; ++j) acc[i][j] = 0.0;

    for (long long rb = r0; rb < r1; rb += GK) {
#pragma unroll
        for (int q = 0; q < (GK * GT) / kThreads; ++q) {
            const int e = threadIdx.x + kThreads * q;
            const int kk = e / GT, c = e % GT;
            const long long r = rb + kk;
            double u = 0.0, v = 0.0;
            if (r < r1) {
                if (cu0 + c < mu) u = *seg_addr(U, r, cu0 + c);
                if (cv0 + c < mv) v = *seg_addr(V, r, cv0 + c);
            }
            Us[kk][c] = u;
            Vs[kk][c] = v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK; ++kk) {
            double a[6], b[6];
#pragma unroll
            for (int i = 0; i < 6; ++i) a[i] = Us[kk][ty * 6 + i];
#pragma unroll
            for (int j = 0; j < 6; ++j) b[j] = Vs[kk][tx * 6 + j];
#pragma unroll
            for (int i = 0; i < 6; ++i)
#pragma unroll
                for (int j = 0; j < 6; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
    double* P = part + (long long)chunk * mu * mv;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        const int gi = cu0 + ty * 6 + i;
        if (gi >= mu) continue;
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const int gj = cv0 + tx * 6 + j;
            if (gj < mv) P[(long long)gi * mv + gj] = acc[i][j];
        }
    }
}

__global__ __launch_bounds__(kThreads) void gram_reduce_kernel(int mu, int mv, int nchunks, int sym,
                                                               const double* __restrict__ part,
                                                               double* __restrict__ C) {
    const long long idx = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (idx >= (long long)mu * mv) return;
    const int i = (int)(idx / mv), j = (int)(idx % mv);
    const long long stride = (long long)mu * mv;
    auto sum = [&](int a, int b) {
        double s = 0.0;
        const double* p = part + (long long)a * mv + b;
        for (int c = 0; c < nchunks; ++c) s += p[c * stride];
        return s;
    };
    double v;
    if (!sym) {
        v = sum(i, j);
    } else {
        const int ti = i / GT, tj = j / GT;
        if (ti < tj)
            v = sum(i, j);
        else if (ti > tj)
            v = sum(j, i);
        else
            v = 0.5 * (sum(i, j) + sum(j, i));
    }
    C[idx] = v;
}

void gram_plan(long long n, int mu, int mv, int sym, int& ntiles, int& nt_v, int& nchunks,
               long long& rows) {
    const int nt_u = (mu + GT - 1) / GT;
    nt_v = (mv + GT - 1) / GT;
    ntiles = sym ? nt_u * (nt_u + 1) / 2 : nt_u * nt_v;
    long long want = (2048 + ntiles - 1) / ntiles;
    const long long maxc = (n + GK - 1) / GK;
    if (want > maxc) want = maxc;
    if (want < 1) want = 1;
    rows = (n + want - 1) / want;
    rows = (rows + GK - 1) / GK * GK;
    if (rows < GK) rows = GK;
    nchunks = (int)((n + rows - 1) / rows);
    if (nchunks < 1) nchunks = 1;
}

// ---------------------------------------------------------------------------
// Basis update Out = beta Out + alpha U C. Workgroup = 64 rows x 96 output columns;
// each thread keeps a 4 x 6 register tile; K is streamed through LDS in steps
// of 16 together with the matching rows of C.
constexpr int UM = 64;
constexpr int UN = 96;
constexpr int UK = 16;

__global__ __launch_bounds__(kThreads) void update_kernel(long long n, Segs U, int K,
                                                          const double* __restrict__ C, int N,
                                                          Segs O, double alpha, double beta,
                                                          int ntn) {
    __shared__ double Us[UK][UM + 2];
    __shared__ double Cs[UK][UN + 2];
    const int lin = xcd_remap(blockIdx.x, gridDim.x);
    const int rb = lin / ntn, tn = lin % ntn;
    const long long r0 = (long long)rb * UM;
    const int n0 = tn * UN;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    double acc[4][6];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 6; ++j) acc[i][j] = 0.0;

    for (int k0 = 0; k0 < K; k0 += UK) {
#pragma unroll
        for (int q = 0; q < (UM * UK) / kThreads; ++q) {
            const int e = threadIdx.x + kThreads * q;
            const int row = e / UK, kk = e % UK;
            const long long r = r0 + row;
            const int kc = k0 + kk;
            Us[kk][row] = (r < n && kc < K) ? *seg_addr(U, r, kc) : 0.0;
        }
#pragma unroll
        for (int q = 0; q < (UK * UN) / kThreads; ++q) {
            const int e = threadIdx.x + kThreads * q;
            const int kk = e / UN, c = e % UN;
            const int kc = k0 + kk;
            Cs[kk][c] = (kc < K && n0 + c < N) ? C[(long long)kc * N + n0 + c] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < UK; ++kk) {
            double a[4], b[6];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = Us[kk][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 6; ++j) b[j] = Cs[kk][tx * 6 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 6; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const long long r = r0 + ty * 4 + i;
        if (r >= n) continue;
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const int c = n0 + tx * 6 + j;
            if (c >= N) continue;
            double* p = const_cast<double*>(seg_addr(O, r, c));
            *p = (beta != 0.0) ? fma(beta, *p, alpha * acc[i][j]) : alpha * acc[i][j];
        }
    }
}

}  // namespace

// ---------------------------------------------------------------------------
hipError_t launch_spmm(hipStream_t st, int n, const int* rowptr, const int* col, const double* val,
                       const double* X, long long ldx, double* Y, long long ldy, int w) {
    if (n <= 0 || w <= 0) return hipSuccess;
    const int half = (w + 1) / 2;
    if (half <= 1) return spmm_launch<1>(st, n, rowptr, col, val, X, ldx, Y, ldy, w);
    if (half <= 2) return spmm_launch<2>(st, n, rowptr, col, val, X, ldx, Y, ldy, w);
    if (half <= 4) return spmm_launch<4>(st, n, rowptr, col, val, X, ldx, Y, ldy, w);
    if (half <= 8) return spmm_launch<8>(st, n, rowptr, col, val, X, ldx, Y, ldy, w);
    if (half <= 16) return spmm_launch<16>(st, n, rowptr, col, val, X, ldx, Y, ldy, w);
    if (half <= 32) return spmm_launch<32>(st, n, rowptr, col, val, X, ldx, Y, ldy, w);
    return spmm_launch<64>(st, n, rowptr, col, val, X, ldx, Y, ldy, w);
}

hipError_t launch_resid_norms(hipStream_t st, long long n, const double* X, const double* AX,
                              long long ld, int k, const double* lam, double* part, double* out) {
    if (k <= 0) return hipSuccess;
    long long rows = 2048;
    long long nchunks = (n + rows - 1) / rows;
    if (nchunks > 4096) {
        nchunks = 4096;
        rows = (n + nchunks - 1) / nchunks;
        nchunks = (n + rows - 1) / rows;
    }
    if (nchunks < 1) nchunks = 1;
    hipLaunchKernelGGL(resid_norms_kernel, dim3((int)nchunks), dim3(kThreads), 0, st, n, X, AX, ld, k,
                       lam, rows, part);
    hipLaunchKernelGGL(sum_partials_kernel, dim3((2 * k + kThreads - 1) / kThreads), dim3(kThreads), 0,
                       st, 2 * k, (int)nchunks, part, out);
    return hipGetLastError();
}

hipError_t launch_form_w(hipStream_t st, long long n, const double* X, const double* AX,
                         long long ld, const double* lam, const int* act, int a, double* W,
                         long long ldw) {
    if (a <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(form_w_kernel, dim3(grid_for(n * a, kThreads, 16384)), dim3(kThreads), 0, st, n,
                       X, AX, ld, lam, act, a, W, ldw);
    return hipGetLastError();
}

hipError_t launch_shift_sub(hipStream_t st, long long n, double* X, const double* AX, long long ld,
                            int k, double sigma) {
    if (k <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(shift_sub_kernel, dim3(grid_for(n * k, kThreads, 16384)), dim3(kThreads), 0, st,
                       n, X, AX, ld, k, sigma);
    return hipGetLastError();
}

hipError_t launch_copy_cols(hipStream_t st, long long n, const double* src, long long lds, int sc,
                            double* dst, long long ldd, int dc, int w) {
    if (w <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy_cols_kernel, dim3(grid_for(n * w, kThreads, 16384)), dim3(kThreads), 0, st,
                       n, src, lds, sc, dst, ldd, dc, w);
    return hipGetLastError();
}

hipError_t launch_colmajor_to_rowmajor(hipStream_t st, long long n, int w, const double* src,
                                       long long ldc, double* dst, long long ldr) {
    if (w <= 0 || n <= 0) return hipSuccess;
    dim3 grid((unsigned)((n + 31) / 32), (unsigned)((w + 31) / 32));
    hipLaunchKernelGGL(c2r_kernel, grid, dim3(32, 8), 0, st, n, w, src, ldc, dst, ldr);
    return hipGetLastError();
}

hipError_t launch_rowmajor_to_colmajor(hipStream_t st, long long n, int w, const double* src,
                                       long long ldr, double* dst, long long ldc) {
    if (w <= 0 || n <= 0) return hipSuccess;
    dim3 grid((unsigned)((n + 31) / 32), (unsigned)((w + 31) / 32));
    hipLaunchKernelGGL(r2c_kernel, grid, dim3(32, 8), 0, st, n, w, src, ldr, dst, ldc);
    return hipGetLastError();
}

size_t gram_scratch_doubles(long long n, int mu, int mv) {
    size_t best = 0;
    for (int sym = 0; sym < 2; ++sym) {
        if (sym && mu != mv) continue;
        int ntiles, nt_v, nchunks;
        long long rows;
        gram_plan(n, mu, mv, sym, ntiles, nt_v, nchunks, rows);
        best = std::max(best, (size_t)nchunks * (size_t)mu * (size_t)mv);
    }
    return best;
}

hipError_t launch_gram(hipStream_t st, long long n, const Segs& U, const Segs& V, int sym,
                       double* part, double* C) {
    const int mu = segs_width(U), mv = segs_width(V);
    if (mu <= 0 || mv <= 0) return hipSuccess;
    if (sym && mu != mv) sym = 0;
    int ntiles, nt_v, nchunks;
    long long rows;
    gram_plan(n, mu, mv, sym, ntiles, nt_v, nchunks, rows);
    if (n <= 0) {
        hipMemsetAsync(C, 0, sizeof(double) * (size_t)mu * mv, st);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(gram_kernel, dim3(nchunks * ntiles), dim3(kThreads), 0, st, n, U, V, mu, mv,
                       nt_v, sym, ntiles, rows, part);
    const long long total = (long long)mu * mv;
    hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)((total + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, st, mu, mv, nchunks, sym, part, C);
    return hipGetLastError();
}

hipError_t launch_update(hipStream_t st, long long n, const Segs& U, const double* C, int N,
                         const Segs& O, double alpha, double beta) {
    const int K = segs_width(U);
    if (N <= 0 || n <= 0) return hipSuccess;
    const int ntn = (N + UN - 1) / UN;
    const long long nrb = (n + UM - 1) / UM;
    hipLaunchKernelGGL(update_kernel, dim3((unsigned)(nrb * ntn)), dim3(kThreads), 0, st, n, U, K, C, N,
                       O, alpha, beta, ntn);
    return hipGetLastError();
}

}  // namespace se
