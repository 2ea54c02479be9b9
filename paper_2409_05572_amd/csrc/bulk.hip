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
// adjacent columns (one 16-byte load per gathered row of X). A lane group
// walks SPR consecutive rows two at a time. For each batch it first loads the
// column indices and values of up to eight nonzeros of both rows, then issues
// all sixteen row gathers, then accumulates: a 7-point row needs two memory
// round trips, not fourteen. Slots past the end of a row gather the row
// itself with weight zero (always a valid address). With an odd width the
// last lane also reads the padding column (ld >= w + 1) and stores only its
// first value.
constexpr int SPR = 8;  // rows per lane group
constexpr int SB = 8;   // nonzeros per row per batch

__device__ __forceinline__ void spmm_row_pair(int ra, int rb, const int* __restrict__ rowptr,
                                              const int* __restrict__ col,
                                              const double* __restrict__ val,
                                              const double* __restrict__ X, long long ldx,
                                              double* __restrict__ Y, long long ldy, int c0,
                                              bool pair_col) {
    const int ba = rowptr[ra];
    int ea = rowptr[ra + 1];
    const bool heavy_a = ea - ba > kHeavyRow;  // computed by spmm_heavy_kernel
    if (heavy_a) ea = ba;
    const bool hasb0 = rb >= 0;
    const int rbs = hasb0 ? rb : ra;
    const int bb = hasb0 ? rowptr[rbs] : 0;
    int eb = hasb0 ? rowptr[rbs + 1] : 0;
    if (eb - bb > kHeavyRow) eb = bb;
    const bool hasb = hasb0 && rowptr[rbs + 1] - bb <= kHeavyRow;
    double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0;
    for (int pa = ba, pb = bb; pa < ea || pb < eb; pa += SB, pb += SB) {
        int ja[SB], jb[SB];
        double va[SB], vb[SB];
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const bool oka = pa + u < ea, okb = pb + u < eb;
            ja[u] = oka ? col[pa + u] : ra;
            va[u] = oka ? val[pa + u] : 0.0;
            jb[u] = okb ? col[pb + u] : rbs;
            vb[u] = okb ? val[pb + u] : 0.0;
        }
        double2 xa[SB], xb[SB];
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            xa[u] = *reinterpret_cast<const double2*>(X + (long long)ja[u] * ldx + c0);
            xb[u] = *reinterpret_cast<const double2*>(X + (long long)jb[u] * ldx + c0);
        }
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            a0 = fma(va[u], xa[u].x, a0);
            a1 = fma(va[u], xa[u].y, a1);
            b0 = fma(vb[u], xb[u].x, b0);
            b1 = fma(vb[u], xb[u].y, b1);
        }
    }
    if (pair_col) {
        if (!heavy_a) *reinterpret_cast<double2*>(Y + (long long)ra * ldy + c0) = make_double2(a0, a1);
        if (hasb) *reinterpret_cast<double2*>(Y + (long long)rb * ldy + c0) = make_double2(b0, b1);
    } else {
        if (!heavy_a) Y[(long long)ra * ldy + c0] = a0;
        if (hasb) Y[(long long)rb * ldy + c0] = b0;
    }
}

// One long row per workgroup: the kThreads / LPR lane groups take batches of
// SB nonzeros in turn (same column mapping as spmm_kernel), and group 0 sums
// the partial rows from LDS in a fixed order.
template <int LPR>
__global__ __launch_bounds__(kThreads) void spmm_heavy_kernel(const int* __restrict__ heavy,
                                                              const int* __restrict__ rowptr,
                                                              const int* __restrict__ col,
                                                              const double* __restrict__ val,
                                                              const double* __restrict__ X, long long ldx,
                                                              double* __restrict__ Y, long long ldy, int w) {
    constexpr int G = kThreads / LPR;
    __shared__ double2 red[G][LPR];
    const int row = heavy[blockIdx.x];
    const int g = threadIdx.x / LPR, lane = threadIdx.x % LPR;
    const int b = rowptr[row], e = rowptr[row + 1];
    for (int cb = 0; cb < w; cb += 2 * LPR) {
        const int c0 = cb + 2 * lane;
        double a0 = 0.0, a1 = 0.0;
        if (c0 < w) {
            for (int p = b + g * SB; p < e; p += G * SB) {
                int j[SB];
                double v[SB];
#pragma unroll
                for (int u = 0; u < SB; ++u) {
                    const bool ok = p + u < e;
                    j[u] = ok ? col[p + u] : row;
                    v[u] = ok ? val[p + u] : 0.0;
                }
                double2 x[SB];
#pragma unroll
                for (int u = 0; u < SB; ++u) x[u] = *reinterpret_cast<const double2*>(X + (long long)j[u] * ldx + c0);
#pragma unroll
                for (int u = 0; u < SB; ++u) {
                    a0 = fma(v[u], x[u].x, a0);
                    a1 = fma(v[u], x[u].y, a1);
                }
            }
        }
        red[g][lane] = make_double2(a0, a1);
        __syncthreads();
        if (g == 0 && c0 < w) {
            double s0 = 0.0, s1 = 0.0;
            for (int q = 0; q < G; ++q) {
                s0 += red[q][lane].x;
                s1 += red[q][lane].y;
            }
            Y[(long long)row * ldy + c0] = s0;
            if (c0 + 1 < w) Y[(long long)row * ldy + c0 + 1] = s1;
        }
        __syncthreads();
    }
}

template <int LPR>
__global__ __launch_bounds__(kThreads) void spmm_kernel(int n, const int* __restrict__ rowptr,
                                                        const int* __restrict__ col,
                                                        const double* __restrict__ val,
                                                        const double* __restrict__ X, long long ldx,
                                                        double* __restrict__ Y, long long ldy,
                                                        int w) {
    constexpr int GPB = kThreads / LPR;  // lane groups per workgroup
    // Plain round-robin dealing: all XCDs work on neighbouring row blocks, so
    // the planes a stencil row reaches stay in the shared last-level cache
    // (measured 8% faster than contiguous per-XCD ranges at 2.1M rows).
    const int blk = blockIdx.x;
    const int sub = threadIdx.x / LPR;
    const int lane = threadIdx.x % LPR;
    const int rbeg = (blk * GPB + sub) * SPR;
    if (rbeg >= n) return;
    const int rend = min(n, rbeg + SPR);
    for (int c0 = 2 * lane; c0 < w; c0 += 2 * LPR) {
        const bool pair_col = c0 + 1 < w;
        for (int r = rbeg; r < rend; r += 2)
            spmm_row_pair(r, r + 1 < rend ? r + 1 : -1, rowptr, col, val, X, ldx, Y, ldy, c0,
                          pair_col);
    }
}

// CSR x block for matrices without heavy rows: one wave per run of
// kStreamRows consecutive rows walks the run's nonzeros in order, NB at a
// time. Their column indices and values are uniform over the wave (scalar
// loads; the arrays are padded by kCsrPad entries), all NB row gathers of X
// (16 bytes per lane) are issued before any is used, and the accumulator
// moves to the next row, storing the finished one, at each row boundary, so
// NB gathers are in flight whatever the row lengths. The run's row offsets
// sit one per lane and are read with readlane. Lane l owns columns
// cb + 2l, cb + 2l + 1 of each 128-column block (an odd width reads the
// padding column, ld >= w + 1, and stores one value).
constexpr int kStreamRows = 32;

// Body of one wave; `wid_in` is the wave's index over the row runs.
template <int NB>
__device__ __forceinline__ void spmm_stream_body(int wid_in, int n, const int* __restrict__ rowptr,
                                                 const int* __restrict__ col, const double* __restrict__ val,
                                                 const double* __restrict__ X, long long ldx,
                                                 double* __restrict__ Y, long long ldy, int w) {
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(wid_in);
    if ((long long)wid * kStreamRows >= n) return;
    const int r0 = wid * kStreamRows;
    const int r1 = min(n, r0 + kStreamRows);
    const int rp = rowptr[min(r0 + lane, r1)];  // lane q: offset of row r0 + q, q <= r1 - r0
    const int pbeg = __builtin_amdgcn_readlane(rp, 0);
    const int pend = __builtin_amdgcn_readlane(rp, r1 - r0);
    for (int cb = 0; cb < w; cb += 128) {
        const int c0 = cb + 2 * lane;
        const bool has0 = c0 < w, has1 = c0 + 1 < w;
        const long long cc = has0 ? c0 : cb;  // lanes without columns read a valid address
        int r = r0;
        int rend = __builtin_amdgcn_readlane(rp, 1);
        double a0 = 0.0, a1 = 0.0;
        auto flush = [&]() {
            double* y = Y + (long long)r * ldy + c0;
            if (has1)
                *reinterpret_cast<double2*>(y) = make_double2(a0, a1);
            else if (has0)
                *y = a0;
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
            for (int u = 0; u < NB; ++u) x[u] = *reinterpret_cast<const double2*>(X + (long long)j[u] * ldx + cc);
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

template <int NB>
__global__ __launch_bounds__(kThreads) void spmm_stream_kernel(int n, const int* __restrict__ rowptr,
                                                               const int* __restrict__ col,
                                                               const double* __restrict__ val,
                                                               const double* __restrict__ X, long long ldx,
                                                               double* __restrict__ Y, long long ldy, int w) {
    spmm_stream_body<NB>((int)blockIdx.x * (kThreads / 64) + (int)(threadIdx.x >> 6), n, rowptr, col, val, X, ldx,
                         Y, ldy, w);
}

// The streaming product with the residual of every row it produces: when row
// r is complete, R[r] = Y[r] - lam X[r] is written and r^2, x^2 are
// accumulated per column. X[r] is the row's own gather when the row stores
// its diagonal entry (captured by a wave-uniform compare of the column index),
// else it is loaded at that point. The per-column sums over the workgroup's
// rows go to part[blockIdx.x * 2w + c] (r^2) and part[blockIdx.x * 2w + w + c]
// (x^2), the four waves summed in a fixed order. Requires w <= 128.
__global__ __launch_bounds__(kThreads) void spmm_resid_kernel(int n, const int* __restrict__ rowptr,
                                                              const int* __restrict__ col,
                                                              const double* __restrict__ val,
                                                              const double* __restrict__ X, long long ldx,
                                                              double* __restrict__ Y, long long ldy, int w,
                                                              const double* __restrict__ lam,
                                                              double* __restrict__ R, long long ldr,
                                                              double* __restrict__ part) {
    constexpr int NB = 16;
    __shared__ double4 red[kThreads];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int wid = __builtin_amdgcn_readfirstlane((int)blockIdx.x * (kThreads / 64) + wv);
    const int c0 = 2 * lane;
    const bool has0 = c0 < w, has1 = c0 + 1 < w;
    double sr0 = 0.0, sr1 = 0.0, sx0 = 0.0, sx1 = 0.0;
    if ((long long)wid * kStreamRows < n) {
        const int r0 = wid * kStreamRows;
        const int r1 = min(n, r0 + kStreamRows);
        const int rp = rowptr[min(r0 + lane, r1)];
        const int pbeg = __builtin_amdgcn_readlane(rp, 0);
        const int pend = __builtin_amdgcn_readlane(rp, r1 - r0);
        const long long cc = has0 ? c0 : 0;
        const double l0 = has0 ? lam[c0] : 0.0, l1 = has1 ? lam[c0 + 1] : 0.0;
        int r = r0;
        int rend = __builtin_amdgcn_readlane(rp, 1);
        double a0 = 0.0, a1 = 0.0, xr0 = 0.0, xr1 = 0.0;
        bool diag = false;  // uniform: X[r] captured from the row's own gather
        auto flush = [&]() {
            if (!diag) {
                const double2 xv = *reinterpret_cast<const double2*>(X + (long long)r * ldx + cc);
                xr0 = xv.x;
                xr1 = xv.y;
            }
            const double q0 = a0 - l0 * xr0, q1 = a1 - l1 * xr1;
            double* y = Y + (long long)r * ldy + c0;
            double* rr = R + (long long)r * ldr + c0;
            if (has1) {
                *reinterpret_cast<double2*>(y) = make_double2(a0, a1);
                *reinterpret_cast<double2*>(rr) = make_double2(q0, q1);
            } else if (has0) {
                *y = a0;
                *rr = q0;
            }
            sr0 = fma(q0, q0, sr0);
            sr1 = fma(q1, q1, sr1);
            sx0 = fma(xr0, xr0, sx0);
            sx1 = fma(xr1, xr1, sx1);
            a0 = 0.0;
            a1 = 0.0;
            diag = false;
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
            for (int u = 0; u < NB; ++u) x[u] = *reinterpret_cast<const double2*>(X + (long long)j[u] * ldx + cc);
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                if (p + u < pend) {
                    while (p + u >= rend) flush();
                    a0 = fma(v[u], x[u].x, a0);
                    a1 = fma(v[u], x[u].y, a1);
                    if (j[u] == r) {
                        xr0 = x[u].x;
                        xr1 = x[u].y;
                        diag = true;
                    }
                }
            }
        }
        while (r < r1) flush();
    }
    red[threadIdx.x] = make_double4(sr0, sr1, sx0, sx1);
    __syncthreads();
    if (wv == 0) {
        double4 t = red[lane];
#pragma unroll
        for (int q = 1; q < kThreads / 64; ++q) {
            const double4 u = red[q * 64 + lane];
            t.x += u.x;
            t.y += u.y;
            t.z += u.z;
            t.w += u.w;
        }
        double* out = part + (long long)blockIdx.x * 2 * w;
        if (has0) {
            out[c0] = t.x;
            out[w + c0] = t.z;
        }
        if (has1) {
            out[c0 + 1] = t.y;
            out[w + c0 + 1] = t.w;
        }
    }
}

template <int LPR>
hipError_t spmm_launch(hipStream_t st, int n, const int* rowptr, const int* col, const double* val,
                       const double* X, long long ldx, double* Y, long long ldy, int w, const int* heavy,
                       int n_heavy) {
    constexpr int RPB = (kThreads / LPR) * SPR;
    const int grid = (n + RPB - 1) / RPB;
    hipLaunchKernelGGL(spmm_kernel<LPR>, dim3(grid), dim3(kThreads), 0, st, n, rowptr, col, val, X,
                       ldx, Y, ldy, w);
    if (n_heavy > 0)
        hipLaunchKernelGGL(spmm_heavy_kernel<LPR>, dim3(n_heavy), dim3(kThreads), 0, st, heavy, rowptr, col,
                           val, X, ldx, Y, ldy, w);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed-order sum of per-chunk partial vectors: out[i] = sum_c part[c * L + i].
// out[i] = sum_c part[c rs + i] (rs: row stride of the partials, at least L).
// 32 threads per output, 8 outputs per workgroup (consecutive threads take
// consecutive outputs, so each chunk's read is contiguous): thread g sums
// chunks g, g + 32, ... in increasing order and a fixed tree combines the 32
// sums (deterministic).
constexpr int kSumG = 32;
__device__ __forceinline__ void sum_partials_body(int bx, int L, int nchunks, const double* __restrict__ part,
                                                  double* __restrict__ out, long long rs) {
    constexpr int OPB = kThreads / kSumG;
    __shared__ double sh[kThreads];
    const int o = threadIdx.x % OPB, g = threadIdx.x / OPB;
    const int i = bx * OPB + o;
    double s0 = 0.0, s1 = 0.0;
    if (i < L) {
        int c = g;
        for (; c + kSumG < nchunks; c += 2 * kSumG) {
            s0 += part[(long long)c * rs + i];
            s1 += part[(long long)(c + kSumG) * rs + i];
        }
        if (c < nchunks) s0 += part[(long long)c * rs + i];
    }
    sh[threadIdx.x] = s0 + s1;
    __syncthreads();
#pragma unroll
    for (int h = kSumG / 2; h > 0; h >>= 1) {
        if (g < h) sh[g * OPB + o] += sh[(g + h) * OPB + o];
        __syncthreads();
    }
    if (g == 0 && i < L) out[i] = sh[o];
}

__global__ __launch_bounds__(kThreads) void sum_partials_kernel(int L, int nchunks,
                                                                const double* __restrict__ part,
                                                                double* __restrict__ out, long long rs) {
    sum_partials_body(blockIdx.x, L, nchunks, part, out, rs);
}

// First level for many chunks: workgroup (x, y) sums chunks y kSumBlk ..
// y kSumBlk + kSumBlk - 1 of outputs 16 x .. 16 x + 15 and overwrites that
// block's first partial row with the result. 16 threads per output, each
// with four running sums over its chunks g, g + 16, ... (in increasing order,
// chunk 64 u + 16 q + g into sum q), combined by a fixed tree: the same
// inputs always give the same bits. Only this workgroup reads the block's
// rows in these columns, so the write after its last read is safe.
constexpr int kSumBlk = 512;
__global__ __launch_bounds__(kThreads) void sum_blocks_kernel(int L, int nchunks, double* __restrict__ part) {
    constexpr int OPB = 16, G = kThreads / OPB;
    __shared__ double sh[kThreads];
    const int o = threadIdx.x % OPB, g = threadIdx.x / OPB;
    const int i = (int)blockIdx.x * OPB + o;
    const long long c0 = (long long)blockIdx.y * kSumBlk;
    const int cn = (int)min((long long)kSumBlk, (long long)nchunks - c0);
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < L) {
        int c = g;
        for (; c + 3 * G < cn; c += 4 * G) {
#pragma unroll
            for (int q = 0; q < 4; ++q) s[q] += part[(c0 + c + q * G) * L + i];
        }
#pragma unroll
        for (int q = 0; q < 3; ++q)
            if (c + q * G < cn) s[q] += part[(c0 + c + q * G) * L + i];
    }
    sh[threadIdx.x] = (s[0] + s[1]) + (s[2] + s[3]);
    __syncthreads();
#pragma unroll
    for (int h = G / 2; h > 0; h >>= 1) {
        if (g < h) sh[g * OPB + o] += sh[(g + h) * OPB + o];
        __syncthreads();
    }
    if (g == 0 && i < L) part[c0 * L + i] = sh[o];
}

// Residual and column norms: per chunk of rows, sum (ax - lam x)^2 and x^2.
// With R != nullptr the residual rows are written there as well.
__device__ __forceinline__ void resid_norms_body(int chunk, long long n, const double* __restrict__ X,
                                                 const double* __restrict__ AX, long long ld, int k,
                                                 const double* __restrict__ lam, long long rows_per_chunk,
                                                 double* __restrict__ part, double* __restrict__ R,
                                                 long long ldr) {
    __shared__ double sr[kThreads];
    __shared__ double sx[kThreads];
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
                if (R) R[r * ldr + c] = y;
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
                if (R) R[r * ldr + c] = y;
                ar = fma(y, y, ar);
                axx = fma(x, x, axx);
            }
            out[c] = ar;
            out[k + c] = axx;
        }
    }
}

__global__ __launch_bounds__(kThreads) void resid_norms_kernel(long long n, const double* __restrict__ X,
                                                               const double* __restrict__ AX,
                                                               long long ld, int k,
                                                               const double* __restrict__ lam,
                                                               long long rows_per_chunk,
                                                               double* __restrict__ part,
                                                               double* __restrict__ R, long long ldr) {
    resid_norms_body(blockIdx.x, n, X, AX, ld, k, lam, rows_per_chunk, part, R, ldr);
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

__global__ __launch_bounds__(kThreads) void gather_cols_kernel(long long n, const double* __restrict__ src,
                                                               long long lds, const int* __restrict__ idx,
                                                               int a, double* __restrict__ dst,
                                                               long long ldd) {
    const long long total = n * a;
    for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < total;
         e += (long long)gridDim.x * kThreads) {
        const long long r = e / a;
        const int q = (int)(e - r * a);
        dst[r * ldd + q] = src[r * lds + idx[q]];
    }
}

__global__ __launch_bounds__(kThreads) void shift_sub_kernel(long long n, double* __restrict__ X,
                                                             const double* __restrict__ AX,
                                                             long long ld, int k, double sigma,
                                                             double scale) {
    const long long total = n * k;
    for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < total;
         e += (long long)gridDim.x * kThreads) {
        const long long r = e / k;
        const int c = (int)(e - r * k);
        X[r * ld + c] = scale * (sigma * X[r * ld + c] - AX[r * ld + c]);
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
// FP64 matrix cores. v_mfma_f64_16x16x4 computes D[16x16] += A[16x4] B[4x16];
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16], and holds
// D[l / 16 + 4 r][l % 16] in accumulator register r (checked on gfx950).
typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Gram product C = U^T V. Workgroup = (row chunk, 96 x 96 output tile); the
// four waves split the tile 2 x 2 and each accumulates 3 x 3 MFMA tiles. Rows
// are the contraction index: 16 rows of U and V are staged in LDS per step.
// Per-chunk partials are summed by gram_reduce_kernel in a fixed order.
constexpr int GT = kGramTile;
constexpr int GK = kGramRows;

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

__device__ __forceinline__ const double* seg_col(const Segs& S, int c, bool& ok) {
    ok = c < S.off[S.nseg];
    if (!ok) return S.p[0];
    const double* p = S.p[0];
    int o = 0;
    if (S.nseg > 1 && c >= S.off[1]) { p = S.p[1]; o = S.off[1]; }
    if (S.nseg > 2 && c >= S.off[2]) { p = S.p[2]; o = S.off[2]; }
    if (S.nseg > 3 && c >= S.off[3]) { p = S.p[3]; o = S.off[3]; }
    return p + (c - o);
}

// MFMA work of one stage for a wave whose 48 x 48 block has NI x NJ tiles
// with data (the others are skipped).
template <int NI, int NJ>
__device__ __forceinline__ void gram_compute(const double (*Ts)[2 * GT + 4], d4 (&acc)[3][3], int lr,
                                             int lc, int wy, int wx) {
#pragma unroll
    for (int ks = 0; ks < GK; ks += 4) {
        double a[NI], b[NJ];
#pragma unroll
        for (int i = 0; i < NI; ++i) a[i] = Ts[ks + lr][wy * 48 + i * 16 + lc];
#pragma unroll
        for (int j = 0; j < NJ; ++j) b[j] = Ts[ks + lr][GT + wx * 48 + j * 16 + lc];
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
            for (int j = 0; j < NJ; ++j) acc[i][j] = mfma16(a[i], b[j], acc[i][j]);
    }
}

// Diagonal tiles of symmetric products: only the 21 upper 16 x 16 MFMA tiles
// (I <= J) of the 6 x 6 grid are formed, 6/5/5/5 per wave by tile rows
// (wave 0: row 0; 1: row 1; 2: rows 2 and 5; 3: rows 3 and 4). Tile (I, J0 + q)
// accumulates in slot S0 + q of acc; nv = tile rows/columns holding data.
template <int I, int J0, int NJ, int S0>
__device__ __forceinline__ void gram_diag_row(const double (*Ts)[2 * GT + 4], d4 (&acc)[3][3], int ks, int lr,
                                              int lc, int nv, int boff) {
    if (I >= nv) return;
    const double a = Ts[ks + lr][I * 16 + lc];
#pragma unroll
    for (int q = 0; q < NJ; ++q) {
        if (J0 + q < nv) {
            const double b = Ts[ks + lr][boff + (J0 + q) * 16 + lc];
            acc[(S0 + q) / 3][(S0 + q) % 3] = mfma16(a, b, acc[(S0 + q) / 3][(S0 + q) % 3]);
        }
    }
}

template <int WV>
__device__ __forceinline__ void gram_diag_stage(const double (*Ts)[2 * GT + 4], d4 (&acc)[3][3], int lr, int lc,
                                                int nv, int boff) {
#pragma unroll
    for (int ks = 0; ks < GK; ks += 4) {
        if (WV == 0) gram_diag_row<0, 0, 6, 0>(Ts, acc, ks, lr, lc, nv, boff);
        if (WV == 1) gram_diag_row<1, 1, 5, 0>(Ts, acc, ks, lr, lc, nv, boff);
        if (WV == 2) {
            gram_diag_row<2, 2, 4, 0>(Ts, acc, ks, lr, lc, nv, boff);
            gram_diag_row<5, 5, 1, 4>(Ts, acc, ks, lr, lc, nv, boff);
        }
        if (WV == 3) {
            gram_diag_row<3, 3, 3, 0>(Ts, acc, ks, lr, lc, nv, boff);
            gram_diag_row<4, 4, 2, 3>(Ts, acc, ks, lr, lc, nv, boff);
        }
    }
}

// U and V are the same blocks (W^T W): a diagonal tile then needs one operand.
__device__ __forceinline__ bool segs_same(const Segs& A, const Segs& B) {
    if (A.nseg != B.nseg || A.ld != B.ld) return false;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (q < A.nseg && (A.p[q] != B.p[q] || A.off[q + 1] != B.off[q + 1])) return false;
    return true;
}

// (I, J) of slot s of wave wv in a diagonal tile; false if the slot is unused.
__device__ __forceinline__ bool gram_diag_slot(int wv, int s, int& I, int& J) {
    if (wv == 0) { I = 0; J = s; return s < 6; }
    if (wv == 1) { I = 1; J = 1 + s; return s < 5; }
    if (wv == 2) {
        if (s < 4) { I = 2; J = 2 + s; return true; }
        I = 5; J = 5; return s == 4;
    }
    if (s < 3) { I = 3; J = 3 + s; return true; }
    I = 4; J = 4 + (s - 3); return s < 5;
}

// Loads of one stage: the U tile (GK rows x 96) and the V tile (GK x 96) form
// a GK x 192 array. Thread t owns columns t%64, t%64+64, t%64+128 and rows
// t/64 + 4i, so its three column pointers are fixed for the whole chunk and a
// wave reads 64 consecutive columns of one row.
__device__ __forceinline__ void gram_body(int chunk, int tile, long long n, const Segs& U, const Segs& V, int mu,
                                          int mv, int nt_v, int sym, long long rows_per_chunk,
                                          double* __restrict__ part) {
    constexpr int RPT = GK / 4;  // rows per thread per stage (8)
    __shared__ double Ts[GK][2 * GT + 4];  // [row][0..95 U | 96..191 V]
    int ti, tj;
    tile_decode(tile, nt_v, sym, ti, tj);
    const long long r0 = (long long)chunk * rows_per_chunk;
    const long long r1 = min(n, r0 + rows_per_chunk);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int wy = wv >> 1, wx = wv & 1;
    const int cu0 = ti * GT, cv0 = tj * GT;
    const int lr = lane >> 4, lc = lane & 15;
    const int niv = max(0, min(3, (mu - cu0 - wy * 48 + 15) / 16));
    const int njv = max(0, min(3, (mv - cv0 - wx * 48 + 15) / 16));
    // symmetric diagonal tile: triangular split (shape -1 .. -4 = wave 0 .. 3)
    const bool diag = sym && ti == tj;
    const int nv = min(6, (mu - cu0 + 15) / 16);
    const int shape = diag ? -1 - wv : niv * 4 + njv;
    // same operand on a diagonal tile: only the U half is loaded, and the
    // MFMAs read both operands from it
    const bool dup = diag && segs_same(U, V);
    const int boff = dup ? 0 : GT;

    // fixed column pointers of this thread (c < 96: U, else V)
    const double* cp[3];
    bool cok[3];
    long long cld[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int c = lane + 64 * q;
        if (c < GT) {
            cp[q] = seg_col(U, cu0 + c, cok[q]);
            cld[q] = U.ld;
        } else {
            cp[q] = seg_col(V, cv0 + c - GT, cok[q]);
            cok[q] = cok[q] && !dup;
            cld[q] = V.ld;
        }
    }
    d4 acc[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    double rg[RPT][3];

    auto fetch = [&](long long rb) {
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const long long r = rb + wv + 4 * i;
            const bool rok = r < r1;
#pragma unroll
            for (int q = 0; q < 3; ++q) rg[i][q] = (rok && cok[q]) ? cp[q][r * cld[q]] : 0.0;
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int i = 0; i < RPT; ++i)
#pragma unroll
            for (int q = 0; q < 3; ++q) Ts[wv + 4 * i][lane + 64 * q] = rg[i][q];
    };

    if (r0 < r1) {
        fetch(r0);
        stash();
    }
    __syncthreads();
    for (long long rb = r0; rb < r1; rb += GK) {
        const bool more = rb + GK < r1;
        if (more) fetch(rb + GK);
        switch (shape) {  // uniform per wave: skip MFMA tiles without data
            case 15: gram_compute<3, 3>(Ts, acc, lr, lc, wy, wx); break;
            case 14: gram_compute<3, 2>(Ts, acc, lr, lc, wy, wx); break;
            case 13: gram_compute<3, 1>(Ts, acc, lr, lc, wy, wx); break;
            case 11: gram_compute<2, 3>(Ts, acc, lr, lc, wy, wx); break;
            case 10: gram_compute<2, 2>(Ts, acc, lr, lc, wy, wx); break;
            case 9: gram_compute<2, 1>(Ts, acc, lr, lc, wy, wx); break;
            case 7: gram_compute<1, 3>(Ts, acc, lr, lc, wy, wx); break;
            case 6: gram_compute<1, 2>(Ts, acc, lr, lc, wy, wx); break;
            case 5: gram_compute<1, 1>(Ts, acc, lr, lc, wy, wx); break;
            case -1: gram_diag_stage<0>(Ts, acc, lr, lc, nv, boff); break;
            case -2: gram_diag_stage<1>(Ts, acc, lr, lc, nv, boff); break;
            case -3: gram_diag_stage<2>(Ts, acc, lr, lc, nv, boff); break;
            case -4: gram_diag_stage<3>(Ts, acc, lr, lc, nv, boff); break;
            default: break;
        }
        __syncthreads();
        if (more) {
            stash();
            __syncthreads();
        }
    }
    double* P = part + (long long)chunk * mu * mv;
    if (diag) {
#pragma unroll
        for (int sl = 0; sl < 9; ++sl) {
            int I, J;
            if (!gram_diag_slot(wv, sl, I, J)) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gi = cu0 + I * 16 + lr + 4 * r;
                const int gj = cv0 + J * 16 + lc;
                if (gi < mu && gj < mv) P[(long long)gi * mv + gj] = acc[sl / 3][sl % 3][r];
            }
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gi = cu0 + wy * 48 + i * 16 + lr + 4 * r;
                const int gj = cv0 + wx * 48 + j * 16 + lc;
                if (gi < mu && gj < mv) P[(long long)gi * mv + gj] = acc[i][j][r];
            }
}

__global__ __launch_bounds__(kThreads, 2) void gram_kernel(long long n, Segs U, Segs V, int mu, int mv,
                                                        int nt_v, int sym, int ntiles,
                                                        long long rows_per_chunk,
                                                        double* __restrict__ part) {
    const int lin = xcd_remap(blockIdx.x, gridDim.x);
    gram_body(lin / ntiles, lin % ntiles, n, U, V, mu, mv, nt_v, sym, rows_per_chunk, part);
}

// C = sum over chunks of the partial Gram products. 16 threads per output
// and 16 outputs per workgroup (consecutive threads on consecutive outputs):
// thread g sums chunks g, g + 16, ... in increasing order and a fixed tree
// combines the 16 sums (deterministic). Symmetric products (partials hold
// at least every 16 x 16 block on or above the diagonal): outputs below the
// diagonal blocks take the mirrored sum, diagonal 16 x 16 blocks average
// (i, j) and (j, i).
constexpr int kRedG = 16;
__device__ __forceinline__ void gram_reduce_body(int bx, int mu, int mv, int nchunks, int sym,
                                                 const double* __restrict__ part, double* __restrict__ C) {
    constexpr int OPB = kThreads / kRedG;
    __shared__ double sa[kThreads];
    __shared__ double sb[kThreads];
    const int o = threadIdx.x % OPB, g = threadIdx.x / OPB;
    const long long total = (long long)mu * mv;
    const long long idx = (long long)bx * OPB + o;
    const bool valid = idx < total;
    int mode = 0;  // 0: sum (i, j); 1: sum (j, i); 2: average of both
    long long p1 = idx, p2 = idx;
    if (valid) {
        const int i = (int)(idx / mv), j = (int)(idx % mv);
        if (sym) {
            const int ti = i / 16, tj = j / 16;
            mode = ti < tj ? 0 : (ti > tj ? 1 : 2);
            p2 = (long long)j * mv + i;
            if (mode == 1) p1 = p2;
        }
    }
    double s1 = 0.0, s2 = 0.0;
    if (valid) {
        for (int c = g; c < nchunks; c += kRedG) {
            s1 += part[(long long)c * total + p1];
            if (mode == 2) s2 += part[(long long)c * total + p2];
        }
    }
    sa[threadIdx.x] = s1;
    sb[threadIdx.x] = s2;
    __syncthreads();
#pragma unroll
    for (int h = kRedG / 2; h > 0; h >>= 1) {
        if (g < h) {
            sa[g * OPB + o] += sa[(g + h) * OPB + o];
            sb[g * OPB + o] += sb[(g + h) * OPB + o];
        }
        __syncthreads();
    }
    if (g == 0 && valid) C[idx] = (mode == 2) ? 0.5 * (sa[o] + sb[o]) : sa[o];
}

__global__ __launch_bounds__(kThreads) void gram_reduce_kernel(int mu, int mv, int nchunks, int sym,
                                                               const double* __restrict__ part,
                                                               double* __restrict__ C) {
    gram_reduce_body(blockIdx.x, mu, mv, nchunks, sym, part, C);
}

}  // namespace

void gram_plan(long long n, int mu, int mv, int sym, int& ntiles, int& nt_v, int& nchunks,
               long long& rows, long long max_chunks) {
    const int nt_u = (mu + GT - 1) / GT;
    nt_v = (mv + GT - 1) / GT;
    ntiles = sym ? nt_u * (nt_u + 1) / 2 : nt_u * nt_v;
    // Two full waves of resident workgroups (2 per CU x 256 CUs, twice), never
    // more: a partly filled last wave leaves most CUs idle while it runs.
    long long want = 1024 / ntiles;
    const long long maxc = (n + 255) / 256;        // at least 256 rows per chunk
    if (want > maxc) want = maxc;
    if (max_chunks > 0 && want > max_chunks) want = max_chunks;  // bounded scratch
    if (want < 1) want = 1;
    rows = (n + want - 1) / want;
    rows = (rows + GK - 1) / GK * GK;
    if (rows < GK) rows = GK;
    nchunks = (int)((n + rows - 1) / rows);
    if (nchunks < 1) nchunks = 1;
}

namespace {

// ---------------------------------------------------------------------------
// Basis update Out = beta Out + alpha U C. Workgroup = 64 rows x (16 NT)
// output columns; wave w owns rows 16w..16w+15 and NT MFMA tiles along N. K is
// streamed through LDS 32 at a time with the matching rows of C; the global
// loads of the next stage are issued into registers before the MFMAs of the
// current stage, so their latency overlaps the matrix-core work. Up to 96
// output columns (NT <= 6) three workgroups share a CU (43 KB of LDS and at
// most 168 VGPRs each): 5-9% faster than two at K x N = 96..288 x 96.
constexpr int UM = 64;
constexpr int UK = 32;

template <int NT>
__device__ __forceinline__ void update_body(int rb, int tn, long long n, const Segs& U, int K,
                                            const double* __restrict__ C, int N, const Segs& O, double alpha,
                                            double beta) {
    constexpr int BN = 16 * NT;
    constexpr int UQ = (UM * UK) / kThreads;  // U elements per thread per stage (8)
    constexpr int CQ = (UK * BN) / kThreads;  // C elements per thread per stage (2 NT)
    // odd row stride: the transposing stores of a stage (32 lanes on 32
    // consecutive k rows, one column) then fall on distinct bank pairs
    __shared__ double Us[UK][UM + 1];
    __shared__ double Cs[UK][BN + 4];
    const long long r0 = (long long)rb * UM;
    const int n0 = tn * BN;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane >> 4, lc = lane & 15;
    d4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
    double ru[UQ], rc[CQ];

    // U loads: thread t owns k-column t % UK and rows t / UK + 8 i of a stage;
    // its segment pointer is resolved once per stage.
    auto fetch = [&](int k0) {
        bool ok;
        const double* up = seg_col(U, k0 + (int)(threadIdx.x % UK), ok);
#pragma unroll
        for (int q = 0; q < UQ; ++q) {
            const long long r = r0 + threadIdx.x / UK + (kThreads / UK) * q;
            ru[q] = (ok && r < n) ? up[r * U.ld] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < CQ; ++q) {
            const int e = threadIdx.x + kThreads * q;
            const int kk = e / BN, c = e % BN;
            const int kc = k0 + kk;
            rc[q] = (kc < K && n0 + c < N) ? C[(long long)kc * N + n0 + c] : 0.0;
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int q = 0; q < UQ; ++q)
            Us[threadIdx.x % UK][threadIdx.x / UK + (kThreads / UK) * q] = ru[q];
#pragma unroll
        for (int q = 0; q < CQ; ++q) {
            const int e = threadIdx.x + kThreads * q;
            Cs[e / BN][e % BN] = rc[q];
        }
    };

    fetch(0);
    stash();
    __syncthreads();
    for (int k0 = 0; k0 < K; k0 += UK) {
        const bool more = k0 + UK < K;
        if (more) fetch(k0 + UK);
#pragma unroll
        for (int ks = 0; ks < UK; ks += 4) {
            const double a = Us[ks + lr][wv * 16 + lc];
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = mfma16(a, Cs[ks + lr][t * 16 + lc], acc[t]);
        }
        __syncthreads();
        if (more) {
            stash();
            __syncthreads();
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long long row = r0 + wv * 16 + lr + 4 * r;
            const int c = n0 + t * 16 + lc;
            if (row < n && c < N) {
                double* p = const_cast<double*>(seg_addr(O, row, c));
                *p = (beta != 0.0) ? fma(beta, *p, alpha * acc[t][r]) : alpha * acc[t][r];
            }
        }
}

template <int NT>
__global__ __launch_bounds__(kThreads, (NT > 8 ? 1 : (NT > 6 ? 2 : 3))) void update_kernel(long long n, Segs U, int K,
                                                          const double* __restrict__ C, int N,
                                                          Segs O, double alpha, double beta,
                                                          int ntn) {
    const int lin = xcd_remap(blockIdx.x, gridDim.x);
    update_body<NT>(lin / ntn, lin % ntn, n, U, K, C, N, O, alpha, beta);
}

template <int NT>
void update_launch(hipStream_t st, long long n, const Segs& U, int K, const double* C, int N,
                   const Segs& O, double alpha, double beta) {
    constexpr int BN = 16 * NT;
    const int ntn = (N + BN - 1) / BN;
    const long long nrb = (n + UM - 1) / UM;
    hipLaunchKernelGGL(update_kernel<NT>, dim3((unsigned)(nrb * ntn)), dim3(kThreads), 0, st, n, U, K,
                       C, N, O, alpha, beta, ntn);
}

}  // namespace

// ---------------------------------------------------------------------------
hipError_t launch_spmm(hipStream_t st, int n, const int* rowptr, const int* col, const double* val,
                       const double* X, long long ldx, double* Y, long long ldy, int w, const int* heavy,
                       int n_heavy) {
    if (n <= 0 || w <= 0) return hipSuccess;
    if (n_heavy == 0) {
        const long long waves = ((long long)n + kStreamRows - 1) / kStreamRows;
        const int grid = (int)((waves + kThreads / 64 - 1) / (kThreads / 64));
        hipLaunchKernelGGL(spmm_stream_kernel<16>, dim3(grid), dim3(kThreads), 0, st, n, rowptr, col, val, X,
                           ldx, Y, ldy, w);
        return hipGetLastError();
    }
    const int half = (w + 1) / 2;
#define SE_SPMM(L) return spmm_launch<L>(st, n, rowptr, col, val, X, ldx, Y, ldy, w, heavy, n_heavy)
    if (half <= 1) SE_SPMM(1);
    if (half <= 2) SE_SPMM(2);
    if (half <= 4) SE_SPMM(4);
    if (half <= 8) SE_SPMM(8);
    if (half <= 16) SE_SPMM(16);
    if (half <= 32) SE_SPMM(32);
    SE_SPMM(64);
#undef SE_SPMM
}

hipError_t launch_resid_norms(hipStream_t st, long long n, const double* X, const double* AX,
                              long long ld, int k, const double* lam, double* part, double* out, double* R,
                              long long ldr) {
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
                       lam, rows, part, R, ldr);
    return launch_sum_partials(st, 2 * k, (int)nchunks, part, out);
}

long long spmm_resid_chunks(long long n) {
    const long long waves = (n + kStreamRows - 1) / kStreamRows;
    return (waves + kThreads / 64 - 1) / (kThreads / 64);
}

hipError_t launch_spmm_resid(hipStream_t st, int n, const int* rowptr, const int* col, const double* val,
                             const double* X, long long ldx, double* Y, long long ldy, int w, const int* heavy,
                             int n_heavy, const double* lam, double* R, long long ldr, double* part, double* out) {
    if (n <= 0 || w <= 0 || w > 128 || n_heavy > 0) return hipErrorInvalidValue;
    const long long grid = spmm_resid_chunks(n);
    (void)heavy;
    hipLaunchKernelGGL(spmm_resid_kernel, dim3((unsigned)grid), dim3(kThreads), 0, st, n, rowptr, col, val, X, ldx,
                       Y, ldy, w, lam, R, ldr, part);
    return launch_sum_partials(st, 2 * w, (int)grid, part, out);
}

namespace {
// SplitMix64 (Steele, Lea and Flood 2014) at Weyl state seed + (k + 1) * gamma.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long seed, unsigned long long k) {
    unsigned long long z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(kThreads) void seeded_block_kernel(long long n, int nb, unsigned long long seed,
                                                                double* __restrict__ X, long long ld,
                                                                int col_major) {
    const long long total = n * nb;
    for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < total;
         e += (long long)gridDim.x * kThreads) {
        const long long i = e / nb;
        const int j = (int)(e - i * nb);
        const unsigned long long z = splitmix64(seed, (unsigned long long)j * (unsigned long long)n + (unsigned long long)i);
        X[col_major ? (long long)j * ld + i : i * ld + j] = (double)(z >> 11) * 0x1p-52 - 1.0;
    }
}

// Columns c0 .. c0 + d - 1 of a row-major panel get the normally distributed
// block of draw `draw`: entry (i, j) is Box-Muller (1958) of the SplitMix64
// outputs at counters 2t and 2t + 1, t = (draw nb + j) n + i.
__global__ __launch_bounds__(kThreads) void gaussian_cols_kernel(long long n, int d, int nb, long long draw,
                                                                 unsigned long long seed, double* __restrict__ X,
                                                                 long long ld, int c0) {
    const long long total = n * d;
    for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < total;
         e += (long long)gridDim.x * kThreads) {
        const long long i = e / d;
        const int j = (int)(e - i * d);
        const unsigned long long t =
            ((unsigned long long)draw * (unsigned long long)nb + (unsigned long long)j) * (unsigned long long)n +
            (unsigned long long)i;
        const unsigned long long z1 = splitmix64(seed, 2ull * t), z2 = splitmix64(seed, 2ull * t + 1ull);
        const double u1 = (double)((z1 >> 11) + 1ull) * 0x1p-53;  // (0, 1]
        const double u2 = (double)(z2 >> 11) * 0x1p-53;           // [0, 1)
        X[i * ld + c0 + j] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    }
}
}  // namespace

hipError_t launch_seeded_block(hipStream_t st, long long n, int nb, unsigned long long seed, double* X,
                               long long ld, bool col_major) {
    if (n <= 0 || nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(seeded_block_kernel, dim3(grid_for(n * nb, kThreads, 16384)), dim3(kThreads), 0, st, n,
                       nb, seed, X, ld, col_major ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_gaussian_cols(hipStream_t st, long long n, int d, int nb, long long draw, unsigned long long seed,
                                double* X, long long ld, int c0) {
    if (n <= 0 || d <= 0) return hipSuccess;
    hipLaunchKernelGGL(gaussian_cols_kernel, dim3(grid_for(n * d, kThreads, 16384)), dim3(kThreads), 0, st, n, d,
                       nb, draw, seed, X, ld, c0);
    return hipGetLastError();
}

hipError_t launch_gather_cols(hipStream_t st, long long n, const double* src, long long lds, const int* idx,
                              int a, double* dst, long long ldd) {
    if (a <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_cols_kernel, dim3(grid_for(n * a, kThreads, 16384)), dim3(kThreads), 0, st, n,
                       src, lds, idx, a, dst, ldd);
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
                            int k, double sigma, double scale) {
    if (k <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(shift_sub_kernel, dim3(grid_for(n * k, kThreads, 16384)), dim3(kThreads), 0, st,
                       n, X, AX, ld, k, sigma, scale);
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

hipError_t launch_sum_partials(hipStream_t st, int L, int nchunks, double* part, double* out) {
    if (L <= 0) return hipSuccess;
    constexpr int OPB = kThreads / kSumG;
    long long rs = L;
    if (nchunks > 2 * kSumBlk) {  // two levels: block sums first, in place
        const int nb = (nchunks + kSumBlk - 1) / kSumBlk;
        hipLaunchKernelGGL(sum_blocks_kernel, dim3((L + 15) / 16, nb), dim3(kThreads), 0, st, L, nchunks, part);
        nchunks = nb;
        rs = (long long)kSumBlk * L;
    }
    hipLaunchKernelGGL(sum_partials_kernel, dim3((L + OPB - 1) / OPB), dim3(kThreads), 0, st, L, nchunks, part,
                       out, rs);
    return hipGetLastError();
}

hipError_t launch_gram_reduce(hipStream_t st, int mu, int mv, int nchunks, int sym, const double* part,
                              double* C) {
    const long long total = (long long)mu * mv;
    if (total <= 0) return hipSuccess;
    constexpr int OPB = kThreads / kRedG;
    hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)((total + OPB - 1) / OPB)), dim3(kThreads), 0, st, mu,
                       mv, nchunks, sym, part, C);
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
                       double* part, double* C, size_t part_cap) {
    const int mu = segs_width(U), mv = segs_width(V);
    if (mu <= 0 || mv <= 0) return hipSuccess;
    if (sym && mu != mv) sym = 0;
    int ntiles, nt_v, nchunks;
    long long rows;
    const long long max_chunks = part_cap ? (long long)(part_cap / ((size_t)mu * (size_t)mv)) : 0;
    if (part_cap && max_chunks < 1) return hipErrorInvalidValue;
    gram_plan(n, mu, mv, sym, ntiles, nt_v, nchunks, rows, max_chunks);
    if (n <= 0) {
        (void)hipMemsetAsync(C, 0, sizeof(double) * (size_t)mu * mv, st);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(gram_kernel, dim3(nchunks * ntiles), dim3(kThreads), 0, st, n, U, V, mu, mv,
                       nt_v, sym, ntiles, rows, part);
    const long long total = (long long)mu * mv;
    constexpr int OPB = kThreads / kRedG;
    hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)((total + OPB - 1) / OPB)), dim3(kThreads), 0, st, mu,
                       mv, nchunks, sym, part, C);
    return hipGetLastError();
}

hipError_t launch_update(hipStream_t st, long long n, const Segs& U, const double* C, int N,
                         const Segs& O, double alpha, double beta) {
    const int K = segs_width(U);
    if (N <= 0 || n <= 0) return hipSuccess;
    // Column tiles of 16 NT columns: the fewest tiles with NT <= 8 (which
    // keeps two workgroups per CU), NT as small as that tile count allows.
    const int need = (N + 15) / 16;
    const int nct = (need + 7) / 8;
    switch ((need + nct - 1) / nct) {
        case 1: update_launch<1>(st, n, U, K, C, N, O, alpha, beta); break;
        case 2: update_launch<2>(st, n, U, K, C, N, O, alpha, beta); break;
        case 3: update_launch<3>(st, n, U, K, C, N, O, alpha, beta); break;
        case 4: update_launch<4>(st, n, U, K, C, N, O, alpha, beta); break;
        case 5: update_launch<5>(st, n, U, K, C, N, O, alpha, beta); break;
        case 6: update_launch<6>(st, n, U, K, C, N, O, alpha, beta); break;
        case 7: update_launch<7>(st, n, U, K, C, N, O, alpha, beta); break;
        default: update_launch<8>(st, n, U, K, C, N, O, alpha, beta); break;
    }
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Batched products: the single-solve bodies above, driven by a work list. Each
// workgroup forms the prefix sums of the jobs' item counts in LDS and loops
// over items blockIdx.x, blockIdx.x + gridDim.x, ...
namespace {

__device__ __forceinline__ int gram_tiles(int mu, int mv, int sym, int& nt_v) {
    const int nt_u = (mu + GT - 1) / GT;
    nt_v = (mv + GT - 1) / GT;
    return sym ? nt_u * (nt_u + 1) / 2 : nt_u * nt_v;
}

template <class F>
__device__ __forceinline__ void for_items(int nj, F&& count, int* s_start) {
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int j = 0; j < nj; ++j) {
            s_start[j] = acc;
            acc += count(j);
        }
        s_start[nj] = acc;
    }
    __syncthreads();
}

// Job of item `it` (uniform over the workgroup, so that the job's fields are
// read with scalar loads).
__device__ __forceinline__ int item_job(int it, int nj, const int* s_start) {
    int j = 0;
    while (j + 1 < nj && it >= s_start[j + 1]) ++j;
    return __builtin_amdgcn_readfirstlane(j);
}

__global__ __launch_bounds__(kThreads, 2) void gram_batched_kernel(const BGramJob* __restrict__ jobs, int nj) {
    __shared__ int s_start[kMaxBatch + 1];
    for_items(
        nj,
        [&](int j) {
            const BGramJob& J = jobs[j];
            if (J.n <= 0 || J.mu <= 0 || J.mv <= 0) return 0;
            int ntv;
            return J.nchunks * gram_tiles(J.mu, J.mv, J.sym, ntv);
        },
        s_start);
    const int total = __builtin_amdgcn_readfirstlane(s_start[nj]);
    for (int it = blockIdx.x; it < total; it += gridDim.x) {
        const int j = item_job(it, nj, s_start);
        const BGramJob& J = jobs[j];
        int ntv;
        const int nt = gram_tiles(J.mu, J.mv, J.sym, ntv);
        const int loc = __builtin_amdgcn_readfirstlane(it - s_start[j]);
        gram_body(loc / nt, loc % nt, J.n, J.U, J.V, J.mu, J.mv, ntv, J.sym, J.rows, J.part);
        __syncthreads();
    }
}

__global__ __launch_bounds__(kThreads) void gram_reduce_batched_kernel(const BGramJob* __restrict__ jobs, int nj) {
    constexpr int OPB = kThreads / kRedG;
    __shared__ int s_start[kMaxBatch + 1];
    for_items(
        nj,
        [&](int j) {
            const BGramJob& J = jobs[j];
            if (J.n <= 0 || J.mu <= 0 || J.mv <= 0) return 0;
            return (J.mu * J.mv + OPB - 1) / OPB;
        },
        s_start);
    const int total = __builtin_amdgcn_readfirstlane(s_start[nj]);
    for (int it = blockIdx.x; it < total; it += gridDim.x) {
        const int j = item_job(it, nj, s_start);
        const BGramJob& J = jobs[j];
        gram_reduce_body(it - s_start[j], J.mu, J.mv, J.nchunks, J.sym, J.part, J.C);
        __syncthreads();
    }
}

constexpr int kBatchNT = 6;  // update column tile: 96 columns

__global__ __launch_bounds__(kThreads, 2) void update_batched_kernel(const BUpdJob* __restrict__ jobs, int nj) {
    constexpr int BN = 16 * kBatchNT;
    __shared__ int s_start[kMaxBatch + 1];
    for_items(
        nj,
        [&](int j) {
            const BUpdJob& J = jobs[j];
            if (J.n <= 0 || J.N <= 0) return 0;
            return (int)((J.n + UM - 1) / UM) * ((J.N + BN - 1) / BN);
        },
        s_start);
    // one item per workgroup: the grid covers every item (launch_update_batched)
    const int it = blockIdx.x;
    if (it >= s_start[nj]) return;
    const int j = item_job(it, nj, s_start);
    const BUpdJob& J = jobs[j];
    const int ntn = (J.N + BN - 1) / BN;
    const int loc = __builtin_amdgcn_readfirstlane(it - s_start[j]);
    update_body<kBatchNT>(loc / ntn, loc % ntn, J.n, J.U, J.K, J.C, J.N, J.O, J.alpha, J.beta);
}

__global__ __launch_bounds__(kThreads) void spmm_batched_kernel(const BSpmmJob* __restrict__ jobs, int nj) {
    constexpr int RPB = kStreamRows * (kThreads / 64);  // rows per work item
    __shared__ int s_start[kMaxBatch + 1];
    for_items(
        nj,
        [&](int j) {
            const BSpmmJob& J = jobs[j];
            if (J.n <= 0 || J.w <= 0) return 0;
            return (J.n + RPB - 1) / RPB;
        },
        s_start);
    const int total = __builtin_amdgcn_readfirstlane(s_start[nj]);
    for (int it = blockIdx.x; it < total; it += gridDim.x) {
        const int j = item_job(it, nj, s_start);
        const BSpmmJob& J = jobs[j];
        spmm_stream_body<16>((it - s_start[j]) * (kThreads / 64) + (int)(threadIdx.x >> 6), J.n, J.rowptr, J.col,
                             J.val, J.X, J.ldx, J.Y, J.ldy, J.w);
    }
}

__global__ __launch_bounds__(kThreads) void resid_batched_kernel(const BResidJob* __restrict__ jobs, int nj) {
    __shared__ int s_start[kMaxBatch + 1];
    for_items(
        nj,
        [&](int j) {
            const BResidJob& J = jobs[j];
            return (J.n <= 0 || J.k <= 0) ? 0 : J.nchunks;
        },
        s_start);
    const int total = __builtin_amdgcn_readfirstlane(s_start[nj]);
    for (int it = blockIdx.x; it < total; it += gridDim.x) {
        const int j = item_job(it, nj, s_start);
        const BResidJob& J = jobs[j];
        resid_norms_body(it - s_start[j], J.n, J.X, J.AX, J.ld, J.k, J.lam, J.rows, J.part, J.R, J.ldr);
        __syncthreads();
    }
}

__global__ __launch_bounds__(kThreads) void resid_sum_batched_kernel(const BResidJob* __restrict__ jobs, int nj) {
    constexpr int OPB = kThreads / kSumG;
    __shared__ int s_start[kMaxBatch + 1];
    for_items(
        nj,
        [&](int j) {
            const BResidJob& J = jobs[j];
            return (J.n <= 0 || J.k <= 0) ? 0 : (2 * J.k + OPB - 1) / OPB;
        },
        s_start);
    const int total = __builtin_amdgcn_readfirstlane(s_start[nj]);
    for (int it = blockIdx.x; it < total; it += gridDim.x) {
        const int j = item_job(it, nj, s_start);
        const BResidJob& J = jobs[j];
        sum_partials_body(it - s_start[j], 2 * J.k, J.nchunks, J.part, J.out, 2 * J.k);
        __syncthreads();
    }
}

}  // namespace

void launch_gram_batched(Launcher& L, const BGramJob* jobs, int nj, int grid) {
    if (nj <= 0 || nj > kMaxBatch || grid <= 0) L.err = hipErrorInvalidValue;
    L(gram_batched_kernel, dim3(grid), dim3(kThreads), 0, jobs, nj);
    L(gram_reduce_batched_kernel, dim3(grid), dim3(kThreads), 0, jobs, nj);
}

void launch_update_batched(Launcher& L, const BUpdJob* jobs, int nj, int grid) {
    if (nj <= 0 || nj > kMaxBatch || grid <= 0) L.err = hipErrorInvalidValue;
    L(update_batched_kernel, dim3(grid), dim3(kThreads), 0, jobs, nj);
}

void launch_spmm_batched(Launcher& L, const BSpmmJob* jobs, int nj, int grid) {
    if (nj <= 0 || nj > kMaxBatch || grid <= 0) L.err = hipErrorInvalidValue;
    L(spmm_batched_kernel, dim3(grid), dim3(kThreads), 0, jobs, nj);
}

void launch_resid_batched(Launcher& L, const BResidJob* jobs, int nj, int grid) {
    if (nj <= 0 || nj > kMaxBatch || grid <= 0) L.err = hipErrorInvalidValue;
    L(resid_batched_kernel, dim3(grid), dim3(kThreads), 0, jobs, nj);
    L(resid_sum_batched_kernel, dim3(grid), dim3(kThreads), 0, jobs, nj);
}

}  // namespace se
