// n-length kernels of the Rayleigh-Ritz step on low-precision panels (FP32 or
// BF16 storage), gfx950.
//
// Storage halves (FP32) or quarters (BF16) the panel traffic of the FP64
// path; arithmetic is FP32, on the matrix cores (v_mfma_f32_16x16x4f32; the
// Gram product of BF16 blocks on v_mfma_f32_16x16x16bf16_1k) for
// the Gram products and basis updates. Their FP32 accumulators are folded
// into FP64 registers every 64 rows (Gram) or 64 terms of K (update), so the
// rounding of a long FP32 sum never exceeds a few units of the storage
// format, and every reduction over n leaves the workgroup in FP64 and is
// summed in a fixed order (bitwise reproducible). Layouts and the row-chunk
// plans follow the FP64 kernels: row-major panels, XCD-contiguous row ranges.
#include <algorithm>
#include <cstdint>

#include "common.h"

namespace se {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ int xcd_remap(int bid, int G) {
    constexpr int NX = 8;
    const int q = G / NX, r = G % NX;
    const int x = bid % NX, i = bid / NX;
    return x * q + min(x, r) + i;
}

inline int grid_for(long long work, int per_block, int cap = 1 << 20) {
    long long g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return static_cast<int>(g);
}

// ---- storage <-> FP32 ------------------------------------------------------
__device__ __forceinline__ float bf2f(uint32_t bits16) { return __uint_as_float(bits16 << 16); }
__device__ __forceinline__ uint32_t f2bf(float f) {  // round to nearest even
    const uint32_t u = __float_as_uint(f);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float ld1(const float* p) { return *p; }
__device__ __forceinline__ float ld1(const bf16_t* p) { return bf2f(*p); }
__device__ __forceinline__ void st1(float* p, float v) { *p = v; }
__device__ __forceinline__ void st1(bf16_t* p, float v) { *p = (bf16_t)f2bf(v); }
// four consecutive elements (16-byte FP32 or 8-byte BF16 access)
__device__ __forceinline__ void ld4(const float* p, float* v) {
    const float4 q = *reinterpret_cast<const float4*>(p);
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
    v[3] = q.w;
}
__device__ __forceinline__ void ld4(const bf16_t* p, float* v) {
    const uint2 q = *reinterpret_cast<const uint2*>(p);
    v[0] = bf2f(q.x & 0xFFFFu);
    v[1] = bf2f(q.x >> 16);
    v[2] = bf2f(q.y & 0xFFFFu);
    v[3] = bf2f(q.y >> 16);
}
__device__ __forceinline__ void st4(float* p, const float* v) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void st4(bf16_t* p, const float* v) {
    uint2 q;
    q.x = f2bf(v[0]) | (f2bf(v[1]) << 16);
    q.y = f2bf(v[2]) | (f2bf(v[3]) << 16);
    *reinterpret_cast<uint2*>(p) = q;
}

template <class T>
__device__ __forceinline__ const T* seg_col(const SegsT<T>& S, int c, bool& ok) {
    ok = c < S.off[S.nseg];
    if (!ok) return S.p[0];
    const T* p = S.p[0];
    int o = 0;
    if (S.nseg > 1 && c >= S.off[1]) { p = S.p[1]; o = S.off[1]; }
    if (S.nseg > 2 && c >= S.off[2]) { p = S.p[2]; o = S.off[2]; }
    if (S.nseg > 3 && c >= S.off[3]) { p = S.p[3]; o = S.off[3]; }
    return p + (c - o);
}

template <class T>
__device__ __forceinline__ T* seg_addr(const SegsT<T>& S, long long row, int c) {
    const T* p = S.p[0];
    int o = 0;
    if (S.nseg > 1 && c >= S.off[1]) { p = S.p[1]; o = S.off[1]; }
    if (S.nseg > 2 && c >= S.off[2]) { p = S.p[2]; o = S.off[2]; }
    if (S.nseg > 3 && c >= S.off[3]) { p = S.p[3]; o = S.off[3]; }
    return const_cast<T*>(p) + row * S.ld + (c - o);
}

// ---------------------------------------------------------------------------
// CSR x block (FP32 values). LPR lanes cooperate on one matrix row and each
// lane owns four adjacent columns (one 16- or 8-byte gather per nonzero). A
// lane group walks SPR rows two at a time with the index / gather / FMA phases
// of up to SB nonzeros per row separated, so a 7-point row costs two memory
// round trips. Slots past the end of a row gather the row itself with weight
// zero. A lane whose four columns straddle w reads padding columns
// (ld >= w rounded up to 8) and stores only the columns below w.
constexpr int SPR = 8;
constexpr int SB = 8;

template <class T>
__device__ __forceinline__ void store_cols(T* p, const float* v, int c0, int w) {
    if (c0 + 4 <= w) {
        st4(p, v);
    } else {
        for (int q = 0; q < w - c0; ++q) st1(p + q, v[q]);
    }
}

template <class T>
__device__ __forceinline__ void spmm_rows(int ra, int rb, const int* __restrict__ rowptr,
                                          const int* __restrict__ col, const float* __restrict__ val,
                                          const T* __restrict__ X, long long ldx, T* __restrict__ Y,
                                          long long ldy, int c0, int w) {
    const int ba = rowptr[ra];
    int ea = rowptr[ra + 1];
    const bool heavy_a = ea - ba > kHeavyRow;  // computed by spmm_lp_heavy_kernel
    if (heavy_a) ea = ba;
    const bool hasb0 = rb >= 0;
    const int rbs = hasb0 ? rb : ra;
    const int bb = hasb0 ? rowptr[rbs] : 0;
    int eb = hasb0 ? rowptr[rbs + 1] : 0;
    if (eb - bb > kHeavyRow) eb = bb;
    const bool hasb = hasb0 && rowptr[rbs + 1] - bb <= kHeavyRow;
    float a[4] = {0.f, 0.f, 0.f, 0.f}, b[4] = {0.f, 0.f, 0.f, 0.f};
    for (int pa = ba, pb = bb; pa < ea || pb < eb; pa += SB, pb += SB) {
        int ja[SB], jb[SB];
        float va[SB], vb[SB];
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const bool oka = pa + u < ea, okb = pb + u < eb;
            ja[u] = oka ? col[pa + u] : ra;
            va[u] = oka ? val[pa + u] : 0.f;
            jb[u] = okb ? col[pb + u] : rbs;
            vb[u] = okb ? val[pb + u] : 0.f;
        }
        float xa[SB][4], xb[SB][4];
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            ld4(X + (long long)ja[u] * ldx + c0, xa[u]);
            ld4(X + (long long)jb[u] * ldx + c0, xb[u]);
        }
#pragma unroll
        for (int u = 0; u < SB; ++u)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a[q] = fmaf(va[u], xa[u][q], a[q]);
                b[q] = fmaf(vb[u], xb[u][q], b[q]);
            }
    }
    if (!heavy_a) store_cols(Y + (long long)ra * ldy + c0, a, c0, w);
    if (hasb) store_cols(Y + (long long)rb * ldy + c0, b, c0, w);
}

// One long row per workgroup (see the FP64 heavy-row kernel): lane groups
// take batches of SB nonzeros in turn, group 0 sums the partials in order.
template <class T, int LPR>
__global__ __launch_bounds__(kThreads) void spmm_lp_heavy_kernel(const int* __restrict__ heavy,
                                                                 const int* __restrict__ rowptr,
                                                                 const int* __restrict__ col,
                                                                 const float* __restrict__ val,
                                                                 const T* __restrict__ X, long long ldx,
                                                                 T* __restrict__ Y, long long ldy, int w) {
    constexpr int G = kThreads / LPR;
    __shared__ float4 red[G][LPR];
    const int row = heavy[blockIdx.x];
    const int g = threadIdx.x / LPR, lane = threadIdx.x % LPR;
    const int b = rowptr[row], e = rowptr[row + 1];
    for (int cb = 0; cb < w; cb += 4 * LPR) {
        const int c0 = cb + 4 * lane;
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        if (c0 < w) {
            for (int p = b + g * SB; p < e; p += G * SB) {
                int j[SB];
                float v[SB];
#pragma unroll
                for (int u = 0; u < SB; ++u) {
                    const bool ok = p + u < e;
                    j[u] = ok ? col[p + u] : row;
                    v[u] = ok ? val[p + u] : 0.f;
                }
                float x[SB][4];
#pragma unroll
                for (int u = 0; u < SB; ++u) ld4(X + (long long)j[u] * ldx + c0, x[u]);
#pragma unroll
                for (int u = 0; u < SB; ++u)
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[q] = fmaf(v[u], x[u][q], acc[q]);
            }
        }
        red[g][lane] = make_float4(acc[0], acc[1], acc[2], acc[3]);
        __syncthreads();
        if (g == 0 && c0 < w) {
            float s[4] = {0.f, 0.f, 0.f, 0.f};
            for (int q = 0; q < G; ++q) {
                s[0] += red[q][lane].x;
                s[1] += red[q][lane].y;
                s[2] += red[q][lane].z;
                s[3] += red[q][lane].w;
            }
            store_cols(Y + (long long)row * ldy + c0, s, c0, w);
        }
        __syncthreads();
    }
}

template <class T, int LPR>
__global__ __launch_bounds__(kThreads) void spmm_lp_kernel(int n, const int* __restrict__ rowptr,
                                                           const int* __restrict__ col,
                                                           const float* __restrict__ val,
                                                           const T* __restrict__ X, long long ldx,
                                                           T* __restrict__ Y, long long ldy, int w) {
    constexpr int GPB = kThreads / LPR;
    const int blk = blockIdx.x;  // round-robin over XCDs, as in the FP64 product
    const int sub = threadIdx.x / LPR;
    const int lane = threadIdx.x % LPR;
    const int rbeg = (blk * GPB + sub) * SPR;
    if (rbeg >= n) return;
    const int rend = min(n, rbeg + SPR);
    for (int c0 = 4 * lane; c0 < w; c0 += 4 * LPR)
        for (int r = rbeg; r < rend; r += 2)
            spmm_rows(r, r + 1 < rend ? r + 1 : -1, rowptr, col, val, X, ldx, Y, ldy, c0, w);
}

// Two consecutive elements (8-byte FP32 or 4-byte BF16 access).
__device__ __forceinline__ void ld2(const float* p, float& a, float& b) {
    const float2 q = *reinterpret_cast<const float2*>(p);
    a = q.x;
    b = q.y;
}
__device__ __forceinline__ void ld2(const bf16_t* p, float& a, float& b) {
    const uint32_t q = *reinterpret_cast<const uint32_t*>(p);
    a = bf2f(q & 0xFFFFu);
    b = bf2f(q >> 16);
}
__device__ __forceinline__ void st2(float* p, float a, float b) {
    *reinterpret_cast<float2*>(p) = make_float2(a, b);
}
__device__ __forceinline__ void st2(bf16_t* p, float a, float b) {
    *reinterpret_cast<uint32_t*>(p) = f2bf(a) | (f2bf(b) << 16);
}

// CSR x block for matrices without heavy rows (the FP64 streaming product
// with FP32 values and arithmetic): one wave per run of kStreamRows rows walks
// the run's nonzeros NB at a time with wave-uniform indices and values, all
// NB gathers in flight, the accumulator moved at row boundaries. Lane l owns
// columns cb + 2l, cb + 2l + 1 of each 128-column block; per row the sum runs
// over the nonzeros in order, as in spmm_lp_kernel.
constexpr int kStreamRows = 32;

template <class T, int NB>
__global__ __launch_bounds__(kThreads) void spmm_lp_stream_kernel(int n, const int* __restrict__ rowptr,
                                                                  const int* __restrict__ col,
                                                                  const float* __restrict__ val,
                                                                  const T* __restrict__ X, long long ldx,
                                                                  T* __restrict__ Y, long long ldy, int w) {
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane((int)blockIdx.x * (kThreads / 64) + (int)(threadIdx.x >> 6));
    if ((long long)wid * kStreamRows >= n) return;
    const int r0 = wid * kStreamRows;
    const int r1 = min(n, r0 + kStreamRows);
    const int rp = rowptr[min(r0 + lane, r1)];
    const int pbeg = __builtin_amdgcn_readlane(rp, 0);
    const int pend = __builtin_amdgcn_readlane(rp, r1 - r0);
    for (int cb = 0; cb < w; cb += 128) {
        const int c0 = cb + 2 * lane;
        const bool has0 = c0 < w, has1 = c0 + 1 < w;
        const long long cc = has0 ? c0 : cb;
        int r = r0;
        int rend = __builtin_amdgcn_readlane(rp, 1);
        float a0 = 0.f, a1 = 0.f;
        auto flush = [&]() {
            T* y = Y + (long long)r * ldy + c0;
            if (has1)
                st2(y, a0, a1);
            else if (has0)
                st1(y, a0);
            a0 = 0.f;
            a1 = 0.f;
            ++r;
            if (r < r1) rend = __builtin_amdgcn_readlane(rp, r - r0 + 1);
        };
        for (int p = pbeg; p < pend; p += NB) {
            int j[NB];
            float v[NB];
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                j[u] = col[p + u];
                v[u] = val[p + u];
            }
            float x0[NB], x1[NB];
#pragma unroll
            for (int u = 0; u < NB; ++u) ld2(X + (long long)j[u] * ldx + cc, x0[u], x1[u]);
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                if (p + u < pend) {
                    while (p + u >= rend) flush();
                    a0 = fmaf(v[u], x0[u], a0);
                    a1 = fmaf(v[u], x1[u], a1);
                }
            }
        }
        while (r < r1) flush();
    }
}

// The streaming product fused with one step of the Chebyshev filter, for
// matrices without heavy rows: at a row's end the lane rounds its two sums to
// the storage format (as the separate product would store them), forms
// alpha (A Y) + beta Y + gamma Z in FP64 from the stored Y and Z of the row,
// and stores Z rounded once. A Y never goes to memory.
__device__ __forceinline__ float stored(const float*, float x) { return x; }
__device__ __forceinline__ float stored(const bf16_t*, float x) { return bf2f(f2bf(x)); }

template <class T, int NB>
__global__ __launch_bounds__(kThreads) void spmm_cheb_lp_kernel(int n, const int* __restrict__ rowptr,
                                                                const int* __restrict__ col,
                                                                const float* __restrict__ val,
                                                                const T* __restrict__ Y, T* __restrict__ Z,
                                                                long long ld, int w, double alpha, double beta,
                                                                double gamma) {
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane((int)blockIdx.x * (kThreads / 64) + (int)(threadIdx.x >> 6));
    if ((long long)wid * kStreamRows >= n) return;
    const int r0 = wid * kStreamRows;
    const int r1 = min(n, r0 + kStreamRows);
    const int rp = rowptr[min(r0 + lane, r1)];
    const int pbeg = __builtin_amdgcn_readlane(rp, 0);
    const int pend = __builtin_amdgcn_readlane(rp, r1 - r0);
    const bool with_z = gamma != 0.0;
    for (int cb = 0; cb < w; cb += 128) {
        const int c0 = cb + 2 * lane;
        const bool has0 = c0 < w, has1 = c0 + 1 < w;
        const long long cc = has0 ? c0 : cb;
        int r = r0;
        int rend = __builtin_amdgcn_readlane(rp, 1);
        float a0 = 0.f, a1 = 0.f;
        auto flush = [&]() {
            const long long o = (long long)r * ld + c0;
            if (has0) {
                float y0, y1, z0 = 0.f, z1 = 0.f;
                ld2(Y + o, y0, y1);  // y1 is the padding column when only has0
                if (with_z) ld2(Z + o, z0, z1);
                const float v0 = (float)(alpha * (double)stored(Y, a0) + beta * (double)y0 + gamma * (double)z0);
                const float v1 = (float)(alpha * (double)stored(Y, a1) + beta * (double)y1 + gamma * (double)z1);
                if (has1)
                    st2(Z + o, v0, v1);
                else
                    st1(Z + o, v0);
            }
            a0 = 0.f;
            a1 = 0.f;
            ++r;
            if (r < r1) rend = __builtin_amdgcn_readlane(rp, r - r0 + 1);
        };
        for (int p = pbeg; p < pend; p += NB) {
            int j[NB];
            float v[NB];
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                j[u] = col[p + u];
                v[u] = val[p + u];
            }
            float x0[NB], x1[NB];
#pragma unroll
            for (int u = 0; u < NB; ++u) ld2(Y + (long long)j[u] * ld + cc, x0[u], x1[u]);
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                if (p + u < pend) {
                    while (p + u >= rend) flush();
                    a0 = fmaf(v[u], x0[u], a0);
                    a1 = fmaf(v[u], x1[u], a1);
                }
            }
        }
        while (r < r1) flush();
    }
}

template <class T, int LPR>
hipError_t spmm_lp_launch(hipStream_t st, int n, const int* rowptr, const int* col, const float* val,
                          const T* X, long long ldx, T* Y, long long ldy, int w, const int* heavy,
                          int n_heavy) {
    constexpr int RPB = (kThreads / LPR) * SPR;
    const int grid = (n + RPB - 1) / RPB;
    hipLaunchKernelGGL((spmm_lp_kernel<T, LPR>), dim3(grid), dim3(kThreads), 0, st, n, rowptr, col, val, X,
                       ldx, Y, ldy, w);
    if (n_heavy > 0)
        hipLaunchKernelGGL((spmm_lp_heavy_kernel<T, LPR>), dim3(n_heavy), dim3(kThreads), 0, st, heavy, rowptr,
                           col, val, X, ldx, Y, ldy, w);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Residual and column norms in FP64: per chunk of rows, sum (ax - lam x)^2
// and x^2 for each column c < k.
template <class T>
__global__ __launch_bounds__(kThreads) void resid_norms_lp_kernel(long long n, const T* __restrict__ X,
                                                                  const T* __restrict__ AX, long long ld,
                                                                  int k, const double* __restrict__ lam,
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
                const double x = ld1(X + r * ld + c);
                const double y = (double)ld1(AX + r * ld + c) - l * x;
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
                const double x = ld1(X + r * ld + c);
                const double y = (double)ld1(AX + r * ld + c) - l * x;
                ar = fma(y, y, ar);
                axx = fma(x, x, axx);
            }
            out[c] = ar;
            out[k + c] = axx;
        }
    }
}

template <class T>
__global__ __launch_bounds__(kThreads) void form_w_lp_kernel(long long n, const T* __restrict__ X,
                                                             const T* __restrict__ AX, long long ld,
                                                             const double* __restrict__ lam,
                                                             const int* __restrict__ act, int a,
                                                             T* __restrict__ W, long long ldw) {
    const long long total = n * a;
    for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < total;
         e += (long long)gridDim.x * kThreads) {
        const long long r = e / a;
        const int jj = (int)(e - r * a);
        const int c = act[jj];
        st1(W + r * ldw + jj, (float)((double)ld1(AX + r * ld + c) - lam[c] * (double)ld1(X + r * ld + c)));
    }
}

template <class T>
__global__ __launch_bounds__(kThreads) void shift_sub_lp_kernel(long long n, T* __restrict__ X,
                                                                const T* __restrict__ AX, long long ld,
                                                                int k, double sigma, double scale) {
    const long long total = n * k;
    for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < total;
         e += (long long)gridDim.x * kThreads) {
        const long long r = e / k;
        const int c = (int)(e - r * k);
        T* px = X + r * ld + c;
        st1(px, (float)(scale * (sigma * (double)ld1(px) - (double)ld1(AX + r * ld + c))));
    }
}

// One step of the Chebyshev filter recurrence on stored blocks: Z = alpha U +
// beta V + gamma Z over the first k columns (Z not read when gamma = 0),
// formed in FP64 from the stored values and rounded once.
template <class T>
__global__ __launch_bounds__(kThreads) void cheb_step_lp_kernel(long long n, int k, double alpha,
                                                                const T* __restrict__ U, double beta,
                                                                const T* __restrict__ V, double gamma,
                                                                T* __restrict__ Z, long long ld) {
    const long long total = n * k;
    const bool with_z = gamma != 0.0;
    for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < total;
         e += (long long)gridDim.x * kThreads) {
        const long long r = e / k;
        const int c = (int)(e - r * k);
        const long long o = r * ld + c;
        const double z = with_z ? (double)ld1(Z + o) : 0.0;
        st1(Z + o, (float)(alpha * (double)ld1(U + o) + beta * (double)ld1(V + o) + gamma * z));
    }
}

template <class T>
__global__ __launch_bounds__(kThreads) void copy_cols_lp_kernel(long long n, const T* __restrict__ src,
                                                                long long lds, int sc, T* __restrict__ dst,
                                                                long long ldd, int dc, int w) {
    const long long total = n * w;
    for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < total;
         e += (long long)gridDim.x * kThreads) {
        const long long r = e / w;
        const int c = (int)(e - r * w);
        dst[r * ldd + dc + c] = src[r * lds + sc + c];
    }
}

// FP64 column-major -> T row-major through 32 x 32 LDS tiles; blockDim (32, 8).
template <class T>
__global__ void c2r_lp_kernel(long long n, int w, const double* __restrict__ src, long long ldc,
                              T* __restrict__ dst, long long ldr) {
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
        if (r < n && c < w) st1(dst + r * ldr + c, (float)tile[threadIdx.x][q]);
    }
}

template <class T>
__global__ __launch_bounds__(kThreads) void rows_to_f64_kernel(long long n, int w, const T* __restrict__ src,
                                                               long long lds, double* __restrict__ dst,
                                                               long long ldd) {
    const long long total = n * w;
    for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < total;
         e += (long long)gridDim.x * kThreads) {
        const long long r = e / w;
        const int c = (int)(e - r * w);
        dst[r * ldd + c] = (double)ld1(src + r * lds + c);
    }
}

__global__ __launch_bounds__(kThreads) void f64_to_f32_kernel(long long count, const double* __restrict__ src,
                                                              float* __restrict__ dst) {
    for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < count;
         e += (long long)gridDim.x * kThreads)
        dst[e] = (float)src[e];
}

// ---------------------------------------------------------------------------
// FP32 matrix cores. v_mfma_f32_16x16x4f32 computes D[16x16] += A[16x4] B[4x16];
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds
// D[4 (l / 16) + r][l % 16] in accumulator register r (checked on gfx950; the
// row order differs from the FP64 instruction's).
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma16f(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr int GT = kGramTile;
constexpr int GK = kGramRows;
constexpr int GFLUSH = 2;  // Gram stages (of GK rows) per FP32 accumulation run

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

template <int NI, int NJ>
__device__ __forceinline__ void gram_lp_compute(const float (*Ts)[2 * GT + 4], f4 (&acc)[3][3], int lr,
                                                int lc, int wy, int wx) {
#pragma unroll
    for (int ks = 0; ks < GK; ks += 4) {
        float a[NI], b[NJ];
#pragma unroll
        for (int i = 0; i < NI; ++i) a[i] = Ts[ks + lr][wy * 48 + i * 16 + lc];
#pragma unroll
        for (int j = 0; j < NJ; ++j) b[j] = Ts[ks + lr][GT + wx * 48 + j * 16 + lc];
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
            for (int j = 0; j < NJ; ++j) acc[i][j] = mfma16f(a[i], b[j], acc[i][j]);
    }
}

// Gram product C = U^T V, the FP64 kernel's tiling (96 x 96 output tile per
// workgroup, four waves of 3 x 3 MFMA tiles, GK rows per stage through LDS
// with register prefetch), FP32 MFMAs folded into FP64 every GFLUSH stages.
template <class T>
__global__ __launch_bounds__(kThreads, 2) void gram_lp_kernel(long long n, SegsT<T> U, SegsT<T> V, int mu,
                                                           int mv, int nt_v, int sym, int ntiles,
                                                           long long rows_per_chunk,
                                                           double* __restrict__ part) {
    constexpr int RPT = GK / 4;
    __shared__ float Ts[GK][2 * GT + 4];
    const int lin = xcd_remap(blockIdx.x, gridDim.x);
    const int chunk = lin / ntiles;
    const int tile = lin % ntiles;
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
    const int shape = niv * 4 + njv;

    const T* cp[3];
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
            cld[q] = V.ld;
        }
    }
    f4 acc[3][3];
    double dacc[3][3][4];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int r = 0; r < 4; ++r) dacc[i][j][r] = 0.0;
        }
    auto flush = [&]() {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
#pragma unroll
                for (int r = 0; r < 4; ++r) dacc[i][j][r] += (double)acc[i][j][r];
                acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
            }
    };
    float rg[RPT][3];
    auto fetch = [&](long long rb) {
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const long long r = rb + wv + 4 * i;
            const bool rok = r < r1;
#pragma unroll
            for (int q = 0; q < 3; ++q) rg[i][q] = (rok && cok[q]) ? ld1(cp[q] + r * cld[q]) : 0.f;
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
    int stage = 0;
    for (long long rb = r0; rb < r1; rb += GK) {
        const bool more = rb + GK < r1;
        if (more) fetch(rb + GK);
        switch (shape) {  // uniform per wave
            case 15: gram_lp_compute<3, 3>(Ts, acc, lr, lc, wy, wx); break;
            case 14: gram_lp_compute<3, 2>(Ts, acc, lr, lc, wy, wx); break;
            case 13: gram_lp_compute<3, 1>(Ts, acc, lr, lc, wy, wx); break;
            case 11: gram_lp_compute<2, 3>(Ts, acc, lr, lc, wy, wx); break;
            case 10: gram_lp_compute<2, 2>(Ts, acc, lr, lc, wy, wx); break;
            case 9: gram_lp_compute<2, 1>(Ts, acc, lr, lc, wy, wx); break;
            case 7: gram_lp_compute<1, 3>(Ts, acc, lr, lc, wy, wx); break;
            case 6: gram_lp_compute<1, 2>(Ts, acc, lr, lc, wy, wx); break;
            case 5: gram_lp_compute<1, 1>(Ts, acc, lr, lc, wy, wx); break;
            default: break;
        }
        if (++stage == GFLUSH) {
            flush();
            stage = 0;
        }
        __syncthreads();
        if (more) {
            stash();
            __syncthreads();
        }
    }
    flush();
    double* P = part + (long long)chunk * mu * mv;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gi = cu0 + wy * 48 + i * 16 + 4 * lr + r;
                const int gj = cv0 + wx * 48 + j * 16 + lc;
                if (gi < mu && gj < mv) P[(long long)gi * mv + gj] = dacc[i][j][r];
            }
}

// ---------------------------------------------------------------------------
// Gram product of BF16 blocks on the BF16 matrix cores:
// v_mfma_f32_16x16x16bf16_1k computes D[16x16] += A[16x16] B[16x16] with FP32
// accumulation; lane l supplies A[l % 16][4 (l / 16) + q] and
// B[4 (l / 16) + q][l % 16] (q < 4, one 8-byte vector each) and holds
// D[4 (l / 16) + r][l % 16] in accumulator register r (checked on gfx950).
// Products of two BF16 values are exact in FP32, so the result equals the
// FP32-MFMA kernel's up to the order of the FP32 additions. The tiling is the
// FP32 kernel's; the stage is kept in LDS transposed (column-major, BF16), so
// the four consecutive rows a lane supplies are one 8-byte read, and a
// 32-row stage is two MFMA steps instead of eight.
typedef short s4bf __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma16bf(s4bf a, s4bf b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

constexpr int GKT = GK + 8;  // row stride (BF16 entries) of the transposed stage

template <int NI, int NJ>
__device__ __forceinline__ void gram_bf16_compute(const bf16_t (*Tt)[GKT], f4 (&acc)[3][3], int lr, int lc,
                                                  int wy, int wx) {
#pragma unroll
    for (int ks = 0; ks < GK; ks += 16) {
        s4bf a[NI], b[NJ];
#pragma unroll
        for (int i = 0; i < NI; ++i)
            a[i] = *reinterpret_cast<const s4bf*>(&Tt[wy * 48 + i * 16 + lc][ks + 4 * lr]);
#pragma unroll
        for (int j = 0; j < NJ; ++j)
            b[j] = *reinterpret_cast<const s4bf*>(&Tt[GT + wx * 48 + j * 16 + lc][ks + 4 * lr]);
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
            for (int j = 0; j < NJ; ++j) acc[i][j] = mfma16bf(a[i], b[j], acc[i][j]);
    }
}

__global__ __launch_bounds__(kThreads, 2) void gram_bf16_kernel(long long n, SegsT<bf16_t> U, SegsT<bf16_t> V,
                                                                int mu, int mv, int nt_v, int sym, int ntiles,
                                                                long long rows_per_chunk,
                                                                double* __restrict__ part) {
    constexpr int RPT = GK / 4;
    __shared__ __align__(16) bf16_t Tt[2 * GT][GKT];  // [column][row]
    const int lin = xcd_remap(blockIdx.x, gridDim.x);
    const int chunk = lin / ntiles;
    const int tile = lin % ntiles;
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
    const int shape = niv * 4 + njv;

    const bf16_t* cp[3];
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
            cld[q] = V.ld;
        }
    }
    f4 acc[3][3];
    double dacc[3][3][4];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int r = 0; r < 4; ++r) dacc[i][j][r] = 0.0;
        }
    auto flush = [&]() {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
#pragma unroll
                for (int r = 0; r < 4; ++r) dacc[i][j][r] += (double)acc[i][j][r];
                acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
            }
    };
    bf16_t rg[RPT][3];
    auto fetch = [&](long long rb) {
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const long long r = rb + wv + 4 * i;
            const bool rok = r < r1;
#pragma unroll
            for (int q = 0; q < 3; ++q) rg[i][q] = (rok && cok[q]) ? cp[q][r * cld[q]] : (bf16_t)0;
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int i = 0; i < RPT; ++i)
#pragma unroll
            for (int q = 0; q < 3; ++q) Tt[lane + 64 * q][wv + 4 * i] = rg[i][q];
    };

    if (r0 < r1) {
        fetch(r0);
        stash();
    }
    __syncthreads();
    int stage = 0;
    for (long long rb = r0; rb < r1; rb += GK) {
        const bool more = rb + GK < r1;
        if (more) fetch(rb + GK);
        switch (shape) {  // uniform per wave
            case 15: gram_bf16_compute<3, 3>(Tt, acc, lr, lc, wy, wx); break;
            case 14: gram_bf16_compute<3, 2>(Tt, acc, lr, lc, wy, wx); break;
            case 13: gram_bf16_compute<3, 1>(Tt, acc, lr, lc, wy, wx); break;
            case 11: gram_bf16_compute<2, 3>(Tt, acc, lr, lc, wy, wx); break;
            case 10: gram_bf16_compute<2, 2>(Tt, acc, lr, lc, wy, wx); break;
            case 9: gram_bf16_compute<2, 1>(Tt, acc, lr, lc, wy, wx); break;
            case 7: gram_bf16_compute<1, 3>(Tt, acc, lr, lc, wy, wx); break;
            case 6: gram_bf16_compute<1, 2>(Tt, acc, lr, lc, wy, wx); break;
            case 5: gram_bf16_compute<1, 1>(Tt, acc, lr, lc, wy, wx); break;
            default: break;
        }
        if (++stage == GFLUSH) {
            flush();
            stage = 0;
        }
        __syncthreads();
        if (more) {
            stash();
            __syncthreads();
        }
    }
    flush();
    double* P = part + (long long)chunk * mu * mv;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gi = cu0 + wy * 48 + i * 16 + 4 * lr + r;
                const int gj = cv0 + wx * 48 + j * 16 + lc;
                if (gi < mu && gj < mv) P[(long long)gi * mv + gj] = dacc[i][j][r];
            }
}

// ---------------------------------------------------------------------------
// Basis update Out = beta Out + alpha U C (C given in FP64, rounded to FP32
// once per call into a K x N scratch that every workgroup streams): the FP64
// kernel's tiling (64 rows x 16 NT columns per workgroup, K streamed UK at a
// time with register prefetch), FP32 MFMAs folded into FP64 every UFLUSH
// stages.
constexpr int UM = 64;
constexpr int UK = 32;
constexpr int UFLUSH = 2;

template <class T, int NT>
__global__ __launch_bounds__(kThreads, 2) void update_lp_kernel(long long n, SegsT<T> U, int K,
                                                             const float* __restrict__ C, int N,
                                                             SegsT<T> O, float alpha, float beta,
                                                             int ntn) {
    constexpr int BN = 16 * NT;
    constexpr int UQ = (UM * UK) / kThreads;
    constexpr int CQ = (UK * BN) / kThreads;
    __shared__ float Us[UK][UM + 4];
    __shared__ float Cs[UK][BN + 4];
    const int lin = xcd_remap(blockIdx.x, gridDim.x);
    const int rb = lin / ntn, tn = lin % ntn;
    const long long r0 = (long long)rb * UM;
    const int n0 = tn * BN;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane >> 4, lc = lane & 15;
    f4 acc[NT];
    double dacc[NT][4];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        acc[t] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int r = 0; r < 4; ++r) dacc[t][r] = 0.0;
    }
    auto flush = [&]() {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
#pragma unroll
            for (int r = 0; r < 4; ++r) dacc[t][r] += (double)acc[t][r];
            acc[t] = f4{0.f, 0.f, 0.f, 0.f};
        }
    };
    float ru[UQ], rc[CQ];
    auto fetch = [&](int k0) {
        bool ok;
        const T* up = seg_col(U, k0 + (int)(threadIdx.x % UK), ok);
#pragma unroll
        for (int q = 0; q < UQ; ++q) {
            const long long r = r0 + threadIdx.x / UK + (kThreads / UK) * q;
            ru[q] = (ok && r < n) ? ld1(up + r * U.ld) : 0.f;
        }
#pragma unroll
        for (int q = 0; q < CQ; ++q) {
            const int e = threadIdx.x + kThreads * q;
            const int kk = e / BN, c = e % BN;
            const int kc = k0 + kk;
            rc[q] = (kc < K && n0 + c < N) ? C[(long long)kc * N + n0 + c] : 0.f;
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int q = 0; q < UQ; ++q) Us[threadIdx.x % UK][threadIdx.x / UK + (kThreads / UK) * q] = ru[q];
#pragma unroll
        for (int q = 0; q < CQ; ++q) {
            const int e = threadIdx.x + kThreads * q;
            Cs[e / BN][e % BN] = rc[q];
        }
    };

    fetch(0);
    stash();
    __syncthreads();
    int stage = 0;
    for (int k0 = 0; k0 < K; k0 += UK) {
        const bool more = k0 + UK < K;
        if (more) fetch(k0 + UK);
#pragma unroll
        for (int ks = 0; ks < UK; ks += 4) {
            const float a = Us[ks + lr][wv * 16 + lc];
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = mfma16f(a, Cs[ks + lr][t * 16 + lc], acc[t]);
        }
        if (++stage == UFLUSH) {
            flush();
            stage = 0;
        }
        __syncthreads();
        if (more) {
            stash();
            __syncthreads();
        }
    }
    flush();
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long long row = r0 + wv * 16 + 4 * lr + r;
            const int c = n0 + t * 16 + lc;
            if (row < n && c < N) {
                T* p = seg_addr(O, row, c);
                double v = (double)alpha * dacc[t][r];
                if (beta != 0.f) v = fma((double)beta, (double)ld1(p), v);
                st1(p, (float)v);
            }
        }
}

template <class T, int NT>
void update_lp_launch(hipStream_t st, long long n, const SegsT<T>& U, int K, const float* C, int N,
                      const SegsT<T>& O, double alpha, double beta) {
    constexpr int BN = 16 * NT;
    const int ntn = (N + BN - 1) / BN;
    const long long nrb = (n + UM - 1) / UM;
    hipLaunchKernelGGL((update_lp_kernel<T, NT>), dim3((unsigned)(nrb * ntn)), dim3(kThreads), 0, st, n, U,
                       K, C, N, O, (float)alpha, (float)beta, ntn);
}

bool ld_ok(long long ld, int w) { return ld % 8 == 0 && ld >= (long long)((w + 7) / 8 * 8); }

}  // namespace

// ---------------------------------------------------------------------------
template <class T>
hipError_t launch_spmm_lp(hipStream_t st, int n, const int* rowptr, const int* col, const float* val,
                          const T* X, long long ldx, T* Y, long long ldy, int w, const int* heavy,
                          int n_heavy) {
    if (n <= 0 || w <= 0) return hipSuccess;
    if (!ld_ok(ldx, w) || !ld_ok(ldy, w)) return hipErrorInvalidValue;
    if (n_heavy == 0) {
        const long long waves = ((long long)n + kStreamRows - 1) / kStreamRows;
        const int grid = (int)((waves + kThreads / 64 - 1) / (kThreads / 64));
        hipLaunchKernelGGL((spmm_lp_stream_kernel<T, 16>), dim3(grid), dim3(kThreads), 0, st, n, rowptr, col, val,
                           X, ldx, Y, ldy, w);
        return hipGetLastError();
    }
    const int quads = (w + 3) / 4;
#define SE_SPMM(L) return spmm_lp_launch<T, L>(st, n, rowptr, col, val, X, ldx, Y, ldy, w, heavy, n_heavy)
    if (quads <= 1) SE_SPMM(1);
    if (quads <= 2) SE_SPMM(2);
    if (quads <= 4) SE_SPMM(4);
    if (quads <= 8) SE_SPMM(8);
    if (quads <= 16) SE_SPMM(16);
    if (quads <= 32) SE_SPMM(32);
    SE_SPMM(64);
#undef SE_SPMM
}

template <class T>
hipError_t launch_resid_norms_lp(hipStream_t st, long long n, const T* X, const T* AX, long long ld, int k,
                                 const double* lam, double* part, double* out) {
    if (k <= 0) return hipSuccess;
    long long rows = 2048;
    long long nchunks = (n + rows - 1) / rows;
    if (nchunks > 4096) {
        nchunks = 4096;
        rows = (n + nchunks - 1) / nchunks;
        nchunks = (n + rows - 1) / rows;
    }
    if (nchunks < 1) nchunks = 1;
    hipLaunchKernelGGL(resid_norms_lp_kernel<T>, dim3((int)nchunks), dim3(kThreads), 0, st, n, X, AX, ld, k,
                       lam, rows, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_sum_partials(st, 2 * k, (int)nchunks, part, out);
}

template <class T>
hipError_t launch_form_w_lp(hipStream_t st, long long n, const T* X, const T* AX, long long ld,
                            const double* lam, const int* act, int a, T* W, long long ldw) {
    if (a <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(form_w_lp_kernel<T>, dim3(grid_for(n * a, kThreads, 16384)), dim3(kThreads), 0, st, n,
                       X, AX, ld, lam, act, a, W, ldw);
    return hipGetLastError();
}

template <class T>
hipError_t launch_shift_sub_lp(hipStream_t st, long long n, T* X, const T* AX, long long ld, int k,
                               double sigma, double scale) {
    if (k <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(shift_sub_lp_kernel<T>, dim3(grid_for(n * k, kThreads, 16384)), dim3(kThreads), 0, st,
                       n, X, AX, ld, k, sigma, scale);
    return hipGetLastError();
}

template <class T>
hipError_t launch_spmm_cheb_lp(hipStream_t st, int n, const int* rowptr, const int* col, const float* val,
                               const T* Y, T* Z, long long ld, int w, int n_heavy, double alpha, double beta,
                               double gamma) {
    if (n <= 0 || w <= 0) return hipSuccess;
    if (n_heavy > 0 || !ld_ok(ld, w)) return hipErrorInvalidValue;
    const long long waves = ((long long)n + kStreamRows - 1) / kStreamRows;
    const int grid = (int)((waves + kThreads / 64 - 1) / (kThreads / 64));
    hipLaunchKernelGGL((spmm_cheb_lp_kernel<T, 16>), dim3(grid), dim3(kThreads), 0, st, n, rowptr, col, val, Y, Z,
                       ld, w, alpha, beta, gamma);
    return hipGetLastError();
}

template <class T>
hipError_t launch_cheb_step_lp(hipStream_t st, long long n, int k, double alpha, const T* U, double beta,
                               const T* V, double gamma, T* Z, long long ld) {
    if (k <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(cheb_step_lp_kernel<T>, dim3(grid_for(n * k, kThreads, 16384)), dim3(kThreads), 0, st,
                       n, k, alpha, U, beta, V, gamma, Z, ld);
    return hipGetLastError();
}

template <class T>
hipError_t launch_copy_cols_lp(hipStream_t st, long long n, const T* src, long long lds, int sc, T* dst,
                               long long ldd, int dc, int w) {
    if (w <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy_cols_lp_kernel<T>, dim3(grid_for(n * w, kThreads, 16384)), dim3(kThreads), 0, st,
                       n, src, lds, sc, dst, ldd, dc, w);
    return hipGetLastError();
}

template <class T>
hipError_t launch_colmajor_to_rows_lp(hipStream_t st, long long n, int w, const double* src, long long ldc,
                                      T* dst, long long ldr) {
    if (w <= 0 || n <= 0) return hipSuccess;
    dim3 grid((unsigned)((n + 31) / 32), (unsigned)((w + 31) / 32));
    hipLaunchKernelGGL(c2r_lp_kernel<T>, grid, dim3(32, 8), 0, st, n, w, src, ldc, dst, ldr);
    return hipGetLastError();
}

template <class T>
hipError_t launch_rows_lp_to_f64(hipStream_t st, long long n, int w, const T* src, long long lds,
                                 double* dst, long long ldd) {
    if (w <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(rows_to_f64_kernel<T>, dim3(grid_for(n * w, kThreads, 16384)), dim3(kThreads), 0, st,
                       n, w, src, lds, dst, ldd);
    return hipGetLastError();
}

template <class T>
hipError_t launch_gram_lp(hipStream_t st, long long n, const SegsT<T>& U, const SegsT<T>& V, int sym,
                          double* part, double* C) {
    const int mu = segs_width(U), mv = segs_width(V);
    if (mu <= 0 || mv <= 0 || n <= 0) return hipSuccess;
    if (sym && mu != mv) sym = 0;
    int ntiles, nt_v, nchunks;
    long long rows;
    gram_plan(n, mu, mv, sym, ntiles, nt_v, nchunks, rows);
    if constexpr (sizeof(T) == 2)  // BF16 storage: BF16 matrix cores
        hipLaunchKernelGGL(gram_bf16_kernel, dim3(nchunks * ntiles), dim3(kThreads), 0, st, n, U, V, mu, mv, nt_v,
                           sym, ntiles, rows, part);
    else
        hipLaunchKernelGGL(gram_lp_kernel<T>, dim3(nchunks * ntiles), dim3(kThreads), 0, st, n, U, V, mu, mv,
                           nt_v, sym, ntiles, rows, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_gram_reduce(st, mu, mv, nchunks, sym, part, C);
}

template <class T>
hipError_t launch_update_lp(hipStream_t st, long long n, const SegsT<T>& U, const double* C64, int N,
                            const SegsT<T>& O, double alpha, double beta, float* C) {
    const int K = segs_width(U);
    if (N <= 0 || n <= 0 || K <= 0) return hipSuccess;
    if (!C) return hipErrorInvalidValue;
    {
        const hipError_t e = launch_f64_to_f32(st, (long long)K * N, C64, C);
        if (e != hipSuccess) return e;
    }
    const int need = (N + 15) / 16;
    const int nct = (need + 7) / 8;
    switch ((need + nct - 1) / nct) {
        case 1: update_lp_launch<T, 1>(st, n, U, K, C, N, O, alpha, beta); break;
        case 2: update_lp_launch<T, 2>(st, n, U, K, C, N, O, alpha, beta); break;
        case 3: update_lp_launch<T, 3>(st, n, U, K, C, N, O, alpha, beta); break;
        case 4: update_lp_launch<T, 4>(st, n, U, K, C, N, O, alpha, beta); break;
        case 5: update_lp_launch<T, 5>(st, n, U, K, C, N, O, alpha, beta); break;
        case 6: update_lp_launch<T, 6>(st, n, U, K, C, N, O, alpha, beta); break;
        case 7: update_lp_launch<T, 7>(st, n, U, K, C, N, O, alpha, beta); break;
        default: update_lp_launch<T, 8>(st, n, U, K, C, N, O, alpha, beta); break;
    }
    return hipGetLastError();
}

hipError_t launch_f64_to_f32(hipStream_t st, long long count, const double* src, float* dst) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(f64_to_f32_kernel, dim3(grid_for(count, kThreads, 16384)), dim3(kThreads), 0, st, count,
                       src, dst);
    return hipGetLastError();
}

#define SE_LP_INSTANTIATE(T)                                                                            \
    template hipError_t launch_spmm_lp<T>(hipStream_t, int, const int*, const int*, const float*, const T*, \
                                          long long, T*, long long, int, const int*, int);               \
    template hipError_t launch_resid_norms_lp<T>(hipStream_t, long long, const T*, const T*, long long, int, \
                                                 const double*, double*, double*);                        \
    template hipError_t launch_form_w_lp<T>(hipStream_t, long long, const T*, const T*, long long,         \
                                            const double*, const int*, int, T*, long long);               \
    template hipError_t launch_shift_sub_lp<T>(hipStream_t, long long, T*, const T*, long long, int, double, \
                                               double);                                                  \
    template hipError_t launch_cheb_step_lp<T>(hipStream_t, long long, int, double, const T*, double,     \
                                               const T*, double, T*, long long);                         \
    template hipError_t launch_spmm_cheb_lp<T>(hipStream_t, int, const int*, const int*, const float*,    \
                                               const T*, T*, long long, int, int, double, double, double); \
    template hipError_t launch_copy_cols_lp<T>(hipStream_t, long long, const T*, long long, int, T*,       \
                                               long long, int, int);                                     \
    template hipError_t launch_colmajor_to_rows_lp<T>(hipStream_t, long long, int, const double*,          \
                                                      long long, T*, long long);                          \
    template hipError_t launch_rows_lp_to_f64<T>(hipStream_t, long long, int, const T*, long long, double*, \
                                                 long long);                                              \
    template hipError_t launch_gram_lp<T>(hipStream_t, long long, const SegsT<T>&, const SegsT<T>&, int,    \
                                          double*, double*);                                              \
    template hipError_t launch_update_lp<T>(hipStream_t, long long, const SegsT<T>&, const double*, int,   \
                                            const SegsT<T>&, double, double, float*);

SE_LP_INSTANTIATE(float)
SE_LP_INSTANTIATE(bf16_t)
#undef SE_LP_INSTANTIATE

}  // namespace se
