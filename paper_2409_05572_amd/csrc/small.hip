// Small dense FP64 kernels of the Rayleigh-Ritz step: the Cholesky-QR
// transform, the spectral decomposition of the projected matrix A_p (only the
// lowest k eigenpairs are formed), and the Hetmaniuk-Lehoucq start block. Each
// works on one matrix of order <= 1024, kept in LDS when it fits and in global
// memory (L2-resident) otherwise.
#include <cfloat>

#include <algorithm>

#include <hip/hip_cooperative_groups.h>

#include "common.h"

namespace se {

namespace {

constexpr int kSmall = 512;  // threads of the single-workgroup kernels
constexpr int kTri = 1024;   // threads of the global-memory tridiagonalization
constexpr int kSWaves = kSmall / 64;
constexpr int kLdsDoubles = 12800;  // 100 KB of dynamic LDS for an in-LDS matrix

// Value of lane `lane` (wave-uniform) in every lane: two v_readlane_b32,
// where __shfl goes through the LDS crossbar (ds_bpermute) and its latency.
__device__ __forceinline__ double bcast_lane(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Lane-permuted copy of v by a DPP move of each 32-bit half (no LDS).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// row_bcast15: rows 1 and 3 of the wave receive lane 15 of rows 0 and 2;
// rows 0 and 2 receive zero (the DPP write is masked and `old` is 0).
__device__ __forceinline__ double dpp_row_bcast15(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x142, 0xA, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x142, 0xA, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes, in every lane; the whole wave must be active. Within
// each row of 16 lanes: swap neighbours (quad_perm 1,0,3,2), then pairs
// (quad_perm 2,3,0,1), then the half-row mirror and the row mirror, after
// which every lane holds its row's sum; the four row sums are read with
// v_readlane and added in a fixed order (deterministic).
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_f64<0xB1>(v);
    v += dpp_f64<0x4E>(v);
    v += dpp_f64<0x141>(v);
    v += dpp_f64<0x140>(v);
    return (bcast_lane(v, 0) + bcast_lane(v, 16)) + (bcast_lane(v, 32) + bcast_lane(v, 48));
}

// Workgroup sum in a fixed order; `sh` holds kSWaves doubles. Two barriers.
__device__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kSWaves; ++q) s += sh[q];
    __syncthreads();
    return s;
}

// ---------------------------------------------------------------------------
// Cholesky-QR transform. Columns are scaled to unit norm (G -> D G D) so the
// pivots measure the part of each column independent of the previous ones.
// With drop_tol2 >= 0 a column whose pivot falls below drop_tol2 is dropped;
// with drop_tol2 < 0 nothing is dropped and tiny pivots are floored (used for
// bases known to be full rank). T = D R^{-1} restricted to the kept columns,
// a x r with leading dimension r. The factor lives in one a x a array: L in
// the lower triangle, R^{-1} in the upper one, their diagonals apart.
//
// With ns_tol > 0 the kernel first measures ||G - I||_F. When it is at most
// ns_tol the block is already orthonormal to that level and one Newton-Schulz
// step T = (3 I - G) / 2 replaces the factorization: the Gram matrix of W T
// is I - (3/4) E^2 - (1/4) E^3 with E = G - I, so ns_tol = 1e-8 leaves an
// error below rounding. The decision is taken on the device, so a caller can
// chain passes without reading anything back.
// kLds: the a x a work matrix lives in dynamic LDS (a^2 <= kLdsDoubles), else
// in `work`; fixed at compile time so every access is a plain LDS or global
// instruction rather than a generic (flat) one.
template <bool kLds>
__device__ __forceinline__ void chol_drop_kernel_body(int bx, int a, const double* __restrict__ G,
                                                           double* __restrict__ T,
                                                           double* __restrict__ work,
                                                           int* __restrict__ info_i,
                                                           double* __restrict__ info_d,
                                                           double drop_tol2, double ns_tol) {
    extern __shared__ double dyn[];
    __shared__ int s_pos[1024];
    __shared__ int s_kept[1024];
    __shared__ double s_D[1024];
    __shared__ double s_dl[1024];  // diagonal of L
    __shared__ double s_dr[1024];  // diagonal of R^{-1}
    __shared__ double s_red[kSWaves];
    __shared__ int s_r;
    double* F = kLds ? dyn : work;  // a x a
    const int t = threadIdx.x;
    const bool can_drop = drop_tol2 >= 0.0;

    const int nth = blockDim.x;
    if (ns_tol > 0.0) {
        double s = 0.0;
        for (size_t e = t; e < (size_t)a * a; e += nth) {
            const double v = G[e] - ((e / a == e % a) ? 1.0 : 0.0);
            s += v * v;
        }
        s = block_sum(s, s_red);  // identical in every thread
        if (s <= ns_tol * ns_tol) {
            for (size_t e = t; e < (size_t)a * a; e += nth)
                T[e] = ((e / a == e % a) ? 1.5 : 0.0) - 0.5 * G[e];
            for (int i = t; i < a; i += nth) info_i[1 + i] = i;
            if (t == 0) {
                info_i[0] = a;
                info_d[0] = 1.0 - sqrt(s);
            }
            return;
        }
    }
    for (int i = t; i < a; i += nth) {
        const double g = G[(size_t)i * a + i];
        s_D[i] = (g > 0.0) ? 1.0 / sqrt(g) : 0.0;
    }
    __syncthreads();
    for (size_t e = t; e < (size_t)a * a; e += nth) {
        const int i = (int)(e / a), j = (int)(e % a);
        if (j <= i) F[e] = G[e] * s_D[i] * s_D[j];
    }
    __syncthreads();

    double minpiv = DBL_MAX;
    // Right-looking elimination. The scaled pivot column is staged in LDS
    // (s_col), and the rank-1 update of the lower triangle runs as wave-rows
    // over contiguous column ranges: one load and one store per element.
    double* s_col = s_dr;  // reused: R^{-1}'s diagonal is formed after the loop
    const int lane = t & 63, wrow = t >> 6, nwave = nth >> 6;
    for (int j = 0; j < a; ++j) {
        double d = F[(size_t)j * a + j];
        const bool drop = can_drop && (!(d > drop_tol2) || s_D[j] == 0.0);
        if (!can_drop && !(d > 1e-300)) d = 1e-300;
        if (drop) {
            for (int i = j + 1 + t; i < a; i += nth) F[(size_t)i * a + j] = 0.0;
            if (t == 0) {
                s_pos[j] = -1;
                s_dl[j] = 0.0;
            }
            __syncthreads();
            continue;
        }
        const double piv = sqrt(d);
        const double inv = 1.0 / piv;
        minpiv = fmin(minpiv, d);
        for (int i = j + 1 + t; i < a; i += nth) {
            const double l = F[(size_t)i * a + j] * inv;
            F[(size_t)i * a + j] = l;
            s_col[i] = l;
        }
        if (t == 0) {
            s_dl[j] = piv;
            s_pos[j] = 0;
        }
        __syncthreads();
        for (int i = j + 1 + wrow; i < a; i += nwave) {
            const double li = s_col[i];
            double* frow = F + (size_t)i * a;
            for (int i2 = j + 1 + lane; i2 <= i; i2 += 64) frow[i2] -= li * s_col[i2];
        }
        __syncthreads();
    }
    if (t == 0) {
        int r = 0;
        for (int j = 0; j < a; ++j) {
            if (s_pos[j] >= 0) {
                s_pos[j] = r;
                s_kept[r] = j;
                info_i[1 + r] = j;
                ++r;
            }
        }
        s_r = r;
        info_i[0] = r;
        info_d[0] = minpiv;
    }
    __syncthreads();
    const int r = s_r;
    // R^{-1} by back substitution, one column per thread: with R[p][u] =
    // L[kept u][kept p], X[p][q] = -(sum_{u=p+1..q} R[p][u] X[u][q]) / R[p][p].
    // X[u][q] (u < q) is stored at F[kept u][kept q] (upper triangle).
    for (int q = t; q < r; q += nth) {
        const int kq = s_kept[q];
        s_dr[q] = 1.0 / s_dl[kq];
        for (int p = q - 1; p >= 0; --p) {
            const int kp = s_kept[p];
            double s = F[(size_t)kq * a + kp] * s_dr[q];
            for (int u = p + 1; u < q; ++u) {
                const int ku = s_kept[u];
                s += F[(size_t)ku * a + kp] * F[(size_t)ku * a + kq];
            }
            F[(size_t)kp * a + kq] = -s / s_dl[kp];
        }
    }
    __syncthreads();
    for (size_t e = t; e < (size_t)a * r; e += nth) {
        const int i = (int)(e / r), q = (int)(e % r);
        const int p = s_pos[i];
        double v = 0.0;
        if (p >= 0 && p <= q) v = s_D[i] * ((p == q) ? s_dr[q] : F[(size_t)i * a + s_kept[q]]);
        T[e] = v;
    }
}

template <bool kLds>
__global__ __launch_bounds__(kSmall) void chol_drop_kernel(int a, const double* __restrict__ G,
                                                           double* __restrict__ T,
                                                           double* __restrict__ work,
                                                           int* __restrict__ info_i,
                                                           double* __restrict__ info_d,
                                                           double drop_tol2, double ns_tol) {
    chol_drop_kernel_body<kLds>(blockIdx.x, a, G, T, work, info_i, info_d, drop_tol2, ns_tol);
}


// Cholesky-QR transform with column drop for a <= kCholBlk (same inputs,
// outputs and drop rule as chol_drop_kernel), blocked so that synchronization
// no longer scales with a: the scaled matrix lives in LDS (odd row stride);
// panels of 16 columns are factorized by one wave (lanes own rows, the pivot
// column broadcast by shuffles), each followed by one workgroup-wide update
// of the trailing lower triangle. The inverse of L over the kept columns
// (dropped rows and columns replaced by the identity, which leaves the kept
// block's inverse unchanged) is formed by 16 x 16 blocks: every diagonal
// block by one wave, then the block diagonals at distance 1, 2, ... from
// products of blocks already formed, two barriers each. L stays in the lower
// triangle, R^{-1} = L^{-T} goes to the upper one.
constexpr int kCholBlk = 112;
constexpr int kCholPanel = 16;
__device__ __forceinline__ void chol_drop_blocked_kernel_body(int bx, int a, const double* __restrict__ G,
                                                                   double* __restrict__ T,
                                                                   int* __restrict__ info_i,
                                                                   double* __restrict__ info_d, double drop_tol2,
                                                                   double ns_tol) {
    extern __shared__ double F[];  // a x FS
    __shared__ int s_pos[kCholBlk];
    __shared__ int s_kept[kCholBlk];
    __shared__ double s_D[kCholBlk];
    __shared__ double s_dl[kCholBlk];  // diagonal of L (0 where dropped)
    __shared__ double s_dm[kCholBlk];  // diagonal of the modified L (1 where dropped)
    __shared__ double s_tmp[(kCholBlk / kCholPanel) * kCholPanel * kCholPanel];
    __shared__ double s_red[kSWaves];
    __shared__ double s_minpiv;
    __shared__ int s_r;
    const int t = threadIdx.x;
    const int nth = blockDim.x;
    const int FS = a | 1;
    const bool can_drop = drop_tol2 >= 0.0;
    const int lane = t & 63, wid = t >> 6, nwave = nth >> 6;
    if (ns_tol > 0.0) {
        double sq = 0.0;
        for (int e = t; e < a * a; e += nth) {
            const double v = G[e] - ((e / a == e % a) ? 1.0 : 0.0);
            sq += v * v;
        }
        sq = block_sum(sq, s_red);
        if (sq <= ns_tol * ns_tol) {
            for (int e = t; e < a * a; e += nth) T[e] = ((e / a == e % a) ? 1.5 : 0.0) - 0.5 * G[e];
            for (int i = t; i < a; i += nth) info_i[1 + i] = i;
            if (t == 0) {
                info_i[0] = a;
                info_d[0] = 1.0 - sqrt(sq);
            }
            return;
        }
    }
    for (int i = t; i < a; i += nth) {
        const double g = G[i * a + i];
        s_D[i] = (g > 0.0) ? 1.0 / sqrt(g) : 0.0;
    }
    __syncthreads();
    for (int e = t; e < a * a; e += nth) {
        const int i = e / a, j = e % a;
        if (j <= i) F[i * FS + j] = G[e] * s_D[i] * s_D[j];
    }
    if (t == 0) s_minpiv = DBL_MAX;
    __syncthreads();

    // ---- blocked right-looking factorization ----
    for (int jb = 0; jb < a; jb += kCholPanel) {
        const int nbw = min(kCholPanel, a - jb);
        if (wid == 0) {
            // rows jb + lane and jb + lane + 64 of the panel's columns
            double P[2][kCholPanel];
            const int i0 = jb + lane, i1 = jb + lane + 64;
#pragma unroll
            for (int c = 0; c < kCholPanel; ++c) {
                P[0][c] = (c < nbw && i0 < a && i0 >= jb + c) ? F[i0 * FS + jb + c] : 0.0;
                P[1][c] = (c < nbw && i1 < a) ? F[i1 * FS + jb + c] : 0.0;
            }
            double minp = DBL_MAX;
            // fully unrolled (no break or continue), so P stays in registers
#pragma unroll
            for (int c = 0; c < kCholPanel; ++c) {
                if (c < nbw) {
                    const int j = jb + c;
                    double dj = bcast_lane(P[0][c], c);
                    const bool drop = can_drop && (!(dj > drop_tol2) || s_D[j] == 0.0);
                    if (!can_drop && !(dj > 1e-300)) dj = 1e-300;
                    if (drop) {
                        if (i0 >= j) P[0][c] = 0.0;
                        P[1][c] = 0.0;
                        if (lane == 0) {
                            s_pos[j] = -1;
                            s_dl[j] = 0.0;
                        }
                    } else {
                        const double piv = sqrt(dj);
                        const double inv = 1.0 / piv;
                        minp = fmin(minp, dj);
                        if (i0 > j) P[0][c] *= inv;
                        if (lane == c) P[0][c] = piv;
                        P[1][c] *= inv;
                        if (lane == 0) {
                            s_pos[j] = 0;
                            s_dl[j] = piv;
                        }
#pragma unroll
                        for (int c2 = c + 1; c2 < kCholPanel; ++c2) {
                            if (c2 < nbw) {
                                const double l2 = bcast_lane(P[0][c], c2);  // L[jb + c2][j]
                                if (i0 >= jb + c2) P[0][c2] -= P[0][c] * l2;
                                P[1][c2] -= P[1][c] * l2;
                            }
                        }
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < kCholPanel; ++c) {
                if (c < nbw && i0 < a && i0 >= jb + c) F[i0 * FS + jb + c] = P[0][c];
                if (c < nbw && i1 < a) F[i1 * FS + jb + c] = P[1][c];
            }
            if (lane == 0) s_minpiv = fmin(s_minpiv, minp);
        }
        __syncthreads();
        // trailing update: F[i][i2] -= sum_c L[i][jb + c] L[i2][jb + c], jb + nbw <= i2 <= i
        const int t0 = jb + nbw;
        for (int i = t0 + wid; i < a; i += nwave) {
            double li[kCholPanel];
#pragma unroll
            for (int c = 0; c < kCholPanel; ++c) li[c] = (c < nbw) ? F[i * FS + jb + c] : 0.0;
            for (int i2 = t0 + lane; i2 <= i; i2 += 64) {
                double sacc = 0.0;
#pragma unroll
                for (int c = 0; c < kCholPanel; ++c)
                    if (c < nbw) sacc = fma(li[c], F[i2 * FS + jb + c], sacc);
                F[i * FS + i2] -= sacc;
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        int r = 0;
        for (int j = 0; j < a; ++j) {
            if (s_pos[j] >= 0) {
                s_pos[j] = r;
                s_kept[r] = j;
                info_i[1 + r] = j;
                ++r;
            }
        }
        s_r = r;
        info_i[0] = r;
        info_d[0] = s_minpiv;
    }
    __syncthreads();
    const int r = s_r;

    // ---- inverse of the modified L by 16 x 16 blocks ----
    // Lm: L over kept rows and columns, identity on dropped ones. Dropped
    // columns are already zero below the diagonal; the rows of dropped
    // columns are zeroed here and the diagonal of Lm goes to s_dm, so that
    // every strictly lower Lm(i, j) is the plain LDS read F[i][j].
    for (int i = t; i < a; i += nth) s_dm[i] = (s_pos[i] < 0) ? 1.0 : s_dl[i];
    for (int e = t; e < a * a; e += nth) {
        const int i = e / a, j = e % a;
        if (j < i && s_pos[i] < 0) F[i * FS + j] = 0.0;
    }
    __syncthreads();
    // Linv(i, j), i >= j, is stored transposed at F[j][i] (its diagonal on
    // F's diagonal, which Lm no longer needs).
    const int nbk = (a + kCholPanel - 1) / kCholPanel;
    // diagonal blocks: wave b inverts block b, lane c forms column c by
    // forward substitution
    for (int b = wid; b < nbk; b += nwave) {
        const int b0 = b * kCholPanel, bs = min(kCholPanel, a - b0);
        const int c = lane;
        if (c < bs) {
            double x[kCholPanel];
#pragma unroll
            for (int rr = 0; rr < kCholPanel; ++rr) {
                double v = 0.0;
                if (rr < bs && rr >= c) {
                    double sacc = (rr == c) ? 1.0 : 0.0;
#pragma unroll
                    for (int q = 0; q < kCholPanel; ++q)
                        if (q >= c && q < rr) sacc -= F[(b0 + rr) * FS + b0 + q] * x[q];
                    v = sacc / s_dm[b0 + rr];
                }
                x[rr] = v;
            }
#pragma unroll
            for (int rr = 0; rr < kCholPanel; ++rr)
                if (rr < bs && rr >= c) F[(b0 + c) * FS + b0 + rr] = x[rr];
        }
    }
    __syncthreads();
    // block diagonals: Linv[I][J] = -Linv[I][I] sum_{K=J}^{I-1} L[I][K] Linv[K][J]
    for (int dist = 1; dist < nbk; ++dist) {
        const int npair = nbk - dist;
        for (int e = t; e < npair * kCholPanel * kCholPanel; e += nth) {
            const int J = e / (kCholPanel * kCholPanel), I = J + dist;
            const int rr = (e / kCholPanel) % kCholPanel, cc = e % kCholPanel;
            const int gi = I * kCholPanel + rr, gj = J * kCholPanel + cc;
            double sacc = 0.0;
            if (gi < a) {
                // reads of 8 steps issued before their FMAs (same order of the sum)
                const double* li = F + (size_t)gi * FS;
                const double* lj = F + (size_t)gj * FS;
                const int gend = I * kCholPanel;
                int gk = gj;
                for (; gk + 8 <= gend; gk += 8) {
                    double lv[8], xv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        lv[u] = li[gk + u];
                        xv[u] = lj[gk + u];
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) sacc = fma(lv[u], xv[u], sacc);
                }
                if (gk < gend) {  // fewer than 8 steps left
                    double lv[8], xv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const bool ok = gk + u < gend;
                        lv[u] = ok ? li[gk + u] : 0.0;
                        xv[u] = ok ? lj[gk + u] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (gk + u < gend) sacc = fma(lv[u], xv[u], sacc);
                }
            }
            s_tmp[e] = sacc;
        }
        __syncthreads();
        for (int e = t; e < npair * kCholPanel * kCholPanel; e += nth) {
            const int J = e / (kCholPanel * kCholPanel), I = J + dist;
            const int rr = (e / kCholPanel) % kCholPanel, cc = e % kCholPanel;
            const int gi = I * kCholPanel + rr, gj = J * kCholPanel + cc;
            if (gi >= a) continue;
            // the rr + 1 <= 16 terms read first, then summed in order
            double xv[kCholPanel], tv[kCholPanel];
#pragma unroll
            for (int q = 0; q < kCholPanel; ++q) {
                const bool ok = q <= rr;
                xv[q] = ok ? F[(I * kCholPanel + q) * FS + gi] : 0.0;
                tv[q] = ok ? s_tmp[J * kCholPanel * kCholPanel + q * kCholPanel + cc] : 0.0;
            }
            double sacc = 0.0;
#pragma unroll
            for (int q = 0; q < kCholPanel; ++q)
                if (q <= rr) sacc = fma(xv[q], tv[q], sacc);
            F[gj * FS + gi] = -sacc;
        }
        __syncthreads();
    }
    // T = D R^{-1} on the kept columns: T[i][q] = D_i X[i][kept q], X = L^{-T}
    for (int e = t; e < a * r; e += nth) {
        const int i = e / r, q = e % r;
        const int p = s_pos[i];
        double v = 0.0;
        if (p >= 0 && p <= q) v = s_D[i] * F[i * FS + s_kept[q]];
        T[e] = v;
    }
}

__global__ __launch_bounds__(kSmall) void chol_drop_blocked_kernel(int a, const double* __restrict__ G,
                                                                   double* __restrict__ T,
                                                                   int* __restrict__ info_i,
                                                                   double* __restrict__ info_d, double drop_tol2,
                                                                   double ns_tol) {
    chol_drop_blocked_kernel_body(blockIdx.x, a, G, T, info_i, info_d, drop_tol2, ns_tol);
}


// ---------------------------------------------------------------------------
// Householder tridiagonalization of the symmetric m x m matrix A (row-major,
// both triangles kept up to date; copied into LDS when it fits). Reflector k
// acts on rows/columns k+1..m-1: H_k = I - tau_k v_k v_k^T with v_k stored in
// Vh row k from column k+1 (leading 1 explicit). d / e = diagonal /
// off-diagonal of the result.
template <bool kInLds>  // the matrix is copied into dynamic LDS (m^2 <= kLdsDoubles)
__device__ __forceinline__ void tridiag_kernel_body(int bx, int m, int kend, double* __restrict__ Ag,
                                                       double* __restrict__ d,
                                                       double* __restrict__ e,
                                                       double* __restrict__ tau,
                                                       double* __restrict__ Vh) {
    constexpr int NTH = kTri;
    constexpr int NW = NTH / 64;
    extern __shared__ double dyn[];
    __shared__ double sv[1024];
    __shared__ double sw[1024];
    __shared__ double sp[NTH];
    __shared__ double sred[NW];
    __shared__ double s_scal[4];
    const int t = threadIdx.x;
    double* A = kInLds ? dyn : Ag;
    if (kInLds) {
        for (size_t q = t; q < (size_t)m * m; q += NTH) dyn[q] = Ag[q];
        __syncthreads();
    }
    const int klast = min(kend, m - 2);
    for (int k = 0; k < klast; ++k) {
        const int L = m - k - 1;
        const double* row = A + (size_t)k * m + (k + 1);
        double part = 0.0;
        for (int i = 1 + t; i < L; i += NTH) part += row[i] * row[i];
        part = wave_sum(part);
        if ((t & 63) == 0) sred[t >> 6] = part;
        __syncthreads();
        if (t == 0) {
            double sigma2 = 0.0;
            for (int q = 0; q < NW; ++q) sigma2 += sred[q];
            const double alpha = row[0];
            double tk = 0.0, beta = alpha, scale = 0.0;
            if (sigma2 > 0.0) {
                beta = -copysign(sqrt(alpha * alpha + sigma2), alpha);
                tk = (beta - alpha) / beta;
                scale = 1.0 / (alpha - beta);
            }
            s_scal[0] = tk;
            s_scal[1] = scale;
            e[k] = beta;
            d[k] = A[(size_t)k * m + k];
            tau[k] = tk;
        }
        __syncthreads();
        const double tk = s_scal[0], scale = s_scal[1];
        for (int i = t; i < L; i += NTH) {
            const double v = (i == 0) ? 1.0 : (tk != 0.0 ? row[i] * scale : 0.0);
            sv[i] = v;
            Vh[(size_t)k * m + k + 1 + i] = v;
        }
        __syncthreads();
        if (tk == 0.0) continue;
        // p = tau * A22 v, A22 = A[k+1:, k+1:]; each column summed by G row
        // groups (G >= 1 since L < m <= 1024)
        const int G = NTH / L;
        {
            const int i = t % L, g = t / L;
            if (g < G) {
                double s = 0.0;
                const double* colp = A + (size_t)(k + 1) * m + (k + 1) + i;
                for (int jj = g; jj < L; jj += G) s = fma(colp[(size_t)jj * m], sv[jj], s);
                sp[g * L + i] = s;
            }
        }
        __syncthreads();
        double pv = 0.0;
        for (int i = t; i < L; i += NTH) {
            double s = 0.0;
            for (int q = 0; q < G; ++q) s += sp[q * L + i];
            s *= tk;
            sw[i] = s;
            pv += s * sv[i];
        }
        pv = wave_sum(pv);
        if ((t & 63) == 0) sred[t >> 6] = pv;
        __syncthreads();
        double pvs = 0.0;
        for (int q = 0; q < NW; ++q) pvs += sred[q];
        const double Kc = 0.5 * tk * pvs;
        for (int i = t; i < L; i += NTH) sw[i] -= Kc * sv[i];
        __syncthreads();
        for (size_t q = t; q < (size_t)L * L; q += NTH) {
            const int jj = (int)(q / L), i = (int)(q % L);
            A[(size_t)(k + 1 + jj) * m + (k + 1 + i)] -= sv[jj] * sw[i] + sw[jj] * sv[i];
        }
        __syncthreads();
    }
    if (klast == m - 2 && t == 0) {
        if (m >= 2) {
            d[m - 2] = A[(size_t)(m - 2) * m + (m - 2)];
            e[m - 2] = A[(size_t)(m - 1) * m + (m - 2)];
        }
        d[m - 1] = A[(size_t)(m - 1) * m + (m - 1)];
    }
}

template <bool kInLds>
__global__ __launch_bounds__(kTri) void tridiag_kernel(int m, int kend, double* __restrict__ Ag,
                                                       double* __restrict__ d,
                                                       double* __restrict__ e,
                                                       double* __restrict__ tau,
                                                       double* __restrict__ Vh) {
    tridiag_kernel_body<kInLds>(blockIdx.x, m, kend, Ag, d, e, tau, Vh);
}


// ---------------------------------------------------------------------------
// Householder tridiagonalization of small matrices (m <= 64) by one wave:
// lane l owns row l of the matrix, kept in LDS with an odd row stride (no
// bank conflicts when the lanes walk a column). Same reflectors and outputs
// as tridiag_kernel; with a single wave the barriers are free, so a
// reflector costs a few passes over the lane's row instead of several
// workgroup-wide synchronizations.
constexpr int kWaveTri = 64;
__device__ __forceinline__ void tridiag_wave_kernel_body(int bx, int m, const double* __restrict__ Ag,
                                                          double* __restrict__ d, double* __restrict__ e,
                                                          double* __restrict__ tau, double* __restrict__ Vh) {
    constexpr int S = kWaveTri + 1;
    __shared__ double A[kWaveTri * S];
    __shared__ double sv[kWaveTri];
    __shared__ double sw[kWaveTri];
    const int l = threadIdx.x;
    for (int q = l; q < m * m; q += 64) A[(q / m) * S + q % m] = Ag[q];
    __syncthreads();
    for (int k = 0; k + 2 < m; ++k) {
        const bool below = l > k && l < m;
        const double xl = below ? A[l * S + k] : 0.0;  // column k under the diagonal
        const double sigma2 = wave_sum((l >= k + 2 && l < m) ? xl * xl : 0.0);
        const double alpha = bcast_lane(xl, k + 1);
        double tk = 0.0, beta = alpha, scale = 0.0;
        if (sigma2 > 0.0) {
            beta = -copysign(sqrt(alpha * alpha + sigma2), alpha);
            tk = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
        if (l == 0) {
            d[k] = A[k * S + k];
            e[k] = beta;
            tau[k] = tk;
        }
        const double v = (l == k + 1) ? 1.0 : ((l > k + 1 && l < m && tk != 0.0) ? xl * scale : 0.0);
        if (below) Vh[(size_t)k * m + l] = v;
        if (tk == 0.0) continue;  // uniform
        sv[l] = v;
        __syncthreads();
        // p = tau A22 v (row l), K = tau/2 p.v, w = p - K v
        double p = 0.0;
        if (below) {
            double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;  // four chains hide the FMA latency
            int j = k + 1;
            for (; j + 3 < m; j += 4) {
                p0 = fma(A[l * S + j], sv[j], p0);
                p1 = fma(A[l * S + j + 1], sv[j + 1], p1);
                p2 = fma(A[l * S + j + 2], sv[j + 2], p2);
                p3 = fma(A[l * S + j + 3], sv[j + 3], p3);
            }
            for (; j < m; ++j) p0 = fma(A[l * S + j], sv[j], p0);
            p = tk * ((p0 + p1) + (p2 + p3));
        }
        const double Kc = 0.5 * tk * wave_sum(p * v);
        const double w = p - Kc * v;
        sw[l] = w;
        __syncthreads();
        // A22 -= v w^T + w v^T
        if (below)
            for (int j = k + 1; j < m; ++j) A[l * S + j] -= v * sw[j] + w * sv[j];
        __syncthreads();
    }
    if (l == 0) {
        if (m >= 2) {
            d[m - 2] = A[(m - 2) * S + (m - 2)];
            e[m - 2] = A[(m - 1) * S + (m - 2)];
        }
        d[m - 1] = A[(m - 1) * S + (m - 1)];
    }
}

__global__ __launch_bounds__(64) void tridiag_wave_kernel(int m, const double* __restrict__ Ag,
                                                          double* __restrict__ d, double* __restrict__ e,
                                                          double* __restrict__ tau, double* __restrict__ Vh) {
    tridiag_wave_kernel_body(blockIdx.x, m, Ag, d, e, tau, Vh);
}


// ---------------------------------------------------------------------------
// Register-resident Householder tridiagonalization for m <= min(16 RR, 32 RC).
// 512 threads form a 16 x 32 grid; thread (ty, tx) owns the elements (r, c)
// with r = 16 i + ty, c = 32 j + tx (i < RR, j < RC) in registers; elements
// past m are zero. Per reflector k: the owners of column k publish it to LDS
// (barrier), every wave reduces the Householder scalars itself, each thread
// forms its share of p = tau A22 v and a row-partial sum per owned row
// (barrier), one thread per row completes p (barrier), every wave reduces
// K = tau/2 p.v, and each thread applies A22 -= v w^T + w v^T to all of its
// elements. v and w are exactly zero outside rows k+1 .. m-1, so the update
// needs no per-element test and leaves the reduced part and the padding
// unchanged. LDS vectors are double-buffered by step parity.
template <int RR, int RC>
__device__ __forceinline__ void tridiag_reg_kernel_body(int bx, int mfull, int k0,
                                                          const double* __restrict__ Ag,
                                                          double* __restrict__ dg,
                                                          double* __restrict__ eg,
                                                          double* __restrict__ taug,
                                                          double* __restrict__ Vhg) {
    // Works on the trailing block A[k0:, k0:] (order m); outputs go to the
    // global positions k0 + k.
    const int m = mfull - k0;
    double* d = dg + k0;
    double* e = eg + k0;
    double* tau = taug + k0;
    constexpr int NT = 512;
    constexpr int MR = 16 * RR, MC = 32 * RC;
    constexpr int ML = MR > MC ? MR : MC;
    __shared__ double sx[2][ML];      // column k (rows owned; zero past m)
    __shared__ double sp[2][ML];      // tau A22 v, zero outside k+1 .. m-1
    __shared__ double rowpart[MR][33];  // per-thread row partials of A22 v
    const int t = threadIdx.x;
    const int tx = t & 31, ty = t >> 5;
    const int lane = t & 63;
    for (int q = t; q < 2 * ML; q += NT) {
        (&sx[0][0])[q] = 0.0;
        (&sp[0][0])[q] = 0.0;
    }
    double a[RR][RC];
#pragma unroll
    for (int i = 0; i < RR; ++i)
#pragma unroll
        for (int j = 0; j < RC; ++j) {
            const int r = 16 * i + ty, c = 32 * j + tx;
            a[i][j] = (r < m && c < m) ? Ag[(size_t)(k0 + r) * mfull + (k0 + c)] : 0.0;
        }
    __syncthreads();
    for (int k = 0; k + 2 < m; ++k) {
        const int par = k & 1;
        const int kj = k >> 5;
        // (1) column k (all owned rows) and the diagonal element; kj is
        // uniform, so the register column is chosen by a scalar branch
        if (tx == (k & 31)) {
            switch (kj) {
#define SE_REG_PUB(J)                                              \
    case J:                                                        \
        if (J < RC) {                                              \
            _Pragma("unroll") for (int i = 0; i < RR; ++i) {       \
                const double x = a[i][J < RC ? J : 0];             \
                sx[par][16 * i + ty] = x;                          \
                if (16 * i + ty == k) d[k] = x;                    \
            }                                                      \
        }                                                          \
        break;
                SE_REG_PUB(0) SE_REG_PUB(1) SE_REG_PUB(2) SE_REG_PUB(3)
                SE_REG_PUB(4) SE_REG_PUB(5) SE_REG_PUB(6) SE_REG_PUB(7)
#undef SE_REG_PUB
                default: break;
            }
        }
        __syncthreads();
        // (2) Householder scalars, reduced redundantly by every wave
        const int L = m - k - 1;
        double part = 0.0;
        for (int r = k + 2 + lane; r < m; r += 64) part += sx[par][r] * sx[par][r];
        const double sigma2 = wave_sum(part);
        const double alpha = sx[par][k + 1];
        double tk = 0.0, beta = alpha, scale = 0.0;
        if (sigma2 > 0.0) {
            beta = -copysign(sqrt(alpha * alpha + sigma2), alpha);
            tk = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
        if (t == 0) {
            e[k] = beta;
            tau[k] = tk;
        }
        for (int q = t; q < L; q += NT) {
            const int r = k + 1 + q;
            Vhg[(size_t)(k0 + k) * mfull + (k0 + r)] = (q == 0) ? 1.0 : (tk != 0.0 ? sx[par][r] * scale : 0.0);
        }
        if (tk == 0.0) continue;  // uniform; the next step uses the other buffers
        // v on this thread's columns: 1 at k+1, x scale on k+2 .. m-1, else 0
        double vc[RC];
#pragma unroll
        for (int j = 0; j < RC; ++j) {
            const int c = 32 * j + tx;
            const double xs = sx[par][c] * scale;
            vc[j] = (c == k + 1) ? 1.0 : ((c > k + 1 && c < m) ? xs : 0.0);
        }
        // (3) row partials of A22 v over this thread's columns
#pragma unroll
        for (int i = 0; i < RR; ++i) {
            double sacc = 0.0;
#pragma unroll
            for (int j = 0; j < RC; ++j) sacc = fma(a[i][j], vc[j], sacc);
            rowpart[16 * i + ty][tx] = sacc;
        }
        __syncthreads();
        if (t < MR) {
            double sacc = 0.0;
#pragma unroll
            for (int q = 0; q < 32; ++q) sacc += rowpart[t][q];
            sp[par][t] = (t > k && t < m) ? tk * sacc : 0.0;
        }
        __syncthreads();
        // (4) K = tau/2 p.v, reduced redundantly by every wave
        double pv = 0.0;
        for (int r = k + 1 + lane; r < m; r += 64)
            pv += sp[par][r] * ((r == k + 1) ? 1.0 : sx[par][r] * scale);
        const double Kc = 0.5 * tk * wave_sum(pv);
        // (5) A22 -= v w^T + w v^T with w = p - K v, on every owned element
        double wc[RC];
#pragma unroll
        for (int j = 0; j < RC; ++j) wc[j] = sp[par][32 * j + tx] - Kc * vc[j];
#pragma unroll
        for (int i = 0; i < RR; ++i) {
            const int r = 16 * i + ty;
            const double xs = sx[par][r] * scale;
            const double vr = (r == k + 1) ? 1.0 : ((r > k + 1 && r < m) ? xs : 0.0);
            const double wr = sp[par][r] - Kc * vr;
#pragma unroll
            for (int j = 0; j < RC; ++j) a[i][j] = fma(-wr, vc[j], fma(-vr, wc[j], a[i][j]));
        }
    }
    // last 2 x 2 block
#pragma unroll
    for (int i = 0; i < RR; ++i)
#pragma unroll
        for (int j = 0; j < RC; ++j) {
            const int r = 16 * i + ty, c = 32 * j + tx;
            if (m >= 2 && r == m - 2 && c == m - 2) d[m - 2] = a[i][j];
            if (m >= 2 && r == m - 1 && c == m - 2) e[m - 2] = a[i][j];
            if (r == m - 1 && c == m - 1) d[m - 1] = a[i][j];
        }
}

template <int RR, int RC>
__global__ __launch_bounds__(512) void tridiag_reg_kernel(int mfull, int k0,
                                                          const double* __restrict__ Ag,
                                                          double* __restrict__ dg,
                                                          double* __restrict__ eg,
                                                          double* __restrict__ taug,
                                                          double* __restrict__ Vhg) {
    tridiag_reg_kernel_body<RR, RC>(blockIdx.x, mfull, k0, Ag, dg, eg, taug, Vhg);
}


// ---------------------------------------------------------------------------
// The k smallest eigenvalues of the symmetric tridiagonal (d, e) by
// multisection: one wave per eigenvalue, each lane evaluates the Sturm count
// at one of 64 interior points of the bracket, so it shrinks 65x per round.
__device__ __forceinline__ int sturm_count(int m, const double* d, const double* e2, double x,
                                           double pivmin) {
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int cnt = q < 0.0;
    for (int t = 1; t < m; ++t) {
        q = d[t] - x - e2[t - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0;
    }
    return cnt;
}

__device__ __forceinline__ void bisect_kernel_body(int bx, int m, int k, const double* __restrict__ dg,
                                                     const double* __restrict__ eg,
                                                     double* __restrict__ w,
                                                     double* __restrict__ scal) {
    __shared__ double d[1024];
    __shared__ double e2[1024];
    __shared__ double ae[1024];
    __shared__ double s_lo[256], s_hi[256], s_em[256];
    __shared__ double s_gl[1], s_gu[1], s_pm[1];
    const int tt = threadIdx.x;
    for (int i = tt; i < m; i += 256) {
        d[i] = dg[i];
        if (i + 1 < m) {
            const double ei = eg[i];
            e2[i] = ei * ei;
            ae[i] = fabs(ei);
        }
    }
    __syncthreads();
    // Gershgorin bounds and the largest e^2 by all threads (min and max are
    // exact in any order, so this equals the sequential scan)
    {
        double gl = DBL_MAX, gu = -DBL_MAX, emax2 = 0.0;
        for (int i = tt; i < m; i += 256) {
            const double ea = (i > 0 ? ae[i - 1] : 0.0) + (i + 1 < m ? ae[i] : 0.0);
            gl = fmin(gl, d[i] - ea);
            gu = fmax(gu, d[i] + ea);
            if (i + 1 < m) emax2 = fmax(emax2, e2[i]);
        }
        s_lo[tt] = gl;
        s_hi[tt] = gu;
        s_em[tt] = emax2;
    }
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tt < h) {
            s_lo[tt] = fmin(s_lo[tt], s_lo[tt + h]);
            s_hi[tt] = fmax(s_hi[tt], s_hi[tt + h]);
            s_em[tt] = fmax(s_em[tt], s_em[tt + h]);
        }
        __syncthreads();
    }
    if (tt == 0) {
        double gl = s_lo[0], gu = s_hi[0];
        const double emax2 = s_em[0];
        const double pivmin = DBL_MIN * fmax(1.0, emax2);
        const double tnorm = fmax(fabs(gl), fabs(gu));
        gl -= 2.0 * DBL_EPSILON * tnorm * m + 4.0 * pivmin;
        gu += 2.0 * DBL_EPSILON * tnorm * m + 4.0 * pivmin;
        s_gl[0] = gl;
        s_gu[0] = gu;
        s_pm[0] = pivmin;
        if (bx == 0) scal[0] = tnorm;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int idx = bx * 4 + (threadIdx.x >> 6);
    if (idx >= k) return;
    double lo = s_gl[0], hi = s_gu[0];
    const double pivmin = s_pm[0];
    for (int it = 0; it < 40; ++it) {
        const double tolr = 4.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + 4.0 * pivmin;
        if (hi - lo <= tolr) break;
        const double x = lo + (hi - lo) * (double)(lane + 1) / 65.0;
        const int c = sturm_count(m, d, e2, x, pivmin);
        const unsigned long long mask = __ballot(c > idx);
        double nlo, nhi;
        if (mask == 0ull) {
            nlo = bcast_lane(x, 63);
            nhi = hi;
        } else {
            const int first = __ffsll((long long)mask) - 1;
            nhi = bcast_lane(x, first);
            nlo = (first > 0) ? bcast_lane(x, first - 1) : lo;
        }
        lo = nlo;
        hi = nhi;
    }
    if (lane == 0) w[idx] = 0.5 * (lo + hi);
}

__global__ __launch_bounds__(256) void bisect_kernel(int m, int k, const double* __restrict__ dg,
                                                     const double* __restrict__ eg,
                                                     double* __restrict__ w,
                                                     double* __restrict__ scal) {
    bisect_kernel_body(blockIdx.x, m, k, dg, eg, w, scal);
}


// ---------------------------------------------------------------------------
// Eigenvectors of the tridiagonal for the k computed eigenvalues by inverse
// iteration (one thread per eigenvalue, two steps from a pseudo-random start,
// LU with partial pivoting of T - shift I). Shifts that coincide to a few ulps
// are separated slightly so that a degenerate cluster yields independent
// vectors; the caller orthonormalizes the block afterwards.
// ZT[j * k + i] = component j of eigenvector i.
__device__ __forceinline__ double hash_unit(unsigned i, unsigned j) {
    unsigned h = i * 0x9E3779B1u ^ (j + 0x7F4A7C15u) * 0x85EBCA77u;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    h *= 0x297A2D39u;
    h ^= h >> 15;
    return (double)(h & 0xFFFFFF) / 8388608.0 - 1.0;
}

__device__ __forceinline__ void invit_kernel_body(int bx, int m, int k, const double* __restrict__ dg,
                                                    const double* __restrict__ eg,
                                                    const double* __restrict__ w,
                                                    const double* __restrict__ scal,
                                                    double* __restrict__ ZT,
                                                    double* __restrict__ work) {
    const int i = bx * 256 + threadIdx.x;
    if (i >= k) return;
    double* DL = work;
    double* DD = DL + (size_t)m * k;
    double* DU = DD + (size_t)m * k;
    double* DU2 = DU + (size_t)m * k;
    int* IP = reinterpret_cast<int*>(DU2 + (size_t)m * k);
    const double tnorm = fmax(scal[0], DBL_MIN);
    const double tiny = DBL_EPSILON * tnorm;
    const double sep = 10.0 * DBL_EPSILON * tnorm;
    int run = 0;
    for (int q = i; q > 0 && w[q] - w[q - 1] <= sep; --q) ++run;
    const double lam = w[i] + run * sep;
    auto guard = [&](double x) { return fabs(x) < tiny ? copysign(tiny, x == 0.0 ? 1.0 : x) : x; };
#define AT(arr, j) arr[(size_t)(j) * k + i]
    // LU factorization with partial pivoting of T - lam I. The diagonal and
    // superdiagonal entries that step j modifies for row j + 1 are carried in
    // registers, so every load reads an input (no store-to-load chain through
    // memory) and each factor entry is stored once.
    double dcur = dg[0] - lam;
    double ucur = (m > 1) ? eg[0] : 0.0;
#pragma unroll 4
    for (int j = 0; j + 1 < m; ++j) {
        const double lj = eg[j];
        const double dn = dg[j + 1] - lam;
        const double un = (j + 2 < m) ? eg[j + 1] : 0.0;
        if (fabs(dcur) >= fabs(lj)) {
            const double f = (dcur != 0.0) ? lj / dcur : 0.0;
            AT(IP, j) = j;
            AT(DL, j) = (dcur != 0.0) ? f : lj;
            AT(DD, j) = guard(dcur);
            AT(DU, j) = ucur;
            AT(DU2, j) = 0.0;
            dcur = (dcur != 0.0) ? dn - f * ucur : dn;
            ucur = un;
        } else {
            const double f = dcur / lj;
            AT(IP, j) = j + 1;
            AT(DD, j) = guard(lj);
            AT(DL, j) = f;
            AT(DU, j) = dn;
            AT(DU2, j) = un;
            dcur = ucur - f * dn;
            ucur = -f * un;
        }
    }
    AT(DD, m - 1) = guard(dcur);
    for (int j = 0; j < m; ++j) AT(ZT, j) = hash_unit((unsigned)i, (unsigned)j);
    for (int it = 0; it < 2; ++it) {
        // forward: apply the row interchanges and L^{-1} (carrying the row
        // being eliminated)
        double bcur = AT(ZT, 0);
#pragma unroll 8
        for (int j = 0; j + 1 < m; ++j) {
            const double bn = AT(ZT, j + 1);
            const double l = AT(DL, j);
            if (AT(IP, j) == j) {
                AT(ZT, j) = bcur;
                bcur = bn - l * bcur;
            } else {
                AT(ZT, j) = bn;
                bcur = bcur - l * bn;
            }
        }
        // back substitution with U (diagonal, first and second superdiagonal)
        double z1 = bcur / AT(DD, m - 1);
        AT(ZT, m - 1) = z1;
        double z2 = 0.0;
        if (m >= 2) {
            const double zz = (AT(ZT, m - 2) - AT(DU, m - 2) * z1) / AT(DD, m - 2);
            AT(ZT, m - 2) = zz;
            z2 = z1;
            z1 = zz;
        }
        double mx = fmax(fabs(z1), fabs(z2));
#pragma unroll 8
        for (int j = m - 3; j >= 0; --j) {
            const double zz = (AT(ZT, j) - AT(DU, j) * z1 - AT(DU2, j) * z2) / AT(DD, j);
            AT(ZT, j) = zz;
            z2 = z1;
            z1 = zz;
            mx = fmax(mx, fabs(zz));
        }
        const double sc = (mx > 0.0) ? 1.0 / mx : 1.0;
        double nr = 0.0;
        for (int j = 0; j < m; ++j) {
            const double v = AT(ZT, j) * sc;
            AT(ZT, j) = v;
            nr += v * v;
        }
        if (it == 1) {
            const double inv = 1.0 / sqrt(nr);
            for (int j = 0; j < m; ++j) AT(ZT, j) *= inv;
        }
    }
#undef AT
}

__global__ __launch_bounds__(256) void invit_kernel(int m, int k, const double* __restrict__ dg,
                                                    const double* __restrict__ eg,
                                                    const double* __restrict__ w,
                                                    const double* __restrict__ scal,
                                                    double* __restrict__ ZT,
                                                    double* __restrict__ work) {
    invit_kernel_body(blockIdx.x, m, k, dg, eg, w, scal, ZT, work);
}


// The same inverse iteration with the factors and the iterate of each
// eigenvalue in LDS (E eigenvalues per workgroup, one per lane of a single
// wave): the recurrences read LDS instead of waiting on L2 at every step.
// Arithmetic identical to invit_kernel. LDS: E (5 m doubles + m bytes).
__global__ __launch_bounds__(64) void invit_lds_kernel(int m, int k, int E, const double* __restrict__ dg,
                                                       const double* __restrict__ eg,
                                                       const double* __restrict__ w,
                                                       const double* __restrict__ scal,
                                                       double* __restrict__ ZT) {
    extern __shared__ double sm[];
    const int lane = threadIdx.x;
    const int i = blockIdx.x * E + lane;
    double* DL = sm;                      // [j][E]
    double* DD = DL + (size_t)m * E;
    double* DU = DD + (size_t)m * E;
    double* DU2 = DU + (size_t)m * E;
    double* Z = DU2 + (size_t)m * E;
    unsigned char* IP = reinterpret_cast<unsigned char*>(Z + (size_t)m * E);
    if (lane >= E || i >= k) return;
    const double tnorm = fmax(scal[0], DBL_MIN);
    const double tiny = DBL_EPSILON * tnorm;
    const double sep = 10.0 * DBL_EPSILON * tnorm;
    int run = 0;
    for (int q = i; q > 0 && w[q] - w[q - 1] <= sep; --q) ++run;
    const double lam = w[i] + run * sep;
    auto guard = [&](double x) { return fabs(x) < tiny ? copysign(tiny, x == 0.0 ? 1.0 : x) : x; };
#define AT(arr, j) arr[(size_t)(j) * E + lane]
    double dcur = dg[0] - lam;
    double ucur = (m > 1) ? eg[0] : 0.0;
#pragma unroll 4
    for (int j = 0; j + 1 < m; ++j) {
        const double lj = eg[j];
        const double dn = dg[j + 1] - lam;
        const double un = (j + 2 < m) ? eg[j + 1] : 0.0;
        if (fabs(dcur) >= fabs(lj)) {
            const double f = (dcur != 0.0) ? lj / dcur : 0.0;
            AT(IP, j) = 0;
            AT(DL, j) = (dcur != 0.0) ? f : lj;
            AT(DD, j) = guard(dcur);
            AT(DU, j) = ucur;
            AT(DU2, j) = 0.0;
            dcur = (dcur != 0.0) ? dn - f * ucur : dn;
            ucur = un;
        } else {
            const double f = dcur / lj;
            AT(IP, j) = 1;
            AT(DD, j) = guard(lj);
            AT(DL, j) = f;
            AT(DU, j) = dn;
            AT(DU2, j) = un;
            dcur = ucur - f * dn;
            ucur = -f * un;
        }
    }
    AT(DD, m - 1) = guard(dcur);
    for (int j = 0; j < m; ++j) AT(Z, j) = hash_unit((unsigned)i, (unsigned)j);
    for (int it = 0; it < 2; ++it) {
        double bcur = AT(Z, 0);
#pragma unroll 8
        for (int j = 0; j + 1 < m; ++j) {
            const double bn = AT(Z, j + 1);
            const double l = AT(DL, j);
            if (AT(IP, j) == 0) {
                AT(Z, j) = bcur;
                bcur = bn - l * bcur;
            } else {
                AT(Z, j) = bn;
                bcur = bcur - l * bn;
            }
        }
        double z1 = bcur / AT(DD, m - 1);
        AT(Z, m - 1) = z1;
        double z2 = 0.0;
        if (m >= 2) {
            const double zz = (AT(Z, m - 2) - AT(DU, m - 2) * z1) / AT(DD, m - 2);
            AT(Z, m - 2) = zz;
            z2 = z1;
            z1 = zz;
        }
        double mx = fmax(fabs(z1), fabs(z2));
#pragma unroll 8
        for (int j = m - 3; j >= 0; --j) {
            const double zz = (AT(Z, j) - AT(DU, j) * z1 - AT(DU2, j) * z2) / AT(DD, j);
            AT(Z, j) = zz;
            z2 = z1;
            z1 = zz;
            mx = fmax(mx, fabs(zz));
        }
        const double sc = (mx > 0.0) ? 1.0 / mx : 1.0;
        double nr = 0.0;
        for (int j = 0; j < m; ++j) {
            const double v = AT(Z, j) * sc;
            AT(Z, j) = v;
            nr += v * v;
        }
        if (it == 1) {
            const double inv = 1.0 / sqrt(nr);
            for (int j = 0; j < m; ++j) ZT[(size_t)j * k + i] = AT(Z, j) * inv;
        }
    }
#undef AT
}

// Eigenvalues per workgroup of invit_lds_kernel for order m (0: the matrix is
// too large for its LDS; use invit_kernel).
int invit_lds_per_block(int m) {
    const size_t per = (size_t)m * (5 * sizeof(double) + 1);
    const int E = (int)std::min<size_t>(64, (150 * 1024) / per);
    return E >= 2 ? E : 0;
}

// Z = Q ZT with Q = H_0 H_1 ... H_{m-3}; one wave per eigenvector, kept in
// registers (m <= 1024 -> 16 values per lane). ZT and Z are m x k (ld k).
// MAXQ = values of a column per lane (rows lane + 64 q < m); tau comes from
// LDS, filled by the whole workgroup.
template <int MAXQ>
__device__ __forceinline__ void backtransform_q(int bx, int m, int k, const double* s_tau,
                                                const double* __restrict__ Vh, const double* __restrict__ ZT,
                                                double* __restrict__ Z) {
    const int lane = threadIdx.x & 63;
    const int i = bx * 4 + (threadIdx.x >> 6);
    if (i >= k) return;
    double z[MAXQ];
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
        const int j = lane + 64 * q;
        z[q] = (j < m) ? ZT[(size_t)j * k + i] : 0.0;
    }
    // Reflector rows are prefetched one step ahead into registers, so their
    // load latency overlaps the previous reflector's dot product and update.
    double vc[MAXQ], vn[MAXQ];
    auto load_v = [&](int kk, double (&dst)[MAXQ]) {
        const double* v = Vh + (size_t)kk * m;  // v[j] valid for j >= kk + 1
#pragma unroll
        for (int q = 0; q < MAXQ; ++q) {
            const int j = lane + 64 * q;
            dst[q] = (j > kk && j < m) ? v[j] : 0.0;
        }
    };
    if (m >= 3) load_v(m - 3, vc);
    for (int kk = m - 3; kk >= 0; --kk) {
        if (kk > 0) load_v(kk - 1, vn);
        const double tk = s_tau[kk];
        if (tk != 0.0) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < MAXQ; ++q) s = fma(vc[q], z[q], s);
            s = wave_sum(s) * tk;
#pragma unroll
            for (int q = 0; q < MAXQ; ++q) z[q] = fma(-s, vc[q], z[q]);
        }
#pragma unroll
        for (int q = 0; q < MAXQ; ++q) vc[q] = vn[q];
    }
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
        const int j = lane + 64 * q;
        if (j < m) Z[(size_t)j * k + i] = z[q];
    }
}

// Z = Q ZT for Q = H_0 ... H_{m-3}: one wave per eigenvector, 256 threads.
// tau is staged in LDS first (each step's scalar was otherwise a dependent
// L2 load), and the per-lane arrays are sized for m (the rows past m are
// zero and added nothing).
__device__ __forceinline__ void backtransform_kernel_body(int bx, int m, int k, const double* __restrict__ tau,
                                                            const double* __restrict__ Vh,
                                                            const double* __restrict__ ZT,
                                                            double* __restrict__ Z) {
    __shared__ double s_tau[1024];
    for (int q = threadIdx.x; q + 2 < m; q += 256) s_tau[q] = tau[q];
    __syncthreads();
    if (m <= 256)
        backtransform_q<4>(bx, m, k, s_tau, Vh, ZT, Z);
    else if (m <= 320)
        backtransform_q<5>(bx, m, k, s_tau, Vh, ZT, Z);
    else if (m <= 512)
        backtransform_q<8>(bx, m, k, s_tau, Vh, ZT, Z);
    else if (m <= 768)
        backtransform_q<12>(bx, m, k, s_tau, Vh, ZT, Z);
    else
        backtransform_q<16>(bx, m, k, s_tau, Vh, ZT, Z);
}

__global__ __launch_bounds__(256) void backtransform_kernel(int m, int k, const double* __restrict__ tau,
                                                            const double* __restrict__ Vh,
                                                            const double* __restrict__ ZT,
                                                            double* __restrict__ Z) {
    backtransform_kernel_body(blockIdx.x, m, k, tau, Vh, ZT, Z);
}


// ---------------------------------------------------------------------------
// Householder tridiagonalization by G cooperating workgroups (a cooperative
// launch, all resident): workgroup g keeps rows [g R, g R + R) of the matrix
// in its LDS, so the trailing matrix is never re-read from memory. Per
// reflector k:
//   A. every workgroup publishes its part of column k (xcol) and of
//      sigma^2 = sum_{i >= k+2} a_ik^2 (partA[g]);        grid barrier
//   B. every workgroup forms the same Householder scalars and v (from xcol,
//      partials summed in order), then p_i = tau (A22 v)_i for its rows
//      (xp) and its part of p^T v (partB[g]);             grid barrier
//   C. w = p - (tau/2)(p^T v) v, and each workgroup applies
//      A22 -= v w^T + w v^T to its own rows.
// Every workgroup runs the same number of barriers. Outputs as tridiag_kernel.
constexpr int kCoopThreads = 1024;

__device__ double block_sum_1024(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kCoopThreads / 64; ++q) s += sh[q];
    __syncthreads();
    return s;
}

// Reflectors 0 .. kend - 1 only; when it stops early (kend < m - 2) each
// workgroup writes its updated rows back to Ag for the kernel that continues.
// Grid-wide barrier of the cooperative kernel. Wave 0 of every workgroup
// has written whatever other workgroups read; it releases those writes at
// agent scope, thread 0 adds one arrival to a counter (zeroed before the
// launch; the n-th barrier completes at n G arrivals) and waits for the
// rest, and wave 0 acquires before the workgroup barrier lets the other waves
// read. Measured 0.8-1.5 us at 5-32 workgroups, against 5-12 us for the
// cooperative-groups grid sync with a device fence in every wave. The wait
// is bounded (about a second) so that a launch that is not co-resident
// cannot hang; the launch is cooperative, so every workgroup arrives.
__device__ __forceinline__ void coop_grid_barrier(unsigned* ctr, unsigned& target) {
    target += gridDim.x;
    if (threadIdx.x < 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (threadIdx.x == 0) {
            __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (int spin = 0; spin < (1 << 24) &&
                               __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target;
                 ++spin)
                __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

__global__ void coop_reset_kernel(unsigned* ctr) { *ctr = 0u; }

// Works on the trailing block A[k0:, k0:] (order m = mfull - k0) of the
// mfull x mfull matrix; reflector k of the block is reflector k0 + k of the
// whole (outputs at the global positions). A launch that stops before the end
// (kend < m - 2) writes its updated rows back, so that a later launch with
// fewer workgroups continues on the smaller trailing block.
__global__ __launch_bounds__(kCoopThreads) void tridiag_coop_kernel(int mfull, int k0, int R, int kend,
                                                                    double* __restrict__ Ag,
                                                                    double* __restrict__ d, double* __restrict__ e,
                                                                    double* __restrict__ tau,
                                                                    double* __restrict__ Vh,
                                                                    double* __restrict__ xcol,
                                                                    double* __restrict__ xp,
                                                                    double* __restrict__ partA,
                                                                    double* __restrict__ partB,
                                                                    unsigned* __restrict__ ctr) {
    extern __shared__ double lds[];
    __shared__ double sred[kCoopThreads / 64];
    unsigned target = 0;
    const int m = mfull - k0;
    d += k0;
    e += k0;
    tau += k0;
    Vh += (size_t)k0 * mfull + k0;  // row stride mfull
    const int g = blockIdx.x, G = gridDim.x, t = threadIdx.x;
    const int r0 = g * R, r1 = min(m, r0 + R), nr = max(0, r1 - r0);
    double* Al = lds;                    // nr x m, row-major
    double* v = Al + (size_t)R * m;      // m
    double* w = v + m;                   // m
    for (size_t q = t; q < (size_t)nr * m; q += kCoopThreads) {
        const size_t i = q / m, j = q % m;
        Al[q] = Ag[(size_t)(k0 + r0 + i) * mfull + k0 + j];
    }
    __syncthreads();
    const int row_sub = t >> 5, lane32 = t & 31;  // 32 row groups of 32 lanes
    // The values other workgroups read (the column, p, the partial sums) are
    // staged in LDS (in w, free at those points) and published by wave 0
    // alone, so that only wave 0 has to release them before the grid barrier.
    for (int k = 0; k < kend && k + 2 < m; ++k) {
        // A: column k of my rows below the diagonal, partial sigma^2
        double s = 0.0;
        for (int i = max(r0, k + 1) + t; i < r1; i += kCoopThreads) {
            const double x = Al[(size_t)(i - r0) * m + k];
            w[i] = x;
            if (i >= k + 2) s = fma(x, x, s);
        }
        s = block_sum_1024(s, sred);
        if (t < 64) {
            for (int i = max(r0, k + 1) + t; i < r1; i += 64) xcol[i] = w[i];
            if (t == 0) {
                partA[g] = s;
                if (k >= r0 && k < r1) d[k] = Al[(size_t)(k - r0) * m + k];
            }
        }
        coop_grid_barrier(ctr, target);
        // B: scalars, v, p = tau A22 v on my rows
        // the G <= 128 partial sums: at most two per lane, then a wave sum
        // (one round trip to L2 instead of G dependent ones)
        const int lane = t & 63;
        double sa = 0.0;
        for (int q = lane; q < G; q += 64) sa += partA[q];
        const double sigma2 = wave_sum(sa);
        const double alpha = xcol[k + 1];
        double tk = 0.0, beta = alpha, scale = 0.0;
        if (sigma2 > 0.0) {
            beta = -copysign(sqrt(alpha * alpha + sigma2), alpha);
            tk = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
        for (int i = k + 1 + t; i < m; i += kCoopThreads)
            v[i] = (i == k + 1) ? 1.0 : (tk != 0.0 ? xcol[i] * scale : 0.0);
        __syncthreads();
        if (g == 0) {
            if (t == 0) {
                e[k] = beta;
                tau[k] = tk;
            }
            for (int i = k + 1 + t; i < m; i += kCoopThreads) Vh[(size_t)k * mfull + i] = v[i];
        }
        double pv = 0.0;
        const int rb = max(r0, k + 1);
        for (int i0 = rb; i0 < r1; i0 += 32) {
            const int i = i0 + row_sub;
            double acc = 0.0;
            if (i < r1 && tk != 0.0) {
                const double* arow = Al + (size_t)(i - r0) * m;
                for (int j = k + 1 + lane32; j < m; j += 32) acc = fma(arow[j], v[j], acc);
            }
            // sum over the 32 lanes of the row group: DPP butterflies within
            // each row of 16 lanes, then row_bcast15 adds row 0's (2's) sum
            // into row 1 (3), so lane 31 of the group holds the total
            acc += dpp_f64<0xB1>(acc);
            acc += dpp_f64<0x4E>(acc);
            acc += dpp_f64<0x141>(acc);
            acc += dpp_f64<0x140>(acc);
            acc += dpp_row_bcast15(acc);
            if (lane32 == 31 && i < r1) {
                const double pi = tk * acc;
                w[i] = pi;
                pv = fma(pi, v[i], pv);
            }
        }
        pv = block_sum_1024(pv, sred);
        if (t < 64) {
            for (int i = rb + t; i < r1; i += 64) xp[i] = w[i];
            if (t == 0) partB[g] = pv;
        }
        coop_grid_barrier(ctr, target);
        // C: w = p - K v and the rank-2 update of my rows
        if (tk != 0.0) {
            double sb = 0.0;
            for (int q = lane; q < G; q += 64) sb += partB[q];
            const double Kc = 0.5 * tk * wave_sum(sb);
            for (int j = k + 1 + t; j < m; j += kCoopThreads) w[j] = xp[j] - Kc * v[j];
            __syncthreads();
            // 32 x 32 thread tile over (my rows, columns > k)
            for (int i = rb + row_sub; i < r1; i += 32) {
                const double vi = v[i], wi = w[i];
                double* arow = Al + (size_t)(i - r0) * m;
                for (int j = k + 1 + lane32; j < m; j += 32) arow[j] -= vi * w[j] + wi * v[j];
            }
        }
        __syncthreads();
    }
    if (kend < m - 2) {
        for (size_t q = t; q < (size_t)nr * m; q += kCoopThreads) {
            const size_t i = q / m, j = q % m;
            Ag[(size_t)(k0 + r0 + i) * mfull + k0 + j] = Al[q];
        }
        return;
    }
    if (t == 0 && m >= 2) {
        if (m - 2 >= r0 && m - 2 < r1) d[m - 2] = Al[(size_t)(m - 2 - r0) * m + (m - 2)];
        if (m - 1 >= r0 && m - 1 < r1) {
            e[m - 2] = Al[(size_t)(m - 1 - r0) * m + (m - 2)];
            d[m - 1] = Al[(size_t)(m - 1 - r0) * m + (m - 1)];
        }
    }
    if (t == 0 && m == 1) d[0] = Al[0];
}

// ---------------------------------------------------------------------------
// Hetmaniuk-Lehoucq start block: B[:, c] = e_{act[c]} (unit vector in
// S-coefficients) and Y[:, c] = Z1[act[c], :]^T, so that B - Z1 Y is the part
// of the old active X columns orthogonal to the new X = S Z1.
__global__ __launch_bounds__(256) void hl_init_kernel(int m, int k, const double* __restrict__ Z1,
                                                      const int* __restrict__ act, int a,
                                                      double* __restrict__ B,
                                                      double* __restrict__ Y) {
    const int total = m * a + k * a;
    for (int q = blockIdx.x * 256 + threadIdx.x; q < total; q += gridDim.x * 256) {
        if (q < m * a) {
            const int i = q / a, c = q % a;
            B[q] = (i == act[c]) ? 1.0 : 0.0;
        } else {
            const int r = q - m * a;
            const int tt = r / a, c = r % a;
            Y[r] = Z1[(size_t)act[c] * k + tt];
        }
    }
}

// Elementwise helpers on small dense matrices.
__global__ __launch_bounds__(256) void axpby_kernel(long long count, double alpha, const double* __restrict__ X,
                                                    double beta, double* __restrict__ Y) {
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < count; e += (long long)gridDim.x * 256)
        Y[e] = alpha * X[e] + beta * Y[e];
}

__global__ __launch_bounds__(256) void add_diag_kernel(int m, double* __restrict__ A, long long ld,
                                                       double alpha) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < m) A[(long long)i * ld + i] += alpha;
}

__global__ __launch_bounds__(256) void fill_kernel(int rows, int cols, double* __restrict__ A, long long ld,
                                                   double v) {
    const long long total = (long long)rows * cols;
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < total; e += (long long)gridDim.x * 256)
        A[(e / cols) * ld + e % cols] = v;
}

// A_p (m x m) from the known block of the leading q columns (Axp, q x q)
// and the product G = S^T (A W) (m x a, a = m - q): A_p[i][j] = Axp[i][j]
// for i, j < q; G[i][j - q] and its mirror for one index >= q; the average
// of G[i][j - q] and G[j][i - q] for both >= q (W^T A W, symmetrized).
__global__ __launch_bounds__(256) void assemble_ap_kernel(int m, int q, const double* __restrict__ Axp,
                                                          const double* __restrict__ G,
                                                          double* __restrict__ Ap) {
    const int a = m - q;
    const long long total = (long long)m * m;
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < total; e += (long long)gridDim.x * 256) {
        const int i = (int)(e / m), j = (int)(e % m);
        double v;
        if (i < q && j < q)
            v = Axp[(long long)i * q + j];
        else if (j >= q && i < q)
            v = G[(long long)i * a + (j - q)];
        else if (i >= q && j < q)
            v = G[(long long)j * a + (i - q)];
        else
            v = 0.5 * (G[(long long)i * a + (j - q)] + G[(long long)j * a + (i - q)]);
        Ap[e] = v;
    }
}

// out (r x r) = in[idx[a]][idx[b]] for a, b < r (in has leading dimension ld).
__global__ __launch_bounds__(256) void gather_sym_kernel(int r, const int* __restrict__ idx,
                                                         const double* __restrict__ in, long long ld,
                                                         double* __restrict__ out) {
    const long long total = (long long)r * r;
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < total; e += (long long)gridDim.x * 256) {
        const int a = (int)(e / r), b = (int)(e % r);
        out[e] = in[(long long)idx[a] * ld + idx[b]];
    }
}

// out[0] = sum of squares of the count entries of X (one workgroup, fixed order).
__global__ __launch_bounds__(kSmall) void sumsq_kernel(long long count, const double* __restrict__ X,
                                                       double* __restrict__ out) {
    __shared__ double sh[kSWaves];
    double s = 0.0;
    for (long long e = threadIdx.x; e < count; e += kSmall) s = fma(X[e], X[e], s);
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[0] = s;
}

// Cholesky-QR transform with column drop for 112 < a <= kCholBig (same
// inputs, outputs and drop rule as chol_drop_kernel): blocked right-looking
// factorization with the scaled matrix in `work` (global memory, L2
// resident). Per panel of 16 columns, one wave factorizes the diagonal block
// (drop decisions and pivots), every thread then solves its rows below the
// block against it (dropped columns give zero entries), and the trailing lower
// triangle takes the rank-16 update with the panel's columns staged in LDS.
// The inverse of L follows by 16 x 16 blocks as in chol_drop_blocked_kernel,
// with the block products in `work` after the matrix. work: a (a | 1) +
// 16 a + 256 doubles.
constexpr int kCholBig = 896;
constexpr int kBigLP = kCholPanel + 1;  // LDS panel row stride (odd: no bank conflicts)
__device__ __forceinline__ void chol_drop_big_body(int a, const double* __restrict__ G, double* __restrict__ T,
                                                   double* __restrict__ work, int* __restrict__ info_i,
                                                   double* __restrict__ info_d, double drop_tol2, double ns_tol) {
    extern __shared__ double lp[];  // a x kBigLP: L's rows in the current panel's columns
    __shared__ int b_pos[kCholBig];
    __shared__ int b_kept[kCholBig];
    __shared__ double b_D[kCholBig];
    __shared__ double b_dl[kCholBig];  // diagonal of L (0 where dropped)
    __shared__ double b_dm[kCholBig];  // diagonal of the modified L (1 where dropped)
    __shared__ double b_red[kSWaves];
    __shared__ double b_minpiv;
    __shared__ int b_r;
    const int t = threadIdx.x;
    const int nth = blockDim.x;
    const int FS = a | 1;
    double* F = work;
    const bool can_drop = drop_tol2 >= 0.0;
    const int lane = t & 63, wid = t >> 6, nwave = nth >> 6;
    if (ns_tol > 0.0) {
        double sq = 0.0;
        for (int e = t; e < a * a; e += nth) {
            const double v = G[e] - ((e / a == e % a) ? 1.0 : 0.0);
            sq += v * v;
        }
        sq = block_sum(sq, b_red);
        if (sq <= ns_tol * ns_tol) {
            for (int e = t; e < a * a; e += nth) T[e] = ((e / a == e % a) ? 1.5 : 0.0) - 0.5 * G[e];
            for (int i = t; i < a; i += nth) info_i[1 + i] = i;
            if (t == 0) {
                info_i[0] = a;
                info_d[0] = 1.0 - sqrt(sq);
            }
            return;
        }
    }
    for (int i = t; i < a; i += nth) {
        const double g = G[(size_t)i * a + i];
        b_D[i] = (g > 0.0) ? 1.0 / sqrt(g) : 0.0;
    }
    __syncthreads();
    for (int e = t; e < a * a; e += nth) {
        const int i = e / a, j = e % a;
        if (j <= i) F[(size_t)i * FS + j] = G[e] * b_D[i] * b_D[j];
    }
    if (t == 0) b_minpiv = DBL_MAX;
    __syncthreads();

    for (int jb = 0; jb < a; jb += kCholPanel) {
        const int nbw = min(kCholPanel, a - jb);
        // diagonal block: lane c < nbw holds row jb + c
        if (wid == 0) {
            double P[kCholPanel];
#pragma unroll
            for (int c = 0; c < kCholPanel; ++c)
                P[c] = (lane < nbw && c <= lane) ? F[(size_t)(jb + lane) * FS + jb + c] : 0.0;
            double minp = DBL_MAX;
#pragma unroll
            for (int c = 0; c < kCholPanel; ++c) {
                if (c < nbw) {
                    const int j = jb + c;
                    double dj = bcast_lane(P[c], c);
                    const bool drop = can_drop && (!(dj > drop_tol2) || b_D[j] == 0.0);
                    if (!can_drop && !(dj > 1e-300)) dj = 1e-300;
                    if (drop) {
                        if (lane >= c) P[c] = 0.0;
                        if (lane == 0) {
                            b_pos[j] = -1;
                            b_dl[j] = 0.0;
                        }
                    } else {
                        const double piv = sqrt(dj);
                        const double inv = 1.0 / piv;
                        minp = fmin(minp, dj);
                        if (lane > c) P[c] *= inv;
                        if (lane == c) P[c] = piv;
                        if (lane == 0) {
                            b_pos[j] = 0;
                            b_dl[j] = piv;
                        }
#pragma unroll
                        for (int c2 = c + 1; c2 < kCholPanel; ++c2) {
                            if (c2 < nbw) {
                                const double l2 = bcast_lane(P[c], c2);  // L[jb + c2][j]
                                if (lane >= c2) P[c2] -= P[c] * l2;
                            }
                        }
                    }
                }
            }
            if (lane < nbw) {
#pragma unroll
                for (int c = 0; c < kCholPanel; ++c) {
                    if (c <= lane) F[(size_t)(jb + lane) * FS + jb + c] = P[c];
                    lp[(jb + lane) * kBigLP + c] = (c <= lane) ? P[c] : 0.0;
                }
            }
            if (lane == 0) b_minpiv = fmin(b_minpiv, minp);
        }
        __syncthreads();
        // rows below the block: x L_D^T = f by forward substitution
        const int t0 = jb + nbw;
        for (int i = t0 + t; i < a; i += nth) {
            double x[kCholPanel];
#pragma unroll
            for (int c = 0; c < kCholPanel; ++c) x[c] = (c < nbw) ? F[(size_t)i * FS + jb + c] : 0.0;
#pragma unroll
            for (int c = 0; c < kCholPanel; ++c) {
                if (c < nbw) {
                    if (b_pos[jb + c] < 0) {
                        x[c] = 0.0;
                    } else {
                        double sacc = x[c];
#pragma unroll
                        for (int q = 0; q < kCholPanel; ++q)
                            if (q < c) sacc -= x[q] * lp[(jb + c) * kBigLP + q];
                        x[c] = sacc / b_dl[jb + c];
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < kCholPanel; ++c) {
                if (c < nbw) F[(size_t)i * FS + jb + c] = x[c];
                lp[i * kBigLP + c] = (c < nbw) ? x[c] : 0.0;
            }
        }
        __syncthreads();
        // trailing update: F[i][i2] -= sum_c L[i][jb + c] L[i2][jb + c], t0 <= i2 <= i.
        // A wave takes rows i and i + nwave together, so the read-modify-writes
        // of F (in L2) of the two rows overlap and each panel row read from
        // LDS serves both.
        for (int i = t0 + wid; i < a; i += 2 * nwave) {
            const int ib = i + nwave;
            const bool two = ib < a;
            double li[kCholPanel], lb[kCholPanel];
#pragma unroll
            for (int c = 0; c < kCholPanel; ++c) {
                li[c] = lp[i * kBigLP + c];
                lb[c] = two ? lp[ib * kBigLP + c] : 0.0;
            }
            const int iend = two ? ib : i;
            for (int i2 = t0 + lane; i2 <= iend; i2 += 64) {
                double s1 = 0.0, s2 = 0.0;
#pragma unroll
                for (int c = 0; c < kCholPanel; ++c) {
                    const double l2 = lp[i2 * kBigLP + c];
                    s1 = fma(li[c], l2, s1);
                    s2 = fma(lb[c], l2, s2);
                }
                if (i2 <= i) F[(size_t)i * FS + i2] -= s1;
                if (two) F[(size_t)ib * FS + i2] -= s2;
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        int r = 0;
        for (int j = 0; j < a; ++j) {
            if (b_pos[j] >= 0) {
                b_pos[j] = r;
                b_kept[r] = j;
                info_i[1 + r] = j;
                ++r;
            }
        }
        b_r = r;
        info_i[0] = r;
        info_d[0] = b_minpiv;
    }
    __syncthreads();
    const int r = b_r;

    // inverse of the modified L (identity on dropped rows and columns) by
    // 16 x 16 blocks. Dropped columns are already zero below the diagonal;
    // the rows of dropped columns are zeroed here and the modified diagonal
    // goes to b_dm, so every strictly lower entry is a plain read of F.
    for (int i = t; i < a; i += nth) b_dm[i] = (b_pos[i] < 0) ? 1.0 : b_dl[i];
    for (int e = t; e < a * a; e += nth) {
        const int i = e / a, j = e % a;
        if (j < i && b_pos[i] < 0) F[(size_t)i * FS + j] = 0.0;
    }
    __syncthreads();
    // X = Lm^{-1}, lower part, row-major in its own array after F (work holds
    // a (a | 1) + a^2 <= 2 a^2 + 2 a doubles): the block products read it
    // along rows, so the lanes of a wave (consecutive columns) read
    // consecutive addresses. Their partial sums use the panel's LDS rows,
    // free once the factorization is done ((nbk - 1) 256 <= a kBigLP).
    double* X = F + (size_t)a * FS;
    double* tmp = lp;
    const int nbk = (a + kCholPanel - 1) / kCholPanel;
    for (int b = wid; b < nbk; b += nwave) {
        const int b0 = b * kCholPanel, bs = min(kCholPanel, a - b0);
        const int c = lane;
        if (c < bs) {
            double x[kCholPanel];
#pragma unroll
            for (int rr = 0; rr < kCholPanel; ++rr) {
                double v = 0.0;
                if (rr < bs && rr >= c) {
                    double sacc = (rr == c) ? 1.0 : 0.0;
#pragma unroll
                    for (int q = 0; q < kCholPanel; ++q)
                        if (q >= c && q < rr) sacc -= F[(size_t)(b0 + rr) * FS + b0 + q] * x[q];
                    v = sacc / b_dm[b0 + rr];
                }
                x[rr] = v;
            }
#pragma unroll
            for (int rr = 0; rr < kCholPanel; ++rr)
                if (rr < bs && rr >= c) X[(size_t)(b0 + rr) * a + b0 + c] = x[rr];
        }
    }
    __syncthreads();
    for (int dist = 1; dist < nbk; ++dist) {
        const int npair = nbk - dist;
        for (int e = t; e < npair * kCholPanel * kCholPanel; e += nth) {
            const int J = e / (kCholPanel * kCholPanel), I = J + dist;
            const int rr = (e / kCholPanel) % kCholPanel, cc = e % kCholPanel;
            const int gi = I * kCholPanel + rr, gj = J * kCholPanel + cc;
            double sacc = 0.0;
            if (gi < a) {
                // loads of 8 steps issued before their FMAs (same order of the sum)
                const double* li = F + (size_t)gi * FS;
                const int gend = I * kCholPanel;
                int gk = gj;
                for (; gk + 8 <= gend; gk += 8) {
                    double lv[8], xv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        lv[u] = li[gk + u];
                        xv[u] = X[(size_t)(gk + u) * a + gj];
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) sacc = fma(lv[u], xv[u], sacc);
                }
                if (gk < gend) {  // fewer than 8 steps left
                    double lv[8], xv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const bool ok = gk + u < gend;
                        lv[u] = ok ? li[gk + u] : 0.0;
                        xv[u] = ok ? X[(size_t)(gk + u) * a + gj] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (gk + u < gend) sacc = fma(lv[u], xv[u], sacc);
                }
            }
            tmp[e] = sacc;
        }
        __syncthreads();
        for (int e = t; e < npair * kCholPanel * kCholPanel; e += nth) {
            const int J = e / (kCholPanel * kCholPanel), I = J + dist;
            const int rr = (e / kCholPanel) % kCholPanel, cc = e % kCholPanel;
            const int gi = I * kCholPanel + rr, gj = J * kCholPanel + cc;
            if (gi >= a) continue;
            // the rr + 1 <= 16 terms loaded first, then summed in order
            double xv[kCholPanel], tv[kCholPanel];
#pragma unroll
            for (int q = 0; q < kCholPanel; ++q) {
                const bool ok = q <= rr;
                xv[q] = ok ? X[(size_t)gi * a + I * kCholPanel + q] : 0.0;
                tv[q] = ok ? tmp[J * kCholPanel * kCholPanel + q * kCholPanel + cc] : 0.0;
            }
            double sacc = 0.0;
#pragma unroll
            for (int q = 0; q < kCholPanel; ++q)
                if (q <= rr) sacc = fma(xv[q], tv[q], sacc);
            X[(size_t)gi * a + gj] = -sacc;
        }
        __syncthreads();
    }
    for (int e = t; e < a * r; e += nth) {
        const int i = e / r, q = e % r;
        const int p = b_pos[i];
        double v = 0.0;
        if (p >= 0 && p <= q) v = b_D[i] * X[(size_t)b_kept[q] * a + i];
        T[e] = v;
    }
}

__global__ __launch_bounds__(kSmall) void chol_drop_big_kernel(int a, const double* __restrict__ G,
                                                               double* __restrict__ T, double* __restrict__ work,
                                                               int* __restrict__ info_i,
                                                               double* __restrict__ info_d, double drop_tol2,
                                                               double ns_tol) {
    chol_drop_big_body(a, G, T, work, info_i, info_d, drop_tol2, ns_tol);
}

}  // namespace

hipError_t launch_chol_drop(hipStream_t st, int a, const double* G, double* T, double* work,
                            int* info_i, double* info_d, double drop_tol2, double ns_tol) {
    if (a <= 0 || a > 1024) return hipErrorInvalidValue;
    if (a <= kCholBlk)
        hipLaunchKernelGGL(chol_drop_blocked_kernel, dim3(1), dim3(kSmall), sizeof(double) * (size_t)a * (a | 1), st,
                           a, G, T, info_i, info_d, drop_tol2, ns_tol);
    else if (a <= kCholBig)
        hipLaunchKernelGGL(chol_drop_big_kernel, dim3(1), dim3(kSmall), sizeof(double) * (size_t)a * kBigLP, st, a,
                           G, T, work, info_i, info_d, drop_tol2, ns_tol);
    else
        hipLaunchKernelGGL(chol_drop_kernel<false>, dim3(1), dim3(kSmall), 0, st, a, G, T, work, info_i, info_d,
                           drop_tol2, ns_tol);
    return hipGetLastError();
}

static int small_grid(long long count) {
    long long g = (count + 255) / 256;
    return (int)std::max(1LL, std::min(g, 4096LL));
}

hipError_t launch_axpby(hipStream_t st, long long count, double alpha, const double* X, double beta, double* Y) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(axpby_kernel, dim3(small_grid(count)), dim3(256), 0, st, count, alpha, X, beta, Y);
    return hipGetLastError();
}

hipError_t launch_add_diag(hipStream_t st, int m, double* A, long long ld, double alpha) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(add_diag_kernel, dim3((m + 255) / 256), dim3(256), 0, st, m, A, ld, alpha);
    return hipGetLastError();
}

hipError_t launch_fill(hipStream_t st, int rows, int cols, double* A, long long ld, double v) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_kernel, dim3(small_grid((long long)rows * cols)), dim3(256), 0, st, rows, cols, A,
                       ld, v);
    return hipGetLastError();
}

hipError_t launch_assemble_ap(hipStream_t st, int m, int q, const double* Axp, const double* G, double* Ap) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(assemble_ap_kernel, dim3(small_grid((long long)m * m)), dim3(256), 0, st, m, q, Axp, G,
                       Ap);
    return hipGetLastError();
}

hipError_t launch_gather_sym(hipStream_t st, int r, const int* idx, const double* in, long long ld,
                             double* out) {
    if (r <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_sym_kernel, dim3(small_grid((long long)r * r)), dim3(256), 0, st, r, idx, in, ld,
                       out);
    return hipGetLastError();
}

hipError_t launch_sumsq(hipStream_t st, long long count, const double* X, double* out) {
    hipLaunchKernelGGL(sumsq_kernel, dim3(1), dim3(kSmall), 0, st, count, X, out);
    return hipGetLastError();
}

size_t syev_work_doubles(int m) {
    // d, e, tau, scal (4m + 16), Vh (m^2), two eigenvector blocks (2 m^2),
    // inverse-iteration factors (4 m^2 doubles + m^2 ints), the Gram matrix
    // and transform of the orthonormalization (2 m^2), its Gram scratch, the
    // Cholesky work (2 m^2 + 2m) and info words.
    const size_t mm = (size_t)m * m;
    // + the cooperative tridiagonalization's exchange vectors (2m + 2 x 128)
    // and its barrier counter
    return 4 * (size_t)m + 16 + mm + 2 * mm + 5 * mm + 2 * mm + gram_scratch_doubles(m, m, m) +
           2 * mm + 2 * (size_t)m + 2 * (size_t)m + 64 + 2 * (size_t)m + 256 + 16;
}

static void launch_invit(hipStream_t st, int m, int k, const double* d, const double* e, const double* w,
                         const double* scal, double* ZT, double* fac) {
    const int E = invit_lds_per_block(m);
    if (E > 0) {
        const size_t lds = (size_t)E * m * (5 * sizeof(double) + 1);
        hipLaunchKernelGGL(invit_lds_kernel, dim3((k + E - 1) / E), dim3(64), lds, st, m, k, E, d, e, w, scal, ZT);
    } else {
        hipLaunchKernelGGL(invit_kernel, dim3((k + 255) / 256), dim3(256), 0, st, m, k, d, e, w, scal, ZT, fac);
    }
}

hipError_t launch_syev_lowest(hipStream_t st, int m, int k, double* A, double* w, double* Z,
                              double* work) {
    if (m <= 0 || m > 1024 || k <= 0 || k > m) return hipErrorInvalidValue;
    const size_t mm = (size_t)m * m;
    double* d = work;
    double* e = d + m;
    double* tau = e + m;
    double* scal = tau + m;
    double* Vh = scal + m + 16;
    double* ZT = Vh + mm;
    double* ZT2 = ZT + mm;
    double* fac = ZT2 + mm;
    double* Gk = fac + 5 * mm;
    double* Tk = Gk + mm;
    double* gpart = Tk + mm;
    double* cwork = gpart + gram_scratch_doubles(m, m, m);
    double* infod = cwork + 2 * mm + 2 * (size_t)m;
    int* infoi = reinterpret_cast<int*>(infod + 8);
    const size_t lds = (mm <= (size_t)kLdsDoubles) ? sizeof(double) * mm : 0;
    // Above order 112: the cooperative kernel (rows spread over workgroups, in
    // LDS) takes the leading reflectors in chunks of kCoopChunk, each chunk
    // on the current trailing block with as few workgroups as its order
    // needs (the grid-wide synchronizations of a reflector cost more with more
    // workgroups); the register kernel takes the last kRegOrder reflectors
    // (below order 192 the faster per reflector, measured at m = 160 .. 288).
    auto coop = [&](int k0, int nref) -> bool {
        const int mt = m - k0;
        // Rows per workgroup so that R mt + 2 mt doubles fit 150 KB of LDS.
        const int R = std::max(1, (int)((150 * 1024 / sizeof(double) - 2 * (size_t)mt) / mt));
        const int G = (mt + R - 1) / R;
        if (G > 128) return false;
        double* xcol = infod + 64;
        double* xp = xcol + m;
        double* partA = xp + m;
        double* partB = partA + 128;
        unsigned* ctr = reinterpret_cast<unsigned*>(partB + 128);
        hipLaunchKernelGGL(coop_reset_kernel, dim3(1), dim3(1), 0, st, ctr);
        const size_t clds = sizeof(double) * ((size_t)R * mt + 2 * (size_t)mt);
        int mf_i = m, k0_i = k0, R_i = R, kend_i = nref;
        void* args[] = {&mf_i, &k0_i, &R_i, &kend_i, &A, &d, &e, &tau, &Vh, &xcol, &xp, &partA, &partB, &ctr};
        const bool ok = hipLaunchCooperativeKernel((void*)tridiag_coop_kernel, dim3(G), dim3(kCoopThreads), args,
                                                   clds, st) == hipSuccess;
        if (!ok) (void)hipGetLastError();  // fall back to the single-workgroup kernels
        return ok;
    };
    constexpr int kRegOrder = 192;
    constexpr int kCoopChunk = 64;
    if (m <= kWaveTri) {
        hipLaunchKernelGGL(tridiag_wave_kernel, dim3(1), dim3(64), 0, st, m, A, d, e, tau, Vh);
    } else if (m <= 112) {
        hipLaunchKernelGGL(tridiag_kernel<true>, dim3(1), dim3(kTri), lds, st, m, m, A, d, e, tau, Vh);
    } else {
        int k0 = 0;
        while (m - k0 > kRegOrder) {
            const int nref = std::min(kCoopChunk, m - k0 - kRegOrder);
            if (!coop(k0, nref)) break;
            k0 += nref;
        }
        if (m - k0 > kRegOrder) {
            if (k0 > 0) return hipErrorLaunchFailure;  // a later chunk is never larger than the first
            // no cooperative launch: the leading reflectors in L2 by one workgroup
            k0 = m - kRegOrder;
            hipLaunchKernelGGL(tridiag_kernel<false>, dim3(1), dim3(kTri), 0, st, m, k0, A, d, e, tau, Vh);
        }
        switch ((m - k0 + 15) / 16) {
            case 8: hipLaunchKernelGGL((tridiag_reg_kernel<8, 4>), dim3(1), dim3(512), 0, st, m, k0, A, d, e, tau, Vh); break;
            case 9: hipLaunchKernelGGL((tridiag_reg_kernel<9, 5>), dim3(1), dim3(512), 0, st, m, k0, A, d, e, tau, Vh); break;
            case 10: hipLaunchKernelGGL((tridiag_reg_kernel<10, 5>), dim3(1), dim3(512), 0, st, m, k0, A, d, e, tau, Vh); break;
            case 11: hipLaunchKernelGGL((tridiag_reg_kernel<11, 6>), dim3(1), dim3(512), 0, st, m, k0, A, d, e, tau, Vh); break;
            default: hipLaunchKernelGGL((tridiag_reg_kernel<12, 6>), dim3(1), dim3(512), 0, st, m, k0, A, d, e, tau, Vh); break;
        }
    }
    hipLaunchKernelGGL(bisect_kernel, dim3((k + 3) / 4), dim3(256), 0, st, m, k, d, e, w, scal);
    launch_invit(st, m, k, d, e, w, scal, ZT, fac);
    // Orthonormalize the k vectors (an m x k block whose rows are vector
    // components): one Cholesky-QR pass without column drop, then two passes
    // that take a Newton-Schulz step when the block is orthonormal to 1e-8
    // and another Cholesky-QR pass otherwise (vectors of a degenerate cluster
    // can leave inverse iteration nearly dependent).
    double* cur = ZT;
    double* nxt = ZT2;
    for (int pass = 0; pass < 3; ++pass) {
        Segs Zs = make_segs(k);
        push_seg(Zs, cur, k);
        hipError_t err = launch_gram(st, m, Zs, Zs, 1, gpart, Gk);
        if (err != hipSuccess) return err;
        err = launch_chol_drop(st, k, Gk, Tk, cwork, infoi, infod, -1.0, pass == 0 ? 0.0 : 1e-8);
        if (err != hipSuccess) return err;
        Segs Os = make_segs(k);
        push_seg(Os, nxt, k);
        err = launch_update(st, m, Zs, Tk, k, Os, 1.0, 0.0);
        if (err != hipSuccess) return err;
        double* tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    hipLaunchKernelGGL(backtransform_kernel, dim3((k + 3) / 4), dim3(256), 0, st, m, k, tau, Vh, cur, Z);
    return hipGetLastError();
}

size_t tridiag_vectors_work_doubles(int m) {
    const size_t mm = (size_t)m * m;
    // scal (16), two vector blocks (2 m^2), inverse-iteration factors (5 m^2),
    // Gram and transform (2 m^2), Gram scratch, Cholesky work (2 m^2 + 2m),
    // info words
    return 16 + 2 * mm + 5 * mm + 2 * mm + gram_scratch_doubles(m, m, m) + 2 * mm + 2 * (size_t)m + 64 +
           2 * (size_t)m + 256;
}

hipError_t launch_tridiag_lowest_vectors(hipStream_t st, int m, int k, const double* d, const double* e,
                                         double* w, double* ZT, double* work) {
    if (m <= 0 || m > 1024 || k <= 0 || k > m) return hipErrorInvalidValue;
    const size_t mm = (size_t)m * m;
    double* scal = work;
    double* B0 = scal + 16;
    double* B1 = B0 + mm;
    double* fac = B1 + mm;
    double* Gk = fac + 5 * mm;
    double* Tk = Gk + mm;
    double* gpart = Tk + mm;
    double* cwork = gpart + gram_scratch_doubles(m, m, m);
    double* infod = cwork + 2 * mm + 2 * (size_t)m;
    int* infoi = reinterpret_cast<int*>(infod + 8);
    hipLaunchKernelGGL(bisect_kernel, dim3((k + 3) / 4), dim3(256), 0, st, m, k, d, e, w, scal);
    launch_invit(st, m, k, d, e, w, scal, B0, fac);
    // the same three orthonormalization passes as launch_syev_lowest, the
    // last one writing ZT
    double* src[3] = {B0, B1, B0};
    double* dst[3] = {B1, B0, ZT};
    for (int pass = 0; pass < 3; ++pass) {
        Segs Zs = make_segs(k);
        push_seg(Zs, src[pass], k);
        hipError_t err = launch_gram(st, m, Zs, Zs, 1, gpart, Gk);
        if (err != hipSuccess) return err;
        err = launch_chol_drop(st, k, Gk, Tk, cwork, infoi, infod, -1.0, pass == 0 ? 0.0 : 1e-8);
        if (err != hipSuccess) return err;
        Segs Os = make_segs(k);
        push_seg(Os, dst[pass], k);
        err = launch_update(st, m, Zs, Tk, k, Os, 1.0, 0.0);
        if (err != hipSuccess) return err;
    }
    return hipGetLastError();
}

hipError_t launch_syev(hipStream_t st, int m, double* A, double* w, double* Z, double* work) {
    return launch_syev_lowest(st, m, m, A, w, Z, work);
}

hipError_t launch_hl_init(hipStream_t st, int m, int k, const double* Z1, const int* act, int a,
                          double* B, double* Y) {
    if (a <= 0) return hipSuccess;
    const int total = m * a + k * a;
    hipLaunchKernelGGL(hl_init_kernel, dim3((total + 255) / 256), dim3(256), 0, st, m, k, Z1, act, a,
                       B, Y);
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Batched small dense operations: the single-workgroup bodies above with one
// job per workgroup row (blockIdx.y). A workgroup whose job has nothing for
// it returns before its first barrier.
namespace {

// C = op(A) B by 32 x 32 output tiles; 256 threads, 4 outputs each.
__global__ __launch_bounds__(256) void small_mm_batched_kernel(const SmallMMJob* __restrict__ jobs) {
    __shared__ double As[32][33];
    __shared__ double Bs[32][33];
    const SmallMMJob& J = jobs[blockIdx.y];
    const int R = J.transA ? J.ca : J.rows;  // output rows
    const int K = J.transA ? J.rows : J.ca;  // contraction
    if (R <= 0 || J.cb <= 0) return;
    const int ntj = (J.cb + 31) / 32;
    const int ntiles = ((R + 31) / 32) * ntj;
    const int t = threadIdx.x, tx = t & 31, ty = t >> 5;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int i0 = (tile / ntj) * 32, j0 = (tile % ntj) * 32;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < K; k0 += 32) {
            for (int q = t; q < 32 * 32; q += 256) {
                const int kk = q >> 5, c = q & 31;  // consecutive threads: consecutive columns
                const int kr = k0 + kk;
                double av = 0.0;
                if (J.transA) {
                    if (kr < K && i0 + c < R) av = J.A[(size_t)kr * J.lda + i0 + c];
                    As[kk][c] = av;
                } else {
                    // A row i0 + kk, contraction index k0 + c
                    if (i0 + kk < R && k0 + c < K) av = J.A[(size_t)(i0 + kk) * J.lda + k0 + c];
                    As[c][kk] = av;
                }
                Bs[kk][c] = (kr < K && j0 + c < J.cb) ? J.B[(size_t)kr * J.ldb + j0 + c] : 0.0;
            }
            __syncthreads();
#pragma unroll 8
            for (int kk = 0; kk < 32; ++kk) {
                const double b = Bs[kk][tx];
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[q] = fma(As[kk][ty + 8 * q], b, acc[q]);
            }
            __syncthreads();
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = i0 + ty + 8 * q, j = j0 + tx;
            if (i < R && j < J.cb) {
                double* c = J.C + (size_t)i * J.ldc + j;
                *c = (J.beta != 0.0) ? fma(J.beta, *c, J.alpha * acc[q]) : J.alpha * acc[q];
            }
        }
    }
}

__global__ __launch_bounds__(kSmall) void chol_batched_kernel(const CholJob* __restrict__ jobs) {
    const CholJob& J = jobs[blockIdx.x];
    if (J.a <= 0) return;
    if (J.a <= kCholBlk)
        chol_drop_blocked_kernel_body(0, J.a, J.G, J.T, J.info_i, J.info_d, J.drop_tol2, J.ns_tol);
    else
        chol_drop_big_body(J.a, J.G, J.T, J.work, J.info_i, J.info_d, J.drop_tol2, J.ns_tol);
}

// Work layout of the batched path for order m (within syev_work_doubles(m)).
struct EigWork {
    double *d, *e, *tau, *scal, *Vh, *ZT, *ZT2, *fac, *Gk, *Tk, *cwork, *infod;
    int* infoi;
};
__device__ __forceinline__ EigWork eig_work(double* work, int m) {
    const size_t mm = (size_t)m * m;
    EigWork W;
    W.d = work;
    W.e = W.d + m;
    W.tau = W.e + m;
    W.scal = W.tau + m;
    W.Vh = W.scal + m + 16;
    W.ZT = W.Vh + mm;
    W.ZT2 = W.ZT + mm;
    W.fac = W.ZT2 + mm;
    W.Gk = W.fac + 5 * mm;
    W.Tk = W.Gk + mm;
    W.cwork = W.Tk + mm;
    W.infod = W.cwork + 2 * mm + 2 * (size_t)m;
    W.infoi = reinterpret_cast<int*>(W.infod + 8);
    return W;
}

// Jobs of the three orthonormalization passes (gram, Cholesky, update) of the
// k inverse-iteration vectors: pass p maps ZT -> ZT2 -> ZT -> ZT2.
__global__ void eig_plan_kernel(const EigJob* __restrict__ jobs, int nj, SmallMMJob* __restrict__ mm,
                                CholJob* __restrict__ ch) {
    const int j = threadIdx.x;
    if (j >= nj) return;
    const EigJob J = jobs[j];
    const bool on = J.m > 0 && J.k > 0;
    const EigWork W = eig_work(J.work, on ? J.m : 1);
    for (int p = 0; p < 3; ++p) {
        double* cur = (p & 1) ? W.ZT2 : W.ZT;
        double* nxt = (p & 1) ? W.ZT : W.ZT2;
        SmallMMJob g{cur, cur, W.Gk, 1.0, 0.0, on ? J.m : 0, J.k, J.k, J.k, J.k, J.k, 1};
        SmallMMJob u{cur, W.Tk, nxt, 1.0, 0.0, on ? J.m : 0, J.k, J.k, J.k, J.k, J.k, 0};
        mm[(2 * p) * kMaxBatch + j] = g;
        mm[(2 * p + 1) * kMaxBatch + j] = u;
        CholJob c{W.Gk, W.Tk, W.cwork, W.infoi, W.infod, -1.0, p == 0 ? 0.0 : 1e-8, on ? J.k : 0};
        ch[p * kMaxBatch + j] = c;
    }
}

__global__ __launch_bounds__(64) void tridiag_wave_batched_kernel(const EigJob* __restrict__ jobs) {
    const EigJob& J = jobs[blockIdx.x];
    if (J.m <= 0 || J.m > kWaveTri || J.k <= 0) return;
    const EigWork W = eig_work(J.work, J.m);
    tridiag_wave_kernel_body(0, J.m, J.A, W.d, W.e, W.tau, W.Vh);
}

// Orders up to 112: the in-LDS kernel; above: the register kernel takes the
// trailing 192 (or fewer) reflectors, the global-memory kernel the ones before
// (as launch_syev_lowest without the cooperative kernel).
constexpr int kBatchRegOrder = 192;
template <bool kInLds>
__global__ __launch_bounds__(kTri) void tridiag_batched_kernel(const EigJob* __restrict__ jobs) {
    const EigJob& J = jobs[blockIdx.x];
    if (J.m <= kWaveTri || J.k <= 0) return;
    const EigWork W = eig_work(J.work, J.m);
    if (kInLds) {
        if (J.m > 112) return;
        tridiag_kernel_body<true>(0, J.m, J.m, J.A, W.d, W.e, W.tau, W.Vh);
    } else {
        if (J.m <= kBatchRegOrder) return;
        tridiag_kernel_body<false>(0, J.m, J.m - kBatchRegOrder, J.A, W.d, W.e, W.tau, W.Vh);
    }
}

template <int RR, int RC>
__global__ __launch_bounds__(512) void tridiag_reg_batched_kernel(const EigJob* __restrict__ jobs) {
    const EigJob& J = jobs[blockIdx.x];
    if (J.m <= 112 || J.k <= 0) return;
    const int k0 = J.m > kBatchRegOrder ? J.m - kBatchRegOrder : 0;
    if ((J.m - k0 + 15) / 16 != RR) return;
    const EigWork W = eig_work(J.work, J.m);
    tridiag_reg_kernel_body<RR, RC>(0, J.m, k0, J.A, W.d, W.e, W.tau, W.Vh);
}

__global__ __launch_bounds__(256) void bisect_batched_kernel(const EigJob* __restrict__ jobs) {
    const EigJob& J = jobs[blockIdx.y];
    if (J.m <= 0 || (int)blockIdx.x * 4 >= J.k) return;
    const EigWork W = eig_work(J.work, J.m);
    bisect_kernel_body(blockIdx.x, J.m, J.k, W.d, W.e, J.w, W.scal);
}

__global__ __launch_bounds__(256) void invit_batched_kernel(const EigJob* __restrict__ jobs) {
    const EigJob& J = jobs[blockIdx.y];
    if (J.m <= 0 || (int)blockIdx.x * 256 >= J.k) return;
    const EigWork W = eig_work(J.work, J.m);
    invit_kernel_body(blockIdx.x, J.m, J.k, W.d, W.e, J.w, W.scal, W.ZT, W.fac);
}

__global__ __launch_bounds__(256) void backtransform_batched_kernel(const EigJob* __restrict__ jobs) {
    const EigJob& J = jobs[blockIdx.y];
    if (J.m <= 0 || (int)blockIdx.x * 4 >= J.k) return;
    const EigWork W = eig_work(J.work, J.m);
    backtransform_kernel_body(blockIdx.x, J.m, J.k, W.tau, W.Vh, W.ZT2, J.Z);
}

}  // namespace

void launch_small_mm_batched(Launcher& L, const SmallMMJob* jobs, int nj) {
    if (nj <= 0 || nj > kMaxBatch) L.err = hipErrorInvalidValue;
    L(small_mm_batched_kernel, dim3(64, nj), dim3(256), 0, jobs);
}

void launch_chol_batched(Launcher& L, const CholJob* jobs, int nj) {
    if (nj <= 0 || nj > kMaxBatch) L.err = hipErrorInvalidValue;
    L(chol_batched_kernel, dim3(nj), dim3(kSmall), sizeof(double) * (size_t)kCholBlk * (kCholBlk | 1), jobs);
}

size_t syev_batched_jobspace_bytes() {
    return sizeof(SmallMMJob) * 6 * kMaxBatch + sizeof(CholJob) * 3 * kMaxBatch;
}

void launch_syev_lowest_batched(Launcher& L, const EigJob* jobs, int nj, void* jobspace) {
    if (nj <= 0 || nj > kMaxBatch) L.err = hipErrorInvalidValue;
    SmallMMJob* mm = static_cast<SmallMMJob*>(jobspace);
    CholJob* ch = reinterpret_cast<CholJob*>(mm + 6 * kMaxBatch);
    L(eig_plan_kernel, dim3(1), dim3(64), 0, jobs, nj, mm, ch);
    // the leading reflectors of orders above 192, then one branch per order class
    L(tridiag_batched_kernel<false>, dim3(nj), dim3(kTri), 0, jobs);
    L.fork();
    L(tridiag_wave_batched_kernel, dim3(nj), dim3(64), 0, jobs);
    L(tridiag_batched_kernel<true>, dim3(nj), dim3(kTri), sizeof(double) * (size_t)kLdsDoubles, jobs);
    L(tridiag_reg_batched_kernel<8, 4>, dim3(nj), dim3(512), 0, jobs);
    L(tridiag_reg_batched_kernel<9, 5>, dim3(nj), dim3(512), 0, jobs);
    L(tridiag_reg_batched_kernel<10, 5>, dim3(nj), dim3(512), 0, jobs);
    L(tridiag_reg_batched_kernel<11, 6>, dim3(nj), dim3(512), 0, jobs);
    L(tridiag_reg_batched_kernel<12, 6>, dim3(nj), dim3(512), 0, jobs);
    L.join();
    constexpr int kb = (kBatchEigMax + 3) / 4;
    L(bisect_batched_kernel, dim3(kb, nj), dim3(256), 0, jobs);
    L(invit_batched_kernel, dim3((kBatchEigMax + 255) / 256, nj), dim3(256), 0, jobs);
    for (int p = 0; p < 3; ++p) {
        launch_small_mm_batched(L, mm + (2 * p) * kMaxBatch, nj);
        launch_chol_batched(L, ch + p * kMaxBatch, nj);
        launch_small_mm_batched(L, mm + (2 * p + 1) * kMaxBatch, nj);
    }
    L(backtransform_batched_kernel, dim3(kb, nj), dim3(256), 0, jobs);
}

}  // namespace se
