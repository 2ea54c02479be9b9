// Small dense FP64 kernels of the Rayleigh-Ritz step: Cholesky-QR transform,
// the spectral decomposition of the projected matrix A_p, and the
// Hetmaniuk-Lehoucq coefficients. Each works on one matrix of order <= 1024
// that lives in global memory (L2-resident at these sizes).
#include <cfloat>

#include "common.h"

namespace se {

namespace {

constexpr int kBig = 1024;  // threads of the single-workgroup kernels
constexpr int kWaves = kBig / 64;

// Sum over the whole workgroup in a fixed order. `sh` holds >= kWaves doubles.
__device__ double block_sum(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double s = 0.0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int q = 0; q < nw; ++q) s += sh[q];
    __syncthreads();
    return s;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return __shfl(v, 0, 64);
}

// ---------------------------------------------------------------------------
// Cholesky-QR transform with column drop. Columns are first scaled to unit
// norm (G -> D G D) so that the pivots measure the part of each column that is
// independent of the previous ones; a column whose pivot is below drop_tol2 is
// dropped. T = D R^{-1} restricted to the kept columns, written a x r with
// leading dimension r.
__global__ __launch_bounds__(kBig) void chol_drop_kernel(int a, const double* __restrict__ G,
                                                         double* __restrict__ T,
                                                         double* __restrict__ work,
                                                         int* __restrict__ info_i,
                                                         double* __restrict__ info_d,
                                                         double drop_tol2) {
    double* L = work;               // a x a, lower triangle used
    double* D = work + (size_t)a * a;  // a
    double* Rinv = D + a;           // a x a (r x r used), row-major ld a
    __shared__ int s_pos[kBig];
    __shared__ int s_kept[kBig];
    __shared__ double s_red[kWaves];
    const int t = threadIdx.x;

    for (int i = t; i < a; i += kBig) {
        const double g = G[(size_t)i * a + i];
        D[i] = (g > 0.0) ? 1.0 / sqrt(g) : 0.0;
    }
    __syncthreads();
    for (size_t e = t; e < (size_t)a * a; e += kBig) {
        const int i = (int)(e / a), j = (int)(e % a);
        if (j <= i) L[e] = G[e] * D[i] * D[j];
    }
    __syncthreads();

    double minpiv = DBL_MAX;
    for (int j = 0; j < a; ++j) {
        const double d = L[(size_t)j * a + j];
        const bool drop = !(d > drop_tol2) || D[j] == 0.0;
        __syncthreads();
        if (drop) {
            for (int i = j + t; i < a; i += kBig) L[(size_t)i * a + j] = 0.0;
            if (t == 0) s_pos[j] = -1;
            __syncthreads();
            continue;
        }
        const double piv = sqrt(d);
        minpiv = fmin(minpiv, d);
        for (int i = j + 1 + t; i < a; i += kBig) L[(size_t)i * a + j] /= piv;
        if (t == 0) {
            L[(size_t)j * a + j] = piv;
            s_pos[j] = 0;
        }
        __syncthreads();
        const int rem = a - j - 1;
        for (size_t e = t; e < (size_t)rem * rem; e += kBig) {
            const int i = j + 1 + (int)(e / rem), i2 = j + 1 + (int)(e % rem);
            if (i2 <= i) L[(size_t)i * a + i2] -= L[(size_t)i * a + j] * L[(size_t)i2 * a + j];
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
        info_i[0] = r;
    }
    __syncthreads();
    const int r = info_i[0];
    // Back substitution per column q of R^{-1}, R[p][q] = L[kept q][kept p].
    for (int q = t; q < r; q += kBig) {
        const int kq = s_kept[q];
        Rinv[(size_t)q * a + q] = 1.0 / L[(size_t)kq * a + kq];
        for (int p = q - 1; p >= 0; --p) {
            const int kp = s_kept[p];
            double s = 0.0;
            for (int u = p + 1; u <= q; ++u) s += L[(size_t)s_kept[u] * a + kp] * Rinv[(size_t)u * a + q];
            Rinv[(size_t)p * a + q] = -s / L[(size_t)kp * a + kp];
        }
    }
    __syncthreads();
    for (size_t e = t; e < (size_t)a * r; e += kBig) {
        const int i = (int)(e / r), q = (int)(e % r);
        const int p = s_pos[i];
        T[e] = (p >= 0 && p <= q) ? D[i] * Rinv[(size_t)p * a + q] : 0.0;
    }
    // smallest pivot over the workgroup (only thread-local copies differ)
    __syncthreads();
    if (t == 0) s_red[0] = minpiv;
    __syncthreads();
    if (t == 0) info_d[0] = s_red[0];
}

// ---------------------------------------------------------------------------
// Householder tridiagonalization of the symmetric m x m matrix A (row-major,
// both triangles kept up to date). Reflector k acts on rows/columns k+1..m-1:
// H_k = I - tau_k v_k v_k^T with v_k stored in Vh row k from column k+1
// (leading 1 explicit). d = diagonal, e = off-diagonal of the result.
__global__ __launch_bounds__(kBig) void tridiag_kernel(int m, double* __restrict__ A,
                                                       double* __restrict__ d,
                                                       double* __restrict__ e,
                                                       double* __restrict__ tau,
                                                       double* __restrict__ Vh) {
    __shared__ double sv[kBig];
    __shared__ double sw[kBig];
    __shared__ double sp[kBig];
    __shared__ double sred[kWaves];
    __shared__ double s_scal[4];
    const int t = threadIdx.x;
    for (int k = 0; k + 2 < m; ++k) {
        const int L = m - k - 1;
        const double* row = A + (size_t)k * m + (k + 1);
        double part = 0.0;
        for (int i = 1 + t; i < L; i += kBig) part += row[i] * row[i];
        const double sigma2 = block_sum(part, sred);
        if (t == 0) {
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
        for (int i = t; i < L; i += kBig) {
            const double v = (i == 0) ? 1.0 : (tk != 0.0 ? row[i] * scale : 0.0);
            sv[i] = v;
            Vh[(size_t)k * m + k + 1 + i] = v;
        }
        __syncthreads();
        if (tk == 0.0) continue;
        // p = tau * A22 v, A22 = A[k+1:, k+1:]
        const int G = kBig / L;  // >= 1 because L < m <= 1024
        {
            const int i = t % L, g = t / L;
            double s = 0.0;
            if (g < G) {
                const double* base = A + (size_t)(k + 1) * m + (k + 1) + i;
                for (int jj = g; jj < L; jj += G) s = fma(base[(size_t)jj * m], sv[jj], s);
            }
            if (g < G) sp[g * L + i] = s;
        }
        __syncthreads();
        double pv = 0.0;
        for (int i = t; i < L; i += kBig) {
            double s = 0.0;
            for (int g = 0; g < G; ++g) s += sp[g * L + i];
            s *= tk;
            sw[i] = s;
            pv += s * sv[i];
        }
        const double Kc = 0.5 * tk * block_sum(pv, sred);
        for (int i = t; i < L; i += kBig) sw[i] -= Kc * sv[i];
        __syncthreads();
        // A22 -= v w^T + w v^T
        for (size_t q = t; q < (size_t)L * L; q += kBig) {
            const int jj = (int)(q / L), i = (int)(q % L);
            double* p = A + (size_t)(k + 1 + jj) * m + (k + 1 + i);
            *p -= sv[jj] * sw[i] + sw[jj] * sv[i];
        }
        __syncthreads();
    }
    if (t == 0) {
        if (m >= 2) {
            d[m - 2] = A[(size_t)(m - 2) * m + (m - 2)];
            e[m - 2] = A[(size_t)(m - 1) * m + (m - 2)];
        }
        d[m - 1] = A[(size_t)(m - 1) * m + (m - 1)];
    }
}

// ---------------------------------------------------------------------------
// Eigenvalues of the symmetric tridiagonal (d, e) by multisection: one wave
// per eigenvalue, each lane evaluates the Sturm count at one of 64 interior
// points of the current bracket, so the bracket shrinks 65x per round.
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

__global__ __launch_bounds__(256) void bisect_kernel(int m, const double* __restrict__ dg,
                                                     const double* __restrict__ eg,
                                                     double* __restrict__ w,
                                                     double* __restrict__ scal) {
    __shared__ double d[kBig];
    __shared__ double e2[kBig];
    __shared__ double s_gl[4], s_gu[4], s_pm[4];
    for (int i = threadIdx.x; i < m; i += 256) {
        d[i] = dg[i];
        if (i + 1 < m) e2[i] = eg[i] * eg[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double gl = DBL_MAX, gu = -DBL_MAX, emax2 = 0.0;
        for (int i = 0; i < m; ++i) {
            const double ea = (i > 0 ? fabs(eg[i - 1]) : 0.0) + (i + 1 < m ? fabs(eg[i]) : 0.0);
            gl = fmin(gl, d[i] - ea);
            gu = fmax(gu, d[i] + ea);
            if (i + 1 < m) emax2 = fmax(emax2, e2[i]);
        }
        const double pivmin = DBL_MIN * fmax(1.0, emax2);
        const double tnorm = fmax(fabs(gl), fabs(gu));
        gl -= 2.0 * DBL_EPSILON * tnorm * m + 4.0 * pivmin;
        gu += 2.0 * DBL_EPSILON * tnorm * m + 4.0 * pivmin;
        s_gl[0] = gl;
        s_gu[0] = gu;
        s_pm[0] = pivmin;
        if (blockIdx.x == 0) scal[0] = tnorm;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int idx = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (idx >= m) return;
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
            nlo = __shfl(x, 63, 64);
            nhi = hi;
        } else {
            const int first = __ffsll((long long)mask) - 1;
            nhi = __shfl(x, first, 64);
            nlo = (first > 0) ? __shfl(x, first - 1, 64) : lo;
        }
        lo = nlo;
        hi = nhi;
    }
    if (lane == 0) w[idx] = 0.5 * (lo + hi);
}

// ---------------------------------------------------------------------------
// Eigenvectors of the tridiagonal by inverse iteration (one thread per
// eigenvalue, LU with partial pivoting of T - lambda I), followed by
// classical Gram-Schmidt twice within clusters of close eigenvalues.
// ZT[j * m + i] = component j of eigenvector i.
__device__ __forceinline__ double hash_unit(unsigned i, unsigned j) {
    unsigned h = i * 0x9E3779B1u ^ (j + 0x7F4A7C15u) * 0x85EBCA77u;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    h *= 0x297A2D39u;
    h ^= h >> 15;
    return (double)(h & 0xFFFFFF) / 8388608.0 - 1.0;
}

__global__ __launch_bounds__(kBig) void invit_kernel(int m, const double* __restrict__ dg,
                                                     const double* __restrict__ eg,
                                                     const double* __restrict__ w,
                                                     const double* __restrict__ scal,
                                                     double* __restrict__ ZT,
                                                     double* __restrict__ work) {
    __shared__ double sred[kWaves];
    __shared__ double scoef[kBig];
    __shared__ int s_c0[1];
    const int M = m;
    double* DL = work;
    double* DD = DL + (size_t)M * M;
    double* DU = DD + (size_t)M * M;
    double* DU2 = DU + (size_t)M * M;
    int* IP = reinterpret_cast<int*>(DU2 + (size_t)M * M);
    const double tnorm = fmax(scal[0], DBL_MIN);
    const double tiny = DBL_EPSILON * tnorm;

    for (int i = threadIdx.x; i < m; i += kBig) {
        const double lam = w[i];
#define AT(arr, j) arr[(size_t)(j) * M + i]
        // factor T - lam I
        for (int j = 0; j < m; ++j) {
            AT(DD, j) = dg[j] - lam;
            if (j + 1 < m) {
                AT(DL, j) = eg[j];
                AT(DU, j) = eg[j];
            }
            if (j + 2 < m) AT(DU2, j) = 0.0;
        }
        for (int j = 0; j + 1 < m; ++j) {
            const double dj = AT(DD, j), lj = AT(DL, j);
            if (fabs(dj) >= fabs(lj)) {
                AT(IP, j) = j;
                if (dj != 0.0) {
                    const double f = lj / dj;
                    AT(DL, j) = f;
                    AT(DD, j + 1) -= f * AT(DU, j);
                }
            } else {
                const double f = dj / lj;
                AT(DD, j) = lj;
                AT(DL, j) = f;
                const double tmp = AT(DU, j);
                AT(DU, j) = AT(DD, j + 1);
                AT(DD, j + 1) = tmp - f * AT(DD, j + 1);
                if (j + 2 < m) {
                    AT(DU2, j) = AT(DU, j + 1);
                    AT(DU, j + 1) = -f * AT(DU, j + 1);
                }
                AT(IP, j) = j + 1;
            }
        }
        for (int j = 0; j < m; ++j)
            if (fabs(AT(DD, j)) < tiny) AT(DD, j) = copysign(tiny, AT(DD, j) == 0.0 ? 1.0 : AT(DD, j));
        // start vector
        for (int j = 0; j < m; ++j) AT(ZT, j) = hash_unit((unsigned)i, (unsigned)j);
        for (int it = 0; it < 3; ++it) {
            for (int j = 0; j + 1 < m; ++j) {
                const double bj = AT(ZT, j), bj1 = AT(ZT, j + 1);
                if (AT(IP, j) == j) {
                    AT(ZT, j + 1) = bj1 - AT(DL, j) * bj;
                } else {
                    AT(ZT, j) = bj1;
                    AT(ZT, j + 1) = bj - AT(DL, j) * bj1;
                }
            }
            AT(ZT, m - 1) /= AT(DD, m - 1);
            if (m >= 2) AT(ZT, m - 2) = (AT(ZT, m - 2) - AT(DU, m - 2) * AT(ZT, m - 1)) / AT(DD, m - 2);
            for (int j = m - 3; j >= 0; --j)
                AT(ZT, j) = (AT(ZT, j) - AT(DU, j) * AT(ZT, j + 1) - AT(DU2, j) * AT(ZT, j + 2)) / AT(DD, j);
            double mx = 0.0;
            for (int j = 0; j < m; ++j) mx = fmax(mx, fabs(AT(ZT, j)));
            const double sc = (mx > 0.0) ? 1.0 / mx : 1.0;
            double nr = 0.0;
            for (int j = 0; j < m; ++j) {
                const double v = AT(ZT, j) * sc;
                AT(ZT, j) = v;
                nr += v * v;
            }
            if (it == 2) {
                const double inv = 1.0 / sqrt(nr);
                for (int j = 0; j < m; ++j) AT(ZT, j) *= inv;
            }
        }
#undef AT
    }
    __syncthreads();

    // Re-orthogonalize within clusters (gap <= 1e-3 ||T||).
    const double ortol = 1e-3 * tnorm;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int c0 = 0;
    for (int q = 1; q < m; ++q) {
        if (w[q] - w[q - 1] > ortol) {
            c0 = q;
            continue;
        }
        for (int pass = 0; pass < 2; ++pass) {
            // coef[l] = z_l . z_q for l in [c0, q): one wave per l
            for (int l = c0 + wid; l < q; l += kWaves) {
                double s = 0.0;
                for (int j = lane; j < m; j += 64) s += ZT[(size_t)j * M + l] * ZT[(size_t)j * M + q];
                s = wave_sum(s);
                if (lane == 0) scoef[l - c0] = s;
            }
            __syncthreads();
            for (int j = threadIdx.x; j < m; j += kBig) {
                double v = ZT[(size_t)j * M + q];
                for (int l = c0; l < q; ++l) v -= scoef[l - c0] * ZT[(size_t)j * M + l];
                ZT[(size_t)j * M + q] = v;
            }
            __syncthreads();
        }
        double part = 0.0;
        for (int j = threadIdx.x; j < m; j += kBig) {
            const double v = ZT[(size_t)j * M + q];
            part += v * v;
        }
        const double nr = block_sum(part, sred);
        const double inv = nr > 0.0 ? 1.0 / sqrt(nr) : 0.0;
        for (int j = threadIdx.x; j < m; j += kBig) ZT[(size_t)j * M + q] *= inv;
        __syncthreads();
    }
    (void)s_c0;
}

// Z = Q ZT with Q = H_0 H_1 ... H_{m-3}; one wave per eigenvector, kept in
// registers (m <= 1024 -> 16 values per lane).
__global__ __launch_bounds__(256) void backtransform_kernel(int m, const double* __restrict__ tau,
                                                            const double* __restrict__ Vh,
                                                            const double* __restrict__ ZT,
                                                            double* __restrict__ Z) {
    constexpr int MAXQ = kBig / 64;
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= m) return;
    double z[MAXQ];
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
        const int j = lane + 64 * q;
        z[q] = (j < m) ? ZT[(size_t)j * m + i] : 0.0;
    }
    for (int k = m - 3; k >= 0; --k) {
        const double tk = tau[k];
        if (tk == 0.0) continue;
        const double* v = Vh + (size_t)k * m;  // v[j] valid for j >= k + 1
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < MAXQ; ++q) {
            const int j = lane + 64 * q;
            if (j > k && j < m) s = fma(v[j], z[q], s);
        }
        s = wave_sum(s) * tk;
#pragma unroll
        for (int q = 0; q < MAXQ; ++q) {
            const int j = lane + 64 * q;
            if (j > k && j < m) z[q] = fma(-s, v[j], z[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
        const int j = lane + 64 * q;
        if (j < m) Z[(size_t)j * m + i] = z[q];
    }
}

// ---------------------------------------------------------------------------
// Hetmaniuk-Lehoucq coefficients. Column c of B is row act[c] of Z2 = Z[:, k:];
// Q_B is built by classical Gram-Schmidt applied twice per column, dropping
// columns whose remaining norm is below drop_tol times their own norm.
// C = [Z1 | Z2 Q_B].
__global__ __launch_bounds__(kBig) void hl_kernel(int m, int k, const double* __restrict__ Z,
                                                  const int* __restrict__ act, int a,
                                                  double* __restrict__ C,
                                                  double* __restrict__ work,
                                                  int* __restrict__ info_i, double drop_tol) {
    __shared__ double sv[kBig];
    __shared__ double scoef[kBig];
    __shared__ double sred[kWaves];
    const int L = m - k;
    double* Q = work;  // column l at Q[l * L + t]
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int r = 0;
    for (int c = 0; c < a; ++c) {
        const int row = act[c];
        double part = 0.0;
        for (int t = threadIdx.x; t < L; t += kBig) {
            const double v = Z[(size_t)row * m + k + t];
            sv[t] = v;
            part += v * v;
        }
        const double n0 = sqrt(block_sum(part, sred));
        for (int pass = 0; pass < 2 && r > 0; ++pass) {
            for (int l = wid; l < r; l += kWaves) {
                double s = 0.0;
                for (int t = lane; t < L; t += 64) s += Q[(size_t)l * L + t] * sv[t];
                s = wave_sum(s);
                if (lane == 0) scoef[l] = s;
            }
            __syncthreads();
            for (int t = threadIdx.x; t < L; t += kBig) {
                double v = sv[t];
                for (int l = 0; l < r; ++l) v -= scoef[l] * Q[(size_t)l * L + t];
                sv[t] = v;
            }
            __syncthreads();
        }
        part = 0.0;
        for (int t = threadIdx.x; t < L; t += kBig) part += sv[t] * sv[t];
        const double n1 = sqrt(block_sum(part, sred));
        if (n0 > 0.0 && n1 > drop_tol * n0) {
            const double inv = 1.0 / n1;
            for (int t = threadIdx.x; t < L; t += kBig) Q[(size_t)r * L + t] = sv[t] * inv;
            ++r;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) info_i[0] = r;
    const int ldo = k + r;  // C is written compactly: m x (k + r)
    for (size_t e = threadIdx.x; e < (size_t)m * k; e += kBig) {
        const int i = (int)(e / k), j = (int)(e % k);
        C[(size_t)i * ldo + j] = Z[(size_t)i * m + j];
    }
    for (size_t e = threadIdx.x; e < (size_t)m * r; e += kBig) {
        const int i = (int)(e / r), l = (int)(e % r);
        double s = 0.0;
        const double* zrow = Z + (size_t)i * m + k;
        const double* ql = Q + (size_t)l * L;
        for (int t = 0; t < L; ++t) s = fma(zrow[t], ql[t], s);
        C[(size_t)i * ldo + k + l] = s;
    }
}

}  // namespace

hipError_t launch_chol_drop(hipStream_t st, int a, const double* G, double* T, double* work,
                            int* info_i, double* info_d, double drop_tol2) {
    if (a <= 0 || a > kBig) return hipErrorInvalidValue;
    hipLaunchKernelGGL(chol_drop_kernel, dim3(1), dim3(kBig), 0, st, a, G, T, work, info_i, info_d,
                       drop_tol2);
    return hipGetLastError();
}

size_t syev_work_doubles(int m) {
    // d, e, tau, scal (4m) + Vh (m^2) + ZT (m^2) + inverse-iteration factors (4 m^2 + m^2/2 ints)
    return (size_t)4 * m + 8 + (size_t)m * m * 2 + (size_t)m * m * 5;
}

hipError_t launch_syev(hipStream_t st, int m, double* A, double* w, double* Z, double* work) {
    if (m <= 0 || m > kBig) return hipErrorInvalidValue;
    double* d = work;
    double* e = d + m;
    double* tau = e + m;
    double* scal = tau + m;
    double* Vh = scal + m + 8;
    double* ZT = Vh + (size_t)m * m;
    double* fac = ZT + (size_t)m * m;
    hipLaunchKernelGGL(tridiag_kernel, dim3(1), dim3(kBig), 0, st, m, A, d, e, tau, Vh);
    hipLaunchKernelGGL(bisect_kernel, dim3((m + 3) / 4), dim3(256), 0, st, m, d, e, w, scal);
    hipLaunchKernelGGL(invit_kernel, dim3(1), dim3(kBig), 0, st, m, d, e, w, scal, ZT, fac);
    hipLaunchKernelGGL(backtransform_kernel, dim3((m + 3) / 4), dim3(256), 0, st, m, tau, Vh, ZT, Z);
    return hipGetLastError();
}

hipError_t launch_hl(hipStream_t st, int m, int k, const double* Z, const int* act, int a, double* C,
                     double* work, int* info_i, double drop_tol) {
    if (m <= 0 || m > kBig || k < 0 || k > m) return hipErrorInvalidValue;
    hipLaunchKernelGGL(hl_kernel, dim3(1), dim3(kBig), 0, st, m, k, Z, act, a, C, work, info_i,
                       drop_tol);
    return hipGetLastError();
}

}  // namespace se
