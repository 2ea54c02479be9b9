// Complex Hermitian kernels (FP64), gfx950.
//
// The paper states the eigenproblem for Hermitian A in C^{n x n} (Section 1)
// and writes X^H throughout Algorithms 1-4. Complex n-length blocks are
// row-major with interleaved (re, im) entries, so an n x w complex block with
// leading dimension ldc is the n x 2w real block with leading dimension 2 ldc
// whose columns are (Re x_0, Im x_0, Re x_1, ...). On that real view:
//  * U^H V = (Ur^T Vr + Ui^T Vi) + i (Ur^T Vi - Ui^T Vr) is a 2 x 2 block
//    combination of the real Gram product of the two views, so the FP64
//    matrix-core Gram kernel serves both (zgram_combine_kernel combines);
//  * U C with complex C (K x N) is the real product of the view of U with
//    the 2K x 2N real embedding [[Re c, Im c], [-Im c, Re c]] of every entry
//    (zembed_kernel), so the FP64 matrix-core update kernel serves both;
//  * elementwise steps with real scalars (residual and norms with real Ritz
//    values, sigma X - A X, column copies) run on the view unchanged.
// New here: the complex CSR product, and the Hermitian small dense steps
// (Cholesky with column drop, Householder tridiagonalization to a real
// tridiagonal, back-transformation of its eigenvectors).
#include <cfloat>

#include <hip/hip_runtime.h>

#include "common.h"

namespace se {

namespace {

constexpr int kZThreads = 256;
constexpr int kZRows = 32;  // rows per wave of the complex CSR product
constexpr int kZNB = 8;     // nonzeros per batch

// Sum over the 64 lanes, in every lane (whole wave active): DPP butterflies
// within each row of 16 lanes (quad_perm 1,0,3,2 and 2,3,0,1, half-row mirror,
// row mirror), then the four row sums by v_readlane in a fixed order.
template <int CTRL>
__device__ __forceinline__ double zdpp(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double zlane(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double zwave_sum(double v) {
    v += zdpp<0xB1>(v);
    v += zdpp<0x4E>(v);
    v += zdpp<0x141>(v);
    v += zdpp<0x140>(v);
    return (zlane(v, 0) + zlane(v, 16)) + (zlane(v, 32) + zlane(v, 48));
}

// ---------------------------------------------------------------------------
// Y = A X for complex CSR A (values interleaved) and complex row-major blocks.
// One wave per run of kZRows rows walks the run's nonzeros kZNB at a time:
// column indices and values are wave-uniform (one scalar load each), the kZNB
// row gathers of X are issued before any is used, and the accumulator moves
// to the next row at each row boundary. Lane l owns complex column cb + l of
// each 64-column block (one 16-byte load per gathered row).
__global__ __launch_bounds__(kZThreads) void spmm_z_kernel(int n, const int* __restrict__ rowptr,
                                                           const int* __restrict__ col,
                                                           const double* __restrict__ val,
                                                           const double* __restrict__ X, long long ldx,
                                                           double* __restrict__ Y, long long ldy, int w) {
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane((int)blockIdx.x * (kZThreads / 64) + (int)(threadIdx.x >> 6));
    if ((long long)wid * kZRows >= n) return;
    const int r0 = wid * kZRows;
    const int r1 = min(n, r0 + kZRows);
    const int rp = rowptr[min(r0 + lane, r1)];  // lane q: offset of row r0 + q, q <= r1 - r0
    const int pbeg = __builtin_amdgcn_readlane(rp, 0);
    const int pend = __builtin_amdgcn_readlane(rp, r1 - r0);
    for (int cb = 0; cb < w; cb += 64) {
        const int c = cb + lane;
        const bool has = c < w;
        const long long cc = has ? c : cb;  // lanes without a column read a valid address
        int r = r0;
        int rend = __builtin_amdgcn_readlane(rp, 1);
        double are = 0.0, aim = 0.0;
        auto flush = [&]() {
            if (has) *reinterpret_cast<double2*>(Y + 2 * ((long long)r * ldy + c)) = make_double2(are, aim);
            are = 0.0;
            aim = 0.0;
            ++r;
            if (r < r1) rend = __builtin_amdgcn_readlane(rp, r - r0 + 1);
        };
        for (int p = pbeg; p < pend; p += kZNB) {
            int j[kZNB];
            double vr[kZNB], vi[kZNB];
#pragma unroll
            for (int u = 0; u < kZNB; ++u) {
                j[u] = col[p + u];
                vr[u] = val[2 * (long long)(p + u)];
                vi[u] = val[2 * (long long)(p + u) + 1];
            }
            double2 x[kZNB];
#pragma unroll
            for (int u = 0; u < kZNB; ++u)
                x[u] = *reinterpret_cast<const double2*>(X + 2 * ((long long)j[u] * ldx + cc));
#pragma unroll
            for (int u = 0; u < kZNB; ++u) {
                if (p + u < pend) {
                    while (p + u >= rend) flush();
                    // (vr + i vi)(xr + i xi)
                    are = fma(vr[u], x[u].x, fma(-vi[u], x[u].y, are));
                    aim = fma(vr[u], x[u].y, fma(vi[u], x[u].x, aim));
                }
            }
        }
        while (r < r1) flush();
    }
}

// C (mu x mv complex, row-major) from the real Gram product P (2mu x 2mv,
// leading dimension 2mv) of the interleaved views: C[a][b] =
// (P[2a][2b] + P[2a+1][2b+1]) + i (P[2a][2b+1] - P[2a+1][2b]). When P is
// exactly symmetric (U = V) the result is exactly Hermitian.
__global__ __launch_bounds__(kZThreads) void zgram_combine_kernel(int mu, int mv, const double* __restrict__ P,
                                                                  double* __restrict__ C) {
    const long long total = (long long)mu * mv;
    const long long ldp = 2LL * mv;
    for (long long e = (long long)blockIdx.x * kZThreads + threadIdx.x; e < total;
         e += (long long)gridDim.x * kZThreads) {
        const long long a = e / mv, b = e % mv;
        const double* p0 = P + (2 * a) * ldp + 2 * b;
        const double* p1 = p0 + ldp;
        C[2 * e] = p0[0] + p1[1];
        C[2 * e + 1] = p0[1] - p1[0];
    }
}

// Real embedding E (2K x 2N, leading dimension 2N) of the complex K x N matrix
// C: E[2a][2b] = E[2a+1][2b+1] = Re c_ab, E[2a][2b+1] = Im c_ab,
// E[2a+1][2b] = -Im c_ab, so that view(U) E = view(U C).
__global__ __launch_bounds__(kZThreads) void zembed_kernel(int K, int N, const double* __restrict__ C,
                                                           double* __restrict__ E) {
    const long long total = (long long)K * N;
    const long long lde = 2LL * N;
    for (long long e = (long long)blockIdx.x * kZThreads + threadIdx.x; e < total;
         e += (long long)gridDim.x * kZThreads) {
        const long long a = e / N, b = e % N;
        const double cr = C[2 * e], ci = C[2 * e + 1];
        double* e0 = E + (2 * a) * lde + 2 * b;
        double* e1 = e0 + lde;
        e0[0] = cr;
        e0[1] = ci;
        e1[0] = -ci;
        e1[1] = cr;
    }
}

// A <- (A + A^H) / 2 for a complex m x m matrix (the diagonal becomes real).
__global__ __launch_bounds__(kZThreads) void zherm_kernel(int m, double* __restrict__ A) {
    const long long total = (long long)m * m;
    for (long long e = (long long)blockIdx.x * kZThreads + threadIdx.x; e < total;
         e += (long long)gridDim.x * kZThreads) {
        const long long i = e / m, j = e % m;
        if (j < i) continue;
        double* aij = A + 2 * (i * m + j);
        double* aji = A + 2 * (j * m + i);
        if (i == j) {
            aij[1] = 0.0;
            continue;
        }
        const double re = 0.5 * (aij[0] + aji[0]);
        const double im = 0.5 * (aij[1] - aji[1]);
        aij[0] = re;
        aij[1] = im;
        aji[0] = re;
        aji[1] = -im;
    }
}

// Hetmaniuk-Lehoucq start block in complex coefficients: B (m x a) holds the
// unit columns e_{act[c]} and Y (k x a) = Z1^H E, Y[i][c] = conj(Z1[act[c]][i]).
__global__ __launch_bounds__(kZThreads) void hl_init_z_kernel(int m, int k, const double* __restrict__ Z1,
                                                              const int* __restrict__ act, int a,
                                                              double* __restrict__ B, double* __restrict__ Y) {
    const int total = m * a + k * a;
    for (int e = blockIdx.x * kZThreads + threadIdx.x; e < total; e += gridDim.x * kZThreads) {
        if (e < m * a) {
            const int i = e / a, c = e % a;
            B[2 * e] = (i == act[c]) ? 1.0 : 0.0;
            B[2 * e + 1] = 0.0;
        } else {
            const int q = e - m * a;
            const int i = q / a, c = q % a;
            const double* z = Z1 + 2 * ((long long)act[c] * k + i);
            Y[2 * q] = z[0];
            Y[2 * q + 1] = -z[1];
        }
    }
}

// ---------------------------------------------------------------------------
// Complex Cholesky-QR transform with column drop. G = W^H W (a x a, Hermitian)
// is scaled to unit diagonal (D G D); the right-looking factorization D G D =
// L L^H drops a column whose pivot falls below drop_tol2 (drop_tol2 < 0:
// nothing is dropped and tiny pivots are floored). T = D R^{-1} (R = L^H)
// restricted to the kept columns, a x r complex with leading dimension r, so
// that W T has orthonormal columns. info_i[0] = r, info_i[1..r] = kept
// columns, info_d[0] = smallest scaled pivot. work holds a^2 complex entries.
constexpr int kZSmall = 512;
__global__ __launch_bounds__(kZSmall) void cholz_kernel(int a, const double* __restrict__ G, double* __restrict__ T,
                                                        double* __restrict__ F, int* __restrict__ info_i,
                                                        double* __restrict__ info_d, double drop_tol2) {
    __shared__ int s_pos[512];
    __shared__ int s_kept[512];
    __shared__ double s_D[512];
    __shared__ double s_dl[512];
    __shared__ double s_dr[512];
    __shared__ double s_cr[512];
    __shared__ double s_ci[512];
    __shared__ int s_r;
    const int t = threadIdx.x;
    const int nth = blockDim.x;
    const bool can_drop = drop_tol2 >= 0.0;
    for (int i = t; i < a; i += nth) {
        const double g = G[2 * ((size_t)i * a + i)];
        s_D[i] = (g > 0.0) ? 1.0 / sqrt(g) : 0.0;
    }
    __syncthreads();
    for (size_t e = t; e < (size_t)a * a; e += nth) {
        const int i = (int)(e / a), j = (int)(e % a);
        if (j <= i) {
            const double s = s_D[i] * s_D[j];
            F[2 * e] = G[2 * e] * s;
            F[2 * e + 1] = G[2 * e + 1] * s;
        }
    }
    __syncthreads();
    double minpiv = DBL_MAX;
    const int lane = t & 63, wrow = t >> 6, nwave = nth >> 6;
    for (int j = 0; j < a; ++j) {
        double d = F[2 * ((size_t)j * a + j)];
        const bool drop = can_drop && (!(d > drop_tol2) || s_D[j] == 0.0);
        if (!can_drop && !(d > 1e-300)) d = 1e-300;
        if (drop) {
            for (int i = j + 1 + t; i < a; i += nth) {
                F[2 * ((size_t)i * a + j)] = 0.0;
                F[2 * ((size_t)i * a + j) + 1] = 0.0;
            }
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
            double* f = F + 2 * ((size_t)i * a + j);
            const double lr = f[0] * inv, li = f[1] * inv;
            f[0] = lr;
            f[1] = li;
            s_cr[i] = lr;
            s_ci[i] = li;
        }
        if (t == 0) {
            s_dl[j] = piv;
            s_pos[j] = 0;
        }
        __syncthreads();
        // F[i][i2] -= l_i conj(l_i2) for j < i2 <= i (lower triangle)
        for (int i = j + 1 + wrow; i < a; i += nwave) {
            const double lir = s_cr[i], lii = s_ci[i];
            double* frow = F + 2 * (size_t)i * a;
            for (int i2 = j + 1 + lane; i2 <= i; i2 += 64) {
                const double br = s_cr[i2], bi = s_ci[i2];
                frow[2 * i2] -= lir * br + lii * bi;
                frow[2 * i2 + 1] -= lii * br - lir * bi;
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
        info_d[0] = minpiv;
    }
    __syncthreads();
    const int r = s_r;
    // X = R^{-1} (upper triangular, r x r over the kept columns), R[p][u] =
    // conj(L[kept u][kept p]). Column q by back substitution:
    // X[p][q] = -(sum_{u = p+1..q} R[p][u] X[u][q]) / R[p][p], X[q][q] = 1 / R[q][q].
    // X[u][q] (u < q) is stored at F[kept u][kept q] (upper triangle, complex).
    for (int q = t; q < r; q += nth) {
        const int kq = s_kept[q];
        s_dr[q] = 1.0 / s_dl[kq];
        for (int p = q - 1; p >= 0; --p) {
            const int kp = s_kept[p];
            // u = q term: R[p][q] X[q][q] = conj(L[kq][kp]) / R[q][q]
            const double* lqp = F + 2 * ((size_t)kq * a + kp);
            double sr = lqp[0] * s_dr[q], si = -lqp[1] * s_dr[q];
            for (int u = p + 1; u < q; ++u) {
                const int ku = s_kept[u];
                const double* lup = F + 2 * ((size_t)ku * a + kp);  // R[p][u] = conj(lup)
                const double* xuq = F + 2 * ((size_t)ku * a + kq);  // X[u][q]
                sr += lup[0] * xuq[0] + lup[1] * xuq[1];
                si += lup[0] * xuq[1] - lup[1] * xuq[0];
            }
            double* xpq = F + 2 * ((size_t)kp * a + kq);
            const double inv = 1.0 / s_dl[kp];
            xpq[0] = -sr * inv;
            xpq[1] = -si * inv;
        }
    }
    __syncthreads();
    for (size_t e = t; e < (size_t)a * r; e += nth) {
        const int i = (int)(e / r), q = (int)(e % r);
        const int p = s_pos[i];
        double vr = 0.0, vi = 0.0;
        if (p >= 0 && p <= q) {
            if (p == q) {
                vr = s_D[i] * s_dr[q];
            } else {
                const double* x = F + 2 * ((size_t)i * a + s_kept[q]);
                vr = s_D[i] * x[0];
                vi = s_D[i] * x[1];
            }
        }
        T[2 * e] = vr;
        T[2 * e + 1] = vi;
    }
}

// ---------------------------------------------------------------------------
// Householder reduction of the Hermitian m x m matrix A (row-major, complex,
// both triangles kept up to date; overwritten) to a real symmetric
// tridiagonal. Reflector k is H_k = I - tau_k v_k v_k^H with real tau_k, v_k
// (complex, leading 1 at position k + 1) stored in Vh row k from column k + 1;
// it maps column k below the diagonal, x, to beta_k e_1 with beta_k =
// -(x_0 / |x_0|) ||x||, so H_k is Hermitian and unitary. The reduced matrix is
// Hermitian tridiagonal with complex subdiagonal beta_k; the diagonal unitary
// D = diag(delta) with delta_0 = 1, delta_{k+1} = delta_k beta_k / |beta_k|
// makes D^H T D real with subdiagonal |beta_k|. Outputs: d (diagonal), e
// (|beta_k|), ph (delta, complex) and tau. Then A = Q D T_real D^H Q^H with
// Q = H_0 H_1 ... H_{m-3}.
constexpr int kZTri = 1024;
template <bool kInLds>
__global__ __launch_bounds__(kZTri) void hetrd_z_kernel(int m, double* __restrict__ Ag, double* __restrict__ d,
                                                        double* __restrict__ e, double* __restrict__ ph,
                                                        double* __restrict__ tau, double* __restrict__ Vh) {
    constexpr int NW = kZTri / 64;
    extern __shared__ double zdyn[];
    __shared__ double svr[512], svi[512], swr[512], swi[512];
    __shared__ double sred[2 * NW];
    __shared__ double s_scal[4];
    __shared__ double s_beta[2 * 512];  // complex beta_k
    const int t = threadIdx.x;
    double* A = kInLds ? zdyn : Ag;
    if (kInLds) {
        for (size_t q = t; q < (size_t)2 * m * m; q += kZTri) zdyn[q] = Ag[q];
        __syncthreads();
    }
    for (int k = 0; k + 2 < m; ++k) {
        const int L = m - k - 1;
        // x = column k below the diagonal: A[k+1+i][k]
        double part = 0.0;
        for (int i = 1 + t; i < L; i += kZTri) {
            const double* x = A + 2 * ((size_t)(k + 1 + i) * m + k);
            part += x[0] * x[0] + x[1] * x[1];
        }
        part = zwave_sum(part);
        if ((t & 63) == 0) sred[t >> 6] = part;
        __syncthreads();
        if (t == 0) {
            double sigma2 = 0.0;
            for (int q = 0; q < NW; ++q) sigma2 += sred[q];
            const double* x0 = A + 2 * ((size_t)(k + 1) * m + k);
            const double ar = x0[0], ai = x0[1];
            const double amod = sqrt(ar * ar + ai * ai);
            double tk = 0.0, ur = 1.0, ui = 0.0, br = ar, bi = ai;
            if (sigma2 > 0.0) {
                const double nrm = sqrt(amod * amod + sigma2);
                const double phr = amod > 0.0 ? ar / amod : 1.0, phi = amod > 0.0 ? ai / amod : 0.0;
                br = -phr * nrm;
                bi = -phi * nrm;
                // u0 = x0 - beta = ph (|x0| + nrm); v_i = x_i / u0 (i >= 1)
                const double u0m = amod + nrm;
                ur = phr * u0m;
                ui = phi * u0m;
                tk = 2.0 / (1.0 + sigma2 / (u0m * u0m));
            }
            s_scal[0] = tk;
            // 1 / u0 = conj(u0) / |u0|^2
            const double den = ur * ur + ui * ui;
            s_scal[1] = ur / den;
            s_scal[2] = -ui / den;
            s_beta[2 * k] = br;
            s_beta[2 * k + 1] = bi;
            d[k] = A[2 * ((size_t)k * m + k)];
            tau[k] = tk;
        }
        __syncthreads();
        const double tk = s_scal[0], ir = s_scal[1], ii = s_scal[2];
        for (int i = t; i < L; i += kZTri) {
            double vr = 1.0, vi = 0.0;
            if (i > 0) {
                if (tk != 0.0) {
                    const double* x = A + 2 * ((size_t)(k + 1 + i) * m + k);
                    vr = x[0] * ir - x[1] * ii;
                    vi = x[0] * ii + x[1] * ir;
                } else {
                    vr = 0.0;
                }
            }
            svr[i] = vr;
            svi[i] = vi;
            double* vh = Vh + 2 * ((size_t)k * m + k + 1 + i);
            vh[0] = vr;
            vh[1] = vi;
        }
        __syncthreads();
        if (tk == 0.0) continue;
        // p = tau A22 v, A22 = A[k+1:, k+1:]. Hermitian: p_i = tau sum_j
        // conj(A22[j][i]) v_j, so thread i walks column i (consecutive threads
        // read consecutive entries of a row).
        double pvr = 0.0;
        for (int i = t; i < L; i += kZTri) {
            const double* colp = A + 2 * ((size_t)(k + 1) * m + (k + 1 + i));
            double sr = 0.0, si = 0.0;
            for (int jj = 0; jj < L; ++jj) {
                const double arr = colp[2 * (size_t)jj * m], aii = colp[2 * (size_t)jj * m + 1];
                // conj(a) v = (ar vr + ai vi) + i (ar vi - ai vr)
                sr = fma(arr, svr[jj], fma(aii, svi[jj], sr));
                si = fma(arr, svi[jj], fma(-aii, svr[jj], si));
            }
            sr *= tk;
            si *= tk;
            swr[i] = sr;
            swi[i] = si;
            // Re(v^H p) = sum vr pr + vi pi (v^H A v is real)
            pvr += svr[i] * sr + svi[i] * si;
        }
        pvr = zwave_sum(pvr);
        if ((t & 63) == 0) sred[t >> 6] = pvr;
        __syncthreads();
        double pvs = 0.0;
        for (int q = 0; q < NW; ++q) pvs += sred[q];
        const double Kc = 0.5 * tk * pvs;
        for (int i = t; i < L; i += kZTri) {
            swr[i] -= Kc * svr[i];
            swi[i] -= Kc * svi[i];
        }
        __syncthreads();
        // A22 -= v w^H + w v^H
        for (size_t q = t; q < (size_t)L * L; q += kZTri) {
            const int r = (int)(q / L), c = (int)(q % L);
            double* a_ = A + 2 * ((size_t)(k + 1 + r) * m + (k + 1 + c));
            // v_r conj(w_c) + w_r conj(v_c)
            const double re = svr[r] * swr[c] + svi[r] * swi[c] + swr[r] * svr[c] + swi[r] * svi[c];
            const double im = svi[r] * swr[c] - svr[r] * swi[c] + swi[r] * svr[c] - swr[r] * svi[c];
            a_[0] -= re;
            a_[1] -= im;
        }
        __syncthreads();
    }
    if (t == 0) {
        if (m >= 2) {
            d[m - 2] = A[2 * ((size_t)(m - 2) * m + (m - 2))];
            s_beta[2 * (m - 2)] = A[2 * ((size_t)(m - 1) * m + (m - 2))];
            s_beta[2 * (m - 2) + 1] = A[2 * ((size_t)(m - 1) * m + (m - 2)) + 1];
        }
        d[m - 1] = A[2 * ((size_t)(m - 1) * m + (m - 1))];
        // phases delta and the real subdiagonal |beta_k|
        double dr = 1.0, di = 0.0;
        ph[0] = 1.0;
        ph[1] = 0.0;
        for (int k = 0; k + 1 < m; ++k) {
            const double br = s_beta[2 * k], bi = s_beta[2 * k + 1];
            const double bm = sqrt(br * br + bi * bi);
            e[k] = bm;
            if (bm > 0.0) {
                const double nr = (dr * br - di * bi) / bm, ni = (dr * bi + di * br) / bm;
                dr = nr;
                di = ni;
            }
            ph[2 * (k + 1)] = dr;
            ph[2 * (k + 1) + 1] = di;
        }
        if (m < 3) {
            for (int k = 0; k < m; ++k) tau[k] = 0.0;
        }
    }
}

// Z = Q D ZT: row j of each real eigenvector of the tridiagonal is scaled by
// delta_j, then H_{m-3}, ..., H_0 are applied. One wave per eigenvector, kept
// in registers (m <= 512: 8 complex values per lane). ZT (m x k real) and Z
// (m x k complex) have leading dimension k.
__global__ __launch_bounds__(256) void zbacktransform_kernel(int m, int k, const double* __restrict__ tau,
                                                             const double* __restrict__ Vh,
                                                             const double* __restrict__ ph,
                                                             const double* __restrict__ ZT,
                                                             double* __restrict__ Z) {
    constexpr int MAXQ = 512 / 64;
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= k) return;
    double zr[MAXQ], zi[MAXQ];
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
        const int j = lane + 64 * q;
        const double y = (j < m) ? ZT[(size_t)j * k + i] : 0.0;
        zr[q] = (j < m) ? y * ph[2 * j] : 0.0;
        zi[q] = (j < m) ? y * ph[2 * j + 1] : 0.0;
    }
    for (int kk = m - 3; kk >= 0; --kk) {
        const double tk = tau[kk];
        if (tk == 0.0) continue;
        const double* v = Vh + 2 * (size_t)kk * m;  // v[j] valid for j >= kk + 1
        double vr[MAXQ], vi[MAXQ];
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int q = 0; q < MAXQ; ++q) {
            const int j = lane + 64 * q;
            const bool ok = j > kk && j < m;
            vr[q] = ok ? v[2 * j] : 0.0;
            vi[q] = ok ? v[2 * j + 1] : 0.0;
            // v^H z = sum conj(v) z
            sr += vr[q] * zr[q] + vi[q] * zi[q];
            si += vr[q] * zi[q] - vi[q] * zr[q];
        }
        sr = zwave_sum(sr) * tk;
        si = zwave_sum(si) * tk;
#pragma unroll
        for (int q = 0; q < MAXQ; ++q) {
            // z -= v s
            zr[q] -= vr[q] * sr - vi[q] * si;
            zi[q] -= vr[q] * si + vi[q] * sr;
        }
    }
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
        const int j = lane + 64 * q;
        if (j < m) {
            Z[2 * ((size_t)j * k + i)] = zr[q];
            Z[2 * ((size_t)j * k + i) + 1] = zi[q];
        }
    }
}

// Layout conversions between a complex column-major n x w block (leading
// dimension n, interleaved) and complex row-major rows (leading dimension
// ldc); rcol_to_zrows takes a real column-major block (imaginary parts 0).
__global__ __launch_bounds__(kZThreads) void zcol_to_rows_kernel(long long n, int w, const double* __restrict__ src,
                                                                 double* __restrict__ dst, long long ldc) {
    const long long total = n * w;
    for (long long e = (long long)blockIdx.x * kZThreads + threadIdx.x; e < total;
         e += (long long)gridDim.x * kZThreads) {
        const long long c = e / n, r = e % n;
        dst[2 * (r * ldc + c)] = src[2 * e];
        dst[2 * (r * ldc + c) + 1] = src[2 * e + 1];
    }
}
__global__ __launch_bounds__(kZThreads) void zrows_to_col_kernel(long long n, int w, const double* __restrict__ src,
                                                                 long long ldc, double* __restrict__ dst) {
    const long long total = n * w;
    for (long long e = (long long)blockIdx.x * kZThreads + threadIdx.x; e < total;
         e += (long long)gridDim.x * kZThreads) {
        const long long c = e / n, r = e % n;
        dst[2 * e] = src[2 * (r * ldc + c)];
        dst[2 * e + 1] = src[2 * (r * ldc + c) + 1];
    }
}
__global__ __launch_bounds__(kZThreads) void rcol_to_zrows_kernel(long long n, int w, const double* __restrict__ src,
                                                                  double* __restrict__ dst, long long ldc) {
    const long long total = n * w;
    for (long long e = (long long)blockIdx.x * kZThreads + threadIdx.x; e < total;
         e += (long long)gridDim.x * kZThreads) {
        const long long c = e / n, r = e % n;
        dst[2 * (r * ldc + c)] = src[e];
        dst[2 * (r * ldc + c) + 1] = 0.0;
    }
}

inline int zgrid(long long work, long long cap = 4096) {
    long long g = (work + kZThreads - 1) / kZThreads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace

hipError_t launch_spmm_z(hipStream_t st, int n, const int* rowptr, const int* col, const double* val,
                         const double* X, long long ldx, double* Y, long long ldy, int w) {
    if (n <= 0 || w <= 0) return hipSuccess;
    const long long waves = ((long long)n + kZRows - 1) / kZRows;
    const int grid = (int)((waves + kZThreads / 64 - 1) / (kZThreads / 64));
    hipLaunchKernelGGL(spmm_z_kernel, dim3(grid), dim3(kZThreads), 0, st, n, rowptr, col, val, X, ldx, Y, ldy, w);
    return hipGetLastError();
}

hipError_t launch_zgram_combine(hipStream_t st, int mu, int mv, const double* P, double* C) {
    hipLaunchKernelGGL(zgram_combine_kernel, dim3(zgrid((long long)mu * mv)), dim3(kZThreads), 0, st, mu, mv, P, C);
    return hipGetLastError();
}

hipError_t launch_zembed(hipStream_t st, int K, int N, const double* C, double* E) {
    hipLaunchKernelGGL(zembed_kernel, dim3(zgrid((long long)K * N)), dim3(kZThreads), 0, st, K, N, C, E);
    return hipGetLastError();
}

hipError_t launch_zherm(hipStream_t st, int m, double* A) {
    hipLaunchKernelGGL(zherm_kernel, dim3(zgrid((long long)m * m)), dim3(kZThreads), 0, st, m, A);
    return hipGetLastError();
}

hipError_t launch_hl_init_z(hipStream_t st, int m, int k, const double* Z1, const int* act, int a, double* B,
                            double* Y) {
    if (a <= 0) return hipSuccess;
    hipLaunchKernelGGL(hl_init_z_kernel, dim3(zgrid((long long)(m + k) * a)), dim3(kZThreads), 0, st, m, k, Z1, act,
                       a, B, Y);
    return hipGetLastError();
}

hipError_t launch_cholz(hipStream_t st, int a, const double* G, double* T, double* work, int* info_i,
                        double* info_d, double drop_tol2) {
    if (a <= 0 || a > 512) return hipErrorInvalidValue;
    hipLaunchKernelGGL(cholz_kernel, dim3(1), dim3(kZSmall), 0, st, a, G, T, work, info_i, info_d, drop_tol2);
    return hipGetLastError();
}

hipError_t launch_zcol_to_rows(hipStream_t st, long long n, int w, const double* src, double* dst, long long ldc) {
    hipLaunchKernelGGL(zcol_to_rows_kernel, dim3(zgrid(n * w, 16384)), dim3(kZThreads), 0, st, n, w, src, dst, ldc);
    return hipGetLastError();
}
hipError_t launch_zrows_to_col(hipStream_t st, long long n, int w, const double* src, long long ldc, double* dst) {
    hipLaunchKernelGGL(zrows_to_col_kernel, dim3(zgrid(n * w, 16384)), dim3(kZThreads), 0, st, n, w, src, ldc, dst);
    return hipGetLastError();
}
hipError_t launch_rcol_to_zrows(hipStream_t st, long long n, int w, const double* src, double* dst, long long ldc) {
    hipLaunchKernelGGL(rcol_to_zrows_kernel, dim3(zgrid(n * w, 16384)), dim3(kZThreads), 0, st, n, w, src, dst, ldc);
    return hipGetLastError();
}

size_t heev_z_work_doubles(int m) {
    // d, e, tau (3m), phases (2m), Vh (2 m^2), the real eigenvectors of the
    // tridiagonal (m k <= m^2), their work, and margins
    return 5 * (size_t)m + 3 * (size_t)m * m + tridiag_vectors_work_doubles(m) + 64;
}

hipError_t launch_heev_lowest_z(hipStream_t st, int m, int k, double* A, double* w, double* Z, double* work) {
    if (m <= 0 || m > 512 || k <= 0 || k > m) return hipErrorInvalidValue;
    double* d = work;
    double* e = d + m;
    double* tau = e + m;
    double* ph = tau + m;
    double* Vh = ph + 2 * (size_t)m;
    double* ZT = Vh + 2 * (size_t)m * m;
    double* twork = ZT + (size_t)m * k;
    const size_t lds = (2 * (size_t)m * m <= 12800) ? sizeof(double) * 2 * (size_t)m * m : 0;
    if (lds)
        hipLaunchKernelGGL(hetrd_z_kernel<true>, dim3(1), dim3(kZTri), lds, st, m, A, d, e, ph, tau, Vh);
    else
        hipLaunchKernelGGL(hetrd_z_kernel<false>, dim3(1), dim3(kZTri), 0, st, m, A, d, e, ph, tau, Vh);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    err = launch_tridiag_lowest_vectors(st, m, k, d, e, w, ZT, twork);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(zbacktransform_kernel, dim3((k + 3) / 4), dim3(256), 0, st, m, k, tau, Vh, ph, ZT, Z);
    return hipGetLastError();
}

}  // namespace se
