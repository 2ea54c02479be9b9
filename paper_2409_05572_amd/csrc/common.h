// Internal declarations shared by the HIP kernels and the host engine.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <tuple>
#include <utility>

namespace se {

// Issues kernel launches on a stream, or appends them to a graph as a chain of
// kernel nodes (each depending on the one before). The graph is built
// explicitly rather than captured from a stream: a capture in progress makes
// other threads' work on the null stream fail, and a serving engine cannot
// keep its callers from using the null stream.
// Between fork() and join() the launches are independent branches (graph
// nodes that depend only on the node before the fork; on a stream they run in
// order); the launch after join() depends on all of them.
struct Launcher {
    hipStream_t st = nullptr;
    hipGraph_t graph = nullptr;  // nullptr: launch on st
    hipGraphNode_t last = nullptr;
    hipError_t err = hipSuccess;

    void fork() {
        forking = true;
        base = last;
        nbranch = 0;
    }
    void join() { forking = false; }

    template <class... P, class... A>
    void operator()(void (*kernel)(P...), dim3 grid, dim3 block, size_t shmem, A... args) {
        if (err != hipSuccess) return;
        if (!graph) {
            hipLaunchKernelGGL(kernel, grid, block, shmem, st, static_cast<P>(args)...);
            err = hipGetLastError();
            return;
        }
        std::tuple<P...> vals(static_cast<P>(args)...);
        void* argv[sizeof...(P) > 0 ? sizeof...(P) : 1];
        fill_args(vals, argv, std::index_sequence_for<P...>{});
        hipKernelNodeParams kp{};
        kp.func = reinterpret_cast<void*>(kernel);
        kp.gridDim = grid;
        kp.blockDim = block;
        kp.sharedMemBytes = (unsigned)shmem;
        kp.kernelParams = argv;
        kp.extra = nullptr;
        hipGraphNode_t node = nullptr;
        if (forking) {
            err = hipGraphAddKernelNode(&node, graph, base ? &base : nullptr, base ? 1 : 0, &kp);
            if (err == hipSuccess && nbranch < kMaxBranch) branch[nbranch++] = node;
            if (nbranch == kMaxBranch) err = hipErrorInvalidValue;
            return;
        }
        if (nbranch > 0) {  // first launch after a join
            err = hipGraphAddKernelNode(&node, graph, branch, (size_t)nbranch, &kp);
            nbranch = 0;
        } else {
            err = hipGraphAddKernelNode(&node, graph, last ? &last : nullptr, last ? 1 : 0, &kp);
        }
        if (err == hipSuccess) last = node;
    }

  private:
    static constexpr int kMaxBranch = 16;
    bool forking = false;
    hipGraphNode_t base = nullptr;
    hipGraphNode_t branch[kMaxBranch] = {};
    int nbranch = 0;

    template <class T, size_t... I>
    static void fill_args(T& vals, void** argv, std::index_sequence<I...>) {
        ((argv[I] = static_cast<void*>(&std::get<I>(vals))), ...);
    }
};

// Up to four column segments of row-major n-row blocks that share one leading
// dimension. Segment s covers logical columns [off[s], off[s] + w[s]) and
// element (i, c) of it lives at p[s][i * ld + (c - off[s])].
struct Segs {
    const double* p[4];
    int w[4];
    int off[5];
    int nseg;
    long long ld;
};

inline Segs make_segs(long long ld) {
    Segs s{};
    s.nseg = 0;
    s.ld = ld;
    s.off[0] = 0;
    return s;
}
inline void push_seg(Segs& s, const double* p, int w) {
    if (w <= 0) return;
    s.p[s.nseg] = p;
    s.w[s.nseg] = w;
    s.off[s.nseg + 1] = s.off[s.nseg] + w;
    s.nseg++;
}
inline int segs_width(const Segs& s) { return s.off[s.nseg]; }

// Low-precision panels: BF16 values are stored as the upper 16 bits of the
// FP32 pattern (rounded to nearest even).
using bf16_t = uint16_t;

// The same column-segment view over FP32 or BF16 panels.
template <class T>
struct SegsT {
    const T* p[4];
    int w[4];
    int off[5];
    int nseg;
    long long ld;
};

template <class T>
inline SegsT<T> make_segs_t(long long ld) {
    SegsT<T> s{};
    s.nseg = 0;
    s.ld = ld;
    s.off[0] = 0;
    return s;
}
template <class T>
inline void push_seg_t(SegsT<T>& s, const T* p, int w) {
    if (w <= 0) return;
    s.p[s.nseg] = p;
    s.w[s.nseg] = w;
    s.off[s.nseg + 1] = s.off[s.nseg] + w;
    s.nseg++;
}
template <class T>
inline int segs_width(const SegsT<T>& s) {
    return s.off[s.nseg];
}

// ---- bulk kernels (bulk.hip) ----
// Rows with more than kHeavyRow nonzeros (power-law graphs) are listed in
// `heavy` and computed by one workgroup each; the row-per-lane-group kernel
// skips them.
constexpr int kHeavyRow = 64;
// The matrix's column and value arrays carry kCsrPad trailing entries
// (column 0, value 0) so that batched loads past the last nonzero stay in
// bounds and name a valid row.
constexpr int kCsrPad = 64;

// Y[:, 0:w] = A X[:, 0:w] for CSR A with int32 row offsets.
hipError_t launch_spmm(hipStream_t st, int n, const int* rowptr, const int* col, const double* val,
                       const double* X, long long ldx, double* Y, long long ldy, int w,
                       const int* heavy, int n_heavy);

// Per-column sums over rows of (AX - lam X)^2 and X^2 for columns [0, k):
// out[c] = ||r_c||^2, out[k + c] = ||x_c||^2. part is scratch of
// gram_partial_doubles(n, 2k) doubles. With R != nullptr the residual block
// R = AX - X diag(lam) is also written (n x k, leading dimension ldr) in the
// same pass.
hipError_t launch_resid_norms(hipStream_t st, long long n, const double* X, const double* AX,
                              long long ld, int k, const double* lam, double* part, double* out,
                              double* R = nullptr, long long ldr = 0);

// Y = A X (streaming product; matrices without heavy rows, w <= 128) and, for
// the rows produced, R = Y - X diag(lam) with out[c] = ||r_c||^2 and
// out[w + c] = ||x_c||^2 (as launch_resid_norms). part is scratch of
// 2 w spmm_resid_chunks(n) doubles.
long long spmm_resid_chunks(long long n);
hipError_t launch_spmm_resid(hipStream_t st, int n, const int* rowptr, const int* col, const double* val,
                             const double* X, long long ldx, double* Y, long long ldy, int w, const int* heavy,
                             int n_heavy, const double* lam, double* R, long long ldr, double* part, double* out);

// n x nb start block, entry (i, j) = 2 u - 1, u = (z >> 11) 2^-53, z =
// SplitMix64 of the state seed + (j n + i + 1) 0x9E3779B97F4A7C15, stored at
// X[i * ld + j] (row-major) or X[j * ld + i] (col_major).
hipError_t launch_seeded_block(hipStream_t st, long long n, int nb, unsigned long long seed, double* X,
                               long long ld, bool col_major);

// Jacobi preconditioner: dinv[r] = 1 / |a_rr| (1 for a missing or zero
// diagonal); W[r, c] *= dinv[r] for c < a (ld even).
hipError_t launch_jacobi(hipStream_t st, int n, const int* rowptr, const int* col, const double* val, double* dinv);
hipError_t launch_row_scale(hipStream_t st, long long n, int a, const double* dinv, double* W, long long ld);

// Column-wise CG for TraceMIN's inner solve (per-column scalars on the device):
// out[c] = U[:, c] . V[:, c];
// D += alpha d (D = alpha d when first), R -= alpha Q, rr_new[c] = R[:, c] . R[:, c],
//   alpha_c = rr_c / dq_c (0 if rr_c = 0 or dq_c <= 0);
// Dir[:, c] = R[:, c] + (rr_new_c / rr_c) Dir[:, c] (beta 0 if rr_c = 0).
// `part` holds 4096 k doubles.
hipError_t launch_col_dots(hipStream_t st, long long n, int k, const double* U, const double* V, long long ld,
                           double* part, double* out);
hipError_t launch_cg_step(hipStream_t st, long long n, int k, const double* rr, const double* dq, const double* Dir,
                          const double* Q, double* D, double* R, long long ld, bool first, double* part,
                          double* rr_new);
hipError_t launch_cg_dir(hipStream_t st, long long n, int k, const double* rr_new, const double* rr, const double* R,
                         double* Dir, long long ld);

// Z[:, c] = alpha U[:, c] + beta V[:, c] + gamma Z[:, c] for c < k (Z is not
// read when gamma = 0): one step of the Chebyshev filter recurrence. ld even.
hipError_t launch_cheb_step(hipStream_t st, long long n, int k, double alpha, const double* U, double beta,
                            const double* V, double gamma, double* Z, long long ld);

// Z <- alpha A Y + beta Y + gamma Z over the first w columns in one pass over
// the CSR rows (the product is never stored); matrices without heavy rows only
// (n_heavy must be 0), CSR arrays padded by kCsrPad entries, ld even and
// >= w + 1 for odd w.
hipError_t launch_spmm_cheb(hipStream_t st, int n, const int* rowptr, const int* col, const double* val,
                            const double* Y, double* Z, long long ld, int w, int n_heavy, double alpha, double beta,
                            double gamma);

// Columns c0 .. c0 + d - 1 of the row-major n-row panel X get the normally
// distributed block of draw `draw`: entry (i, j) is sqrt(-2 ln u1) cos(2 pi u2)
// (Box-Muller) with u1 = ((z1 >> 11) + 1) 2^-53, u2 = (z2 >> 11) 2^-53 and z1,
// z2 the SplitMix64 outputs at counters 2t and 2t + 1, t = (draw nb + j) n + i.
hipError_t launch_gaussian_cols(hipStream_t st, long long n, int d, int nb, long long draw, unsigned long long seed,
                                double* X, long long ld, int c0);

// dst[:, q] = src[:, idx[q]] for q < a (dst must not overlap src).
hipError_t launch_gather_cols(hipStream_t st, long long n, const double* src, long long lds, const int* idx,
                              int a, double* dst, long long ldd);

// W[:, jj] = AX[:, act[jj]] - lam[act[jj]] X[:, act[jj]], jj < a.
hipError_t launch_form_w(hipStream_t st, long long n, const double* X, const double* AX,
                         long long ld, const double* lam, const int* act, int a, double* W,
                         long long ldw);

// X[:, c] = scale (sigma X[:, c] - AX[:, c]) for c < k.
hipError_t launch_shift_sub(hipStream_t st, long long n, double* X, const double* AX, long long ld,
                            int k, double sigma, double scale = 1.0);

// dst[:, dc + c] = src[:, sc + c] for c < w.
hipError_t launch_copy_cols(hipStream_t st, long long n, const double* src, long long lds, int sc,
                            double* dst, long long ldd, int dc, int w);

// Column-major (leading dimension ldc) <-> row-major (leading dimension ldr).
hipError_t launch_colmajor_to_rowmajor(hipStream_t st, long long n, int w, const double* src,
                                       long long ldc, double* dst, long long ldr);
hipError_t launch_rowmajor_to_colmajor(hipStream_t st, long long n, int w, const double* src,
                                       long long ldr, double* dst, long long ldc);

// Gram product C = U^T V (mu x mv row-major). With sym != 0 the result is
// taken as symmetric (mu == mv): only upper tiles are formed, the lower
// triangle mirrors the upper and diagonal tiles are averaged with their
// transpose. part is scratch of gram_scratch_doubles(n, mu, mv) doubles, or,
// with part_cap > 0, of part_cap doubles: the row chunks are then limited to
// part_cap / (mu mv) (hipErrorInvalidValue when mu mv > part_cap), which only
// changes the chunking (and so the summation order), not the result's bound.
size_t gram_scratch_doubles(long long n, int mu, int mv);
hipError_t launch_gram(hipStream_t st, long long n, const Segs& U, const Segs& V, int sym,
                       double* part, double* C, size_t part_cap = 0);

// Out = beta Out + alpha U C with C (K x N row-major, leading dimension N).
// Out segments must not alias U segments.
hipError_t launch_update(hipStream_t st, long long n, const Segs& U, const double* C, int N,
                         const Segs& Out, double alpha, double beta);

// Fixed-order sum of per-chunk partial vectors: out[i] = sum_c part[c L + i].
// part is scratch: with more than 1024 chunks, block sums overwrite some of
// its rows.
hipError_t launch_sum_partials(hipStream_t st, int L, int nchunks, double* part, double* out);

// Gram output tile (columns of U and of V per workgroup) and rows per stage,
// shared by the FP64 and low-precision Gram kernels.
constexpr int kGramTile = 96;
constexpr int kGramRows = 32;

// Row-chunk plan shared by the FP64 and low-precision Gram kernels, and the
// fixed-order FP64 sum of their per-chunk partials (C is mu x mv; with sym
// the lower tile triangle mirrors the upper one).
void gram_plan(long long n, int mu, int mv, int sym, int& ntiles, int& nt_v, int& nchunks,
               long long& rows, long long max_chunks = 0);
hipError_t launch_gram_reduce(hipStream_t st, int mu, int mv, int nchunks, int sym, const double* part,
                              double* C);

// ---- low-precision bulk kernels (bulk_lp.hip), T = float or bf16_t ----
// Storage is T, arithmetic FP32 (matrix cores for Gram and update), and every
// reduction over n leaves the workgroup in FP64. Leading dimensions must be
// multiples of 8 and at least the width rounded up to 8.
template <class T>
hipError_t launch_spmm_lp(hipStream_t st, int n, const int* rowptr, const int* col, const float* val,
                          const T* X, long long ldx, T* Y, long long ldy, int w, const int* heavy,
                          int n_heavy);
template <class T>
hipError_t launch_resid_norms_lp(hipStream_t st, long long n, const T* X, const T* AX, long long ld,
                                 int k, const double* lam, double* part, double* out);
template <class T>
hipError_t launch_form_w_lp(hipStream_t st, long long n, const T* X, const T* AX, long long ld,
                            const double* lam, const int* act, int a, T* W, long long ldw);
// X = scale (sigma X - AX) and the Chebyshev filter step Z = alpha U + beta V +
// gamma Z, both formed in FP64 from the stored values and rounded once.
template <class T>
hipError_t launch_shift_sub_lp(hipStream_t st, long long n, T* X, const T* AX, long long ld, int k,
                               double sigma, double scale = 1.0);
template <class T>
hipError_t launch_cheb_step_lp(hipStream_t st, long long n, int k, double alpha, const T* U, double beta,
                               const T* V, double gamma, T* Z, long long ld);
// The product A Y fused with that step (no heavy rows; FP32 values val32).
template <class T>
hipError_t launch_spmm_cheb_lp(hipStream_t st, int n, const int* rowptr, const int* col, const float* val,
                               const T* Y, T* Z, long long ld, int w, int n_heavy, double alpha, double beta,
                               double gamma);
template <class T>
hipError_t launch_copy_cols_lp(hipStream_t st, long long n, const T* src, long long lds, int sc, T* dst,
                               long long ldd, int dc, int w);
// FP64 column-major (ldc) -> T row-major (ldr), and T row-major -> FP64 row-major.
template <class T>
hipError_t launch_colmajor_to_rows_lp(hipStream_t st, long long n, int w, const double* src,
                                      long long ldc, T* dst, long long ldr);
template <class T>
hipError_t launch_rows_lp_to_f64(hipStream_t st, long long n, int w, const T* src, long long lds,
                                 double* dst, long long ldd);
template <class T>
hipError_t launch_gram_lp(hipStream_t st, long long n, const SegsT<T>& U, const SegsT<T>& V, int sym,
                          double* part, double* C);
// c32: scratch of K x N floats (K = width of U) that receives C rounded to FP32.
template <class T>
hipError_t launch_update_lp(hipStream_t st, long long n, const SegsT<T>& U, const double* C, int N,
                            const SegsT<T>& O, double alpha, double beta, float* c32);
hipError_t launch_f64_to_f32(hipStream_t st, long long count, const double* src, float* dst);

// ---- small dense kernels (small.hip), one matrix per call, FP64 ----
// Cholesky-QR transform with column drop: given G = W^T W (a x a), writes T
// (a x r, leading dimension r) such that W T has orthonormal columns, r into
// info_i[0] and the kept input columns (ascending) into info_i[1..r], the
// smallest scaled pivot into info_d[0]. Columns whose scaled pivot falls below
// drop_tol2 are dropped (zero rows of T); drop_tol2 < 0 drops nothing.
// ns_tol > 0: when ||G - I||_F <= ns_tol the kernel writes the Newton-Schulz
// transform T = (3 I - G) / 2 instead (r = a, info_d[0] = 1 - ||G - I||_F).
// work needs 2 a^2 + 2 a doubles.
hipError_t launch_chol_drop(hipStream_t st, int a, const double* G, double* T, double* work,
                            int* info_i, double* info_d, double drop_tol2, double ns_tol = 0.0);

// Symmetric eigensolver for the k algebraically smallest eigenpairs of the
// m x m matrix A (row-major, overwritten): w[0..k) ascending, Z row-major
// m x k (leading dimension k, eigenvector c in column c). work needs
// syev_work_doubles(m). launch_syev is the k = m case.
// Small dense helpers: Y = alpha X + beta Y over count entries; A[i][i] +=
// alpha for i < m; fill a rows x cols block; out[0] = sum of squares.
hipError_t launch_axpby(hipStream_t st, long long count, double alpha, const double* X, double beta, double* Y);
hipError_t launch_add_diag(hipStream_t st, int m, double* A, long long ld, double alpha);
hipError_t launch_fill(hipStream_t st, int rows, int cols, double* A, long long ld, double v);
hipError_t launch_sumsq(hipStream_t st, long long count, const double* X, double* out);
// A_p from its known leading q x q block Axp and G = S^T (A W) (m x (m - q)),
// symmetrized; and the symmetric gather out[a][b] = in[idx[a]][idx[b]].
hipError_t launch_assemble_ap(hipStream_t st, int m, int q, const double* Axp, const double* G, double* Ap);
hipError_t launch_gather_sym(hipStream_t st, int r, const int* idx, const double* in, long long ld,
                             double* out);

size_t syev_work_doubles(int m);
hipError_t launch_syev_lowest(hipStream_t st, int m, int k, double* A, double* w, double* Z,
                              double* work);
hipError_t launch_syev(hipStream_t st, int m, double* A, double* w, double* Z, double* work);

// The k lowest eigenpairs of the real symmetric tridiagonal (d, e) of order
// m: w ascending, ZT (m x k row-major, leading dimension k) orthonormal
// eigenvectors (bisection, inverse iteration, orthonormalization as in
// launch_syev_lowest). work needs tridiag_vectors_work_doubles(m).
size_t tridiag_vectors_work_doubles(int m);
hipError_t launch_tridiag_lowest_vectors(hipStream_t st, int m, int k, const double* d, const double* e,
                                         double* w, double* ZT, double* work);

// ---- complex Hermitian kernels (complex.hip), FP64, interleaved (re, im) ----
// Y = A X for complex CSR A (2 nnz + 2 kCsrPad values) and complex row-major
// blocks (leading dimensions in complex entries; 16-byte aligned).
hipError_t launch_spmm_z(hipStream_t st, int n, const int* rowptr, const int* col, const double* val,
                         const double* X, long long ldx, double* Y, long long ldy, int w);
// C (mu x mv complex) = U^H V from the real Gram product P (2mu x 2mv) of the
// interleaved views of U and V.
hipError_t launch_zgram_combine(hipStream_t st, int mu, int mv, const double* P, double* C);
// E (2K x 2N real) = the real embedding of the complex K x N matrix C, so
// that a real update of an interleaved view by E is the complex update by C.
hipError_t launch_zembed(hipStream_t st, int K, int N, const double* C, double* E);
// A <- (A + A^H) / 2 (complex m x m).
hipError_t launch_zherm(hipStream_t st, int m, double* A);
// Hetmaniuk-Lehoucq start block in complex coefficients (as launch_hl_init,
// with Y = Z1^H E).
hipError_t launch_hl_init_z(hipStream_t st, int m, int k, const double* Z1, const int* act, int a, double* B,
                            double* Y);
// Complex Cholesky-QR transform with column drop (a <= 512): T (a x r complex,
// leading dimension r) with W T orthonormal for G = W^H W; info as
// launch_chol_drop. work holds 2 a^2 doubles.
hipError_t launch_cholz(hipStream_t st, int a, const double* G, double* T, double* work, int* info_i,
                        double* info_d, double drop_tol2);
// Complex column-major (leading dimension n) <-> complex rows (leading
// dimension ldc); a real column-major block into complex rows (imaginary 0).
hipError_t launch_zcol_to_rows(hipStream_t st, long long n, int w, const double* src, double* dst, long long ldc);
hipError_t launch_zrows_to_col(hipStream_t st, long long n, int w, const double* src, long long ldc, double* dst);
hipError_t launch_rcol_to_zrows(hipStream_t st, long long n, int w, const double* src, double* dst, long long ldc);
// The k lowest eigenpairs of the Hermitian m x m complex matrix A (m <= 512;
// overwritten): w ascending (real), Z (m x k complex, leading dimension k).
size_t heev_z_work_doubles(int m);
hipError_t launch_heev_lowest_z(hipStream_t st, int m, int k, double* A, double* w, double* Z, double* work);

// Hetmaniuk-Lehoucq start block from Z1 (m x k, ld k) and the positions
// act[0..a) of the unlocked old X columns: B (m x a, ld a) = unit columns
// e_{act[c]}, Y (k x a, ld a) = rows act[c] of Z1, transposed.
hipError_t launch_hl_init(hipStream_t st, int m, int k, const double* Z1, const int* act, int a,
                          double* B, double* Y);

// ---------------------------------------------------------------------------
// Batched products for several resident solves. One launch serves a list of
// jobs (one per solve, at most kMaxBatch), each with its own sizes and
// pointers, read from device memory when the launch runs: a job's sizes may
// be written by an earlier kernel of the same stream, so a captured sequence
// of launches stays valid while the widths change. A job with no rows or no
// columns does nothing. Workgroups loop over the (job, row range, tile) work
// items of all jobs; each job's items and their reduction order depend only
// on that job, so its result does not depend on the others.
constexpr int kMaxBatch = 16;

struct BGramJob {  // C = U^T V (mu x mv); sym: U and V are the same block
    Segs U, V;
    long long n, rows;  // rows of U and V; rows per chunk (multiple of kGramRows)
    int mu, mv, sym, nchunks;
    double* part;  // nchunks x mu x mv partials
    double* C;
};
struct BUpdJob {  // O = beta O + alpha U C, C is K x N with leading dimension N
    Segs U, O;
    long long n;
    int K, N;
    const double* C;
    double alpha, beta;
};
struct BSpmmJob {  // Y = A X (w columns); CSR padded by kCsrPad, ldx >= w + 1 for odd w
    const int* rowptr;
    const int* col;
    const double* val;
    const double* X;
    double* Y;
    long long ldx, ldy;
    int n, w;
};
struct BResidJob {  // R = AX - X diag(lam) (k columns); out = [sum r^2, sum x^2] per column
    const double* X;
    const double* AX;
    const double* lam;
    double* R;
    double* part;  // nchunks x 2k
    double* out;   // 2k
    long long n, ld, ldr, rows;
    int k, nchunks;
};
// `grid` workgroups loop over the work items of the first nj jobs (the
// update takes one item per workgroup: grid must cover them all). Errors are
// left in L.err (1 <= nj <= kMaxBatch).
void launch_gram_batched(Launcher& L, const BGramJob* jobs, int nj, int grid);
void launch_update_batched(Launcher& L, const BUpdJob* jobs, int nj, int grid);
void launch_spmm_batched(Launcher& L, const BSpmmJob* jobs, int nj, int grid);
void launch_resid_batched(Launcher& L, const BResidJob* jobs, int nj, int grid);

// Batched small dense operations (one workgroup or a few per job).
struct SmallMMJob {  // C = alpha op(A) B + beta C; op(A) = A^T when transA (A: rows x ca), else A (rows x ca, B: ca x cb)
    const double* A;
    const double* B;
    double* C;
    double alpha, beta;
    int rows, ca, cb, lda, ldb, ldc, transA;
};
struct CholJob {  // launch_chol_drop's operation on one a x a Gram matrix (a <= 896; work: 2 a^2 + 2a doubles)
    const double* G;
    double* T;
    double* work;
    int* info_i;
    double* info_d;
    double drop_tol2, ns_tol;
    int a;
};
struct EigJob {  // launch_syev_lowest's operation; work holds syev_work_doubles(m) doubles; m <= 288
    double* A;
    double* w;
    double* Z;
    double* work;
    int m, k;
};
constexpr int kBatchEigMax = 288;
void launch_small_mm_batched(Launcher& L, const SmallMMJob* jobs, int nj);
void launch_chol_batched(Launcher& L, const CholJob* jobs, int nj);
// `jobspace`: device memory of syev_batched_jobspace_bytes() for the
// orthonormalization passes' job lists.
size_t syev_batched_jobspace_bytes();
void launch_syev_lowest_batched(Launcher& L, const EigJob* jobs, int nj, void* jobspace);

}  // namespace se
