/*
 * se.h - shrink-and-expand block eigensolvers for MI355X (gfx950).
 *
 * Computes the n_ev algebraically smallest eigenpairs A V = V Lambda of a large
 * sparse real symmetric matrix A (the problem statement of arXiv 2409.05572,
 * Section 1) with LOBPCG (Algorithm 3, Section 2.3) or subspace iteration
 * (Algorithm 1, Section 2.1), optionally shrinking and expanding the block
 * between iterations (Algorithm 5, Section 3.1) by the fix / slope / slopek
 * strategies (Algorithms 6 and 7, Section 3.2).
 *
 * Conventions for every call:
 *   - Return value se_status: 0 = SE_OK, > 0 warning (outputs valid),
 *     < 0 error (output buffers untouched unless stated otherwise).
 *   - No call aborts or exits the process; no C++ exception crosses this ABI.
 *   - "device pointer" means memory on the context's GPU (hipMalloc or any
 *     allocator of the same HIP runtime); "host pointer" means pageable or
 *     pinned host memory.
 *   - All work is enqueued on the context's stream. Calls that return results
 *     to the caller (se_solve) synchronize that stream before returning.
 *   - A context is not thread-safe: one host thread uses a context at a time.
 *     Different contexts are independent.
 */
#ifndef SE_H
#define SE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int se_status;

#define SE_OK 0
#define SE_NOT_CONVERGED 1      /* max_iter or time limit reached; best iterate returned */
#define SE_ERR_INVALID_ARG (-1) /* bad sizes, malformed CSR, non-finite values, NULL */
#define SE_ERR_OOM (-2)         /* device allocation failed */
#define SE_ERR_HIP (-3)         /* a HIP runtime call failed (see se_info.hip_error) */
#define SE_ERR_BREAKDOWN (-4)   /* orthogonalization lost every column */
#define SE_ERR_REJECTED (-5)    /* request larger than the configured memory budget */
#define SE_ERR_UNSUPPORTED (-6) /* option or size not supported */

typedef struct se_ctx se_ctx;
typedef struct se_matrix se_matrix;

/* Solvers. */
#define SE_LOBPCG 0 /* Algorithm 3 with soft locking and the Hetmaniuk-Lehoucq basis */
#define SE_SI 1     /* Algorithm 1 with the shifted power step X <- sigma X - A X */
#define SE_SD 2     /* Algorithm 2 (block steepest descent): S = [X, W], no P; soft locking
                       and expansion as in LOBPCG (X_drop orthonormalized against S) */
#define SE_TRACEMIN 3 /* Algorithm 4 (TraceMIN): X <- X - D with D from params.cg_steps
                         conjugate-gradient steps on P A P D = P R, P = I - X X^T, per column;
                         FP64, block <= 512; A must be positive definite */

/* Vectors appended at an expansion (Section 6, the vectors appended in the
 * expansion). SE_EXPAND_RANDOM is FP64 only (SE_ERR_UNSUPPORTED with a mixed
 * precision); the powered X_drop also runs in the low-precision phase. */
#define SE_EXPAND_XDROP 0   /* the vectors dropped at the last shrink (the paper's choice) */
#define SE_EXPAND_RANDOM 1  /* a normally distributed block of the same width, drawn on the
                               device: entry (i, j) of the e-th expansion (e = 1, 2, ...) is
                               Box-Muller of SplitMix64 counters 2t, 2t + 1 with
                               t = (e nb + j) n + i under params.seed (LOBPCG: the first
                               columns replace X_drop, the rest P_drop) */
#define SE_EXPAND_POWERED 2 /* subspace iteration only (SE_ERR_INVALID_ARG otherwise): the
                               held X_drop takes one power step sigma X - A X per iteration,
                               without orthogonalization, divided by sigma - theta_1
                               (theta_1 the smallest current Ritz value) */

/* Preconditioner T of W <- T R (Algorithms 2 and 3; LOBPCG and SD, FP64). */
#define SE_PRECOND_NONE 0   /* T = I (the paper's experiments) */
#define SE_PRECOND_JACOBI 1 /* T = diag(1 / |a_ii|) (1 where a_ii = 0); W is then projected
                               against [X, P] twice before it is orthonormalized */

/* Shrink-and-expand strategies (Section 3.2). */
#define SE_STRAT_NONE 0
#define SE_STRAT_FIX 1    /* Algorithm 6 */
#define SE_STRAT_SLOPE 2  /* Algorithm 7 with eq. (ckslope) */
#define SE_STRAT_SLOPEK 3 /* Algorithm 7 with eq. (ckslopek) */

/* Arithmetic of the bulk (n-length) work. */
#define SE_FP64 0
#define SE_FP32_MIXED 1 /* FP32 panels until r(j) <= r_switch, then FP64 */
#define SE_BF16_MIXED 2 /* BF16 panels until r(j) <= r_switch, then FP64 */

/* Where X0, V and lambda of se_solve live. */
#define SE_PTR_HOST 0
#define SE_PTR_DEVICE 1

/* se_matrix_create_csr flags. */
#define SE_MATRIX_HOST 0x0   /* rowptr/colind/val are host pointers */
#define SE_MATRIX_DEVICE 0x1 /* rowptr/colind/val are device pointers */

/* Columns of one history row (se_params.history). */
#define SE_HISTORY_FIELDS 8
/* j, r(j) by eq. (rk), max stop ratio, width k, width p, active a, locked, flags
 * (bit 0 = expanded this iteration, bit 1 = shrunk this iteration, bit 2 = iteration of
 * the low-precision phase of a mixed-precision solve, bit 3 = FP64 LOBPCG iteration whose
 * residual block was orthonormalized implicitly, by whitening the Gram matrix of
 * [X, P, W] in coefficient space) */

/* Kernel classes of se_info.kern_* */
#define SE_K_SPMM 0   /* CSR sparse x block (also fused with a Chebyshev filter step) */
#define SE_K_GRAM 1   /* tall-skinny Gram products and their fixed-order reduction */
#define SE_K_UPDATE 2 /* basis updates X <- S C, W <- W - [X,P] G, Cholesky-QR apply */
#define SE_K_RESID 3  /* residual norms, forming W, shifted power step, Chebyshev filter steps,
                         TraceMIN's column CG kernels, Jacobi scaling */
#define SE_K_EIG 4    /* dense eigensolve of the projected matrix */
#define SE_K_SMALL 5  /* Cholesky-QR transform and Hetmaniuk-Lehoucq coefficients */
#define SE_K_COPY 6   /* layout changes and column copies */
#define SE_K_CLASSES 8

typedef struct se_params {
    int32_t solver;      /* SE_LOBPCG, SE_SI, SE_SD or SE_TRACEMIN */
    int32_t strategy;    /* SE_STRAT_* */
    int32_t precision;   /* SE_FP64, SE_FP32_MIXED or SE_BF16_MIXED */
    int32_t ptr_mode;    /* SE_PTR_HOST or SE_PTR_DEVICE for X0, V, lambda */
    int32_t n_ev;        /* wanted eigenpairs, >= 1 */
    int32_t n_extra;     /* extra block columns: block size nb = n_ev + n_extra <= n */
    int32_t n_es;        /* width kept at a shrink; 0 = n_ev + min(5, n_extra - 1) */
    int32_t soft_lock;   /* LOBPCG: 1 = lock converged pairs (Section 6.2 setting) */
    int32_t j_e;         /* fix: expansion period (paper: 12) */
    int32_t j_s;         /* iterations from an expansion to the next shrink (paper: 2) */
    int32_t j_p;         /* slopek averaging window (paper: 10) */
    int32_t j_warm;      /* warm-up: first shrink not before iteration j_warm (paper: 5) */
    int32_t max_iter;    /* iteration cap (default 1000 LOBPCG, 20000 SI) */
    int32_t profile;     /* 1 = time every kernel launch with HIP events (se_info.kern_*) */
    double mu;           /* slope threshold (paper: 1.1) */
    double r_warm;       /* warm-up: first shrink once r(j) <= r_warm (paper: 1e-4) */
    double tol;          /* stop when ||A x_i - lambda_i x_i|| <= tol ||A|| ||x_i||, i <= n_ev */
    double sigma;        /* SI shift, must bound lambda_max from above; 0 = ||A|| */
    double time_limit_s; /* wall-clock cap; <= 0 = none */
    double r_switch;     /* mixed precision: leave the low-precision phase once r(j) <= r_switch
                            (or r(j) stops improving); 0 = 1e-5 (FP32), 4e-2 (BF16) */
    double implicit_pivot; /* FP64 LOBPCG: smallest scaled pivot of the Schur complement of W^T W
                              for which the residual block is orthonormalized implicitly (by
                              whitening in coefficient space) rather than projected and
                              orthonormalized over n; 0 = 1e-2; > 1 = always explicit */
    uint64_t seed;       /* start block generated when se_solve gets X0 = NULL, and the
                            blocks drawn by SE_EXPAND_RANDOM */
    double* history;     /* optional host buffer of history_cap x SE_HISTORY_FIELDS doubles */
    int32_t history_cap; /* rows available in history */
    int32_t expand_vectors; /* SE_EXPAND_XDROP (default), SE_EXPAND_RANDOM or SE_EXPAND_POWERED */
    int32_t filter_degree;  /* subspace iteration: 0 = the shifted power step sigma X - A X;
                               d in 1..64 = the Chebyshev filter of degree d (Zhou and Saad 2007)
                               that damps [theta_k, sigma] and is one at theta_1 (theta the
                               current Ritz values of the k-column block), by the scaled
                               three-term recurrence: d - 1 extra sparse products per
                               iteration. A powered X_drop takes the same filter. Falls back
                               to the shifted step at an iteration where sigma <= theta_k. In
                               the low-precision phase of a mixed solve every intermediate
                               block is stored in FP32 / BF16 (steps formed in FP64). */
    int32_t cg_steps;       /* SE_TRACEMIN: inner CG steps per iteration (0 = 5, the paper's) */
    int32_t precond;        /* SE_PRECOND_NONE (default) or SE_PRECOND_JACOBI */
    int32_t reserved;       /* must be 0 */
} se_params;

typedef struct se_info {
    int32_t iterations;     /* iterations performed */
    int32_t converged;      /* 1 if every pair i <= n_ev met the stopping test */
    int32_t n_shrinks;
    int32_t n_expands;
    double max_stop_ratio;  /* max_i ||A x_i - lambda_i x_i|| / (||A|| ||x_i||), fresh product */
    double max_paper_ratio; /* eq. (rk) on the returned pairs, fresh product */
    double time_ms;         /* wall time of the solve on the stream */
    /* Per kernel class SE_K_* (filled when params.profile = 1): summed device
     * time from HIP events around each launch, launch count, and algorithmic
     * HBM bytes / flops (every operand read and written exactly once). */
    double kern_ms[SE_K_CLASSES];
    double kern_bytes[SE_K_CLASSES];
    double kern_flops[SE_K_CLASSES];
    int32_t kern_calls[SE_K_CLASSES];
    uint64_t workspace_bytes; /* device workspace held by the context after the call */
    int32_t hip_error;      /* first failing hipError_t, 0 if none */
    int32_t history_len;    /* rows written to params.history */
    int32_t lp_iterations;  /* mixed precision: iterations of the low-precision phase */
    int32_t n_reprojections; /* LOBPCG: iterations whose residual block needed a second
                                projection against [X, P] (a column kept < 1/2 of its
                                squared norm after the first) */
} se_info;

/* Fill *p with the defaults of the paper's experiments (Section 6.1-6.2):
 * LOBPCG, no strategy, soft locking on, j_e = 12, j_s = 2, mu = 1.1, j_p = 10,
 * j_warm = 5, r_warm = 1e-4, tol = 1e-8, max_iter = 1000, host pointers. */
void se_params_default(se_params* p);

/* The last failing hipError_t of a call on this context (0 if none), and the
 * runtime's name for a hipError_t value (for messages). */
int32_t se_ctx_last_hip_error(const se_ctx* ctx);
const char* se_hip_error_name(int32_t e);

/* Create a context bound to HIP device `device` and stream `stream`
 * (a hipStream_t; NULL = the device's null stream). The stream is borrowed:
 * it must outlive the context. Errors: SE_ERR_INVALID_ARG (bad device or
 * out == NULL), SE_ERR_HIP. */
se_status se_ctx_create(int device, void* stream, se_ctx** out);
/* Release the context and its workspace. NULL is ignored. */
void se_ctx_destroy(se_ctx* ctx);

/* Create a real symmetric CSR matrix on the context's device (Section 1: the
 * Hermitian A; real case). The full symmetric pattern must be stored.
 *   n      rows (= columns), >= 1
 *   nnz    stored entries, rowptr[n] == nnz
 *   rowptr n + 1 int64 offsets, non-decreasing, rowptr[0] == 0
 *   colind nnz int32 column indices in [0, n)
 *   val    nnz finite doubles
 *   anorm  ||A||_2 or an upper bound of it (used by the stopping test and as
 *          the default SI shift); 0 = the library takes the Gershgorin bound
 *          max_i sum_j |a_ij| (>= ||A||_2 for symmetric A); must be >= 0
 * The library copies the arrays (host or device per `flags`); the caller's
 * buffers may be freed after the call. Offsets, index range and finiteness are
 * validated on the host in both modes (device arrays are copied back for it).
 * Errors: SE_ERR_INVALID_ARG, SE_ERR_OOM, SE_ERR_HIP. */
se_status se_matrix_create_csr(se_ctx* ctx, int64_t n, int64_t nnz, const int64_t* rowptr,
                               const int32_t* colind, const double* val, uint32_t flags,
                               double anorm, se_matrix** out);
/* Release the matrix. It may be called before or after se_ctx_destroy of the
 * context it was created with (it uses only the device id). NULL is ignored. */
void se_matrix_destroy(se_matrix* m);
int64_t se_matrix_n(const se_matrix* m);
/* The ||A||_2 bound the matrix uses (given or estimated). */
double se_matrix_anorm(const se_matrix* m);

/* Solve for the n_ev smallest eigenpairs (Algorithms 1 / 3 with Algorithm 5).
 *   X0     n x nb starting block, column-major, leading dimension n,
 *          nb = n_ev + n_extra; must have full column rank. NULL: the library
 *          generates it from params->seed: entry (i, j) = 2 u - 1 with
 *          u = (z >> 11) 2^-53 and z the SplitMix64 output (Steele, Lea and
 *          Flood 2014) of the state seed + (j n + i + 1) 0x9E3779B97F4A7C15
 *          mod 2^64 (exact in FP64, so host copies of the block match)
 *   V      output n x n_ev eigenvectors, column-major, leading dimension n
 *   lambda output n_ev eigenvalues, ascending
 * X0, V and lambda are host or device pointers per params->ptr_mode and are
 * owned by the caller. info may be NULL. Returns SE_OK when converged,
 * SE_NOT_CONVERGED with the best iterate in V/lambda when max_iter or the time
 * limit is reached, or an error (< 0) with V/lambda untouched. */
se_status se_solve(se_ctx* ctx, const se_matrix* A, const se_params* params, const double* X0,
                   double* V, double* lambda, se_info* info);

/* ---- Building blocks of one Rayleigh-Ritz step (device pointers, FP64) ----
 * Blocks are row-major: element (i, c) of an n x w block B with leading
 * dimension ld is B[i * ld + c]; ld must be even and >= w, pointers 16-byte
 * aligned. These calls enqueue on the context's stream and do not synchronize
 * except where a host output is written. */

/* Y = A X: the sparse-times-block product behind A_p = S^T A S (Algorithm 3)
 * and the SI update (Algorithm 1). X and Y are n x w, w in [1, 256]. */
se_status se_op_spmm(se_ctx* ctx, const se_matrix* A, const double* X, int64_t ldx, double* Y,
                     int64_t ldy, int32_t w);

/* C = U^T V (mu x mv, row-major, leading dimension mv), the tall-skinny Gram
 * products of the orthogonalization and projection steps. U is n x mu, V is
 * n x mv, 1 <= mu, mv <= 1024. Summation order is fixed (deterministic).
 * When V is U (same pointer, leading dimension and width) the product is
 * formed as symmetric: blocks on and above the diagonal are computed and
 * mirrored, so C is exactly symmetric. */
se_status se_op_gram(se_ctx* ctx, int64_t n, const double* U, int64_t ldu, int32_t mu,
                     const double* V, int64_t ldv, int32_t mv, double* C);

/* se_op_gram for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same product C = U^T V with the same arguments, limits and errors, but the
 * per-chunk partial products live in a fixed 32 MiB device array of the
 * library (one per device, held until the process ends) instead of the
 * context's workspace; the call never allocates. The row chunking is limited
 * to what that array holds, so the summation order (not the accuracy) may
 * differ from se_op_gram's for large n. Calls that overlap on one device
 * (any context, any stream) share the array and race: serialize them. */
se_status se_op_gram_noalloc(se_ctx* ctx, int64_t n, const double* U, int64_t ldu, int32_t mu,
                             const double* V, int64_t ldv, int32_t mv, double* C);

/* Out = beta * Out + U C: the basis updates X <- S Z, W <- W - [X,P] G and the
 * Cholesky-QR apply. U is n x K, C is K x N row-major (leading dimension N),
 * Out is n x N; 1 <= K, N <= 1024; beta is 0 or 1; Out must not overlap U. */
se_status se_op_update(se_ctx* ctx, int64_t n, const double* U, int64_t ldu, int32_t K,
                       const double* C, int32_t N, double* Out, int64_t ldo, double beta);

/* ---- Low-precision building blocks (the bulk steps of the mixed-precision
 * phase) ----
 * precision SE_FP32_MIXED: the blocks hold float; SE_BF16_MIXED: bfloat16
 * stored as 16-bit patterns. Arithmetic is FP32 (matrix cores for Gram and
 * update), every reduction over n is FP64, and the outputs are rounded to the
 * block format (C of the Gram product is FP64). ld must be a multiple of 8 and
 * >= w rounded up to 8; pointers 16-byte aligned. Same semantics and limits as
 * the FP64 calls above; the matrix's FP32 copy of its values is made on first
 * use and freed with the matrix. */
se_status se_op_spmm_lp(se_ctx* ctx, int32_t precision, const se_matrix* A, const void* X, int64_t ldx,
                        void* Y, int64_t ldy, int32_t w);
se_status se_op_gram_lp(se_ctx* ctx, int32_t precision, int64_t n, const void* U, int64_t ldu,
                        int32_t mu, const void* V, int64_t ldv, int32_t mv, double* C);
se_status se_op_update_lp(se_ctx* ctx, int32_t precision, int64_t n, const void* U, int64_t ldu,
                          int32_t K, const double* C, int32_t N, void* Out, int64_t ldo, double beta);

/* Symmetric eigendecomposition A = Z diag(w) Z^T of an m x m matrix (the
 * spectral decomposition of A_p in Algorithms 1 and 3), 1 <= m <= 1024.
 * A (row-major, symmetric) is overwritten; w ascending; Z row-major with
 * eigenvector c in column c. Synchronizes the stream. */
se_status se_op_syev(se_ctx* ctx, int32_t m, double* A, double* w, double* Z);

/* The k lowest eigenpairs of a symmetric m x m matrix (Algorithm 3 keeps only
 * the n_es lowest Ritz pairs of A_p), 1 <= k <= m <= 1024. A (row-major,
 * symmetric) is overwritten; w (k) ascending; Z row-major m x k with
 * eigenvector c in column c, orthonormal columns also inside degenerate
 * eigenvalue clusters. Synchronizes the stream. */
se_status se_op_syev_lowest(se_ctx* ctx, int32_t m, int32_t k, double* A, double* w, double* Z);

/* Orthonormalize the w columns of the n x w block W in place by Cholesky-QR
 * applied twice, dropping numerically dependent columns (the "orthogonalize"
 * step of Algorithms 1 and 3). *rank receives the number of columns kept;
 * they are compacted to the front. Synchronizes the stream. */
se_status se_op_cholqr(se_ctx* ctx, int64_t n, double* W, int64_t ldw, int32_t w, int32_t* rank);

/* ---- Complex Hermitian A (Section 1 states the problem for Hermitian
 * A in C^{n x n}; Algorithms 1 and 3 with X^H for the transposes) ----
 * Complex values are interleaved (re, im) doubles throughout. FP64 only. */

/* Create a complex Hermitian CSR matrix (full pattern, a_ji = conj(a_ij)).
 * As se_matrix_create_csr, with val holding 2 nnz doubles (entry e is
 * val[2e] + i val[2e + 1]); anorm 0 = the Gershgorin bound max_i sum_j |a_ij|.
 * The matrix is usable with se_solve_z and the *_z building blocks only. */
se_status se_matrix_create_csr_z(se_ctx* ctx, int64_t n, int64_t nnz, const int64_t* rowptr,
                                 const int32_t* colind, const double* val, uint32_t flags,
                                 double anorm, se_matrix** out);

/* The n_ev smallest eigenpairs of a complex Hermitian matrix: LOBPCG
 * (Algorithm 3, soft locking, HL basis) or SI (Algorithm 1, the shifted power
 * step X <- sigma X - A X), shrink-and-expand with any strategy, X_drop as
 * the expansion vectors. params as se_solve; precision must be SE_FP64,
 * expand_vectors SE_EXPAND_XDROP, filter_degree 0 and precond none
 * (otherwise SE_ERR_UNSUPPORTED); nb <= 170 for LOBPCG, <= 512 for SI.
 *   X0     n x nb complex start block, column-major (leading dimension n
 *          complex entries, 2 n nb doubles); NULL: the real seeded block of
 *          se_solve (imaginary parts zero)
 *   V      output n x n_ev complex eigenvectors, column-major
 *   lambda output n_ev real eigenvalues, ascending
 * Pointers per params->ptr_mode; return values as se_solve. */
se_status se_solve_z(se_ctx* ctx, const se_matrix* A, const se_params* params, const double* X0,
                     double* V, double* lambda, se_info* info);

/* Complex building blocks on device pointers: complex row-major blocks with
 * leading dimensions counted in complex entries (even), 16-byte aligned.
 * se_op_spmm_z: Y = A X (w in [1, 512]).
 * se_op_gram_z: C = U^H V (mu x mv complex, leading dimension mv; mu, mv <=
 *   512); exactly Hermitian when V is U.
 * se_op_update_z: Out = beta Out + U C (C K x N complex, leading dimension
 *   N; K, N <= 512; beta 0 or 1; Out must not overlap U).
 * se_op_heev_lowest_z: the k lowest eigenpairs of the Hermitian m x m
 *   complex matrix A (m <= 512; overwritten): w (k real) ascending, Z (m x k
 *   complex, leading dimension k) orthonormal. Synchronizes the stream. */
se_status se_op_spmm_z(se_ctx* ctx, const se_matrix* A, const double* X, int64_t ldx, double* Y,
                       int64_t ldy, int32_t w);
se_status se_op_gram_z(se_ctx* ctx, int64_t n, const double* U, int64_t ldu, int32_t mu,
                       const double* V, int64_t ldv, int32_t mv, double* C);
se_status se_op_update_z(se_ctx* ctx, int64_t n, const double* U, int64_t ldu, int32_t K,
                         const double* C, int32_t N, double* Out, int64_t ldo, double beta);
se_status se_op_heev_lowest_z(se_ctx* ctx, int32_t m, int32_t k, double* A, double* w, double* Z);

/* Replay the shrink-and-expand controller (the strategy and warm-up rule of
 * Section 3.2 selected in params) on a scripted sequence r(1..count) of
 * eq. (rk) values, without a matrix or a GPU. flags[j-1] receives bit 0 when
 * iteration j expands and bit 1 when it shrinks. Host-only. */
se_status se_strategy_replay(const se_params* params, int32_t count, const double* r,
                             int32_t* flags);

/* ---- Serving: many solves resident on one GPU ----
 * A server runs up to max_slots solves at once, each on its own stream,
 * workspace and host worker thread, and starts queued requests as soon as a
 * slot is free (continuous batching, first come first served). Admission is by
 * HBM footprint: a request starts only if the device workspace held by all
 * slots, after the chosen slot grows to the request's footprint
 * (se_solve_footprint), stays within hbm_budget_bytes; slots keep their
 * workspace between requests. Results are the same as se_solve's on the same
 * inputs (FP64 solves are bitwise identical alone and in a mix).
 * The matrix of a request must have been created on a context of the server's
 * device and must outlive the request; X0, V, lambda (and params.history) are
 * the caller's and must stay valid until se_wait returns. */
typedef struct se_server se_server;
typedef uint64_t se_ticket;

/* Device memory a solve of this shape allocates: panels, small dense
 * workspace and, for mixed precision, the FP32 copy of the matrix values. */
uint64_t se_solve_footprint(int64_t n, int64_t nnz, int32_t n_ev, int32_t n_extra, int32_t precision,
                            int32_t solver);

/* 1 <= max_slots <= 16; hbm_budget_bytes > 0. The server uses ctx's device. */
se_status se_server_create(se_ctx* ctx, uint64_t hbm_budget_bytes, int32_t max_slots, se_server** out);

/* Batched server (1 <= max_slots <= 16): one engine thread advances every
 * resident solve by one LOBPCG iteration per step, each phase of the step one
 * launch over the work of all of them (Algorithm 3 with soft locking, the
 * Hetmaniuk-Lehoucq basis of Section 2.3 and the shrink-and-expand controller
 * of Section 3). Sizes that change inside a step (dropped columns, the rank
 * of the HL block) are planned on the device, so a step is a fixed sequence
 * of launches: issued directly, or (environment SE_BATCH_GRAPH=1 at creation)
 * replayed from a graph built once per server. The slots form two lanes on
 * two streams, so one lane's small dense phase overlaps the other's products
 * over n. New requests join at step boundaries; one host synchronization per
 * step serves every solve.
 * Takes FP64 LOBPCG requests with nb <= 96, no preconditioner, X_drop
 * expansion and a matrix without rows of more than 64 nonzeros; se_submit
 * returns SE_ERR_UNSUPPORTED for others. Admission by se_batched_footprint
 * against hbm_budget_bytes. A solve's arithmetic depends only on its own
 * inputs (its work split and reduction order are fixed by its own size), so it
 * is bitwise the same alone and in any mix. It follows the reference
 * algorithm's steps directly (the residual block projected twice against
 * [X, P], two Cholesky-QR passes, Rayleigh-Ritz on [X, P, W]) rather than
 * se_solve's implicit variants, so its iterates match se_solve's to rounding,
 * not bitwise. se_submit, se_poll, se_wait and se_server_destroy work on both
 * kinds of server. */
se_status se_server_create_batched(se_ctx* ctx, uint64_t hbm_budget_bytes, int32_t max_slots, se_server** out);
/* Device memory a batched solve of this shape holds. */
uint64_t se_batched_footprint(int64_t n, int32_t n_ev, int32_t n_extra);
/* Steps run so far by a batched server's engine, and how many of them were
 * replays of the captured graph (the rest ran as direct launches, after a
 * capture failed). Either pointer may be NULL. SE_ERR_INVALID_ARG for a
 * server not made by se_server_create_batched. */
se_status se_server_batch_stats(se_server* srv, int64_t* steps, int64_t* graph_steps);

/* Queue one solve; never blocks on the GPU. X0 may be NULL (seeded start
 * block, as in se_solve). Returns SE_ERR_INVALID_ARG like se_solve,
 * SE_ERR_REJECTED when its footprint alone exceeds the budget. */
se_status se_submit(se_server* srv, const se_matrix* A, const se_params* params, const double* X0,
                    double* V, double* lambda, se_ticket* ticket);

/* *done = 1 once the request has finished. */
se_status se_poll(se_server* srv, se_ticket ticket, int32_t* done);

/* Block until the request finishes; fills info (may be NULL) with its
 * se_info, queue_ms (submit to start) and run_ms (start to end, host clock;
 * either may be NULL) and returns the solve's status. The ticket is
 * released. */
se_status se_wait(se_server* srv, se_ticket ticket, se_info* info, double* queue_ms, double* run_ms);

/* Finish the running solves, fail the queued ones with SE_ERR_REJECTED (their
 * tickets stay waitable until destroy), release every slot. NULL is ignored. */
void se_server_destroy(se_server* srv);

/* Static description of a status code. */
const char* se_status_string(se_status s);

#ifdef __cplusplus
}
#endif

#endif /* SE_H */
