// Batched serving engine: device state of the resident solves and the
// macro-step that advances every one of them by one LOBPCG iteration
// (Algorithm 3 with soft locking, the Hetmaniuk-Lehoucq basis of Section 2.3
// and shrink-and-expand, Section 3) with one launch per phase for all of them.
#pragma once

#include "common.h"

namespace se {

constexpr int kBNbMax = 96;            // block width nb of a batched solve
constexpr int kBWMax = 2 * kBNbMax;    // residual block plus expansion columns
constexpr int kBMMax = 3 * kBNbMax;    // order of the Rayleigh-Ritz step
constexpr int kBGridBulk = 2048;       // workgroups of the looping bulk launches

enum { BMODE_IDLE = 0, BMODE_INIT = 1, BMODE_ITER = 2 };

// Per-solve constants, written by the host when the solve is admitted. Every
// panel is row-major n x ldw: [X | P] keeps X in columns 0.. and P from
// column poff, so that X, P and W are segments of one leading dimension.
struct BFix {
    const int* rowptr;
    const int* col;
    const double* val;
    double* xp[2];   // [X | P] (current / next, swapped by the device)
    double* axp[2];  // [AX | AP]
    double* xpd;     // dropped columns [X_drop | P_drop]
    double* w[2];    // residual block W and its orthonormalized copy
    double* aw;      // A W
    double* part;    // Gram partials: nch_g x kBMMax x kBMMax
    double* rpart;   // residual partials: nch_r x 2 kBNbMax
    double* sm;      // small matrices (layout: BSmall)
    double anorm;
    long long rows_g, rows_r;  // rows per chunk of the Gram and residual products
    int n, nb, n_es, ldw, poff, nch_g, nch_r;  // poff: first column of P in [X | P]
};

// Per-step decisions of the host (Section 3.2's controller, soft locking).
struct BCtl {
    int mode;    // BMODE_*
    int a;       // unlocked columns of X (positions act[0..a))
    int expand;  // append the dropped columns this step
    int shrink;  // keep n_es columns of X and P after this step
    int act[kBNbMax];
};

// Device state of a solve. The host sets it at admission and reads it after
// every step; in between only the device writes it.
struct BDyn {
    int cur;                // which of xp/axp and w hold the current blocks
    int wcur;
    int k, p, w, dx, dp;    // widths of X, P, W and of the dropped blocks
    int wa;                 // residual columns at the head of the W block
    int kk, pp, m, cx;      // after the Rayleigh-Ritz step: widths of X and P, its order, kept X_drop columns
    int nhl;                // Hetmaniuk-Lehoucq positions
    int map[kBWMax];        // source column (in the gathered W block) of each kept W column
    int hlpos[kBNbMax];
    double theta[kBMMax];   // Ritz values of the step, ascending
    double lam[kBNbMax];    // Ritz values of the current X
    double sums[2 * kBNbMax];  // per column: ||r||^2 (k), ||x||^2 (k)
    double stop[kBNbMax];   // ||r_i|| / (||A|| ||x_i||)
    double paper[kBNbMax];  // ||r_i|| / (||A|| ||x_i|| + |lambda_i| ||x_i||)
};

// Small matrices of one solve, offsets in doubles from BFix::sm.
struct BSmall {
    static constexpr size_t G = 0;                                        // kBMMax^2: Gram outputs
    static constexpr size_t GW = G + (size_t)kBMMax * kBMMax;             // kBWMax^2: W^T W
    static constexpr size_t T = GW + (size_t)kBWMax * kBWMax;             // kBWMax^2: Cholesky-QR transform
    static constexpr size_t CW = T + (size_t)kBWMax * kBWMax;             // Cholesky work
    static constexpr size_t INFO = CW + 2 * (size_t)kBWMax * kBWMax + 2 * kBWMax;  // ints, then doubles
    static constexpr size_t Z = INFO + kBWMax + 64;                       // kBMMax x kBNbMax
    static constexpr size_t B = Z + (size_t)kBMMax * kBNbMax;             // kBMMax x kBNbMax
    static constexpr size_t B2 = B + (size_t)kBMMax * kBNbMax;
    static constexpr size_t GB = B2 + (size_t)kBMMax * kBNbMax;           // kBNbMax^2
    static constexpr size_t TB = GB + (size_t)kBNbMax * kBNbMax;
    static constexpr size_t C = TB + (size_t)kBNbMax * kBNbMax;           // kBMMax x kBWMax
    static constexpr size_t EIG = C + (size_t)kBMMax * kBWMax;            // syev work
};
size_t bsmall_doubles();

// Device memory of the job lists of one macro-step (all slots).
size_t batch_jobs_bytes();

// The launches of one macro-step for slots 0..ns-1, issued on L's stream or
// added to L's graph (no host synchronization, no allocation). jobs: device memory
// of batch_jobs_bytes(). upd_grid: workgroups of the basis updates, at least
// the sum over the slots of 2 ceil(n / 64) (one work item each).
hipError_t launch_batch_step(Launcher& L, int ns, const BFix* fix, const BCtl* ctl, BDyn* dyn, void* jobs,
                             int upd_grid);

}  // namespace se
