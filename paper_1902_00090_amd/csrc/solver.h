// Internal structures of the batched data-driven GMRES solver.
#pragma once

#include "op.h"

#define DD_MAX_K 64
#define DD_MAX_M 256
// reduced values per (problem, launch): 2 reals per coefficient + slack
#define DD_NV_MAX (2 * (DD_MAX_K + DD_MAX_M + 1) + 32)

// Per-problem descriptor (device copy).  Vector storage of one problem:
//   basis: [kmax + max(m+1, kmax)] slots of Dp elements in the inner
//          precision.  C occupies the kmax-k .. kmax-1 slots (right-aligned),
//          the Krylov vectors Q_0, Q_1, ... follow from slot kmax, so that the
//          Gram-Schmidt basis [C, Q_0..Q_j] is one contiguous run of slots.
//   V:     [kmax] slots, V_v = the caller's v-th augmenting vector (padded).
//   r:     FP64 residual scratch.
struct ProbDesc {
  int nx, ny, D, Dp;
  int blk0, nblk;   // chunk range of this problem in every field sweep
  int k, _pad;      // number of augmenting columns (incl. dropped ones)
  double omega2;
  const float* eps32;
  const double* eps64;
  const float2* cf32;
  const double2* cf64;
  void* basis;
  void* V;
  double2* r;
  const double2* b;  // caller's right-hand side [D]
  double2* x;        // caller's solution [D]
  // diagonal preconditioner A' = P_L A P_R (NULL when absent), [Dp] each:
  // inner-precision copies for the Arnoldi sweeps, FP64 for the residual and x
  const void* pl;
  const void* pr;
  const double2* pl64;
  const double2* pr64;
  // fused Arnoldi sweep: this problem's tiles [t0, t0 + nt) of the tile list,
  // and two [Dp] inner-precision buffers for A q~ (the current and the next)
  int t0, nt;
  void* Z;
};

// One tile of the fused sweep: the columns [x0, x0 + DD_FUSED_SW) (clipped to
// nx) of rows [y0, y1) of problem p, walked downwards (dir = 1); its dots go
// to partial row `row` (tiles of a problem have consecutive rows).  p < 0 is
// a padding tile.
struct FusedTile {
  int p, x0, y0, y1, dir, row;
};

// Integer state per problem
enum { ST_ACTIVE = 0, ST_J, ST_ITERS, ST_CYCLES, ST_DONE, ST_PENDING, ST_NCOMB, ST_FLAGS, ST_REORTH,
       ST_NREORTH, ST_NI };
// ST_DONE values
enum { DONE_RUNNING = 0, DONE_CONVERGED = 1, DONE_BUDGET = 2, DONE_NONFINITE = 3 };
// ST_FLAGS bits
enum { FLAG_ZERO_B = 1 };
// FP64 state per problem
// SD_NSUM / SD_NSUM2: sums over Arnoldi steps of the basis length n = k + j + 1
// (all steps / steps with a second pass), for the algorithmic byte counts.
// SD_PRHO / SD_PBNORM: ||P_L r|| and ||P_L b|| (= SD_RHO, SD_BNORM without a
// left preconditioner), the norms of the preconditioned cycle.
enum { SD_BNORM = 0, SD_RHO, SD_BETA, SD_TRUE, SD_EST, SD_NSUM, SD_NSUM2, SD_PRHO, SD_PBNORM,
       SD_ND = 10 };

enum { MODE_START = 0, MODE_ARNOLDI = 1 };

struct PlanDev {
  const ProbDesc* desc;
  const int* blk2prob;
  int* stI;          // [nb][ST_NI]
  double* stD;       // [nb][SD_ND]
  double2* H;        // [nb][m][m+1] rotated Hessenberg (column-major)
  double2* Hraw;     // [nb][m][m+1] as built
  double2* Bc;       // [nb][m][kmax]  B = C^H A Q
  double2* g;        // [nb][m+1]
  double* cs;        // [nb][m]
  double2* sn;       // [nb][m]
  double2* c0;       // [nb][kmax]
  double2* coefA;    // [nb][NC]
  double2* coefB;    // [nb][NC]
  double2* coefA2;   // [nb][NC] one-sweep steps: raw dots of odd steps (coefA: even)
  double* hscale;    // [nb][m+1]
  double2* comb;     // [nb][kmax + m]
  double2* Rinv;     // [nb][kmax][kmax]
  double2* Tm;       // [nb][kmax][kmax] current CholQR factor L^{-H}
  double2* Gm;       // [nb][kmax][kmax] Gram matrix
  unsigned long long* keep;  // [nb] column mask kept by the last CholQR pass
  unsigned long long* bad;   // [nb] columns with non-finite entries
  void* partial;     // [nchunks][NV] inner-precision partial sums
  double* gpart;     // Gram partials [nb][GB][ntiles][32]
  double* hist;      // [nb][hist_cap]
  int nb, m, kmax, NC, NV, hist_cap, GB, qslots;
  int reorth_mode;   // 0 one Gram-Schmidt pass, 1 always two, 2 two where needed
  const double* ctl;  // device [tol, maxit] of the current solve (kernel arguments
                      // stay constant, so captured graphs remain valid)
  int fused;          // 1: one-sweep Arnoldi steps (k_fused_sweep / k_post_fused)
  const FusedTile* tiles;
};
