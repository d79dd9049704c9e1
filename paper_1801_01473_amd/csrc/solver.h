// Device-side state of the CG / multi-shift CG solver.
#pragma once

#include "common.h"

namespace lqcd {

constexpr int kMaxShift = 32;
constexpr int kScalarThreads = 1024;  // one workgroup runs every scalar recurrence

// Deferred shift updates: within a window of at most kMaxWin iterations a
// shifted x_s and p_s are combinations of p_s at the window start (index 0)
// and of the base residuals after each iteration of the window (1..wpos).
constexpr int kMaxWin = 31;
constexpr int kWinRow = kMaxWin + 1;  // coefficients per shift and vector
static_assert(kMaxShift * kWinRow == kScalarThreads, "one thread per window coefficient");

// Window coefficients of one system: x_s += sum_q cx[s][q] v_q, p_s = sum_q cp[s][q] v_q.
struct WinCoef {
  double cx[kMaxShift][kWinRow];
  double cp[kMaxShift][kWinRow];
};

// Scalars of one system (one right-hand side of the main solve, or one
// refined (right-hand side, shift) pair).  All FP64.
struct alignas(16) SysState {
  double rho;      // |r|^2 of the current (iterated or recomputed) residual
  double pp;       // |p|^2 of the base search direction
  double a;        // CG step of the base system
  double a_old, b_old;
  double bnorm2;   // |b|^2
  double target2;  // (tol |b|)^2
  double m2s;      // base diagonal m^2 + sigma_0
  double r2ref;    // |r|^2 at the last reliable update (or start)
  double rho_iter; // iterated |r|^2 just before the last reliable update
  int iters;       // Krylov iterations done
  int done;        // stopped (converged or out of iterations)
  int live;        // = !done, read by the D_oe kernel
  int upd_any;     // this iteration's update is to be applied
  int rel;         // takes part in the current reliable update
  int nrel;        // reliable updates done
  int conv;        // converged on the FP64 recomputed residual
  int err;         // non-finite or non-positive curvature seen
  int restart;     // directions are rebuilt from the recomputed residual
  int lowres;      // residual below the FP64 -> FP32 switch level
  int iters64;     // iterations run in FP64 arithmetic
  int wpos;        // iterations in the current window of deferred shift updates
  long long upd64, upd32;  // shift updates applied (sum over iterations of updated shifts)
  long long fsh64, fsh32;  // shifts materialised by window flushes
  long long fsl64, fsl32;  // residuals combined by window flushes
  double zeta[kMaxShift], zeta_old[kMaxShift], zeta_new[kMaxShift];
  double a_s[kMaxShift], b_s[kMaxShift], delta[kMaxShift];
  int active[kMaxShift];  // shift still iterating
  int upd[kMaxShift];     // shift updated in this iteration
  int dirty[kMaxShift];   // low-precision solution changed since the last reliable update
  int wdirty[kMaxShift];  // updated in the current window
};

static_assert(sizeof(SysState) % 8 == 0, "state stride must be a whole number of doubles");

struct alignas(16) GlobalFlags {
  int all_done;
  int error;
  int rel_req;     // some system's residual fell by the reliable-update factor
  int phase_done;  // every system is below the switch level or done
};

constexpr int kStateStrideD = int(sizeof(SysState) / sizeof(double));
constexpr int kStateStrideI = int(sizeof(SysState) / sizeof(int));

}  // namespace lqcd
