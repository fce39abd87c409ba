// Outer LR-ADI state shared by the ADI kernels and the host driver.
#pragma once

#include "internal.h"

namespace lradi {

// Read-only description of one Sylvester problem in a batch (problem p owns
// inner systems 2p: A side and 2p+1: B side).
struct AdiDesc {
  int n, m, r, kmax, nshifts;
  int selection, backlook, paper_abs, rescale;  // rescale 2: controller in the balanced frame
  int setup;              // 1: the setup kernels initialise this problem
  int sym;                // Lyapunov case B = A^T, C = M^T, g = f, equal shifts:
                          // system 2p+1 is an idle mirror (no workgroups), the
                          // A side's solve serves both sides, T = W, Yf = Zf
  double tol, eps_in, delta_min, delta_max, xi, delta_fixed, rho;
  const double* shiftsA;  // device, nshifts
  const double* shiftsB;  // device, nshifts
  // complex shifts (Sec. 3.2.4's complex form of the iteration): imaginary
  // parts (device, nshifts); W, T, Zf, Yf then hold stacked blocks
  // [re; im] of 2n (2m) rows and gam two doubles (re, im) per step
  int cplx;
  const double* shiftsA_im;
  const double* shiftsB_im;
  const double* f;        // device, n x r
  const double* g;        // device, m x r
  double* W;              // residual factor w_k, n x r
  double* T;              // residual factor t_k, m x r
  double* Zf;             // factor blocks z_1..z_kmax, kmax x n x r
  double* Yf;             // factor blocks y_1..y_kmax, kmax x m x r
  double* gam;            // gamma_1..gamma_kmax
  double* hist;           // kmax x LRADI_HIST_COLS
  int* host_done;         // host-visible flag set to 1 when the problem finishes
};

// Mutable outer state of one problem.
struct AdiCtl {
  int k;        // completed steps
  int done;     // 1 once converged, out of steps or failed
  int status;   // LRADI_OK / LRADI_WNOCONV / LRADI_ENAN
  int winner;   // some inner solve hit its step cap
  double norm_fg, eps, nw, nt, u, v, res, sf, sg, dA, dB;
};

// Setup of the problems flagged `setup`: rescaling, norms, W = sf f,
// T = sg g, and arming of step 1.
int adi_launch_setup(hipStream_t st, const Batch& b, const AdiDesc* ad, AdiCtl* ac, int nprob);
// End of an outer step for every problem whose two inner solves have both
// finished: residual-factor update, norms, stop test, arming of the next
// step.  Issued after every tick, so problems advance independently.
int adi_launch_step_end(hipStream_t st, const Batch& b, const AdiDesc* ad, AdiCtl* ac, int nprob);

}  // namespace lradi
