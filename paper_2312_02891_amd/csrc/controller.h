// Dynamic inner-solve tolerances of the inexact LR-ADI iteration
// (Sec. 3.2): eqs. (ADI_relax1_prak), (ADI_relax2_prak), (bound_tols),
// (simple_tols), (one_side), the equal pair on the boundary of the first
// two, and the gap recursion (upd_resgap).
// __host__ __device__ so that the host self-test runs the same code.
#pragma once

#include <cmath>

#include "../../include/lradi.h"
#include "small.h"

namespace lradi {

struct CtlParams {
  double eps;        // absolute residual-gap budget
  double delta_min, delta_max, xi, delta_fixed, rho;
  int kmax, selection, backlook, paper_abs;
  int balance;  // evaluate the dynamic selections in the balanced frame
};

// c = 2 + sqrt(2): bound on max(||C_k(A)||, ||C_k(B)||) + 1 from the
// Crouzeix-Palencia estimate (Sec. 3.2.1).
LRADI_HD inline double ctl_c() { return 2.0 + sqrt(2.0); }

// eps_hat_k of eq. (ADI_relax1_prak) (backlook = 0) or eq. (ADI_relax2_prak)
// (backlook = 1); k is the 1-based outer step, u, v = u_{k-1}, v_{k-1}.
LRADI_HD inline double ctl_eps_hat(const CtlParams& p, int k, double u, double v) {
  const double c = ctl_c();
  if (!p.backlook) return p.xi * p.eps / (2.0 * c * c * (double)p.kmax);
  double x = p.xi * (double)k * p.eps / (2.0 * c * (double)p.kmax) - u - v;
  x = p.paper_abs ? fabs(x) : fmax(x, 0.0);
  return x / c;
}

// (delta^A_k, delta^B_k) from ||w_{k-1}||, ||t_{k-1}||, u_{k-1}, v_{k-1}.
LRADI_HD inline void ctl_tolerances(const CtlParams& p, int k, double nw, double nt, double u,
                                    double v, double* dA, double* dB) {
  if (p.selection == LRADI_SEL_RELATIVE) {
    *dA = p.rho * nw;
    *dB = p.rho * nt;
    return;
  }
  if (p.selection == LRADI_SEL_FIXED) {
    *dA = p.delta_fixed;
    *dB = p.delta_fixed;
    return;
  }
  const double eh = ctl_eps_hat(p, k, u, v);
  const double lo = p.delta_min, hi = p.delta_max;
  // Balanced frame: (s w, t / s) with s = sqrt(||t|| / ||w||) has equal
  // factor norms and the same w t^T; the left-hand side of the admissibility
  // condition is invariant, so a selection made there and mapped back
  // (delta^A / s, delta^B s) stays admissible, with the clamps of
  // eq. (bound_tols) acting on the balanced pair.
  double s = 1.0;
  if (p.balance && nw > 0.0 && nt > 0.0) {
    s = sqrt(nt / nw);
    nw = nt = sqrt(nw * nt);
  }
  double a, b;
  if (p.selection == LRADI_SEL_TIGHT_A) {
    a = lo;
    b = fmax(fmin((eh - a * nt) / (2.0 * a + nw), hi), lo);
  } else if (p.selection == LRADI_SEL_TIGHT_B) {
    b = lo;
    a = fmax(fmin((eh - b * nw) / (2.0 * b + nt), hi), lo);
  } else if (p.selection == LRADI_SEL_SYM) {
    // a = b on the boundary: 2 a^2 + a (||w|| + ||t||) = eh, positive root
    const double sw = nw + nt;
    a = fmax(fmin((-sw + sqrt(sw * sw + 8.0 * eh)) / 4.0, hi), lo);
    b = a;
  } else {  // LRADI_SEL_MID: eq. (simple_tols) as printed
    a = fmax(0.5 * (fmin(hi, eh / nt) - lo), lo);
    b = fmax(fmin((eh - a * nt) / (2.0 * a + nw), hi), lo);
  }
  *dA = a / s;
  *dB = b * s;
}

// eq. (upd_resgap) with M = C = I.
LRADI_HD inline void ctl_update_gap(double* u, double* v, double gamma, double nz, double ny,
                                    double rA, double rB) {
  *u += fabs(gamma) * nz * rB;
  *v += fabs(gamma) * ny * rA;
}

}  // namespace lradi
