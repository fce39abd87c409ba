"""Oracle (test infrastructure only): the dynamic inner-solve tolerances of
Sec. 3.2 for the inexact LR-ADI iteration (Algorithm 1).

Quantities at outer step k (1-based), all in FP64:
  nw = ||w_{k-1}||, nt = ||t_{k-1}||   spectral norms of the residual factors
  u, v = u_{k-1}, v_{k-1}               residual-gap estimates, eq. (upd_resgap)
  eps                                   absolute residual-gap budget
  kmax, xi                              step budget and safeguard constant

Selections (which point of the admissible region, Sec. 3.2.3):
  "relative": delta^A = rho*nw, delta^B = rho*nt (an exact-tolerance
              baseline, not from the paper)
  "fixed":    delta^A = delta^B = const (the "fixed" rows of Table 2)
  "mid":      eq. (simple_tols)
  "tightA":   eq. (one_side): delta^A = delta_min, delta^B as in (simple_tols)
  "tightB":   the mirrored rule stated after eq. (one_side): delta^B =
              delta_min and the largest admissible delta^A
The "B" rows of Table 2 spend more inner iterations on the B systems, which
is "tightB" here.

Only tests/, the smoke check and the bench's CPU baseline use this module.
"""
from __future__ import annotations

import math

# bound on the constant c_k of Theorem 3 obtained from the Crouzeix-Palencia
# estimate of ||C_k|| (Sec. 3.2.1)
C_BOUND = 2.0 + math.sqrt(2.0)


def eps_hat_1(eps: float, kmax: int, xi: float = 1.0) -> float:
    """Right-hand side of eq. (ADI_relax1_prak): xi * eps / (2 c^2 kmax)."""
    c = C_BOUND
    return xi * eps / (2.0 * c * c * kmax)


def eps_hat_2(eps: float, kmax: int, k: int, u: float, v: float, xi: float = 1.0,
              paper_abs: bool = False) -> float:
    """Right-hand side of eq. (ADI_relax2_prak) (back-looking):
    (1/c) * | xi k eps / (2 c kmax) - u_{k-1} - v_{k-1} |.

    The paper takes the absolute value; with paper_abs=False a negative
    bracket (gap budget already spent) gives 0 instead, so the caller falls
    back to delta_min."""
    c = C_BOUND
    x = xi * k * eps / (2.0 * c * kmax) - u - v
    if paper_abs:
        x = abs(x)
    else:
        x = max(x, 0.0)
    return x / c


def select_mid(eh: float, nw: float, nt: float, dmin: float, dmax: float):
    """eq. (simple_tols), taken literally:
    delta^A = max( (min(dmax, eh/nt) - dmin)/2 , dmin )
    delta^B = max( min( (eh - delta^A nt) / (2 delta^A + nw), dmax ), dmin )."""
    dA = max(0.5 * (min(dmax, eh / nt) - dmin), dmin)
    dB = max(min((eh - dA * nt) / (2.0 * dA + nw), dmax), dmin)
    return dA, dB


def select_tightA(eh: float, nw: float, nt: float, dmin: float, dmax: float):
    """eq. (one_side): delta^A = delta_min, delta^B from the second line of
    eq. (simple_tols) with that delta^A."""
    dA = dmin
    dB = max(min((eh - dA * nt) / (2.0 * dA + nw), dmax), dmin)
    return dA, dB


def select_tightB(eh: float, nw: float, nt: float, dmin: float, dmax: float):
    """Mirror of eq. (one_side): delta^B = delta_min and the largest admissible
    delta^A, i.e. eq. (tolBfromtolA) solved for ||r^A|| with the roles of
    (A, w) and (B, t) exchanged, then clamped as in eq. (bound_tols)."""
    dB = dmin
    dA = max(min((eh - dB * nw) / (2.0 * dB + nt), dmax), dmin)
    return dA, dB


def select_sym(eh: float, nw: float, nt: float, dmin: float, dmax: float):
    """Equal tolerances delta^A = delta^B = delta, the largest equal pair on
    the boundary of the condition of eq. (ADI_relax1_prak)/(ADI_relax2_prak):
    delta (||t|| + ||w||) + 2 delta^2 = eh, the positive root of that
    quadratic, clamped as in eq. (bound_tols).  A single inner solve that
    serves both sides (the Lyapunov case B = A^T, g = f of the related
    equations of Sec. 3.2.4) needs exactly such a pair."""
    s = nw + nt
    d = (-s + math.sqrt(s * s + 8.0 * eh)) / 4.0
    d = max(min(d, dmax), dmin)
    return d, d


def tolerances(selection: str, k: int, nw: float, nt: float, u: float, v: float,
               eps: float, kmax: int = 50, xi: float = 1.0, dmin: float = 5e-10,
               dmax: float = 0.1, backlook: bool = True, fixed: float = 5e-10,
               rho: float = 1e-12, paper_abs: bool = False, balance: bool = False):
    """(delta^A_k, delta^B_k) for outer step k.

    balance (an extension; the paper balances only f and g, Sec. 4): the
    dynamic selections are evaluated for the pair (s w, t / s) with
    s = sqrt(||t|| / ||w||), i.e. both factors at the norm sqrt(||w|| ||t||),
    and mapped back (delta^A / s, delta^B s).  The product w t^T, every ADI
    iterate and the left-hand side of eqs. (ADI_relax1_prak)/(ADI_relax2_prak)
    do not change under that rescaling, so admissibility carries over; only
    the clamps of eq. (bound_tols) and the split of eq. (simple_tols) now act
    in the balanced frame."""
    if selection == "relative":
        return rho * nw, rho * nt
    if selection == "fixed":
        return fixed, fixed
    if backlook:
        eh = eps_hat_2(eps, kmax, k, u, v, xi, paper_abs)
    else:
        eh = eps_hat_1(eps, kmax, xi)
    s = 1.0
    if balance and nw > 0.0 and nt > 0.0:
        s = math.sqrt(nt / nw)
        nw = nt = math.sqrt(nw * nt)
    if selection == "mid":
        dA, dB = select_mid(eh, nw, nt, dmin, dmax)
    elif selection == "tightA":
        dA, dB = select_tightA(eh, nw, nt, dmin, dmax)
    elif selection == "tightB":
        dA, dB = select_tightB(eh, nw, nt, dmin, dmax)
    elif selection == "sym":
        dA, dB = select_sym(eh, nw, nt, dmin, dmax)
    else:
        raise ValueError(selection)
    return dA / s, dB * s


def update_gap(u: float, v: float, gamma: float, nz: float, ny: float,
               rA: float, rB: float):
    """eq. (upd_resgap) with M = C = I:
    u_k = u_{k-1} + |gamma_k| ||z_k|| ||r^B_k||,
    v_k = v_{k-1} + |gamma_k| ||y_k|| ||r^A_k||."""
    return u + abs(gamma) * nz * rB, v + abs(gamma) * ny * rA


def gap_lhs(rA: float, rB: float, nw: float, nt: float) -> float:
    """Left-hand side of eqs. (ADI_relax1_prak)/(ADI_relax2_prak):
    ||r^A|| ||t|| + ||r^B|| ||w|| + 2 ||r^A|| ||r^B||."""
    return rA * nt + rB * nw + 2.0 * rA * rB
