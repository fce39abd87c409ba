"""Pins of the oracle's inner-tolerance controller (Sec. 3.2)."""
import math
import os

import numpy as np
import pytest

from oracle import controller as C

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_norm_bound_constant():
    """Sec. 3.2.1: c = 2 + sqrt(2) (Crouzeix-Palencia constant 1 + sqrt(2) plus 1);
    with kmax = 50 the no-back-looking threshold is eps / 1165.685."""
    assert C.C_BOUND == pytest.approx(3.414213562373095, rel=1e-15)
    assert 2 * C.C_BOUND ** 2 * 50 == pytest.approx(1165.685424949238, rel=1e-14)
    assert C.eps_hat_1(1e-8, 50) == pytest.approx(8.578643762690485e-12, rel=1e-13)


def test_backlooking_equals_plain_at_first_step():
    """u_0 = v_0 = 0 makes eq. (ADI_relax2_prak) equal eq. (ADI_relax1_prak) at
    k = 1; the paper's Ex. 1 data show the same (Fig. 3: identical BL and
    no-BL inner residuals in the first steps; Fig. 4: identical cumulative
    inner iteration counts through step 5)."""
    for eps, kmax, xi in [(1e-8, 50, 1.0), (3e-4, 100, 0.1), (1.0, 7, 0.5)]:
        assert C.eps_hat_2(eps, kmax, 1, 0.0, 0.0, xi) == pytest.approx(
            C.eps_hat_1(eps, kmax, xi), rel=1e-15)


def test_backlooking_budget_grows_and_is_consumed():
    e1 = C.eps_hat_2(1.0, 10, 3, 0.0, 0.0)
    e2 = C.eps_hat_2(1.0, 10, 4, 0.0, 0.0)
    assert e2 > e1
    spent = C.eps_hat_2(1.0, 10, 4, 0.01, 0.005)
    assert spent < e2
    # budget exhausted: clamped to 0 by default, |.| as printed with paper_abs
    big = 10.0
    assert C.eps_hat_2(1.0, 10, 1, big, 0.0) == 0.0
    c = C.C_BOUND
    assert C.eps_hat_2(1.0, 10, 1, big, 0.0, paper_abs=True) == pytest.approx(
        (big - 1.0 / (2 * c * 10)) / c, rel=1e-14)


def _fig1():
    vals = {}
    with open(os.path.join(GOLDEN, "paper_fig1_admissible_region.txt")) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split("=")
                vals[k.strip()] = float(v)
    return vals


def test_fig1_intercepts():
    """Fig. 1 (region of admissible inner residual norms) is drawn with
    c_check = 3, eps_check = 1e-8, ||t|| = 1e-5, ||w|| = 2e-3; its axis ticks are
    eps_check/(c_check ||t||) and eps_check/(c_check ||w||).  With the
    threshold eh = eps_check / c_check and no clamping, the one-sided
    selections reach exactly these intercepts of the curve Psi = 0."""
    g = _fig1()
    eh = g["eps_check"] / g["c_check"]
    dA, dB = C.select_tightA(eh, g["norm_w"], g["norm_t"], 0.0, 1.0)
    assert dA == 0.0
    assert dB == pytest.approx(g["eps_check"] / (g["c_check"] * g["norm_w"]), rel=1e-14)
    assert dB == pytest.approx(1.6666666666666667e-06, rel=1e-12)
    dA, dB = C.select_tightB(eh, g["norm_w"], g["norm_t"], 0.0, 1.0)
    assert dB == 0.0
    assert dA == pytest.approx(g["eps_check"] / (g["c_check"] * g["norm_t"]), rel=1e-14)
    assert dA == pytest.approx(3.3333333333333335e-04, rel=1e-12)


def test_fig1_mid_selection_first_line():
    """The first line of eq. (simple_tols) on Fig. 1's data: with delta_min = 0
    and no delta_max cap, delta^A is half the delta^A-axis intercept of the
    admissible region, eps_check/(c_check ||t||)/2 = 1.6667e-4, a value the
    caption's numbers fix.  ||t|| and ||w|| differ by a factor of 200 there,
    so a delta^A built from ||w|| instead (8.33e-7) or the midpoint with
    +delta_min read the wrong way round cannot pass.  delta^B then lies on the
    boundary Psi = 0, i.e. eq. (tolBfromtolA) evaluated at that delta^A."""
    g = _fig1()
    eh = g["eps_check"] / g["c_check"]
    nw, nt = g["norm_w"], g["norm_t"]
    dA, dB = C.select_mid(eh, nw, nt, 0.0, math.inf)
    assert dA == pytest.approx(1.6666666666666666e-04, rel=1e-12)
    assert dA == pytest.approx(0.5 * g["eps_check"] / (g["c_check"] * nt), rel=1e-14)
    assert abs(dA - 0.5 * g["eps_check"] / (g["c_check"] * nw)) > 1e-4
    # eq. (tolBfromtolA) with the caption's numbers: (eps - c dA ||t||) / (c (2 dA + ||w||))
    want_dB = (g["eps_check"] - g["c_check"] * dA * nt) / (g["c_check"] * (2 * dA + nw))
    assert dB == pytest.approx(want_dB, rel=1e-13)
    assert dB == pytest.approx(7.142857142857143e-07, rel=1e-12)
    # the pair is on the curve Psi = 0 of eq. (relax_AB) in the caption's form
    psi = g["c_check"] * (dA * (nt + dB) + dB * (nw + dA))
    assert psi == pytest.approx(g["eps_check"], rel=1e-13)
    # a positive delta_min lowers delta^A by half of it (eq. (simple_tols))
    dA2, _ = C.select_mid(eh, nw, nt, 1e-5, math.inf)
    assert dA2 == pytest.approx(dA - 0.5e-5, rel=1e-13)


@pytest.mark.parametrize("seed", range(20))
def test_mid_selection_lies_on_boundary_curve(seed):
    """eq. (simple_tols) picks delta^A inside the box of eq. (relax_AB) and
    delta^B from eq. (tolBfromtolA), so unless a clamp of eq. (bound_tols) is
    active the pair satisfies eq. (ADI_relax1_prak) with equality."""
    rng = np.random.default_rng(seed)
    nw, nt = 10 ** rng.uniform(-4, 3, 2)
    eh = 10 ** rng.uniform(-14, -6)
    dmin, dmax = 1e-16, 1e3
    dA, dB = C.select_mid(eh, nw, nt, dmin, dmax)
    assert dmin <= dA <= dmax and dmin <= dB <= dmax
    assert dA == pytest.approx(0.5 * (eh / nt - dmin), rel=1e-12)
    assert C.gap_lhs(dA, dB, nw, nt) == pytest.approx(eh, rel=1e-12)
    for sel in (C.select_tightA, C.select_tightB):
        a, b = sel(eh, nw, nt, dmin, dmax)
        assert C.gap_lhs(a, b, nw, nt) == pytest.approx(eh, rel=1e-9)


def test_mid_selection_clamps():
    """eq. (bound_tols): tolerances never leave [delta_min, delta_max]."""
    dA, dB = C.select_mid(1e-30, 1.0, 1.0, 5e-10, 0.1)
    assert dA == 5e-10 and dB == 5e-10
    dA, dB = C.select_mid(1e3, 1e-6, 1e-6, 5e-10, 0.1)
    assert dA == pytest.approx(0.5 * (0.1 - 5e-10)) and dB == 0.1


def test_paper_experiment_settings():
    """Sec. 4 settings: delta_min = eps/20, delta_max = 0.1, kmax = 50, xi = 1
    (Ex. 4: eps/100, 100, 0.1); the fixed-tolerance runs use eps/20."""
    dA, dB = C.tolerances("fixed", 3, 1.0, 1.0, 0.0, 0.0, eps=1.0, fixed=1e-8 / 20)
    assert dA == dB == 5e-10
    dA, dB = C.tolerances("relative", 1, 4.0, 2.0, 0.0, 0.0, eps=1.0, rho=1e-12)
    assert dA == 4e-12 and dB == 2e-12


def test_gap_update_recurrence():
    """eq. (upd_resgap): u += |gamma| ||z|| ||r^B||, v += |gamma| ||y|| ||r^A||."""
    u, v = 0.0, 0.0
    steps = [(-3.0, 2.0, 5.0, 1e-3, 2e-3), (7.0, 0.5, 0.25, 4e-4, 1e-4)]
    for gam, nz, ny, rA, rB in steps:
        u, v = C.update_gap(u, v, gam, nz, ny, rA, rB)
    assert u == pytest.approx(3 * 2 * 2e-3 + 7 * 0.5 * 1e-4)
    assert v == pytest.approx(3 * 5 * 1e-3 + 7 * 0.25 * 4e-4)


# --- balanced frame (an extension: the selection evaluated for (s w, t / s)) ---

@pytest.mark.parametrize("sel", ["mid", "tightA", "tightB"])
def test_balance_is_identity_for_equal_norms(sel):
    for nw in (1e-3, 1.0, 37.0):
        a = C.tolerances(sel, 4, nw, nw, 1e-12, 2e-12, eps=1e-6)
        b = C.tolerances(sel, 4, nw, nw, 1e-12, 2e-12, eps=1e-6, balance=True)
        assert a == pytest.approx(b, rel=1e-15)


@pytest.mark.parametrize("sel", ["mid", "tightA", "tightB"])
def test_balance_is_scale_covariant(sel):
    # w -> c w, t -> t / c leaves w t^T unchanged; the balanced tolerances
    # must follow as (c delta^A, delta^B / c)
    nw, nt = 3.0e2, 4.0e-3
    dA, dB = C.tolerances(sel, 7, nw, nt, 1e-11, 3e-11, eps=1e-5, balance=True)
    for c in (1e-4, 0.5, 3.0, 1e5):
        eA, eB = C.tolerances(sel, 7, nw * c, nt / c, 1e-11, 3e-11, eps=1e-5, balance=True)
        assert eA == pytest.approx(dA * c, rel=1e-13)
        assert eB == pytest.approx(dB / c, rel=1e-13)


def test_balance_mid_lies_on_the_boundary_curve():
    # unclamped "mid" picks delta^B on the boundary of eq. (ADI_relax2_prak);
    # the left-hand side is invariant under the rescaling, so it equals
    # eps_hat in the original frame too
    nw, nt, k, eps, u, v = 2.6e4, 5.9e-4, 6, 2.7e-5, 1e-9, 2e-9
    eh = C.eps_hat_2(eps, 50, k, u, v, 1.0, False)
    dA, dB = C.tolerances("mid", k, nw, nt, u, v, eps, dmin=1e-16, balance=True)
    assert C.gap_lhs(dA, dB, nw, nt) == pytest.approx(eh, rel=1e-12)


def test_balance_keeps_unbalanced_factors_admissible():
    # ||w|| >> ||t||: in the original frame delta^B falls below delta_min and
    # the clamp breaks the budget; in the balanced frame the same delta_min
    # is admissible
    nw, nt, k, eps, dmin = 2.6e4, 5.9e-4, 6, 2.7e-5, 5e-10
    eh = C.eps_hat_2(eps, 50, k, 0.0, 0.0, 1.0, False)
    dA, dB = C.tolerances("mid", k, nw, nt, 0.0, 0.0, eps, dmin=dmin)
    assert dB == dmin and C.gap_lhs(dA, dB, nw, nt) > 10 * eh
    dA, dB = C.tolerances("mid", k, nw, nt, 0.0, 0.0, eps, dmin=dmin, balance=True)
    assert C.gap_lhs(dA, dB, nw, nt) <= eh * (1 + 1e-12)


@pytest.mark.parametrize("seed", range(6))
def test_sym_selection_is_largest_equal_pair(seed):
    """The symmetric selection lies on the boundary of the admissibility
    condition (left-hand side == eps_hat), and bisection on that left-hand
    side over equal pairs finds the same delta (brute force, independent of
    the closed-form root)."""
    rng = np.random.default_rng(seed)
    nw, nt = 10 ** rng.uniform(-4, 1), 10 ** rng.uniform(-4, 1)
    eh = 10 ** rng.uniform(-14, -9)
    d, d2 = C.select_sym(eh, nw, nt, 1e-300, 1e300)
    assert d == d2
    assert C.gap_lhs(d, d, nw, nt) == pytest.approx(eh, rel=1e-12)
    lo, hi = 0.0, eh / (nw + nt) * 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if C.gap_lhs(mid, mid, nw, nt) <= eh:
            lo = mid
        else:
            hi = mid
    assert d == pytest.approx(lo, rel=1e-12)


def test_sym_selection_clamps_and_dispatch():
    assert C.select_sym(1e6, 1e-3, 1e-3, 5e-10, 0.1) == (0.1, 0.1)
    assert C.select_sym(0.0, 1.0, 1.0, 5e-10, 0.1) == (5e-10, 5e-10)
    eh = C.eps_hat_2(1e-8, 50, 3, 1e-12, 2e-12)
    dA, dB = C.tolerances("sym", 3, 0.02, 0.5, 1e-12, 2e-12, 1e-8)
    assert (dA, dB) == C.select_sym(eh, 0.02, 0.5, 5e-10, 0.1)
    # with ||w|| = ||t|| the balanced frame changes nothing
    assert C.tolerances("sym", 3, 0.3, 0.3, 0.0, 0.0, 1e-8, balance=True) == \
        C.tolerances("sym", 3, 0.3, 0.3, 0.0, 0.0, 1e-8)
