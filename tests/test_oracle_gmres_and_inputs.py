"""Pins of the oracle's block minimal-residual iterate and of the shared
input generators."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle.convdiff import convdiff_matrix
from oracle.gmres_ref import block_gmres_iterate, block_krylov_basis
from paper_2312_02891_amd import workloads as WL


def test_full_space_gives_exact_solve():
    """When K_j(S, W) is the whole space the minimiser is S^{-1} W."""
    A = convdiff_matrix(2, 4, (3, -2))          # n = 16
    rng = np.random.default_rng(0)
    W = rng.standard_normal((16, 2))
    Z = block_gmres_iterate(A, -5.0, W, 8)      # 8 blocks of 2 = 16 vectors
    S = (A - 5.0 * sp.identity(16)).toarray()
    assert np.allclose(Z, np.linalg.solve(S, W), rtol=1e-9, atol=1e-12)


def test_r1_small_space_matches_scipy_gmres_without_restart():
    """For one right-hand side, block GMRES is textbook GMRES: compare the
    j-step iterate with SciPy's GMRES run for j steps (no restart)."""
    A = convdiff_matrix(2, 10, (5, 2))
    rng = np.random.default_rng(1)
    w = rng.standard_normal((100, 1))
    S = (A - 30.0 * sp.identity(100)).tocsr()
    for j in (3, 7):
        Z = block_gmres_iterate(A, -30.0, w, j)
        x, _ = spla.gmres(S, w[:, 0], rtol=1e-300, atol=0.0, restart=j, maxiter=1)
        assert np.allclose(Z[:, 0], x, rtol=1e-8, atol=1e-10 * np.abs(x).max())


def test_optimality_and_monotone_residual():
    """The residual is orthogonal to S K_j and never grows with j."""
    A = convdiff_matrix(3, 5, (2, -1, 3))
    rng = np.random.default_rng(2)
    W = rng.standard_normal((125, 3))
    S = (A - 100.0 * sp.identity(125)).tocsr()
    prev = np.inf
    for j in range(1, 6):
        Z = block_gmres_iterate(A, -100.0, W, j)
        R = W - S @ Z
        V = block_krylov_basis(S, W, j)
        assert np.abs((S @ V).T @ R).max() <= 1e-9 * np.abs(W).max() * np.linalg.norm(S.toarray(), 2)
        nr = np.linalg.norm(R)
        assert nr <= prev * (1 + 1e-12)
        prev = nr


def test_rhs_factors_are_seeded_standard_normal():
    f, g = WL.rhs_factors(1, 400, 300, 2)
    f2, g2 = WL.rhs_factors(1, 400, 300, 2)
    assert f.shape == (400, 2) and g.shape == (300, 2)
    assert np.array_equal(f, f2) and np.array_equal(g, g2)
    rng = np.random.default_rng(1)
    assert np.array_equal(f, rng.standard_normal((400, 2)))
    assert abs(f.mean()) < 0.2 and abs(f.std() - 1) < 0.1


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_shifts_in_the_right_intervals(name):
    """pA (added to A) lies in B's interval and pB (added to B^T) in A's: the
    zeros of each Cayley factor sit over its own spectrum (eq. (adi_shift))."""
    P = WL.CONFIGS[name]
    pA, pB = WL.wachspress_shifts(P.A, P.B, P.nshifts)
    la, ha = WL.numerical_range_interval(P.A)
    lb, hb = WL.numerical_range_interval(P.B)
    assert len(pA) == len(pB) == P.nshifts
    assert np.all((-pA >= lb * (1 - 1e-9)) & (-pA <= hb * (1 + 1e-9)))
    assert np.all((-pB >= la * (1 - 1e-9)) & (-pB <= ha * (1 + 1e-9)))


def test_single_shift_is_geometric_mean_on_symmetric_intervals():
    """For identical intervals [a,b] and J = 1 the optimal shift is sqrt(ab)."""
    op = WL._op(2, 15, (0.0, 0.0))
    pA, pB = WL.wachspress_shifts(op, op, 1, interval="spectrum")
    a, b = WL.spectral_interval(op)
    assert pA[0] == pytest.approx(-math.sqrt(a * b), rel=1e-10)
    assert pB[0] == pytest.approx(-math.sqrt(a * b), rel=1e-10)


def test_spectral_interval_matches_dense():
    op = WL._op(2, 12, (9.0, -4.0))
    A = convdiff_matrix(2, 12, op.omega).toarray()
    ev = np.linalg.eigvals(A).real
    lo, hi = WL.spectral_interval(op)
    assert -ev.max() == pytest.approx(lo, rel=1e-10)
    assert -ev.min() == pytest.approx(hi, rel=1e-10)
    H = 0.5 * (A + A.T)
    evh = np.linalg.eigvalsh(H)
    lo2, hi2 = WL.numerical_range_interval(op)
    assert -evh.max() == pytest.approx(lo2, rel=1e-10)
    assert -evh.min() == pytest.approx(hi2, rel=1e-10)


def test_batch_and_serving_generators():
    probs = WL.batch_problems(16)
    assert len(probs) == 16
    for p in probs:
        assert 32 <= p.A.N <= 128 and 32 <= p.B.N <= 128 and p.r in (1, 2, 4)
        assert all(-40 <= w <= 40 for w in p.A.omega + p.B.omega)
    reqs = WL.serving_requests(50)
    ts = [t for t, _ in reqs]
    assert all(b >= a for a, b in zip(ts, ts[1:]))
    for _, p in reqs:
        assert 1 <= p.r <= 8 and 1e-10 <= p.tol <= 1e-6 and p.A.dim in (2, 3)
