"""Pins of the Lyapunov oracle (A X M^T + M X A^T = -f f^T, the case
B = A^T, C = M^T, g = f of eq. (gsylv)): a closed form for diagonal
matrices, the exact-solve residual identity, dense solutions from SciPy's
Lyapunov solver, and agreement with the Sylvester oracle run on
(A, A^T, f, f) with equal shifts."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import fadi as OF
from oracle import lyap as OL
from oracle.convdiff import convdiff_matrix
from paper_2312_02891_amd import workloads as WL


def _mass(dim, N):
    rp, ci, v = WL.mass_csr(dim, N)
    n = len(rp) - 1
    return sp.csr_matrix((v, ci, rp), shape=(n, n))


def test_diagonal_closed_form_every_iterate():
    """For A = diag(a), M = diag(m): X_ij = -(f f^T)_ij / (a_i m_j + m_i a_j)
    and each step multiplies w by (lambda_i - p)/(lambda_i + p) with
    lambda_i = a_i / m_i, so X_k = X o (1 - q_i q_j).  A sign error in
    gamma = -2p, a missing M in the update or a shift with the wrong sign
    fails."""
    rng = np.random.default_rng(2)
    n, r = 10, 3
    a, mm = -rng.uniform(1.0, 80.0, n), rng.uniform(0.3, 2.0, n)
    f = rng.standard_normal((n, r))
    p = -rng.uniform(1.0, 80.0, 7)
    X = -(f @ f.T) / (a[:, None] * mm[None, :] + mm[:, None] * a[None, :])
    lam = a / mm
    for k in range(1, 8):
        res = OL.lyap_adi(sp.diags(a), f, p, kfixed=k, M=sp.diags(mm))
        q = np.prod([(lam - p[l]) / (lam + p[l]) for l in range(k)], axis=0)
        Xk = X * (1.0 - q[:, None] * q[None, :])
        assert np.allclose(res.X(), Xk, rtol=1e-12, atol=1e-14 * np.abs(X).max())


def test_exact_solves_residual_equals_factor_product():
    """A X_k M^T + M X_k A^T + f f^T = w_k w_k^T with exact solves."""
    A = convdiff_matrix(2, 9, (10.0, -6.0))
    M = _mass(2, 9)
    f = np.random.default_rng(4).standard_normal((81, 2))
    p = WL.wachspress_shifts(WL._op(2, 9, (10, -6)), WL._op(2, 9, (-10, 6)), 6,
                             massA=True, massB=True)[0]
    res = OL.lyap_adi(A, f, p, kfixed=5, M=M)
    X = res.X()
    R = A @ X @ M.T + M @ X @ A.T + f @ f.T
    assert np.linalg.norm(R - res.W @ res.W.T) <= 1e-12 * np.linalg.norm(f @ f.T)


@pytest.mark.parametrize("mass", [False, True])
def test_converged_solution_matches_dense_lyapunov(mass):
    """The converged factored solution equals SciPy's dense solution of
    (M^-1 A) X + X (M^-1 A)^T = -M^-1 f f^T M^-T to the level of tau."""
    N = 10
    A = convdiff_matrix(2, N, (20.0, 8.0))
    M = _mass(2, N) if mass else None
    f = np.random.default_rng(8).standard_normal((N * N, 2))
    op = WL._op(2, N, (20, 8))
    p = WL.wachspress_shifts(op, WL._op(2, N, (-20, -8)), 12, massA=mass, massB=mass)[0]
    res = OL.lyap_adi(A, f, p, tol=1e-11, kmax=200, M=M)
    Ad = A.toarray()
    if mass:
        Mi = np.linalg.inv(M.toarray())
        Xd = sla.solve_continuous_lyapunov(Mi @ Ad, -Mi @ f @ f.T @ Mi.T)
    else:
        Xd = sla.solve_continuous_lyapunov(Ad, -f @ f.T)
    assert res.k < 200 and res.res_hist[-1] < 1e-11
    assert np.linalg.norm(res.X() - Xd) <= 1e-8 * np.linalg.norm(Xd)
    assert np.allclose(res.X(), res.X().T, rtol=0, atol=1e-14 * np.abs(Xd).max())


@pytest.mark.parametrize("mass", [False, True])
def test_matches_sylvester_oracle_with_b_equal_a_transpose(mass):
    """The Sylvester iteration of eq. (lradi_g) on (A, A^T, f, f) with
    alpha_k = beta_k and C = M^T produces y_k = z_k: same Z, gammas and
    computed residuals as the Lyapunov form."""
    A = convdiff_matrix(2, 8, (-15.0, 9.0))
    M = _mass(2, 8) if mass else None
    f = np.random.default_rng(6).standard_normal((64, 3))
    p = WL.wachspress_shifts(WL._op(2, 8, (-15, 9)), WL._op(2, 8, (15, -9)), 6,
                             massA=mass, massB=mass)[0]
    ly = OL.lyap_adi(A, f, p, tol=1e-10, kmax=60, M=M)
    sy = OF.fadi(A, A.T, f, f, p, p, tol=1e-10, kmax=60, rescale=False,
                 M=M, C=None if M is None else M.T)
    assert ly.k == sy.k
    assert np.allclose(ly.Z, sy.Z, rtol=1e-12, atol=1e-13 * np.abs(ly.Z).max())
    assert np.allclose(sy.Y, sy.Z, rtol=1e-12, atol=1e-13 * np.abs(ly.Z).max())
    assert np.allclose(ly.gammas, sy.gammas, rtol=1e-15)
    assert np.allclose(ly.res_hist, sy.res_hist, rtol=1e-9)
    assert ly.norm_ff == pytest.approx(sy.norm_fg, rel=1e-12)
