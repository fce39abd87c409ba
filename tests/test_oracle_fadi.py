"""Pins of the oracle LR-ADI (Algorithm 1 with direct solves) against
closed forms, dense Bartels-Stewart and the identities of Sec. 2."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fadi as OF
from oracle.convdiff import convdiff_matrix
from paper_2312_02891_amd import workloads as WL


def _rng(seed):
    return np.random.default_rng(seed)


def diag_problem(n=9, m=7, r=2, seed=0):
    rng = _rng(seed)
    a = -rng.uniform(1.0, 50.0, n)
    b = -rng.uniform(2.0, 400.0, m)   # deliberately different interval
    f = rng.standard_normal((n, r))
    g = rng.standard_normal((m, r))
    return a, b, f, g


def test_diagonal_closed_form_every_iterate():
    """For diagonal A, B the exact solution is X_ij = -(f g^T)_ij/(a_i + b_j)
    and, by eq. (fadi_error) with X_0 = 0, the k-th ADI iterate is
    X_k = X o (1 - p_i q_j) with p_i = prod_l (a_i - alpha_l)/(a_i + beta_l)
    and q_j = prod_l (b_j - beta_l)/(b_j + alpha_l).  Here beta = pA (added to
    A) and alpha = pB (added to B^T), so a swap of the two shift roles or a
    wrong gamma sign fails."""
    a, b, f, g = diag_problem()
    A, B = sp.diags(a), sp.diags(b)
    rng = _rng(5)
    pA = -rng.uniform(2.0, 400.0, 6)    # from B's interval
    pB = -rng.uniform(1.0, 50.0, 6)     # from A's interval
    X = -(f @ g.T) / (a[:, None] + b[None, :])
    for k in range(1, 7):
        res = OF.fadi(A, B, f, g, pA, pB, rescale=False, kfixed=k)
        p = np.prod([(a - pB[l]) / (a + pA[l]) for l in range(k)], axis=0)
        q = np.prod([(b - pA[l]) / (b + pB[l]) for l in range(k)], axis=0)
        Xk = X * (1.0 - p[:, None] * q[None, :])
        assert np.allclose(res.X(), Xk, rtol=1e-12, atol=1e-14 * np.abs(X).max())


def test_residual_factors_equal_true_residual_exact_solves():
    """eq. (adi_resexact): with exact solves A X_k + X_k B + f g^T = w_k t_k^T."""
    P = WL.SMALL_2D
    A = convdiff_matrix(P.A.dim, 9, (12, -7))
    B = convdiff_matrix(P.B.dim, 8, (-9, 4))
    rng = _rng(3)
    f = rng.standard_normal((81, 2))
    g = rng.standard_normal((64, 2))
    pA, pB = WL.wachspress_shifts(WL._op(2, 9, (12, -7)), WL._op(2, 8, (-9, 4)), 6)
    res = OF.fadi(A, B, f, g, pA, pB, rescale=False, kfixed=5)
    R = OF.true_residual_dense(A, B, f, g, res.X())
    assert np.linalg.norm(R - res.W @ res.T.T) <= 1e-12 * np.linalg.norm(f @ g.T)


def test_config1_matches_bartels_stewart():
    """Config 1 (n = m = 400): the converged factored solution agrees with
    the dense Bartels-Stewart solution to the level the residual allows."""
    P = WL.C1
    A = convdiff_matrix(P.A.dim, P.A.N, P.A.omega)
    B = convdiff_matrix(P.B.dim, P.B.N, P.B.omega)
    f, g = WL.rhs_factors(P.seed, P.A.n, P.B.n, P.r)
    pA, pB = WL.wachspress_shifts(P.A, P.B, P.nshifts)
    res = OF.fadi(A, B, f, g, pA, pB, tol=P.tol)
    X = OF.bartels_stewart(A, B, f, g)
    assert res.k <= P.nshifts
    assert res.res_hist[-1] < P.tol
    err = np.linalg.norm(res.X() - X) / np.linalg.norm(X)
    assert err < 1e-6
    # the dense true residual equals the computed one (exact solves)
    R = OF.true_residual_dense(A, B, f, g, res.X())
    rel = np.linalg.norm(R, 2) / np.linalg.norm(f @ g.T, 2)
    assert abs(rel - res.res_hist[-1]) <= 1e-3 * rel + 1e-14


def _planted_inexact(seed=7, kfix=5):
    A = convdiff_matrix(2, 8, (6, -3))
    B = convdiff_matrix(2, 7, (-4, 5))
    rng = _rng(seed)
    f = rng.standard_normal((64, 2))
    g = rng.standard_normal((49, 2))
    pA, pB = WL.wachspress_shifts(WL._op(2, 8, (6, -3)), WL._op(2, 7, (-4, 5)), 5)
    pert = _rng(seed + 1)

    def noisy(M):
        def solve(k, s, rhs):
            n = M.shape[0]
            z = np.linalg.solve((M + s * sp.identity(n)).toarray(), rhs)
            return z + 1e-3 * np.linalg.norm(z) * pert.standard_normal(z.shape)
        return solve

    res = OF.fadi(A, B, f, g, pA, pB, rescale=False, kfixed=kfix,
                  solve_A=noisy(A), solve_B=noisy(B.T.tocsr()))
    return A, B, f, g, pA, pB, res


def test_theorem2_true_residual_with_planted_inexact_solves():
    """eq. (adi_res_inexact): R_true = w_k t_k^* - S^A Gamma Y^* - Z Gamma (S^B)^*
    for arbitrary (here deliberately inaccurate) inner solutions."""
    A, B, f, g, pA, pB, res = _planted_inexact()
    D = res.D()
    SA = np.hstack(res.rA)
    SB = np.hstack(res.rB)
    Rtrue = OF.true_residual_dense(A, B, f, g, res.X())
    Rthm = res.W @ res.T.T - (SA * D) @ res.Y.T - (res.Z * D) @ SB.T
    assert np.linalg.norm(Rtrue - Rthm) <= 1e-11 * np.linalg.norm(Rtrue)
    # and the gap is not small, so the identity is not trivially satisfied
    assert np.linalg.norm(Rtrue - res.W @ res.T.T) > 1e-4 * np.linalg.norm(Rtrue)


def test_theorem1_identity_and_gamma_equation():
    """eq. (adi_AZ_BTY) with M = I: A Z_k = Z_k sigma^alpha + w_k E_k^T - S^A_k,
    and Gamma_k solves sigma^alpha G + G (sigma^beta)^* + gamma gamma^T = 0."""
    A, B, f, g, pA, pB, res = _planted_inexact(seed=9, kfix=4)
    k = res.k
    r = f.shape[1]
    alpha = np.array([pB[i % len(pB)] for i in range(k)])   # zeros over Lambda(A)
    beta = np.array([pA[i % len(pA)] for i in range(k)])
    gam = res.gammas
    sa = np.zeros((k, k))
    sb = np.zeros((k, k))
    for i in range(k):
        sa[i, i] = alpha[i]
        sb[i, i] = beta[i]
        for j in range(i):
            sa[i, j] = -gam[i]
            sb[i, j] = -gam[i]
    I = np.eye(r)
    SA = np.hstack(res.rA)
    E = np.kron(np.ones((k, 1)), I)
    lhs = A @ res.Z
    rhs = res.Z @ np.kron(sa, I) + res.W @ E.T - SA
    assert np.linalg.norm(lhs - rhs) <= 1e-11 * np.linalg.norm(lhs)
    SB = np.hstack(res.rB)
    lhsB = B.T @ res.Y
    rhsB = res.Y @ np.kron(sb, I) + res.T @ E.T - SB
    assert np.linalg.norm(lhsB - rhsB) <= 1e-11 * np.linalg.norm(lhsB)
    G = np.diag(gam)
    gv = gam[:, None]
    assert np.linalg.norm(sa @ G + G @ sb.T + gv @ gv.T) <= 1e-12 * np.linalg.norm(gv @ gv.T)


def test_lowrank_norm_helpers_match_dense():
    rng = _rng(11)
    W = rng.standard_normal((50, 3))
    T = rng.standard_normal((40, 3))
    assert np.isclose(OF.lowrank_product_norm(W, T), np.linalg.norm(W @ T.T, 2), rtol=1e-13)
    Z1, Y1, d1 = rng.standard_normal((50, 6)), rng.standard_normal((40, 6)), rng.standard_normal(6)
    Z2, Y2, d2 = rng.standard_normal((50, 4)), rng.standard_normal((40, 4)), rng.standard_normal(4)
    dense = (Z1 * d1) @ Y1.T - (Z2 * d2) @ Y2.T
    assert np.isclose(OF.lowrank_diff_fro(Z1, d1, Y1, Z2, d2, Y2), np.linalg.norm(dense), rtol=1e-12)
    assert np.isclose(OF.lowrank_fro(Z1, d1, Y1), np.linalg.norm((Z1 * d1) @ Y1.T), rtol=1e-12)


def test_lowrank_residual_norm_matches_dense():
    A = convdiff_matrix(2, 7, (3, 1))
    B = convdiff_matrix(2, 6, (-2, 4))
    rng = _rng(13)
    f, g = rng.standard_normal((49, 2)), rng.standard_normal((36, 2))
    Z, Y, d = rng.standard_normal((49, 6)), rng.standard_normal((36, 6)), rng.standard_normal(6)
    X = (Z * d) @ Y.T
    dense = np.linalg.norm(OF.true_residual_dense(A, B, f, g, X), 2)
    assert np.isclose(OF.lowrank_residual_norm(A, B, f, g, Z, d, Y), dense, rtol=1e-12)


def test_rescale_keeps_product_and_equalises_norms():
    rng = _rng(17)
    f, g = rng.standard_normal((30, 3)) * 7.0, rng.standard_normal((20, 3))
    f2, g2 = OF.rescale_rhs(f, g)
    assert np.allclose(f2 @ g2.T, f @ g.T, rtol=1e-13, atol=1e-13)
    assert np.isclose(np.linalg.norm(f2, 2), np.linalg.norm(g2, 2), rtol=1e-13)


def test_zero_rhs_terminates_immediately():
    """A zero residual factor stops Algorithm 1 before the first step."""
    A = convdiff_matrix(2, 4, (1, 1))
    f = np.zeros((16, 1))
    g = np.ones((16, 1))
    with np.errstate(all="ignore"):
        res = OF.fadi(A, A, f, g, np.array([-10.0]), np.array([-10.0]), rescale=False)
    assert res.k == 0
