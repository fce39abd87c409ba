"""Pins of the oracle for the generalized equation A X C + M X B = -f g^T
(eq. (gsylv)) and its low-rank ADI iteration (eq. (lradi_g)): closed forms
for diagonal matrices, the exact-solve residual identity, a dense solve, the
reduction to M = C = I, and the mass-matrix inputs."""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import fadi as OF
from oracle.convdiff import convdiff_matrix
from paper_2312_02891_amd import workloads as WL


def _mass(dim, N):
    rp, ci, v = WL.mass_csr(dim, N)
    n = len(rp) - 1
    return sp.csr_matrix((v, ci, rp), shape=(n, n))


def test_diagonal_closed_form_every_iterate():
    """For diagonal A, M, B, C the exact solution is
    X_ij = -(f g^T)_ij / (a_i c_j + m_i b_j), and by eq. (lradi_g_wt) each
    step multiplies w by (lambda_i - alpha)/(lambda_i + beta) with
    lambda_i = a_i/m_i and t by (mu_j - beta)/(mu_j + alpha) with
    mu_j = b_j/c_j, so X_k = X o (1 - p_i q_j).  beta = pA, alpha = pB; a
    swapped M and C, a missing M in the update or a wrong shift role fails."""
    rng = np.random.default_rng(7)
    n, m, r = 9, 7, 2
    a, b = -rng.uniform(1.0, 50.0, n), -rng.uniform(2.0, 400.0, m)
    mm, cc = rng.uniform(0.3, 2.0, n), rng.uniform(0.5, 3.0, m)
    f, g = rng.standard_normal((n, r)), rng.standard_normal((m, r))
    A, B, M, C = sp.diags(a), sp.diags(b), sp.diags(mm), sp.diags(cc)
    pA = -rng.uniform(2.0, 400.0, 6)
    pB = -rng.uniform(1.0, 50.0, 6)
    X = -(f @ g.T) / (a[:, None] * cc[None, :] + mm[:, None] * b[None, :])
    lam, mu = a / mm, b / cc
    for k in range(1, 7):
        res = OF.fadi(A, B, f, g, pA, pB, rescale=False, kfixed=k, M=M, C=C)
        p = np.prod([(lam - pB[l]) / (lam + pA[l]) for l in range(k)], axis=0)
        q = np.prod([(mu - pA[l]) / (mu + pB[l]) for l in range(k)], axis=0)
        Xk = X * (1.0 - p[:, None] * q[None, :])
        assert np.allclose(res.X(), Xk, rtol=1e-12, atol=1e-14 * np.abs(X).max())


def test_exact_solves_residual_equals_factor_product():
    """With exact solves A X_k C + M X_k B + f g^T = w_k t_k^T (the
    generalized form of eq. (adi_resexact)) on conv-diff operators with
    mass matrices."""
    A = convdiff_matrix(2, 9, (12.0, -7.0))
    B = convdiff_matrix(2, 8, (-9.0, 4.0))
    M, C = _mass(2, 9), _mass(2, 8)
    rng = np.random.default_rng(3)
    f, g = rng.standard_normal((81, 2)), rng.standard_normal((64, 2))
    pA, pB = WL.wachspress_shifts(WL._op(2, 9, (12, -7)), WL._op(2, 8, (-9, 4)), 6,
                                  massA=True, massB=True)
    res = OF.fadi(A, B, f, g, pA, pB, rescale=False, kfixed=5, M=M, C=C)
    R = OF.true_residual_dense(A, B, f, g, res.X(), M=M, C=C)
    assert np.linalg.norm(R - res.W @ res.T.T) <= 1e-12 * np.linalg.norm(f @ g.T)


def test_converged_solution_matches_dense_solve():
    """The converged factored solution equals the dense solution of
    (M^-1 A) X + X (B C^-1) = -M^-1 f g^T C^-1 to the level of tau."""
    P = WL.GEN_SMALL
    NA, NB = 11, 9
    A = convdiff_matrix(2, NA, P.A.omega)
    B = convdiff_matrix(2, NB, P.B.omega)
    M, C = _mass(2, NA), _mass(2, NB)
    f, g = WL.rhs_factors(P.seed, NA * NA, NB * NB, P.r)
    pA, pB = WL.wachspress_shifts(WL._op(2, NA, P.A.omega), WL._op(2, NB, P.B.omega), 12,
                                  massA=True, massB=True)
    res = OF.fadi(A, B, f, g, pA, pB, tol=1e-10, kmax=100, M=M, C=C)
    Md, Cd = M.toarray(), C.toarray()
    Xd = sla.solve_sylvester(np.linalg.solve(Md, A.toarray()), B.toarray() @ np.linalg.inv(Cd),
                             -np.linalg.solve(Md, f @ g.T) @ np.linalg.inv(Cd))
    assert res.k < 100
    assert np.linalg.norm(res.X() - Xd) <= 1e-8 * np.linalg.norm(Xd)


def test_identity_mass_reproduces_plain_iteration():
    """M = C = I given explicitly gives the plain iteration's factors bit for
    bit (the same LU of A + p I, and M z = z)."""
    P = WL.SMALL_2D
    A = convdiff_matrix(2, 9, P.A.omega)
    B = convdiff_matrix(2, 8, P.B.omega)
    f, g = WL.rhs_factors(5, 81, 64, 2)
    pA, pB = WL.wachspress_shifts(WL._op(2, 9, P.A.omega), WL._op(2, 8, P.B.omega), 6)
    plain = OF.fadi(A, B, f, g, pA, pB, kfixed=6)
    ident = OF.fadi(A, B, f, g, pA, pB, kfixed=6, M=sp.identity(81, format="csr"),
                    C=sp.identity(64, format="csr"))
    assert np.array_equal(plain.Z, ident.Z) and np.array_equal(plain.Y, ident.Y)
    assert np.array_equal(plain.gammas, ident.gammas)


def test_generalized_lowrank_residual_matches_dense():
    A = convdiff_matrix(2, 7, (3.0, -2.0))
    B = convdiff_matrix(2, 6, (-1.0, 4.0))
    M, C = _mass(2, 7), _mass(2, 6)
    rng = np.random.default_rng(11)
    f, g = rng.standard_normal((49, 2)), rng.standard_normal((36, 2))
    Z, Y = rng.standard_normal((49, 6)), rng.standard_normal((36, 6))
    d = rng.uniform(1.0, 5.0, 6)
    X = (Z * d) @ Y.T
    dense = np.linalg.norm(OF.true_residual_dense(A, B, f, g, X, M=M, C=C), 2)
    assert np.isclose(OF.lowrank_residual_norm(A, B, f, g, Z, d, Y, M=M, C=C), dense, rtol=1e-12)


def test_mass_matrix_input():
    """The mass matrix is the Kronecker product of tridiag(1, 4, 1)/6
    (checked against numpy's dense kron) and its eigenvalues fill
    mass_interval."""
    T = (np.diag(np.full(5, 4.0)) + np.diag(np.ones(4), 1) + np.diag(np.ones(4), -1)) / 6.0
    for dim in (1, 2, 3):
        D = T
        for _ in range(dim - 1):
            D = np.kron(T, D)
        M = _mass(dim, 5).toarray()
        assert np.array_equal(M, D)
        e = np.linalg.eigvalsh(M)
        lo, hi = WL.mass_interval(dim, 5)
        assert np.isclose(e.min(), lo, rtol=1e-12) and np.isclose(e.max(), hi, rtol=1e-12)
