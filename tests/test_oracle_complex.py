"""Pins of the oracle's complex form of the LR-ADI iteration (complex shift
parameters, Sec. 3.2.4 keeps the complex formulation; iteration as in
eq. (lradi_basic) and Algorithm 1 with complex alpha_k, beta_k) and of the
central-difference test operators whose spectra are complex."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import fadi as OF
from oracle.convdiff import convdiff_matrix
from paper_2312_02891_amd import workloads as WL


@pytest.mark.parametrize("dim,N,omega", [(2, 9, (40.0, -31.0)), (2, 12, (5.0, 60.0)), (3, 5, (30.0, -20.0, 25.0))])
def test_central_spectrum_closed_form(dim, N, omega):
    """The central-difference operator's eigenvalues are the Kronecker sum of
    the axis factors' d + 2 sqrt(l u) cos(j pi/(N+1)) (complex square root
    when l u < 0): dense eigenvalues of the generated matrix equal it."""
    op = WL.Operator(dim, N, tuple(omega), "central")
    A = convdiff_matrix(dim, N, omega, scheme="central").toarray()
    ev = np.linalg.eigvals(-A)                      # eigenvalues of L_h
    cf = WL.central_spectrum(op)
    key = lambda z: (np.round(z.real, 6), np.round(z.imag, 6))   # noqa: E731
    a = np.array(sorted(ev, key=key))
    b = np.array(sorted(cf, key=key))
    assert np.max(np.abs(a - b)) <= 1e-9 * np.max(np.abs(b))
    if all(abs(w) / (N + 1) / 2 > 1 for w in omega):
        assert np.max(np.abs(ev.imag)) > 1.0       # complex spectrum


def test_central_scheme_stencil_values():
    """Central differences: neighbours -ih2 -+ w ih / 2, diagonal 2 d ih2
    (before negation), and the matrix minus its transpose is the convection
    part alone (the diffusion part is symmetric)."""
    N, w = 7, (10.0, -6.0)
    A = convdiff_matrix(2, N, w, scheme="central")
    ih = N + 1.0
    L = -A.toarray()
    assert L[0, 0] == pytest.approx(4 * ih * ih)
    assert L[1, 0] == pytest.approx(-ih * ih - w[0] * ih / 2)     # u_{p - s_0} in row p = 1
    assert L[0, 1] == pytest.approx(-ih * ih + w[0] * ih / 2)
    assert L[N, 0] == pytest.approx(-ih * ih - w[1] * ih / 2)
    S = L - L.T
    assert np.allclose(np.diag(L), 4 * ih * ih)
    assert np.allclose(S + S.T, 0.0)
    assert np.abs(S).max() == pytest.approx(abs(w[0]) * ih, rel=1e-12) or \
        np.abs(S).max() == pytest.approx(abs(w[1]) * ih, rel=1e-12)


def _diag_case(seed):
    rng = np.random.default_rng(seed)
    n, m, r = 7, 5, 2
    a = -rng.uniform(1, 10, n) + 1j * rng.uniform(-5, 5, n)
    b = -rng.uniform(1, 10, m) + 1j * rng.uniform(-5, 5, m)
    f = rng.standard_normal((n, r)) + 1j * rng.standard_normal((n, r))
    g = rng.standard_normal((m, r)) + 1j * rng.standard_normal((m, r))
    al = -rng.uniform(1, 10, 6) + 1j * rng.uniform(-5, 5, 6)   # zeros over Lambda(A)
    be = -rng.uniform(1, 10, 6) + 1j * rng.uniform(-5, 5, 6)   # poles' negatives over Lambda(B)
    return a, b, f, g, al, be


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_complex_shifts_diagonal_closed_form(seed):
    """For diagonal A, B every iterate is known in closed form: with
    X_ij = -(f g^*)_ij / (a_i + b_j), eq. (fadi_error) gives
    X_k = X o (1 - c_A(i) c_B(j)), c_A(i) = prod (a_i - alpha)/(a_i + beta),
    c_B(j) = prod (b_j - beta)/(b_j + alpha).  Complex a, b, f, g and
    unpaired complex shifts: a missing conjugate (alpha for conj(alpha) in
    gamma, B^T for B^*, gamma for conj(gamma) in t) breaks it."""
    a, b, f, g, al, be = _diag_case(seed)
    A, B = sp.diags(a).tocsr(), sp.diags(b).tocsr()
    X = -(f @ g.conj().T) / (a[:, None] + b[None, :])
    pA, pB = be, np.conj(al)
    for k in range(1, 7):
        res = OF.fadi(A, B, f, g, pA, pB, rescale=False, kfixed=k)
        cA = np.prod([(a - al[i]) / (a + be[i]) for i in range(k)], axis=0)
        cB = np.prod([(b - be[i]) / (b + al[i]) for i in range(k)], axis=0)
        Xk = X * (1.0 - cA[:, None] * cB[None, :])
        assert np.linalg.norm(res.X() - Xk) <= 1e-12 * np.linalg.norm(X)


def test_complex_shifts_exact_residual_identity():
    """With exact solves the residual is the low-rank product of the factors:
    A X_k + X_k B + f g^T = w_k t_k^* (eq. (adi_resexact)), complex shifts on
    a real central-difference problem."""
    opA = WL.Operator(2, 8, (60.0, 45.0), "central")
    opB = WL.Operator(2, 6, (-50.0, 40.0), "central")
    A = convdiff_matrix(2, 8, opA.omega, scheme="central")
    B = convdiff_matrix(2, 6, opB.omega, scheme="central")
    f, g = WL.rhs_factors(7, A.shape[0], B.shape[0], 2)
    pA, pB = WL.complex_shifts(opA, opB, 6)
    for k in (1, 2, 3, 6):
        res = OF.fadi(A, B, f, g, pA, pB, rescale=False, kfixed=k)
        R = OF.true_residual_dense(A, B, f, g, res.X())
        assert np.linalg.norm(R - res.W @ res.T.conj().T) <= 1e-11 * np.linalg.norm(f @ g.T)


def test_conjugate_pairs_keep_the_iterate_real():
    """Real A, B, f, g and shifts in conjugate pairs: after every completed
    pair the iterate is real (to rounding); in between it is not."""
    opA = WL.Operator(2, 10, (70.0, -40.0), "central")
    opB = WL.Operator(2, 8, (45.0, 55.0), "central")
    A = convdiff_matrix(2, 10, opA.omega, scheme="central")
    B = convdiff_matrix(2, 8, opB.omega, scheme="central")
    f, g = WL.rhs_factors(8, A.shape[0], B.shape[0], 2)
    pA, pB = WL.complex_shifts(opA, opB, 8)
    assert np.all(np.abs(pA.imag) > 0) and np.allclose(pA[1::2], np.conj(pA[0::2]))
    for k in range(1, 9):
        X = OF.fadi(A, B, f, g, pA, pB, kfixed=k).X()
        im = np.linalg.norm(X.imag) / np.linalg.norm(X)
        if k % 2 == 0:
            assert im <= 1e-13
        else:
            assert im >= 1e-6


def test_complex_fadi_converges_to_bartels_stewart():
    """Converged complex-shift iteration against a dense Bartels-Stewart
    solution of the same real equation."""
    opA = WL.Operator(2, 14, (90.0, 70.0), "central")
    opB = WL.Operator(2, 11, (-80.0, 60.0), "central")
    A = convdiff_matrix(2, 14, opA.omega, scheme="central")
    B = convdiff_matrix(2, 11, opB.omega, scheme="central")
    f, g = WL.rhs_factors(9, A.shape[0], B.shape[0], 2)
    pA, pB = WL.complex_shifts(opA, opB, 12)
    res = OF.fadi(A, B, f, g, pA, pB, tol=1e-10, kmax=200)
    Xbs = OF.bartels_stewart(A, B, f, g)
    err = np.linalg.norm(res.X().real - Xbs) / np.linalg.norm(Xbs)
    assert res.k < 200 and err <= 1e-8


def test_real_shifts_as_complex_equal_the_real_path():
    """Real shifts passed with complex dtype run the complex arithmetic and
    reproduce the real iteration."""
    P = WL.SMALL_2D
    A = convdiff_matrix(P.A.dim, P.A.N, P.A.omega)
    B = convdiff_matrix(P.B.dim, P.B.N, P.B.omega)
    f, g = WL.rhs_factors(P.seed, P.A.n, P.B.n, P.r)
    pA, pB = WL.wachspress_shifts(P.A, P.B, P.nshifts)
    re = OF.fadi(A, B, f, g, pA, pB, kfixed=8)
    cx = OF.fadi(A, B, f, g, pA.astype(complex), pB.astype(complex), kfixed=8)
    assert np.abs(cx.gammas.imag).max() == 0.0
    assert np.linalg.norm(cx.X() - re.X()) <= 1e-13 * np.linalg.norm(re.X())
    assert np.allclose(cx.res_hist, re.res_hist, rtol=1e-12)
