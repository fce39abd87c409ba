"""Pins of the red-black ILU(0) right preconditioner oracle and of the
right-preconditioned block GMRES definition: the grid colouring in closed
form, equality with the textbook ILU(0) factors of the red-black permuted
matrix, convergence of the Schur sweeps to the exact inverse, and the
exact-preconditioner special case of GMRES."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import precond as OP
from oracle.convdiff import convdiff_matrix
from oracle.gmres_ref import block_gmres_iterate
from paper_2312_02891_amd import workloads as WL


@pytest.mark.parametrize("dim,N", [(2, 5), (2, 6), (3, 4)])
def test_grid_coloring_is_index_parity(dim, N):
    """On the lexicographic grid (first axis fastest) the colour of point
    (i_1, ..., i_d) is the parity of i_1 + ... + i_d: the unique 2-colouring
    with point 0 red."""
    A = convdiff_matrix(dim, N, tuple([3.0] * dim))
    col = OP.two_coloring(A)
    idx = np.indices([N] * dim).reshape(dim, -1, order="F")
    # the first axis varies fastest in the lexicographic order
    par = idx.sum(axis=0) % 2
    assert np.array_equal(col, par)


def test_non_bipartite_patterns_are_rejected():
    tri = sp.csr_matrix(np.array([[2.0, 1, 1], [1, 2.0, 1], [1, 1, 2.0]]))
    assert OP.two_coloring(tri) is None
    rp, ci, v = WL.mass_csr(2, 5)
    M = sp.csr_matrix((v, ci, rp), shape=(25, 25))
    assert OP.two_coloring(M) is None
    with pytest.raises(ValueError):
        OP.rb_precond_apply(M, 1.0, np.ones((25, 1)))


@pytest.mark.parametrize("dim,N,omega,shift", [(2, 5, (7.0, -3.0), -40.0), (3, 3, (2.0, 5.0, -1.0), -12.0),
                                               (2, 6, (-20.0, 9.0), -3.0)])
def test_zero_sweeps_equals_textbook_ilu0_in_red_black_order(dim, N, omega, shift):
    """With no sweeps M = (L U)^{-1} where L U is the ILU(0) of
    P (A + s I) P^T computed by the generic IKJ algorithm (P: red rows
    first), undone by the same permutation."""
    A = convdiff_matrix(dim, N, omega)
    n = A.shape[0]
    col = OP.two_coloring(A)
    perm = np.concatenate([np.where(col == 0)[0], np.where(col == 1)[0]])
    S = (A + shift * sp.identity(n)).toarray()[np.ix_(perm, perm)]
    L, U = OP.ilu0_dense(S)
    nz = S != 0.0
    assert np.allclose((L @ U)[nz], S[nz], rtol=1e-13, atol=1e-12 * np.abs(S).max())
    V = np.random.default_rng(1).standard_normal((n, 3))
    want = np.empty_like(V)
    want[perm] = np.linalg.solve(U, np.linalg.solve(L, V[perm]))
    got = OP.rb_precond_apply(A, shift, V, sweeps=0)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-13 * np.abs(want).max())


def test_sweeps_converge_to_the_exact_inverse():
    """Jacobi on the Schur complement converges for this diagonally
    dominant shifted operator, so M V -> (A + s I)^{-1} V."""
    A = convdiff_matrix(2, 8, (10.0, -6.0))
    s = -400.0
    n = A.shape[0]
    V = np.random.default_rng(2).standard_normal((n, 2))
    X = spla.spsolve((A + s * sp.identity(n)).tocsc(), V)
    errs = [np.linalg.norm(OP.rb_precond_apply(A, s, V, k) - X) / np.linalg.norm(X) for k in (0, 2, 8, 60)]
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] < 1e-12


def test_preconditioned_gmres_definition():
    """An exact right preconditioner gives the solution after one block
    step.  With the red-black preconditioner the j-step iterate lies in
    M K_j(S M, W) and its residual is orthogonal to S M K_j(S M, W) (the
    least-squares optimality condition), checked on a basis built here by
    plain repeated products; it also beats the unpreconditioned iterate."""
    A = convdiff_matrix(2, 9, (25.0, -12.0))
    n = A.shape[0]
    s = -30.0
    S = (A + s * sp.identity(n)).tocsc()
    W = np.random.default_rng(3).standard_normal((n, 2))
    exact = lambda X: spla.spsolve(S, X).reshape(X.shape)
    Z1 = block_gmres_iterate(A, s, W, 1, precond=exact)
    assert np.allclose(Z1, exact(W), rtol=1e-10, atol=1e-12)
    pre = lambda X: OP.rb_precond_apply(A, s, X, 1)
    for j in (2, 4):
        Zp = block_gmres_iterate(A, s, W, j, precond=pre)
        Zn = block_gmres_iterate(A, s, W, j)
        # Krylov blocks W, (S M) W, ..., (S M)^{j-1} W, orthonormalised once
        blocks, cur = [], W
        for _ in range(j):
            blocks.append(cur)
            cur = S @ pre(cur)
        K, _ = np.linalg.qr(np.hstack(blocks))
        MK = pre(K)
        C, *_ = np.linalg.lstsq(MK, Zp, rcond=None)
        assert np.linalg.norm(MK @ C - Zp) <= 1e-9 * np.linalg.norm(Zp)
        res = W - S @ Zp
        SMK = S @ MK
        assert np.linalg.norm(SMK.T @ res) <= 1e-9 * np.linalg.norm(SMK) * np.linalg.norm(res)
        assert np.linalg.norm(res) < np.linalg.norm(W - S @ Zn)


def test_lumped_mass_pencil_preconditioner():
    """For a pencil the preconditioner is the red-black ILU(0) of
    A + s diag(M 1): equal to the plain form applied to the matrix
    A + s diag(M 1) with shift 0, to the textbook ILU(0) of that matrix, and
    for M = I to the plain preconditioner bit for bit."""
    A = convdiff_matrix(2, 6, (9.0, -4.0))
    n = A.shape[0]
    rp, ci, v = WL.mass_csr(2, 6)
    M = sp.csr_matrix((v, ci, rp), shape=(n, n))
    s = -35.0
    V = np.random.default_rng(12).standard_normal((n, 2))
    lump = np.asarray(M.sum(axis=1)).ravel()
    As = (A + s * sp.diags(lump)).tocsr()
    for k in (0, 3):
        got = OP.rb_precond_apply(A, s, V, k, mass=M)
        assert np.allclose(got, OP.rb_precond_apply(As, 0.0, V, k), rtol=1e-13, atol=1e-15)
    col = OP.two_coloring(A)
    perm = np.concatenate([np.where(col == 0)[0], np.where(col == 1)[0]])
    Sd = As.toarray()[np.ix_(perm, perm)]
    Lf, Uf = OP.ilu0_dense(Sd)
    want = np.empty_like(V)
    want[perm] = np.linalg.solve(Uf, np.linalg.solve(Lf, V[perm]))
    assert np.allclose(OP.rb_precond_apply(A, s, V, 0, mass=M), want, rtol=1e-12, atol=1e-14)
    I = sp.identity(n, format="csr")
    assert np.array_equal(OP.rb_precond_apply(A, s, V, 2, mass=I), OP.rb_precond_apply(A, s, V, 2))


def test_pencil_gmres_definition_with_exact_preconditioner():
    """block_gmres_iterate with M: an exact right preconditioner of the
    pencil solves in one block step."""
    A = convdiff_matrix(2, 7, (5.0, 3.0))
    n = A.shape[0]
    rp, ci, v = WL.mass_csr(2, 7)
    M = sp.csr_matrix((v, ci, rp), shape=(n, n))
    s = -60.0
    S = (A + s * M).tocsc()
    W = np.random.default_rng(13).standard_normal((n, 2))
    exact = lambda X: spla.spsolve(S, X).reshape(X.shape)
    Z1 = block_gmres_iterate(A, s, W, 1, precond=exact, M=M)
    assert np.allclose(Z1, exact(W), rtol=1e-10, atol=1e-12)


def _schur_dense(S, col):
    """Schur complement on the black rows of a small dense S (definition)."""
    r, b = np.where(col == 0)[0], np.where(col == 1)[0]
    return S[np.ix_(b, b)] - S[np.ix_(b, r)] @ np.linalg.solve(S[np.ix_(r, r)], S[np.ix_(r, b)])


@pytest.mark.parametrize("dim,N,omega,shift", [(2, 9, (25.0, -12.0), -30.0), (2, 10, (4.0, 7.0), -3.0),
                                               (3, 5, (20.0, 10.0, 5.0), -40.0), (3, 6, (-10.0, 15.0, 5.0), 0.0)])
def test_chebyshev_bounds_enclose_the_real_spectrum(dim, N, omega, shift):
    """For upwind convection-diffusion operators (diagonally similar to
    symmetric ones) J = I - diag(T)^{-1} T has a real spectrum, and the two
    Gershgorin-type bounds enclose it."""
    A = convdiff_matrix(dim, N, omega)
    S = (A + shift * sp.identity(A.shape[0])).toarray()
    col = OP.two_coloring(A)
    T = _schur_dense(S, col)
    J = np.eye(T.shape[0]) - T / np.diag(T)[:, None]
    ev = np.linalg.eigvals(J)
    assert np.abs(ev.imag).max() < 1e-10
    lo, hi = OP.schur_poly_bounds(sp.csr_matrix(T), np.diag(S)[col == 1])
    assert lo <= ev.real.min() + 1e-12 and ev.real.max() <= hi + 1e-12
    assert lo <= 0.0 < hi < 1.0


def test_chebyshev_error_is_the_scaled_chebyshev_polynomial():
    """After k Chebyshev steps from zero the black-row error is
    T_{k+1}(G / sigma) / T_{k+1}(1 / sigma) applied to the exact Schur solve,
    G = I - gamma diag(T)^{-1} T: evaluated here through G's eigenvectors and
    numpy's Chebyshev series, independently of the three-term recurrence."""
    A = convdiff_matrix(2, 9, (25.0, -12.0))
    n = A.shape[0]
    s = -30.0
    S = (A + s * sp.identity(n)).toarray()
    col = OP.two_coloring(A)
    blk = col == 1
    T = _schur_dense(S, col)
    V = np.random.default_rng(21).standard_normal((n, 2))
    xs = np.linalg.solve(S, V)[blk]  # black part of S^{-1} V = T^{-1} y_b
    lo, hi = OP.schur_poly_bounds(sp.csr_matrix(T), np.diag(S)[blk])
    gamma = 2.0 / (2.0 - lo - hi)
    sigma = (hi - lo) / (2.0 - lo - hi)
    G = np.eye(T.shape[0]) - gamma * T / np.diag(T)[:, None]
    mu, X = np.linalg.eig(G)
    for k in (1, 2, 5, 9):
        c = np.zeros(k + 2)
        c[k + 1] = 1.0
        p = np.polynomial.chebyshev.chebval(mu / sigma, c) / np.polynomial.chebyshev.chebval(1.0 / sigma, c)
        err = (X @ (p[:, None] * np.linalg.solve(X, xs))).real
        got = OP.rb_precond_apply(A, s, V, k, poly="chebyshev")[blk]
        assert np.linalg.norm((xs - got) - err) <= 1e-10 * np.linalg.norm(xs)


def test_chebyshev_beats_jacobi_and_converges():
    """Past a few steps the Chebyshev error falls below the Jacobi one (for
    very few steps Jacobi can be ahead: it damps the oscillatory modes
    faster than the uniform Chebyshev bound), and both reach the exact
    inverse."""
    A = convdiff_matrix(3, 6, (20.0, 10.0, 5.0))
    n = A.shape[0]
    s = -15.0
    V = np.random.default_rng(22).standard_normal((n, 3))
    X = spla.spsolve((A + s * sp.identity(n)).tocsc(), V)
    e = lambda k, poly: np.linalg.norm(OP.rb_precond_apply(A, s, V, k, poly=poly) - X) / np.linalg.norm(X)
    for k in (10, 16):
        assert e(k, "chebyshev") < 0.5 * e(k, "jacobi")
    assert e(80, "chebyshev") < 1e-12
    # no steps: the ILU(0) step whichever the polynomial
    assert np.array_equal(OP.rb_precond_apply(A, s, V, 0, poly="chebyshev"), OP.rb_precond_apply(A, s, V, 0))


def test_chebyshev_falls_back_to_jacobi_without_diagonal_dominance():
    """The 1-D Laplacian stencil (-1, 2, -1) without a shift: interior rows of
    J sum to exactly 1, so hi = 1 and the steps are the Jacobi ones."""
    n = 31
    A = sp.diags([-np.ones(n - 1), 2.0 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr")
    col = OP.two_coloring(A)
    T = _schur_dense(A.toarray(), col)
    assert OP.schur_poly_bounds(sp.csr_matrix(T), np.full(int(col.sum()), 2.0))[1] == 1.0
    V = np.random.default_rng(23).standard_normal((n, 2))
    assert np.array_equal(OP.rb_precond_apply(A, 0.0, V, 5, poly="chebyshev"), OP.rb_precond_apply(A, 0.0, V, 5))
    with pytest.raises(ValueError):
        OP.rb_precond_apply(A, 0.0, V, 5, poly="cg")
