"""Pins of the oracle's CSR generator (Sec. 4, eq. (ex:convdiff)) against
facts that do not come from the generator itself."""
import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.convdiff import convdiff_csr, convdiff_matrix


def closed_form_eigs(dim, N, omega):
    """Eigenvalues of L_h: Kronecker sum of constant tridiagonals
    tridiag(l, d, u) with eigenvalues d - 2 sqrt(l u) cos(j pi/(N+1))."""
    ih = N + 1.0
    axes = []
    for w in omega:
        l = ih * ih + max(w, 0) * ih
        u = ih * ih + max(-w, 0) * ih
        d = 2 * ih * ih + abs(w) * ih
        j = np.arange(1, N + 1)
        axes.append(d - 2 * math.sqrt(l * u) * np.cos(j * math.pi / (N + 1)))
    ev = [sum(c) for c in itertools.product(*axes)]
    return np.sort(np.array(ev))


@pytest.mark.parametrize("dim,N", [(2, 1), (2, 2), (2, 7), (3, 1), (3, 4), (2, 20), (3, 9)])
def test_nnz_formula_and_structure(dim, N):
    omega = [3.0, -2.0, 1.0][:dim]
    rp, ci, v = convdiff_csr(dim, N, omega)
    n = N ** dim
    assert rp.dtype == np.int32 and ci.dtype == np.int32 and v.dtype == np.float64
    assert rp[0] == 0 and rp[-1] == len(ci) == len(v)
    assert len(ci) == (2 * dim + 1) * N ** dim - 2 * dim * N ** (dim - 1)
    for i in range(n):
        row = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) > 0), "columns must ascend within a row"
        assert i in row


@pytest.mark.parametrize("dim,N,omega", [(2, 20, (10, 5)), (2, 20, (-5, 8)), (2, 12, (0, 0)),
                                         (3, 6, (20, 10, 5)), (3, 5, (-10, 15, 5))])
def test_spectrum_closed_form(dim, N, omega):
    """Dense eigenvalues of A = -L_h equal minus the Kronecker-sum closed form."""
    A = convdiff_matrix(dim, N, omega).toarray()
    ev = np.linalg.eigvals(A)
    assert np.max(np.abs(ev.imag)) < 1e-6 * np.max(np.abs(ev.real))
    got = np.sort(-ev.real)
    want = closed_form_eigs(dim, N, omega)
    assert np.allclose(got, want, rtol=1e-9, atol=1e-9 * want.max())


def test_config1_interval_values():
    """Spectral intervals of the two config-1 operators (N=20, omega=(10,5)
    and (-5,8)), from the closed form: Lambda(A) in [-4109.086, -48.914] and
    Lambda(B) in [-4032.334, -41.666]."""
    for omega, lo, hi in [((10, 5), 48.914027, 4109.085973), ((-5, 8), 41.666095, 4032.333905)]:
        A = convdiff_matrix(2, 20, omega).toarray()
        ev = np.linalg.eigvals(A).real
        assert abs(-ev.max() - lo) < 1e-5 and abs(-ev.min() - hi) < 1e-5


@pytest.mark.parametrize("dim,N,omega", [(2, 9, (10, -5)), (3, 5, (3, -7, 2)), (2, 16, (-30, 40))])
def test_transpose_is_negated_convection_bitwise(dim, N, omega):
    """B^T of the upwind operator equals the operator with -omega, bit for bit
    (the B-side systems of Algorithm 1 are solved with B^*)."""
    B = convdiff_matrix(dim, N, omega)
    Bt = B.T.tocsr()
    Bt.sort_indices()
    rp, ci, v = convdiff_csr(dim, N, [-w for w in omega])
    assert np.array_equal(Bt.indptr.astype(np.int32), rp)
    assert np.array_equal(Bt.indices.astype(np.int32), ci)
    assert np.array_equal(Bt.data.view(np.uint64), v.view(np.uint64))


def test_zero_convection_is_five_point_laplacian_exactly():
    """omega = 0 gives -(1/h^2) (I kron T + T kron I), T = tridiag(-1, 2, -1)."""
    N = 11
    h2 = float((N + 1) ** 2)
    T = sp.diags([-np.ones(N - 1), 2 * np.ones(N), -np.ones(N - 1)], [-1, 0, 1])
    I = sp.identity(N)
    L = (sp.kron(I, T) + sp.kron(T, I)) * h2
    A = convdiff_matrix(2, N, (0.0, 0.0))
    assert np.array_equal(A.toarray(), -L.toarray())


@pytest.mark.parametrize("w", [7.0, -7.0])
def test_upwind_direction_on_quadratic(w):
    """For u = x^2 the upwind difference gives omega (2x - h) for omega > 0
    (backward) and omega (2x + h) for omega < 0 (forward); -Lap_h u = -2
    exactly.  So in interior rows A u = 2 - omega (2x -+ h)."""
    N = 15
    h = 1.0 / (N + 1)
    A = convdiff_matrix(2, N, (w, 0.0)).toarray()
    idx = np.arange(N * N)
    ix, iy = idx % N, idx // N
    x = (ix + 1) * h
    u = x ** 2
    Au = A @ u
    interior = (ix > 0) & (ix < N - 1) & (iy > 0) & (iy < N - 1)
    side = -1.0 if w > 0 else 1.0
    want = 2.0 - w * (2 * x + side * h)
    assert np.allclose(Au[interior], want[interior], rtol=1e-9, atol=1e-7)
