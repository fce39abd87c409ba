"""CPU checks of the native library: exported symbols, the C++ CSR generator
against the oracle's (bit for bit), and a host build of the small dense
routines and of the tolerance controller that the GPU kernels execute."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import controller as OC
from oracle.convdiff import convdiff_csr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2312_02891_amd", "liblradi.so")
HEADER = os.path.join(ROOT, "include", "lradi.h")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lradi_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB):
        pytest.fail("liblradi.so not built: run `python -m paper_2312_02891_amd.build`")
    from paper_2312_02891_amd import lradi
    return lradi


def test_library_exports_every_declared_symbol(L):
    lib = ctypes.CDLL(L.LIB_PATH)
    syms = declared_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(lib, s), s


@pytest.mark.parametrize("dim,N,omega", [(2, 1, (1.0, 2.0)), (2, 20, (10, 5)), (2, 20, (5, -8)),
                                         (2, 256, (50, 20)), (2, 192, (30, -40)),
                                         (3, 13, (6, -3, 2)), (3, 48, (10, -15, -5)),
                                         (3, 9, (0.0, -0.0, 0.0)), (2, 37, (12.3456789, -7.25))])
def test_generator_bit_exact_against_oracle(L, dim, N, omega):
    A = L.convdiff(dim, N, omega)
    rp, ci, v = convdiff_csr(dim, N, omega)
    assert np.array_equal(A.rowptr, rp)
    assert np.array_equal(A.colind, ci)
    assert np.array_equal(A.val.view(np.uint64), v.view(np.uint64))


@pytest.mark.parametrize("dim,N,omega", [(2, 1, (1.0, 2.0)), (2, 40, (150.0, 100.0)), (2, 30, (-120.0, 90.0)),
                                         (3, 14, (70.0, -50.0, 40.0)), (2, 37, (12.3456789, -7.25))])
def test_central_generator_bit_exact_against_oracle(L, dim, N, omega):
    A = L.convdiff(dim, N, omega, scheme=L.SCHEME_CENTRAL)
    rp, ci, v = convdiff_csr(dim, N, omega, scheme="central")
    assert np.array_equal(A.rowptr, rp)
    assert np.array_equal(A.colind, ci)
    assert np.array_equal(A.val.view(np.uint64), v.view(np.uint64))


def test_generator_rejects_bad_arguments(L):
    lib = L.lib()
    n = ctypes.c_int64()
    nnz = ctypes.c_int64()
    assert lib.lradi_convdiff_size(4, 10, ctypes.byref(n), ctypes.byref(nnz)) == L.EINVAL
    assert lib.lradi_convdiff_size(2, 0, ctypes.byref(n), ctypes.byref(nnz)) == L.EINVAL
    assert lib.lradi_convdiff_size(3, 64, ctypes.byref(n), ctypes.byref(nnz)) == L.OK
    assert n.value == 262144 and nnz.value == 1810432
    assert b"dim" in lib.lradi_strerror(L.EINVAL) or lib.lradi_strerror(L.EINVAL)


def test_default_options_are_the_paper_settings(L):
    o = L.default_opts()
    assert o.tol == 1e-8 and o.delta_min == 1e-8 / 20 and o.delta_max == 0.1
    assert o.kmax == 50 and o.xi == 1.0 and o.selection == L.SEL_MID and o.backlook == 1
    # the dynamic selections run in the balanced frame unless rescale = 1 asks
    # for the paper's own frame
    assert o.rescale == 2
    # no preconditioner unless asked for; its sweeps run in pairs where they tile
    assert o.precond == L.PRECOND_NONE and o.precond_pairs == 1


# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def ST(tmp_path_factory):
    d = tmp_path_factory.mktemp("st")
    so = str(d / "st.so")
    src = os.path.join(ROOT, "tests", "native", "selftest_small.cpp")
    subprocess.run(["g++", "-O2", "-shared", "-fPIC", "-std=c++17", "-ffp-contract=off",
                    "-o", so, src], check=True)
    lib = ctypes.CDLL(so)
    D = ctypes.c_double
    P = ctypes.POINTER(D)
    lib.st_lmax.restype = D
    lib.st_lmax_ms16.restype = D
    lib.st_lmax_ms64.restype = D
    lib.st_lmax_prod.restype = D
    lib.st_lmax_prod_chol.restype = D
    lib.st_tol.argtypes = [ctypes.c_int] * 4 + [D] * 5 + [ctypes.c_int] + [D] * 5 + [ctypes.c_int, P, P]
    lib.st_gap.argtypes = [P, P] + [D] * 5
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _spd(rng, n, cond=1e3):
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.geomspace(1.0, cond, n)
    return (Q * ev) @ Q.T


@pytest.mark.parametrize("n", range(1, 9))
def test_cholesky_and_inverse(ST, n):
    rng = np.random.default_rng(n)
    G = np.ascontiguousarray(_spd(rng, n))
    S = np.zeros((n, n))
    assert ST.st_chol(_p(G), _p(S), n, ctypes.c_double(1e-24)) == 0
    assert np.allclose(S, np.linalg.cholesky(G).T, rtol=1e-12, atol=1e-12)
    X = np.zeros((n, n))
    ST.st_trinv(_p(S), _p(X), n)
    assert np.allclose(X @ S, np.eye(n), atol=1e-12)


def test_cholesky_regularises_dependent_columns(ST):
    rng = np.random.default_rng(3)
    U = rng.standard_normal((50, 4))
    U[:, 2] = U[:, 0] + U[:, 1]              # exactly dependent column
    G = np.ascontiguousarray(U.T @ U)
    S = np.zeros((4, 4))
    reg = ST.st_chol(_p(G), _p(S), 4, ctypes.c_double(1e-24))
    assert reg >= 1 and np.all(np.isfinite(S)) and np.all(np.diag(S) > 0)
    G[1, 1] = np.nan
    assert ST.st_chol(_p(G), _p(S), 4, ctypes.c_double(1e-24)) == -1


@pytest.mark.parametrize("n", range(1, 9))
def test_jacobi_eigen(ST, n):
    rng = np.random.default_rng(10 + n)
    A = rng.standard_normal((n, n))
    A = np.ascontiguousarray(A + A.T)
    want = np.linalg.eigvalsh(A)
    W = A.copy()
    Q = np.zeros((n, n))
    ST.st_jacobi(_p(W), _p(Q), n)
    assert np.allclose(np.sort(np.diag(W)), want, rtol=1e-12, atol=1e-12 * np.abs(want).max())
    assert np.allclose(Q @ np.diag(np.diag(W)) @ Q.T, A, atol=1e-11 * np.abs(A).max())
    G = np.ascontiguousarray(_spd(rng, n, 1e6))
    assert ST.st_lmax(_p(G), n) == pytest.approx(np.linalg.eigvalsh(G).max(), rel=1e-13)


@pytest.mark.parametrize("n", range(1, 9))
def test_lambda_max_of_gram_product_is_lowrank_norm(ST, n):
    rng = np.random.default_rng(20 + n)
    Wm, Tm = rng.standard_normal((40, n)), rng.standard_normal((30, n))
    Gw, Gt = np.ascontiguousarray(Wm.T @ Wm), np.ascontiguousarray(Tm.T @ Tm)
    got = np.sqrt(ST.st_lmax_prod(_p(Gw), _p(Gt), n))
    assert got == pytest.approx(np.linalg.norm(Wm @ Tm.T, 2), rel=1e-12)


@pytest.mark.parametrize("n", range(1, 9))
def test_lambda_max_of_gram_product_through_cholesky(ST, n):
    """The step end's form of ||W T^T||_2^2: L^T (T^T T) L with W^T W = L L^T,
    also for rank-deficient W (a repeated and a zero column) and T = 0."""
    rng = np.random.default_rng(30 + n)
    Wm, Tm = rng.standard_normal((40, n)), rng.standard_normal((30, n))
    cases = [(Wm, Tm)]
    if n >= 3:
        Wd = Wm.copy()
        Wd[:, 1] = Wd[:, 0]
        Wd[:, 2] = 0.0
        cases.append((Wd, Tm))
    cases.append((Wm, np.zeros_like(Tm)))
    for W, T in cases:
        Gw, Gt = np.ascontiguousarray(W.T @ W), np.ascontiguousarray(T.T @ T)
        got = np.sqrt(max(ST.st_lmax_prod_chol(_p(Gw), _p(Gt), n), 0.0))
        want = np.linalg.norm(W @ T.T, 2)
        assert got == pytest.approx(want, rel=1e-12, abs=1e-14 * np.linalg.norm(W) * np.linalg.norm(T))


@pytest.mark.parametrize("n", range(1, 9))
def test_householder_block(ST, n):
    rng = np.random.default_rng(30 + n)
    M0 = rng.standard_normal((2 * n, n))
    M0[n:] = np.triu(M0[n:])
    M = np.ascontiguousarray(M0.copy())
    Q = np.zeros((2 * n, 2 * n))
    ST.st_house(_p(M), _p(Q), n)
    assert np.allclose(Q.T @ Q, np.eye(2 * n), atol=1e-14)
    assert np.allclose(Q.T @ M0, M, atol=1e-13)
    assert np.allclose(M[n:], 0.0) and np.allclose(np.tril(M[:n], -1), 0.0)


@pytest.mark.parametrize("seed", range(30))
def test_controller_matches_oracle(ST, seed):
    rng = np.random.default_rng(seed)
    sel_names = ["relative", "fixed", "mid", "tightA", "tightB", "sym"]
    sel = int(rng.integers(0, 6))
    bl = int(rng.integers(0, 2))
    pabs = int(rng.integers(0, 2))
    k = int(rng.integers(1, 60))
    nw, nt = 10 ** rng.uniform(-6, 3, 2)
    u, v = 10 ** rng.uniform(-14, -6, 2)
    eps = 10 ** rng.uniform(-10, -2)
    kmax, xi = int(rng.integers(10, 120)), float(rng.uniform(0.1, 1.0))
    dmin, dmax, dfix, rho = 5e-10, 0.1, 5e-10, 1e-12
    dA, dB = ctypes.c_double(), ctypes.c_double()
    bal = int(rng.integers(0, 2))
    ST.st_tol(sel, bl, pabs, k, nw, nt, u, v, eps, kmax, xi, dmin, dmax, dfix, rho, bal,
              ctypes.byref(dA), ctypes.byref(dB))
    wA, wB = OC.tolerances(sel_names[sel], k, nw, nt, u, v, eps, kmax=kmax, xi=xi, dmin=dmin,
                           dmax=dmax, backlook=bool(bl), fixed=dfix, rho=rho,
                           paper_abs=bool(pabs), balance=bool(bal))
    assert dA.value == pytest.approx(wA, rel=1e-13)
    assert dB.value == pytest.approx(wB, rel=1e-13)
    uu, vv = ctypes.c_double(u), ctypes.c_double(v)
    ST.st_gap(ctypes.byref(uu), ctypes.byref(vv), -7.5, nw, nt, 1e-9, 3e-9)
    wu, wv = OC.update_gap(u, v, -7.5, nw, nt, 1e-9, 3e-9)
    assert uu.value == pytest.approx(wu, rel=1e-14) and vv.value == pytest.approx(wv, rel=1e-14)


@pytest.mark.parametrize("n", range(1, 9))
def test_lambda_max_sym_hard_cases(ST, n):
    """The largest eigenvalue to 1e-13 relative on PSD matrices of wide
    condition, rank-deficient ones, repeated eigenvalues, diagonal ones, and
    scales near the ends of the double range; the zero matrix gives 0.  The
    same for the multisection the GPU spreads over 16 and 64 lanes (its
    rounds run here one point after another)."""
    rng = np.random.default_rng(300 + n)
    cases = [_spd(rng, n, 1e12), np.diag(rng.uniform(0.1, 5.0, n)), np.eye(n) * 3.7]
    X = rng.standard_normal((n, max(1, n // 2)))
    cases.append(X @ X.T)                      # rank n // 2
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.full(n, 2.0)
    ev[0] = 1e-9
    cases.append(Q @ np.diag(ev) @ Q.T)        # repeated top eigenvalue
    B = _spd(rng, n, 1e3)
    cases += [B * 1e-280, B * 1e280]
    for G in cases:
        G = np.ascontiguousarray((G + G.T) / 2)
        want = np.linalg.eigvalsh(G).max()
        for f in (ST.st_lmax, ST.st_lmax_ms16, ST.st_lmax_ms64):
            assert f(_p(G), n) == pytest.approx(want, rel=1e-13, abs=1e-300)
    Z = np.zeros((n, n))
    for f in (ST.st_lmax, ST.st_lmax_ms16, ST.st_lmax_ms64):
        assert f(_p(Z), n) == 0.0
