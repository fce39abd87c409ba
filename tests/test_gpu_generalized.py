"""GPU parity of the generalized equation A X C + M X B = -f g^T (eq. (gsylv),
iteration (lradi_g)) against the oracle, through the C ABI."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import controller as OC
from oracle import fadi as OF
from oracle.convdiff import convdiff_matrix
from paper_2312_02891_amd import workloads as WL

from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_2312_02891_amd import lradi
    return lradi


@pytest.fixture(scope="module")
def ctx(L):
    c = L.Context(0)
    yield c
    c.close()


def _mass(dim, N):
    rp, ci, v = WL.mass_csr(dim, N)
    n = len(rp) - 1
    return (rp, ci, v), sp.csr_matrix((v, ci, rp), shape=(n, n))


def setup(P, L):
    HA = L.convdiff(P.A.dim, P.A.N, P.A.omega)
    HB = L.convdiff(P.B.dim, P.B.N, P.B.omega)
    A = convdiff_matrix(P.A.dim, P.A.N, P.A.omega)
    B = convdiff_matrix(P.B.dim, P.B.N, P.B.omega)
    (mrp, mci, mv), M = _mass(P.A.dim, P.A.N)
    (crp, cci, cv), C = _mass(P.B.dim, P.B.N)
    HM, HC = L.HostCsr(mrp, mci, mv), L.HostCsr(crp, cci, cv)
    f, g = WL.rhs_factors(P.seed, P.A.n, P.B.n, P.r)
    pA, pB = WL.wachspress_shifts(P.A, P.B, P.nshifts, massA=True, massB=True)
    return HA, HB, HM, HC, A, B, M, C, f, g, pA, pB


@pytest.mark.parametrize("name,precision", [("GEN_SMALL", "fp64"), ("GEN_SMALL", "fp32"),
                                            ("GEN_SMALL_3D", "fp64"), ("GEN_SMALL_3D", "fp32")])
def test_generalized_matches_oracle(L, ctx, name, precision):
    """Relaxed inner tolerances: the run takes the oracle's steps (+-1), X is
    within 1e-6 of the direct-solve iterate at the same step, the true
    residual of eq. (gsylv) is below tau, and the recorded tolerances and gap
    estimates (with ||M z||, ||C^T y||) follow the oracle's formulas."""
    say("generalized", name, precision)
    P = getattr(WL, name)
    HA, HB, HM, HC, A, B, M, C, f, g, pA, pB = setup(P, L)
    o = L.default_opts(tol=P.tol, precision=precision)
    res = ctx.solve(HA, HB, to_dev(f), to_dev(g), pA, pB, o, M=HM, C=HC)
    assert res.status == L.OK
    full = OF.fadi(A, B, f, g, pA, pB, tol=P.tol, kmax=200, M=M, C=C)
    ora = OF.fadi(A, B, f, g, pA, pB, tol=P.tol, kmax=200, kfixed=res.k, M=M, C=C)
    Zg, dg, Yg = res.factors()
    xerr = OF.lowrank_diff_fro(Zg, dg, Yg, ora.Z, ora.D(), ora.Y) / OF.lowrank_fro(ora.Z, ora.D(), ora.Y)
    fs, gs = OF.rescale_rhs(f, g)
    true = OF.lowrank_residual_norm(A, B, fs, gs, Zg, dg, Yg, M=M, C=C) / ora.norm_fg
    say("  k", res.k, "oracle", full.k, "X err", xerr, "true", true)
    assert abs(res.k - full.k) <= 1
    assert xerr <= 1e-6
    assert true <= P.tol
    assert res.norm_fg == pytest.approx(ora.norm_fg, rel=1e-12)
    u = v = 0.0
    eps = P.tol * res.norm_fg
    for row in res.history():
        dA, dB = OC.tolerances("mid", int(row[0]), row[10], row[11], u, v, eps, balance=True)
        assert row[2] == pytest.approx(dA, rel=1e-12) and row[3] == pytest.approx(dB, rel=1e-12)
        assert row[4] <= row[2] * (1 + 1e-12) and row[5] <= row[3] * (1 + 1e-12)
        u, v = OC.update_gap(u, v, row[14], row[12], row[13], row[4], row[5])
        assert row[8] == pytest.approx(u, rel=1e-12) and row[9] == pytest.approx(v, rel=1e-12)


def test_generalized_true_residual_matches_oracle(L, ctx):
    """lradi_residual_gen (Golub-Kahan-Lanczos through the factors, with M
    and C) equals the oracle's exact low-rank evaluation, for the converged
    solution and for arbitrary factors with a large residual."""
    P = WL.GEN_SMALL
    HA, HB, HM, HC, A, B, M, C, f, g, pA, pB = setup(P, L)
    fd, gd = to_dev(f), to_dev(g)
    res = ctx.solve(HA, HB, fd, gd, pA, pB, L.default_opts(tol=P.tol), M=HM, C=HC)
    gpu = ctx.residual(HA, HB, fd, gd, res, M=HM, C=HC)
    Z, d, Y = res.factors()
    ora = OF.lowrank_residual_norm(A, B, f, g, Z, d, Y, M=M, C=C) / OF.lowrank_product_norm(f, g)
    say("  residual gpu", gpu, "oracle", ora)
    assert gpu == pytest.approx(ora, rel=1e-6)
    rng = np.random.default_rng(9)
    k, r = 3, P.r
    Zs, Ys = rng.standard_normal((k, P.A.n, r)), rng.standard_normal((k, P.B.n, r))
    gam = rng.uniform(1.0, 40.0, k)
    fake = type("R", (), {})()
    import torch
    Zd = torch.from_numpy(np.ascontiguousarray(Zs)).cuda()
    Yd = torch.from_numpy(np.ascontiguousarray(Ys)).cuda()
    fake.Zptr, fake.Yptr, fake.k = Zd.data_ptr(), Yd.data_ptr(), k
    fake.gammas = lambda: gam
    gpu2 = ctx.residual(HA, HB, fd, gd, fake, M=HM, C=HC)
    Zc = np.concatenate(list(Zs), axis=1)
    Yc = np.concatenate(list(Ys), axis=1)
    ora2 = OF.lowrank_residual_norm(A, B, f, g, Zc, np.repeat(gam, r), Yc, M=M, C=C) / \
        OF.lowrank_product_norm(f, g)
    assert gpu2 == pytest.approx(ora2, rel=1e-9)


def test_exact_tolerance_reproduces_direct_iteration(L, ctx):
    """Inner solves to 1e-12 relative: every step's computed residual equals
    the oracle's and the norms ||M z_k||, ||C^T y_k|| recorded on the device
    equal the oracle's."""
    P = WL.GEN_SMALL
    HA, HB, HM, HC, A, B, M, C, f, g, pA, pB = setup(P, L)
    o = L.default_opts(tol=P.tol, selection="relative", rho=1e-12)
    res = ctx.solve(HA, HB, to_dev(f), to_dev(g), pA, pB, o, M=HM, C=HC)
    ora = OF.fadi(A, B, f, g, pA, pB, tol=P.tol, kmax=200, M=M, C=C)
    assert res.k == ora.k
    h = res.history()
    assert np.allclose(h[:, 15], ora.res_hist, rtol=1e-7)
    assert np.allclose(h[:, 12], ora.nMz, rtol=1e-9)
    assert np.allclose(h[:, 13], ora.nCy, rtol=1e-9)


def test_identity_mass_matches_plain_solve(L, ctx):
    """M = C = I given as matrices (so the pencil path runs) gives the plain
    iteration's steps and X to rounding."""
    P = WL.SMALL_2D
    HA = L.convdiff(2, P.A.N, P.A.omega)
    HB = L.convdiff(2, P.B.N, P.B.omega)
    n, m = P.A.n, P.B.n
    I_n = L.HostCsr(np.arange(n + 1), np.arange(n), np.ones(n))
    I_m = L.HostCsr(np.arange(m + 1), np.arange(m), np.ones(m))
    f, g = WL.rhs_factors(P.seed, n, m, P.r)
    pA, pB = WL.wachspress_shifts(P.A, P.B, P.nshifts)
    o = L.default_opts(tol=P.tol)
    plain = ctx.solve(HA, HB, to_dev(f), to_dev(g), pA, pB, o)
    gen = ctx.solve(HA, HB, to_dev(f), to_dev(g), pA, pB, o, M=I_n, C=I_m)
    assert gen.k == plain.k
    Zp, dp, Yp = plain.factors()
    Zg, dg, Yg = gen.factors()
    assert OF.lowrank_diff_fro(Zg, dg, Yg, Zp, dp, Yp) <= 1e-9 * OF.lowrank_fro(Zp, dp, Yp)


def test_generalized_transposed_inputs_and_batch(L, ctx):
    """B^T and C^T passed with b_is_transposed give the same bits as B and C;
    a batch mixing generalized and plain problems equals their solo runs."""
    P = WL.GEN_SMALL
    HA, HB, HM, HC, A, B, M, C, f, g, pA, pB = setup(P, L)
    fd, gd = to_dev(f), to_dev(g)
    o = L.default_opts(tol=P.tol)
    ref = ctx.solve(HA, HB, fd, gd, pA, pB, o, M=HM, C=HC)
    Bt = sp.csr_matrix(B.T)
    Ct = sp.csr_matrix(C.T)
    Bt.sort_indices()
    Ct.sort_indices()
    HBt = L.HostCsr(Bt.indptr, Bt.indices, Bt.data)
    HCt = L.HostCsr(Ct.indptr, Ct.indices, Ct.data)
    ot = L.default_opts(tol=P.tol, b_is_transposed=1)
    tr = ctx.solve(HA, HBt, fd, gd, pA, pB, ot, M=HM, C=HCt)
    for a, b in zip(ref.factors(), tr.factors()):
        assert np.array_equal(a, b)
    Q = WL.SMALL_3D
    HA2, HB2 = L.convdiff(3, Q.A.N, Q.A.omega), L.convdiff(3, Q.B.N, Q.B.omega)
    f2, g2 = WL.rhs_factors(Q.seed, Q.A.n, Q.B.n, Q.r)
    pA2, pB2 = WL.wachspress_shifts(Q.A, Q.B, Q.nshifts)
    f2d, g2d = to_dev(f2), to_dev(g2)
    solo2 = ctx.solve(HA2, HB2, f2d, g2d, pA2, pB2, L.default_opts(tol=Q.tol))
    res, st = ctx.batch_solve([(HA, HB, fd, gd, pA, pB, P.tol, HM, HC),
                               (HA2, HB2, f2d, g2d, pA2, pB2, Q.tol)], o)
    for a, b in zip(res[0].factors(), ref.factors()):
        assert np.array_equal(a, b)
    for a, b in zip(res[1].factors(), solo2.factors()):
        assert np.array_equal(a, b)
