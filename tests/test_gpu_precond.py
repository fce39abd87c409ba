"""GPU parity of the right-preconditioned inner block GMRES (red-black
ILU(0) with Jacobi sweeps on the Schur complement) against the oracle's
preconditioner and the preconditioned block minimal-residual definition,
and of the LR-ADI iteration run with it."""
import ctypes

import numpy as np
import pytest

from oracle import controller as OC
from oracle import fadi as OF
from oracle import precond as OP
from oracle.convdiff import convdiff_matrix
from oracle.gmres_ref import block_gmres_iterate
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


@pytest.mark.parametrize("dim,N,omega", [(2, 15, (8.0, -5.0)), (3, 7, (4.0, -2.0, 6.0))])
@pytest.mark.parametrize("r,j,sweeps", [(1, 1, 0), (2, 3, 0), (4, 6, 0), (3, 4, 2), (8, 3, 1), (4, 5, 5),
                                         (2, 4, 24), (1, 3, 7)])
def test_first_cycle_equals_preconditioned_minres_definition(L, ctx, dim, N, omega, r, j, sweeps):
    """restart = j, step cap j: the returned Z is the minimiser of
    ||W - S Z||_F over M K_j(S M, W), with M the oracle's red-black ILU(0)
    (plus sweeps), to 1e-9."""
    say("precond first cycle", dim, N, r, j, sweeps)
    H = L.convdiff(dim, N, omega)
    A = convdiff_matrix(dim, N, omega)
    W = np.random.default_rng(300 + r * 10 + j).standard_normal((H.n, r))
    shift = -300.0
    o = L.default_opts(restart=j, max_inner=j, precond="rbilu0", precond_sweeps=sweeps)
    Zs, stats, st = ctx.shifted_solve([H], [shift], [to_dev(W)], [0.0], o)
    Z = Zs[0].cpu().numpy()
    want = block_gmres_iterate(A, shift, W, j, precond=lambda X: OP.rb_precond_apply(A, shift, X, sweeps))
    assert stats[0]["steps"] == j
    assert np.linalg.norm(Z - want) <= 1e-9 * np.linalg.norm(want)


@pytest.mark.parametrize("r,j,sweeps", [(2, 3, 5), (4, 4, 24), (1, 2, 2), (8, 2, 3)])
def test_first_cycle_with_paired_sweeps_equals_definition(L, ctx, r, j, sweeps):
    """A 2-D grid above the pairing size (182^2 = 33124 rows, sweeps run two
    per launch, an odd count ending with a single one): the first cycle's Z
    is the oracle's preconditioned block minimal-residual iterate, to 1e-9."""
    say("precond first cycle, paired", r, j, sweeps)
    dim, N, omega = 2, 182, (30.0, -12.0)
    H = L.convdiff(dim, N, omega)
    A = convdiff_matrix(dim, N, omega)
    W = np.random.default_rng(500 + r * 10 + j).standard_normal((H.n, r))
    shift = -2000.0
    o = L.default_opts(restart=j, max_inner=j, precond="rbilu0", precond_sweeps=sweeps, profile=1)
    ctx.profile_reset()
    Zs, stats, st = ctx.shifted_solve([H], [shift], [to_dev(W)], [0.0], o)
    launches = ctx.profile_read(L.PROF_PRECOND)[1]
    Z = Zs[0].cpu().numpy()
    want = block_gmres_iterate(A, shift, W, j, precond=lambda X: OP.rb_precond_apply(A, shift, X, sweeps))
    say("  preconditioner launches", launches)
    assert stats[0]["steps"] == j
    assert np.linalg.norm(Z - want) <= 1e-9 * np.linalg.norm(want)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shift", [-2.0e5, -3.0e3, -25.0])
def test_preconditioned_solve_reaches_delta_with_fewer_steps(L, ctx, prec, shift):
    """Config 2's A (n = 65536, r = 4): the FP64 residual of the returned
    block is below delta (checked by the oracle's sparse product), and the
    preconditioned solve needs fewer block steps than the plain one."""
    P = WL.C2
    H = L.convdiff(P.A.dim, P.A.N, P.A.omega)
    A = convdiff_matrix(P.A.dim, P.A.N, P.A.omega)
    W = np.random.default_rng(7).standard_normal((H.n, 4))
    delta = 1e-9 * np.linalg.norm(W, 2)
    steps = {}
    for sweeps in (None, 0, 2):
        kw = {} if sweeps is None else dict(precond="rbilu0", precond_sweeps=sweeps)
        o = L.default_opts(precision=prec, restart=30, max_inner=6000, **kw)
        Zs, stats, st = ctx.shifted_solve([H], [shift], [to_dev(W)], [delta], o)
        Z = Zs[0].cpu().numpy()
        rn = np.linalg.norm(W - (A @ Z + shift * Z), 2)
        assert st == L.OK and stats[0]["status"] == 0
        assert rn <= delta * (1 + 1e-8)
        steps[sweeps] = stats[0]["steps"]
    say("  steps plain / rbilu0 / +2 sweeps", prec, shift, steps[None], steps[0], steps[2])
    assert steps[0] < steps[None] and steps[2] < steps[0]


@pytest.mark.parametrize("steps", [dict(precond_sweeps=1), dict(precond_sweeps=6, precond_poly=1)],
                         ids=["jacobi1", "chebyshev6"])
def test_preconditioned_batch_equals_solo_runs(L, ctx, steps):
    """Systems of different n, r, dimension and shift share launches with
    the preconditioner (Jacobi sweeps, or Chebyshev steps whose bounds each
    system computes for its own shift); each result is bit-identical to its
    solo run."""
    specs = [(2, 21, (4.0, -9.0), 1, -50.0), (2, 40, (-20.0, 3.0), 3, -900.0),
             (3, 9, (2.0, 2.0, -1.0), 8, -120.0), (2, 64, (30.0, 30.0), 5, -4000.0)]
    mats, Ws, shifts, deltas = [], [], [], []
    for i, (dim, N, om, r, s) in enumerate(specs):
        H = L.convdiff(dim, N, om)
        mats.append(H)
        Ws.append(to_dev(np.random.default_rng(400 + i).standard_normal((H.n, r))))
        shifts.append(s)
        deltas.append(1e-9 * float(np.linalg.norm(Ws[-1].cpu().numpy(), 2)))
    o = L.default_opts(restart=12, max_inner=3000, precond="rbilu0", **steps)
    Zb, sb, _ = ctx.shifted_solve(mats, shifts, Ws, deltas, o)
    for i in range(len(specs)):
        Zi, si, _ = ctx.shifted_solve([mats[i]], [shifts[i]], [Ws[i]], [deltas[i]], o)
        assert si[0]["steps"] == sb[i]["steps"]
        assert np.array_equal(Zi[0].cpu().numpy(), Zb[i].cpu().numpy())


@pytest.mark.parametrize("name,precision,sweeps,poly", [("SMALL_2D", "fp64", 0, 0), ("SMALL_2D", "fp32", 2, 0),
                                                        ("SMALL_3D", "fp64", 2, 0), ("SMALL_3D", "fp32", 0, 0),
                                                        ("SMALL_2D", "fp64", 24, 0), ("SMALL_2D", "fp32", 9, 0),
                                                        ("SMALL_2D", "fp64", 12, 1), ("SMALL_3D", "fp32", 8, 1)])
def test_adi_with_preconditioned_inner_solves_matches_oracle(L, ctx, name, precision, sweeps, poly):
    """Algorithm 1 with preconditioned inner solves: the oracle's steps
    (+-1), X within 1e-6 of the direct-solve iterate, true residual below
    tau, tolerances and gap estimates as the oracle's formulas."""
    say("adi precond", name, precision, sweeps, poly)
    P = getattr(WL, name)
    HA = L.convdiff(P.A.dim, P.A.N, P.A.omega)
    HB = L.convdiff(P.B.dim, P.B.N, P.B.omega)
    A = convdiff_matrix(P.A.dim, P.A.N, P.A.omega)
    B = convdiff_matrix(P.B.dim, P.B.N, P.B.omega)
    f, g = WL.rhs_factors(P.seed, P.A.n, P.B.n, P.r)
    pA, pB = WL.wachspress_shifts(P.A, P.B, P.nshifts)
    o = L.default_opts(tol=P.tol, precision=precision, precond="rbilu0", precond_sweeps=sweeps, precond_poly=poly)
    res = ctx.solve(HA, HB, to_dev(f), to_dev(g), pA, pB, o)
    assert res.status == L.OK
    full = OF.fadi(A, B, f, g, pA, pB, tol=P.tol, kmax=100)
    ora = OF.fadi(A, B, f, g, pA, pB, kfixed=res.k)
    Z, d, Y = res.factors()
    xerr = OF.lowrank_diff_fro(Z, d, Y, ora.Z, ora.D(), ora.Y) / OF.lowrank_fro(ora.Z, ora.D(), ora.Y)
    true = OF.lowrank_residual_norm(A, B, f, g, Z, d, Y) / ora.norm_fg
    say("  k", res.k, "oracle", full.k, "X err", xerr, "true", true)
    assert abs(res.k - full.k) <= 1 and xerr <= 1e-6 and true <= P.tol
    u = v = 0.0
    eps = P.tol * res.norm_fg
    for row in res.history():
        dA, dB = OC.tolerances("mid", int(row[0]), row[10], row[11], u, v, eps, balance=True)
        assert row[2] == pytest.approx(dA, rel=1e-12) and row[3] == pytest.approx(dB, rel=1e-12)
        assert row[4] <= row[2] * (1 + 1e-12) and row[5] <= row[3] * (1 + 1e-12)
        u, v = OC.update_gap(u, v, row[14], row[12], row[13], row[4], row[5])


@pytest.mark.parametrize("steps", [dict(precond_sweeps=1), dict(precond_sweeps=8, precond_poly=1)],
                         ids=["jacobi1", "chebyshev8"])
def test_preconditioned_lyapunov_equals_its_oracle(L, ctx, steps):
    """The Lyapunov path with the preconditioner: X within 1e-6 of the
    Lyapunov oracle, true residual below tau."""
    from oracle import lyap as OL
    P = WL.LYAP_SMALL
    HA = L.convdiff(P.A.dim, P.A.N, P.A.omega)
    A = convdiff_matrix(P.A.dim, P.A.N, P.A.omega)
    f, p = WL.lyap_inputs(P)
    o = L.default_opts(tol=P.tol, selection="sym", precond="rbilu0", **steps)
    res = ctx.solve_lyap(HA, to_dev(f), p, o)
    ora = OL.lyap_adi(A, f, p, kfixed=res.k)
    Z, d, _ = res.factors()
    xerr = OF.lowrank_diff_fro(Z, d, Z, ora.Z, ora.D(), ora.Z) / OF.lowrank_fro(ora.Z, ora.D(), ora.Z)
    true = OF.lowrank_residual_norm(A, A.T, f, f, Z, d, Z) / OF.lowrank_product_norm(f, f)
    assert res.status == L.OK and xerr <= 1e-6 and true <= P.tol


def test_preconditioner_argument_errors(L, ctx):
    """A non-bipartite pattern and an out-of-range sweep count give
    LRADI_EINVAL before any launch."""
    P = WL.GEN_SMALL
    HA = L.convdiff(P.A.dim, P.A.N, P.A.omega)
    HM = L.HostCsr(*WL.mass_csr(P.A.dim, P.A.N))
    o = L.default_opts(precond="rbilu0")
    W = to_dev(np.ones((HM.n, 1)))
    with pytest.raises(L.LradiError) as e:
        ctx.shifted_solve([HM], [1.0], [W], [1e-8], o)
    assert e.value.status == L.EINVAL
    with pytest.raises(L.LradiError) as e:
        ctx.shifted_solve([HA], [-10.0], [to_dev(np.ones((HA.n, 1)))], [1e-8],
                          L.default_opts(precond="rbilu0", precond_sweeps=65))
    assert e.value.status == L.EINVAL
    with pytest.raises(L.LradiError) as e:
        ctx.shifted_solve([HA], [-10.0], [to_dev(np.ones((HA.n, 1)))], [1e-8],
                          L.default_opts(precond="rbilu0", precond_pairs=2))
    assert e.value.status == L.EINVAL


def _gen_setup(L, P):
    import scipy.sparse as sp
    HA = L.convdiff(P.A.dim, P.A.N, P.A.omega)
    HB = L.convdiff(P.B.dim, P.B.N, P.B.omega)
    A = convdiff_matrix(P.A.dim, P.A.N, P.A.omega)
    B = convdiff_matrix(P.B.dim, P.B.N, P.B.omega)
    mA, mB = WL.mass_csr(P.A.dim, P.A.N), WL.mass_csr(P.B.dim, P.B.N)
    HM, HC = L.HostCsr(*mA), L.HostCsr(*mB)
    M = sp.csr_matrix((mA[2], mA[1], mA[0]), shape=(P.A.n, P.A.n))
    C = sp.csr_matrix((mB[2], mB[1], mB[0]), shape=(P.B.n, P.B.n))
    f, g = WL.rhs_factors(P.seed, P.A.n, P.B.n, P.r)
    pA, pB = WL.wachspress_shifts(P.A, P.B, P.nshifts, massA=True, massB=True)
    return HA, HB, HM, HC, A, B, M, C, f, g, pA, pB


@pytest.mark.parametrize("name,precision,sweeps,poly", [("GEN_SMALL", "fp64", 4, 0), ("GEN_SMALL", "fp32", 0, 0),
                                                        ("GEN_SMALL_3D", "fp64", 2, 0), ("GEN_SMALL_3D", "fp32", 5, 0),
                                                        ("GEN_SMALL", "fp64", 10, 1), ("GEN_SMALL_3D", "fp32", 6, 1)])
def test_generalized_with_lumped_mass_preconditioner_matches_oracle(L, ctx, name, precision, sweeps, poly):
    """Pencils A + s M preconditioned by the red-black ILU(0) of
    A + s diag(M 1): the generalized iteration keeps the oracle's steps
    (+-1), X within 1e-6 of the direct-solve iterate and a true residual
    below tau, with fewer inner steps than unpreconditioned."""
    say("generalized precond", name, precision, sweeps, poly)
    P = getattr(WL, name)
    HA, HB, HM, HC, A, B, M, C, f, g, pA, pB = _gen_setup(L, P)
    fd, gd = to_dev(f), to_dev(g)
    o = L.default_opts(tol=P.tol, precision=precision, precond="rbilu0", precond_sweeps=sweeps, precond_poly=poly)
    res = ctx.solve(HA, HB, fd, gd, pA, pB, o, M=HM, C=HC)
    plain = ctx.solve(HA, HB, fd, gd, pA, pB, L.default_opts(tol=P.tol, precision=precision), M=HM, C=HC)
    assert res.status == L.OK
    full = OF.fadi(A, B, f, g, pA, pB, tol=P.tol, kmax=200, M=M, C=C)
    ora = OF.fadi(A, B, f, g, pA, pB, tol=P.tol, kmax=200, kfixed=res.k, M=M, C=C)
    Z, d, Y = res.factors()
    xerr = OF.lowrank_diff_fro(Z, d, Y, ora.Z, ora.D(), ora.Y) / OF.lowrank_fro(ora.Z, ora.D(), ora.Y)
    fs, gs = OF.rescale_rhs(f, g)
    true = OF.lowrank_residual_norm(A, B, fs, gs, Z, d, Y, M=M, C=C) / ora.norm_fg
    hp, hn = res.history(), plain.history()
    say("  k", res.k, "oracle", full.k, "X err", xerr, "true", true, "inner", hp[:, 6].sum() + hp[:, 7].sum(),
        "plain", hn[:, 6].sum() + hn[:, 7].sum())
    assert abs(res.k - full.k) <= 1 and xerr <= 1e-6 and true <= P.tol
    assert hp[:, 6].sum() + hp[:, 7].sum() < hn[:, 6].sum() + hn[:, 7].sum()


@pytest.mark.parametrize("name,precision,sweeps,gen,poly", [("C2", "fp64", 24, False, 0), ("C2", "fp32", 5, False, 0),
                                                            ("C2", "fp64", 2, False, 0), ("C2", "fp64", 7, True, 0),
                                                            ("SMALL_2D", "fp64", 24, False, 0),
                                                            ("SMALL_3D", "fp64", 3, False, 0),
                                                            ("C2", "fp64", 48, False, 1), ("C2", "fp32", 5, False, 1),
                                                            ("C2", "fp64", 2, False, 1), ("C2", "fp32", 16, False, 1),
                                                            ("C2", "fp64", 7, True, 1),
                                                            ("SMALL_2D", "fp64", 9, False, 1)])
def test_paired_sweeps_equal_single_sweeps_bitwise(L, ctx, name, precision, sweeps, gen, poly):
    """Two Jacobi sweeps or Chebyshev steps per launch (the first over each
    tile's region into workgroup memory) give the same factors, history and
    inner step counts as one per launch, bit for bit (Chebyshev steps: the
    paired run keeps its iterates in four blocks, the single one in two,
    and an odd count ends with a single step in the four blocks).  The pairs
    are taken on 2-D grids of at least 32768 rows (fewer preconditioner
    launches, counted by the profiler); not on smaller matrices (no tiles)
    nor on 3-D grids, whose regions are about twice their tiles."""
    say("paired sweeps", name, precision, sweeps, "chebyshev" if poly else "jacobi")
    P = getattr(WL, name)
    if gen:
        HA, HB, HM, HC, *_rest = _gen_setup(L, P)
        f, g = WL.rhs_factors(P.seed, P.A.n, P.B.n, P.r)
        pA, pB = WL.wachspress_shifts(P.A, P.B, P.nshifts, massA=True, massB=True)
        kw = dict(M=HM, C=HC)
    else:
        HA = L.convdiff(P.A.dim, P.A.N, P.A.omega)
        HB = L.convdiff(P.B.dim, P.B.N, P.B.omega)
        f, g = WL.rhs_factors(P.seed, P.A.n, P.B.n, P.r)
        pA, pB = WL.wachspress_shifts(P.A, P.B, P.nshifts)
        kw = {}
    fd, gd = to_dev(f), to_dev(g)
    runs = []
    for pairs in (1, 0):
        o = L.default_opts(tol=P.tol, precision=precision, precond="rbilu0", precond_sweeps=sweeps,
                           precond_pairs=pairs, precond_poly=poly, profile=1, kmax=100)
        ctx.profile_reset()
        res = ctx.solve(HA, HB, fd, gd, pA, pB, o, **kw)
        assert res.status == L.OK
        # preconditioner launches per tick: the number of ticks the host
        # issues depends on how far ahead of the device it runs, so the
        # launches are counted per shifted-product launch (one per tick and
        # tiling group, the same groups in both runs)
        runs.append((res, ctx.profile_read(L.PROF_PRECOND)[1] / ctx.profile_read(L.PROF_SPMM)[1]))
    (a, la), (b, lb) = runs
    say("  k", a.k, "preconditioner launches per product launch: paired", la, "single", lb)
    assert a.k == b.k
    assert np.array_equal(a.history(), b.history())
    for x, y in zip(a.factors(), b.factors()):
        assert np.array_equal(x, y)
    # 2-D tiles pair (regions about 1.4 times the tile); 3-D ones and
    # matrices below 32768 rows do not
    expect = P.A.dim == 2 and min(P.A.n, P.B.n) >= 32768
    if expect:
        assert la < lb
    else:
        assert la == pytest.approx(lb, rel=1e-12)


def test_identity_mass_preconditioned_equals_plain(L, ctx):
    """M = C = I given as matrices: the lumped weights are 1, so the
    preconditioned pencil run reproduces the plain preconditioned run's
    steps and X to rounding."""
    P = WL.SMALL_2D
    HA = L.convdiff(2, P.A.N, P.A.omega)
    HB = L.convdiff(2, P.B.N, P.B.omega)
    n, m = P.A.n, P.B.n
    I_n = L.HostCsr(np.arange(n + 1), np.arange(n), np.ones(n))
    I_m = L.HostCsr(np.arange(m + 1), np.arange(m), np.ones(m))
    f, g = WL.rhs_factors(P.seed, n, m, P.r)
    pA, pB = WL.wachspress_shifts(P.A, P.B, P.nshifts)
    o = L.default_opts(tol=P.tol, precond="rbilu0", precond_sweeps=3)
    plain = ctx.solve(HA, HB, to_dev(f), to_dev(g), pA, pB, o)
    gen = ctx.solve(HA, HB, to_dev(f), to_dev(g), pA, pB, o, M=I_n, C=I_m)
    assert gen.k == plain.k
    Zp, dp, Yp = plain.factors()
    Zg, dg, Yg = gen.factors()
    assert OF.lowrank_diff_fro(Zg, dg, Yg, Zp, dp, Yp) <= 1e-9 * OF.lowrank_fro(Zp, dp, Yp)


def test_prepared_matrix_cache_is_keyed_by_contents(L, ctx):
    """A context reuses the preconditioner data of a matrix it has prepared
    before (same contents: bit-identical results); a matrix with the same
    pattern but other values is prepared afresh (its result equals a fresh
    context's)."""
    H = L.convdiff(2, 33, (6.0, -11.0))
    W = to_dev(np.random.default_rng(500).standard_normal((H.n, 3)))
    o = L.default_opts(restart=10, max_inner=400, precond="rbilu0", precond_sweeps=2)
    d = [1e-10 * float(np.linalg.norm(W.cpu().numpy(), 2))]
    Z1 = ctx.shifted_solve([H], [-80.0], [W], d, o)[0][0].cpu().numpy()
    Z2 = ctx.shifted_solve([H], [-80.0], [W], d, o)[0][0].cpu().numpy()
    assert np.array_equal(Z1, Z2)
    H2 = L.HostCsr(H.rowptr, H.colind, H.val * 1.5)
    Z3 = ctx.shifted_solve([H2], [-80.0], [W], d, o)[0][0].cpu().numpy()
    c2 = L.Context(0)
    try:
        Z4 = c2.shifted_solve([H2], [-80.0], [W], d, o)[0][0].cpu().numpy()
    finally:
        c2.close()
    assert np.array_equal(Z3, Z4)
    assert not np.array_equal(Z3, Z1)


def test_preconditioner_degenerate_patterns(L, ctx):
    """Edge cases of the colouring: a diagonal matrix (every row isolated,
    all red, no black rows: the preconditioner is the exact inverse, one
    block step), a 1-D chain (tridiagonal, alternating colours) and n = 1.
    Each solve reaches delta, checked on the host; a block wider than the
    system (r > n) is rejected."""
    import scipy.sparse as sp
    rng = np.random.default_rng(600)
    cases = []
    d = rng.uniform(2.0, 5.0, 37)
    cases.append(("diagonal", sp.diags(d).tocsr(), 1))
    n = 29
    T = sp.diags([-np.ones(n - 1) * 1.3, np.full(n, 4.0), -np.ones(n - 1) * 0.7], [-1, 0, 1]).tocsr()
    cases.append(("chain", T, None))
    cases.append(("one", sp.csr_matrix(np.array([[3.0]])), 1))
    for name, A, steps in cases:
        A.sort_indices()
        H = L.HostCsr(A.indptr, A.indices, A.data)
        W = rng.standard_normal((A.shape[0], min(2, A.shape[0])))
        delta = 1e-10 * np.linalg.norm(W, 2)
        for sweeps in (0, 3):
            o = L.default_opts(restart=8, max_inner=200, precond="rbilu0", precond_sweeps=sweeps)
            Zs, st, rc = ctx.shifted_solve([H], [-1.5], [to_dev(W)], [delta], o)
            Z = Zs[0].cpu().numpy()
            rn = np.linalg.norm(W - (A @ Z - 1.5 * Z), 2)
            say("  degenerate", name, sweeps, "steps", st[0]["steps"], "rn", rn)
            assert rc == L.OK and rn <= delta * (1 + 1e-8)
            if steps is not None:
                assert st[0]["steps"] == steps
    H1 = L.HostCsr(np.array([0, 1]), np.array([0]), np.array([3.0]))
    with pytest.raises(L.LradiError) as e:
        ctx.shifted_solve([H1], [-1.5], [to_dev(np.ones((1, 2)))], [1e-10],
                          L.default_opts(precond="rbilu0"))
    assert e.value.status == L.EINVAL


def test_preconditioned_mixed_batch_and_server_equal_solo(L, ctx):
    """2-D and 3-D problems (different slot widths) with the preconditioner,
    batched and then served: each result equals its solo run bit for bit."""
    o = L.default_opts(precond="rbilu0", precond_sweeps=6)
    probs, solos = [], []
    for name in ("SMALL_2D", "SMALL_3D", "C1"):
        P = getattr(WL, name)
        HA = L.convdiff(P.A.dim, P.A.N, P.A.omega)
        HB = L.convdiff(P.B.dim, P.B.N, P.B.omega)
        f, g = WL.rhs_factors(P.seed, P.A.n, P.B.n, P.r)
        pA, pB = WL.wachspress_shifts(P.A, P.B, P.nshifts)
        fd, gd = to_dev(f), to_dev(g)
        probs.append((HA, HB, fd, gd, pA, pB, P.tol))
        solos.append(ctx.solve(HA, HB, fd, gd, pA, pB, o))
    res, st = ctx.batch_solve(probs, o)
    assert st == L.OK
    for a, b in zip(res, solos):
        assert a.k == b.k
        for x, y in zip(a.factors(), b.factors()):
            assert np.array_equal(x, y)
    c2 = L.Context(0)
    srv = L.Server(c2, o)
    try:
        import time
        tickets = [srv.submit(*p) for p in probs]
        got, t0 = {}, time.time()
        while len(got) < len(tickets) and time.time() - t0 < 60:
            for t in tickets:
                if t not in got:
                    r = srv.poll(t)
                    if r is not None:
                        got[t] = r[0]
            time.sleep(0.01)
        assert len(got) == len(tickets)
        for t, ref in zip(tickets, solos):
            for x, y in zip(got[t].factors(), ref.factors()):
                assert np.array_equal(x, y)
    finally:
        srv.close()
        c2.close()


def test_pairs_only_for_batches_that_leave_the_chip_idle(L, ctx):
    """Sweeps pair while a batch's preconditioned black rows stay within
    262144 (latency-bound launches): two 256^2 systems pair, nine (294912
    black rows) run one sweep per launch; both give the same bits as the
    single-sweep option."""
    H = L.convdiff(2, 256, (50.0, 20.0))
    rng = np.random.default_rng(77)
    for count, pairs_expected in ((2, True), (9, False)):
        say("pair rule", count)
        Ws = [to_dev(rng.standard_normal((H.n, 1))) for _ in range(count)]
        shifts = [-100.0 * (s + 1) for s in range(count)]
        runs = []
        for pairs in (1, 0):
            o = L.default_opts(precond="rbilu0", precond_sweeps=6, precond_pairs=pairs, profile=1)
            ctx.profile_reset()
            Zs, stats, st = ctx.shifted_solve([H] * count, shifts, Ws, [1e-8] * count, o)
            assert st == L.OK
            runs.append(([z.cpu().numpy() for z in Zs], ctx.profile_read(L.PROF_PRECOND)[1]))
        (za, la), (zb, lb) = runs
        say("  launches paired option", la, "single", lb)
        for x, y in zip(za, zb):
            assert np.array_equal(x, y)
        assert (la < lb) == pairs_expected


def test_paired_sweeps_lyapunov_and_mixed_widths_equal_single_sweeps(L, ctx):
    """Pairs on the Lyapunov path (one inner system per step beside an idle
    mirror) and in a batch of mixed block widths (the kernels that dispatch
    on r, with the columns read from the table) give the same bits as one
    sweep per launch, with fewer launches."""
    import torch
    P = WL.LYAP_C2
    HA = L.convdiff(P.A.dim, P.A.N, P.A.omega)
    f, shifts = WL.lyap_inputs(P)
    fd = torch.from_numpy(np.ascontiguousarray(f)).cuda()
    runs = []
    for pairs in (1, 0):
        o = L.default_opts(tol=P.tol, selection="sym", precond="rbilu0", precond_sweeps=9, precond_pairs=pairs,
                           profile=1)
        ctx.profile_reset()
        res = ctx.solve_lyap(HA, fd, shifts, o)
        assert res.status == L.OK
        runs.append((res, ctx.profile_read(L.PROF_PRECOND)[1]))
    (a, la), (b, lb) = runs
    say("  lyapunov k", a.k, "launches", la, lb)
    assert a.k == b.k and la < lb
    for x, y in zip(a.factors(), b.factors()):
        assert np.array_equal(x, y)
    H = L.convdiff(2, 256, (50.0, 20.0))
    rng = np.random.default_rng(78)
    Ws = [to_dev(rng.standard_normal((H.n, r))) for r in (1, 2, 3)]
    runs = []
    for pairs in (1, 0):
        o = L.default_opts(precond="rbilu0", precond_sweeps=6, precond_pairs=pairs, profile=1)
        ctx.profile_reset()
        Zs, stats, st = ctx.shifted_solve([H] * 3, [-150.0, -900.0, -40.0], Ws, [1e-8] * 3, o)
        assert st == L.OK
        runs.append(([z.cpu().numpy() for z in Zs], ctx.profile_read(L.PROF_PRECOND)[1]))
    (za, la), (zb, lb) = runs
    say("  mixed widths launches", la, lb)
    assert la < lb
    for x, y in zip(za, zb):
        assert np.array_equal(x, y)
