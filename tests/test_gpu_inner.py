"""GPU parity of the shifted SpMM and of the batched block GMRES(m)-IR inner
solver against the oracle (called through the C ABI)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

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
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    c = L.Context(0)
    yield c
    c.close()


SHAPES = [(2, 7, (3.0, -2.0)), (2, 37, (12.0, -7.0)), (3, 13, (6.0, -3.0, 2.0)),
          (2, 256, (50.0, 20.0)), (3, 48, (10.0, -15.0, -5.0))]


@pytest.mark.parametrize("dim,N,omega", SHAPES)
@pytest.mark.parametrize("r", [1, 2, 3, 4, 8])
def test_spmm_fp64_matches_oracle(L, ctx, dim, N, omega, r):
    say("spmm fp64", dim, N, r)
    H = L.convdiff(dim, N, omega)
    A = convdiff_matrix(dim, N, omega)
    rng = np.random.default_rng(N * 10 + r)
    X = rng.standard_normal((H.n, r))
    s = -1234.5
    Y = ctx.spmm(H, s, to_dev(X)).cpu().numpy()
    want = A @ X + s * X
    scale = (abs(A) @ np.abs(X) + abs(s) * np.abs(X)).max()
    assert np.abs(Y - want).max() <= 1e-14 * scale


@pytest.mark.parametrize("dim,N,omega", SHAPES)
@pytest.mark.parametrize("r", [1, 4, 8])
def test_spmm_fp32_matches_oracle(L, ctx, dim, N, omega, r):
    import torch
    say("spmm fp32", dim, N, r)
    H = L.convdiff(dim, N, omega)
    A = convdiff_matrix(dim, N, omega)
    A32 = sp.csr_matrix((A.data.astype(np.float32).astype(np.float64), A.indices, A.indptr), A.shape)
    rng = np.random.default_rng(N * 10 + r + 1)
    X = rng.standard_normal((H.n, r)).astype(np.float32)
    s = np.float32(-777.25)
    Y = ctx.spmm(H, float(s), to_dev(X)).cpu().numpy().astype(np.float64)
    Xd = X.astype(np.float64)
    want = A32 @ Xd + float(s) * Xd
    scale = (abs(A32) @ np.abs(Xd) + abs(float(s)) * np.abs(Xd)).max()
    assert np.abs(Y - want).max() <= 2e-6 * scale


def _wide_csr(n, per_row, seed):
    """Random sparse matrix with per_row nonzeros in every row (plus the
    diagonal): a 256-row tile holds more nonzeros than fit in LDS."""
    rng = np.random.default_rng(seed)
    rows = []
    for i in range(n):
        cols = np.unique(np.concatenate([[i], rng.integers(0, n, per_row)]))
        rows.append(cols)
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(c) for c in rows])
    ci = np.concatenate(rows)
    v = rng.standard_normal(len(ci))
    return rp, ci, v


TILING_CASES = [("cd3", 4, "f64"), ("cd3", 8, "f64"), ("cd3", 8, "f32"), ("cd3", 6, "f64"),
                ("cd2", 2, "f32"), ("cd2", 4, "f64"), ("wide", 4, "f64"), ("wide", 8, "f32")]


@pytest.mark.parametrize("mat,r,prec", TILING_CASES)
def test_spmm_tilings_are_bitwise_identical(L, ctx, mat, r, prec):
    """Every admissible tiling (1, 2, 4 lanes per row) gives the same bits as
    the default one, on stencil matrices with a ragged last tile and on a
    matrix whose tiles overflow the LDS staging buffer; the product also
    matches the oracle's matrix."""
    import torch
    say("spmm tilings", mat, r, prec)
    if mat == "cd3":
        H = L.convdiff(3, 29, (10.0, -15.0, -5.0))
        A = convdiff_matrix(3, 29, (10.0, -15.0, -5.0))
    elif mat == "cd2":
        H = L.convdiff(2, 301, (50.0, 20.0))
        A = convdiff_matrix(2, 301, (50.0, 20.0))
    else:
        rp, ci, v = _wide_csr(3001, 40, 7)
        H = L.HostCsr(rp, ci, v)
        A = sp.csr_matrix((v, ci, rp), shape=(3001, 3001))
    dt = torch.float64 if prec == "f64" else torch.float32
    rng = np.random.default_rng(r)
    X = torch.from_numpy(rng.standard_normal((H.n, r))).to(dt).cuda()
    s = -321.75
    ref = ctx.spmm(H, s, X)
    outs = []
    for lanes in (1, 2, 4):
        if r % lanes:
            continue
        Y = torch.empty_like(X)
        ctx.spmm_bench(H, s, X, reps=1, lanes=lanes, out=Y)
        torch.cuda.synchronize()
        outs.append((lanes, Y))
    for lanes, Y in outs:
        assert torch.equal(Y, ref), f"lanes={lanes} differs"
    Xd = X.double().cpu().numpy()
    Ad = A if prec == "f64" else sp.csr_matrix(
        (A.data.astype(np.float32).astype(np.float64), A.indices, A.indptr), A.shape)
    want = Ad @ Xd + s * Xd
    scale = (abs(Ad) @ np.abs(Xd) + abs(s) * np.abs(Xd)).max()
    tol = 1e-14 if prec == "f64" else 2e-6
    assert np.abs(ref.double().cpu().numpy() - want).max() <= tol * scale


def _ragged_csr(n, seed):
    """Rows of every length the sliced layout has to pad: empty rows, runs of
    empty rows spanning whole 32-row slices, single entries, a row of 300
    nonzeros and random short rows; n not a multiple of 32."""
    rng = np.random.default_rng(seed)
    rows = []
    for i in range(n):
        if 64 <= i < 160 or i % 7 == 3:
            cols = np.array([], dtype=np.int64)
        elif i == 200:
            cols = np.unique(rng.integers(0, n, 300))
        elif i % 5 == 1:
            cols = np.array([i])
        else:
            cols = np.unique(np.concatenate([[i], rng.integers(0, n, rng.integers(1, 12))]))
        rows.append(cols)
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(c) for c in rows])
    ci = np.concatenate(rows).astype(np.int64)
    v = rng.standard_normal(len(ci))
    return rp, ci, v


@pytest.mark.parametrize("r,prec", [(1, "f64"), (4, "f64"), (8, "f64"), (8, "f32"), (6, "f32")])
def test_spmm_sliced_layout_ragged_rows(L, ctx, r, prec):
    """The sliced ELL copy of a matrix with empty rows (also whole empty
    slices), one-entry rows, a 300-entry row and a ragged last slice: every
    tiling gives the same bits, and the product matches the oracle's."""
    import torch
    say("spmm ragged", r, prec)
    n = 1001
    rp, ci, v = _ragged_csr(n, 5 + r)
    H = L.HostCsr(rp, ci, v)
    A = sp.csr_matrix((v, ci, rp), shape=(n, n))
    dt = torch.float64 if prec == "f64" else torch.float32
    X = torch.from_numpy(np.random.default_rng(r).standard_normal((n, r))).to(dt).cuda()
    s = 17.5
    ref = ctx.spmm(H, s, X)
    for lanes in (1, 2, 4):
        if r % lanes:
            continue
        Y = torch.empty_like(X)
        ctx.spmm_bench(H, s, X, reps=1, lanes=lanes, out=Y)
        torch.cuda.synchronize()
        assert torch.equal(Y, ref), f"lanes={lanes} differs"
    Xd = X.double().cpu().numpy()
    Ad = A if prec == "f64" else sp.csr_matrix((A.data.astype(np.float32).astype(np.float64), A.indices,
                                                A.indptr), A.shape)
    want = Ad @ Xd + s * Xd
    scale = (abs(Ad) @ np.abs(Xd) + abs(s) * np.abs(Xd)).max()
    tol = 1e-14 if prec == "f64" else 2e-6
    assert np.abs(ref.double().cpu().numpy() - want).max() <= tol * scale


def test_spmm_autotuner_choice_is_valid_and_cached(L, ctx):
    """The tuner returns an admissible tiling for a product above its size
    threshold, and the same one again from its cache."""
    say("spmm tune")
    H = L.convdiff(3, 64, (20.0, 10.0, 5.0))
    for r, prec in ((8, L.FP32_INNER), (4, L.FP64), (3, L.FP64)):
        a = ctx.spmm_tune(H, r, prec)
        assert a in (1, 2, 4) and r % a == 0
        assert ctx.spmm_tune(H, r, prec) == a


@pytest.mark.parametrize("r", [1, 2, 3, 4, 8])
@pytest.mark.parametrize("j", [1, 3, 7])
def test_first_cycle_equals_block_minres_definition(L, ctx, r, j):
    """With restart = j and a step cap of j, the returned Z is block GMRES's
    j-step iterate: the minimiser of ||W - S Z||_F over the block Krylov space
    (oracle written as that definition)."""
    say("first cycle", r, j)
    dim, N, omega = 2, 15, (8.0, -5.0)
    H = L.convdiff(dim, N, omega)
    A = convdiff_matrix(dim, N, omega)
    rng = np.random.default_rng(100 + r * 10 + j)
    W = rng.standard_normal((H.n, r))
    shift = -300.0
    o = L.default_opts(restart=j, max_inner=j)
    Zs, stats, st = ctx.shifted_solve([H], [shift], [to_dev(W)], [0.0], o)
    Z = Zs[0].cpu().numpy()
    want = block_gmres_iterate(A, shift, W, j)
    assert stats[0]["steps"] == j
    assert np.linalg.norm(Z - want) <= 1e-9 * np.linalg.norm(want)


@pytest.mark.parametrize("prec,rel", [("fp64", 1e-11), ("fp32", 1e-11), ("fp32", 1e-5)])
@pytest.mark.parametrize("shift", [-2.0e5, -3.0e3, -25.0])
def test_solve_reaches_delta_config2_shape(L, ctx, prec, rel, shift):
    """A 2-D operator of config 2's shape (n = 65536, r = 4): the FP64 residual
    of the returned block satisfies ||W - (A + s I) Z||_2 <= delta, checked by
    the oracle's sparse product."""
    say("solve", prec, rel, shift)
    P = WL.C2
    H = L.convdiff(P.A.dim, P.A.N, P.A.omega)
    A = convdiff_matrix(P.A.dim, P.A.N, P.A.omega)
    rng = np.random.default_rng(7)
    W = rng.standard_normal((H.n, 4))
    delta = rel * np.linalg.norm(W, 2)
    o = L.default_opts(precision=prec, restart=30, max_inner=6000)
    Zs, stats, st = ctx.shifted_solve([H], [shift], [to_dev(W)], [delta], o)
    Z = Zs[0].cpu().numpy()
    R = W - (A @ Z + shift * Z)
    rn = np.linalg.norm(R, 2)
    say("  steps", stats[0]["steps"], "cycles", stats[0]["cycles"], "rnorm", rn, "delta", delta)
    assert st == L.OK and stats[0]["status"] == 0
    assert rn <= delta * (1 + 1e-8)
    assert stats[0]["rnorm"] == pytest.approx(rn, rel=1e-6)


def test_batch_of_uneven_systems_equals_solo_runs(L, ctx):
    """Systems of different n, r and shift share launches; each result is
    bit-identical to solving that system alone."""
    say("batch vs solo")
    specs = [(2, 21, (4.0, -9.0), 1, -50.0), (2, 40, (-20.0, 3.0), 3, -900.0),
             (3, 9, (2.0, 2.0, -1.0), 8, -120.0), (2, 64, (30.0, 30.0), 5, -4000.0),
             (3, 12, (-5.0, 1.0, 7.0), 2, -60.0)]
    mats, Ws, shifts, deltas = [], [], [], []
    for i, (dim, N, om, r, s) in enumerate(specs):
        H = L.convdiff(dim, N, om)
        W = np.random.default_rng(200 + i).standard_normal((H.n, r))
        mats.append(H)
        Ws.append(to_dev(W))
        shifts.append(s)
        deltas.append(1e-9 * np.linalg.norm(W, 2))
    o = L.default_opts(restart=12, max_inner=3000)
    Zb, sb, _ = ctx.shifted_solve(mats, shifts, Ws, deltas, o)
    for i in range(len(specs)):
        Zi, si, _ = ctx.shifted_solve([mats[i]], [shifts[i]], [Ws[i]], [deltas[i]], o)
        assert si[0]["steps"] == sb[i]["steps"]
        assert np.array_equal(Zi[0].cpu().numpy(), Zb[i].cpu().numpy())
        A = convdiff_matrix(specs[i][0], specs[i][1], specs[i][2])
        W = Ws[i].cpu().numpy()
        Z = Zb[i].cpu().numpy()
        assert np.linalg.norm(W - (A @ Z + shifts[i] * Z), 2) <= deltas[i] * (1 + 1e-8)


def test_zero_rhs_and_rank_deficient_block(L, ctx):
    """Degenerate inputs: W = 0 returns Z = 0 at once; a block with two equal
    columns still converges (the Cholesky-QR regularisation replaces the lost
    direction)."""
    say("degenerate")
    H = L.convdiff(2, 20, (3.0, 4.0))
    A = convdiff_matrix(2, 20, (3.0, 4.0))
    W0 = np.zeros((H.n, 2))
    Zs, stats, _ = ctx.shifted_solve([H], [-100.0], [to_dev(W0)], [1e-12], L.default_opts())
    assert stats[0]["steps"] == 0 and np.all(Zs[0].cpu().numpy() == 0)
    W = np.random.default_rng(5).standard_normal((H.n, 3))
    W[:, 2] = W[:, 0]
    delta = 1e-10 * np.linalg.norm(W, 2)
    Zs, stats, st = ctx.shifted_solve([H], [-100.0], [to_dev(W)], [delta], L.default_opts())
    Z = Zs[0].cpu().numpy()
    assert np.linalg.norm(W - (A @ Z - 100.0 * Z), 2) <= delta * (1 + 1e-8)
