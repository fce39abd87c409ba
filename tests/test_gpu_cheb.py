"""Chebyshev steps on the Schur complement (opts.precond_poly = 1) against
the oracle's definition: the first restart cycle's iterate equals the
preconditioned block minimal-residual iterate with the oracle's Chebyshev
preconditioner; without diagonal dominance the steps are the Jacobi ones
bit for bit; paired launches equal single ones bit for bit.  The ADI
parity of the reduced and full 3-D configuration with these steps is in
test_gpu_config3.py."""
import numpy as np
import pytest

from oracle import precond as OP
from oracle.convdiff import convdiff_matrix
from oracle.gmres_ref import block_gmres_iterate

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


@pytest.mark.parametrize("dim,N,omega,shift", [(2, 15, (8.0, -5.0), -300.0), (3, 7, (4.0, -2.0, 6.0), -300.0),
                                               (3, 9, (20.0, 10.0, 5.0), -40.0)])
@pytest.mark.parametrize("r,j,sweeps", [(1, 2, 1), (2, 3, 2), (4, 4, 5), (8, 3, 8), (3, 2, 13), (8, 2, 16),
                                         (7, 2, 6), (5, 3, 4)])
def test_first_cycle_with_chebyshev_steps_equals_definition(L, ctx, dim, N, omega, shift, r, j, sweeps):
    """restart = j, step cap j: Z minimises ||W - S Z||_F over M K_j(S M, W)
    with M the oracle's red-black ILU(0) and `sweeps` Chebyshev steps, to
    1e-9, far closer than the Jacobi-step iterate where that one differs."""
    say("chebyshev first cycle", dim, N, r, j, sweeps)
    H = L.convdiff(dim, N, omega)
    A = convdiff_matrix(dim, N, omega)
    W = np.random.default_rng(700 + r * 10 + j).standard_normal((H.n, r))
    o = L.default_opts(restart=j, max_inner=j, precond="rbilu0", precond_sweeps=sweeps, precond_poly=1)
    Zs, stats, st = ctx.shifted_solve([H], [shift], [to_dev(W)], [0.0], o)
    Z = Zs[0].cpu().numpy()
    want = block_gmres_iterate(A, shift, W, j,
                               precond=lambda X: OP.rb_precond_apply(A, shift, X, sweeps, poly="chebyshev"))
    assert stats[0]["steps"] == j
    err = np.linalg.norm(Z - want) / np.linalg.norm(want)
    # the oracle's iterate with Jacobi sweeps: where the two definitions
    # differ visibly, the GPU's iterate is the Chebyshev one
    wj = block_gmres_iterate(A, shift, W, j, precond=lambda X: OP.rb_precond_apply(A, shift, X, sweeps))
    gap = np.linalg.norm(wj - want) / np.linalg.norm(want)
    say("  err %.2e, Jacobi-step iterate at %.2e" % (err, gap))
    assert err <= 1e-9
    if gap > 1e-6:
        assert err < 1e-3 * gap


def _laplace_1d(L, n):
    rp = [0]
    ci, v = [], []
    for i in range(n):
        for j, a in ((i - 1, -1.0), (i, 2.0), (i + 1, -1.0)):
            if 0 <= j < n:
                ci.append(j)
                v.append(a)
        rp.append(len(ci))
    return L.HostCsr(np.array(rp), np.array(ci), np.array(v))


def test_chebyshev_without_dominance_is_jacobi_bitwise(L, ctx):
    """The 1-D stencil (-1, 2, -1) without a shift: the symmetrised row sums
    of I - diag(T)^{-1} T reach exactly 1, so the steps fall back to Jacobi
    and the solve equals the Jacobi-step solve bit for bit."""
    H = _laplace_1d(L, 301)
    W = to_dev(np.random.default_rng(71).standard_normal((H.n, 2)))
    out = []
    for poly in (0, 1):
        o = L.default_opts(restart=10, max_inner=40, precond="rbilu0", precond_sweeps=6, precond_poly=poly)
        Zs, stats, st = ctx.shifted_solve([H], [0.0], [W], [1e-9], o)
        out.append((Zs[0].cpu().numpy(), stats[0]["steps"]))
    assert out[0][1] == out[1][1]
    assert np.array_equal(out[0][0], out[1][0])


@pytest.mark.parametrize("prec,r", [("fp64", 4), ("fp32", 4), ("fp64", 2), ("fp32", 1), ("fp64", 3)])
def test_chebyshev_steps_run_in_pairs(L, ctx, prec, r):
    """A 2-D grid above the pairing size: the Chebyshev steps run two per
    launch (fewer preconditioner launches per product launch) with the same
    bits as one per launch, and a relaxed-accuracy solve needs fewer block
    steps than with as many Jacobi sweeps."""
    dim, N, omega = 2, 182, (30.0, -12.0)
    H = L.convdiff(dim, N, omega)
    W = to_dev(np.random.default_rng(72).standard_normal((H.n, r)))
    delta = 1e-8 * float(np.linalg.norm(W.cpu().numpy(), 2))
    res = {}
    for poly, pairs in ((1, 1), (1, 0), (0, 1)):
        o = L.default_opts(precision=prec, restart=30, max_inner=3000, precond="rbilu0", precond_sweeps=8,
                           precond_poly=poly, precond_pairs=pairs, profile=1)
        ctx.profile_reset()
        Zs, stats, st = ctx.shifted_solve([H], [-60.0], [W], [delta], o)
        assert st == L.OK and stats[0]["status"] == 0
        per = ctx.profile_read(L.PROF_PRECOND)[1] / ctx.profile_read(L.PROF_SPMM)[1]
        res[(poly, pairs)] = (Zs[0].cpu().numpy(), stats[0]["steps"], per)
    say("  steps chebyshev / jacobi", prec, r, res[(1, 1)][1], res[(0, 1)][1], "launches per product, paired",
        res[(1, 1)][2], "single", res[(1, 0)][2])
    assert np.array_equal(res[(1, 1)][0], res[(1, 0)][0])
    assert res[(1, 1)][2] < res[(1, 0)][2]
    assert res[(1, 1)][1] < res[(0, 1)][1]


def test_chebyshev_four_block_single_steps_equal_pairs(L, ctx):
    """Systems set up for paired Chebyshev steps (four iterate blocks) in a
    batch with more than 262144 black rows, which is not paired, take their
    steps one per launch in the same four blocks: each result equals the
    system's solo paired solve bit for bit."""
    H = L.convdiff(2, 182, (30.0, -12.0))
    nsys = 17  # 17 x 16562 black rows
    rng = np.random.default_rng(73)
    Ws = [to_dev(rng.standard_normal((H.n, 2))) for _ in range(nsys)]
    shifts = [-60.0 - 7.0 * k for k in range(nsys)]
    deltas = [1e-7 * float(np.linalg.norm(W.cpu().numpy(), 2)) for W in Ws]
    o = L.default_opts(restart=30, max_inner=3000, precond="rbilu0", precond_sweeps=7, precond_poly=1,
                       precond_pairs=1)
    Zs, stats, st = ctx.shifted_solve([H] * nsys, shifts, Ws, deltas, o)
    assert st == L.OK
    for k in (0, 8, 16):
        Zk, sk, st = ctx.shifted_solve([H], [shifts[k]], [Ws[k]], [deltas[k]], o)
        assert st == L.OK and sk[0]["steps"] == stats[k]["steps"]
        assert np.array_equal(Zk[0].cpu().numpy(), Zs[k].cpu().numpy())


def test_precond_poly_argument_errors(L, ctx):
    H = L.convdiff(2, 8, (1.0, 2.0))
    W = to_dev(np.ones((H.n, 1)))
    with pytest.raises(L.LradiError) as e:
        ctx.shifted_solve([H], [-10.0], [W], [1e-8],
                          L.default_opts(precond="rbilu0", precond_sweeps=4, precond_poly=2))
    assert e.value.status == L.EINVAL
