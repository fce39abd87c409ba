"""Failure paths of the solve, forced from the host with ordinary inputs and
options (every kernel still runs to its normal end): a NaN in f ends the
solve with LRADI_ENAN, inner solves stopped by their step cap give
LRADI_WINNER, and the context stays usable afterwards."""
import numpy as np
import pytest

from paper_2312_02891_amd import workloads as WL

from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_2312_02891_amd import lradi
    return lradi


def inputs(L, P):
    HA = L.convdiff(P.A.dim, P.A.N, P.A.omega)
    HB = L.convdiff(P.B.dim, P.B.N, P.B.omega)
    f, g = WL.rhs_factors(P.seed, P.A.n, P.B.n, P.r)
    pA, pB = WL.wachspress_shifts(P.A, P.B, P.nshifts)
    return HA, HB, f, g, pA, pB


def test_nan_in_f_gives_enan(L):
    """||f g^T|| of a right-hand side with a NaN entry is NaN: the setup marks
    the problem failed (Sec. 4's scaled residual is undefined) and no step
    runs; the next solve on the same context is unaffected."""
    say("failure: NaN in f")
    P = WL.SMALL_2D
    HA, HB, f, g, pA, pB = inputs(L, P)
    ctx = L.Context(0)
    bad = f.copy()
    bad[17, 1] = np.nan
    with pytest.raises(L.LradiError) as ei:
        ctx.solve(HA, HB, to_dev(bad), to_dev(g), pA, pB, L.default_opts(tol=P.tol))
    assert ei.value.status == L.ENAN
    res = ctx.solve(HA, HB, to_dev(f), to_dev(g), pA, pB, L.default_opts(tol=P.tol))
    assert res.status == L.OK
    # in a batch the failed problem does not disturb its neighbour
    rs, st = ctx.batch_solve([(HA, HB, to_dev(bad), to_dev(g), pA, pB),
                              (HA, HB, to_dev(f), to_dev(g), pA, pB)], L.default_opts(tol=P.tol))
    say("  batch statuses", [r.status for r in rs], "call", st)
    assert rs[0].status == L.ENAN and rs[1].status == L.OK and st == L.ENAN
    Z1, _, _ = rs[1].factors()
    Z0, _, _ = res.factors()
    assert rs[1].k == res.k and np.array_equal(Z1, Z0)
    ctx.close()


def test_inner_step_cap_gives_winner(L):
    """max_inner = 1: every inner solve stops after one block Arnoldi step.
    With a strong preconditioner the outer iteration still converges in the
    computed residual, and the result carries LRADI_WINNER; the history shows
    inner residuals above their requested tolerances."""
    say("failure: inner step cap")
    P = WL.C1
    HA, HB, f, g, pA, pB = inputs(L, P)
    ctx = L.Context(0)
    o = L.default_opts(tol=P.tol, max_inner=1, precond="rbilu0", precond_sweeps=32)
    res = ctx.solve(HA, HB, to_dev(f), to_dev(g), pA, pB, o)
    h = res.history()
    over = int(np.sum((h[:, 4] > h[:, 2]) | (h[:, 5] > h[:, 3])))
    say("  status", res.status, "k", res.k, "steps over tolerance", over,
        "max inner steps", int(h[:, 6:8].max()))
    assert res.status == L.WINNER
    assert over > 0
    assert h[:, 6:8].max() <= 1
    # the inner solver on its own reports the cap in its statistics
    _, stats, st = ctx.shifted_solve([HA], [pA[0]], [to_dev(f)], [1e-12], L.default_opts(max_inner=1))
    say("  shifted_solve stats", stats, "status", st)
    assert stats[0]["status"] == 1 and st == L.WINNER
    res2 = ctx.solve(HA, HB, to_dev(f), to_dev(g), pA, pB, L.default_opts(tol=P.tol))
    assert res2.status == L.OK
    ctx.close()
