"""GPU tests of the continuous-batching server: requests submitted while
others run are admitted as memory and slots free up, every result equals
the same problem solved alone (bit for bit) and meets its residual target,
oversized requests are rejected at admission, and cancellation works."""
import time

import numpy as np
import pytest

from oracle import fadi as OF
from oracle.convdiff import convdiff_matrix
from paper_2312_02891_amd import workloads as WL

from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_2312_02891_amd import lradi
    return lradi


def small_requests(L, count, seed=5):
    out = []
    for t, P in WL.serving_requests(count, seed=seed, nmin=64, nmax=2500):
        HA = L.convdiff(P.A.dim, P.A.N, P.A.omega)
        HB = L.convdiff(P.B.dim, P.B.N, P.B.omega)
        f, g = WL.rhs_factors(P.seed, P.A.n, P.B.n, P.r)
        pA, pB = WL.wachspress_shifts(P.A, P.B, P.nshifts)
        out.append((t, P, HA, HB, f, g, pA, pB))
    return out


def test_mixed_stream_equals_solo_runs(L):
    say("serving mix")
    reqs = small_requests(L, 10)
    o = L.default_opts()
    ctx = L.Context(0)
    solo = []
    for (_, P, HA, HB, f, g, pA, pB) in reqs:
        # alone: the same problem (with its own tolerance) as a batch of one
        rs, _ = ctx.batch_solve([(HA, HB, to_dev(f), to_dev(g), pA, pB, P.tol)], o)
        solo.append(rs[0])
    srv = L.Server(ctx, o, hbm_budget=0, max_active=4)
    tickets = []
    t0 = time.perf_counter()
    for (t, P, HA, HB, f, g, pA, pB) in reqs:
        while time.perf_counter() - t0 < t:          # Poisson arrival times
            time.sleep(0.001)
        tickets.append(srv.submit(HA, HB, to_dev(f), to_dev(g), pA, pB, tol=P.tol))
    results = {}
    deadline = time.perf_counter() + 120
    while len(results) < len(tickets) and time.perf_counter() < deadline:
        for tk in tickets:
            if tk not in results:
                got = srv.poll(tk)
                if got is not None:
                    results[tk] = got
        time.sleep(0.002)
    stats = srv.stats()
    srv.close()
    say("  stats", stats)
    assert len(results) == len(tickets)
    lat = [results[tk][1] for tk in tickets]
    say("  latency p50 %.4f p99 %.4f" % (np.percentile(lat, 50), np.percentile(lat, 99)))
    for (_, P, HA, HB, f, g, pA, pB), tk, rs in zip(reqs, tickets, solo):
        rm, _ = results[tk]
        assert rm.status == L.OK
        Zm, dm, Ym = rm.factors()
        Zs, ds, Ys = rs.factors()
        assert rm.k == rs.k and np.array_equal(Zm, Zs) and np.array_equal(Ym, Ys)
        A = convdiff_matrix(P.A.dim, P.A.N, P.A.omega)
        B = convdiff_matrix(P.B.dim, P.B.N, P.B.omega)
        fs, gs = OF.rescale_rhs(f, g)
        nfg = OF.lowrank_product_norm(f, g)
        true = OF.lowrank_residual_norm(A, B, fs, gs, Zm, dm, Ym) / nfg
        # Def. 1 and eq. (upd_resgap): ||R_true|| <= ||w t^T|| + u_k + v_k
        h = rm.history()
        bound = rm.rel_res + (h[-1, 8] + h[-1, 9]) / nfg
        say("  tol %.2e comp %.2e true %.2e bound %.2e" % (P.tol, rm.rel_res, true, bound))
        assert rm.rel_res < P.tol
        assert true <= bound * (1 + 1e-6) + 1e-14
    ctx.close()


def test_admission_rejects_oversized_and_cancel(L):
    say("serving reject/cancel")
    reqs = small_requests(L, 3, seed=9)
    ctx = L.Context(0)
    srv = L.Server(ctx, L.default_opts(), hbm_budget=1 << 16, max_active=0)
    (_, P, HA, HB, f, g, pA, pB) = reqs[0]
    with pytest.raises(L.LradiError) as ei:
        srv.submit(HA, HB, to_dev(f), to_dev(g), pA, pB, tol=P.tol)
    assert ei.value.status == L.ENOMEM
    srv.close()
    srv = L.Server(ctx, L.default_opts(), hbm_budget=0, max_active=1)
    tks = [srv.submit(HA, HB, to_dev(f), to_dev(g), pA, pB, tol=P.tol) for _ in range(3)]
    srv.cancel(tks[2])                       # still queued behind the single slot
    done = {}
    deadline = time.perf_counter() + 60
    while len(done) < 3 and time.perf_counter() < deadline:
        for tk in tks:
            if tk not in done:
                got = srv.poll(tk)
                if got is not None:
                    done[tk] = got
        time.sleep(0.002)
    srv.close()
    assert done[tks[2]][0].status == L.ECANCELED
    assert done[tks[0]][0].status == L.OK and done[tks[1]][0].status == L.OK
    ctx.close()
