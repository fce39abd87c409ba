"""The stored config-1 values (tests/golden/config1_oracle.json, written by
tests/golden/make_golden.py from the oracle alone): the oracle still
reproduces them on the CPU, and the GPU solve with exact-tolerance inner
solves reproduces them too (same step count, residual history, ||f g^T||
and gammas)."""
import json
import os

import numpy as np
import pytest

from oracle import fadi as OF
from oracle.convdiff import convdiff_matrix
from paper_2312_02891_amd import workloads as WL

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "config1_oracle.json")


@pytest.fixture(scope="module")
def stored():
    with open(GOLDEN) as fh:
        return json.load(fh)


def _inputs():
    P = WL.C1
    A = convdiff_matrix(P.A.dim, P.A.N, P.A.omega)
    B = convdiff_matrix(P.B.dim, P.B.N, P.B.omega)
    f, g = WL.rhs_factors(P.seed, P.A.n, P.B.n, P.r)
    pA, pB = WL.wachspress_shifts(P.A, P.B, P.nshifts)
    return P, A, B, f, g, pA, pB


def test_oracle_reproduces_stored_config1(stored):
    P, A, B, f, g, pA, pB = _inputs()
    assert np.array_equal(pA, np.array(stored["pA"])) and np.array_equal(pB, np.array(stored["pB"]))
    res = OF.fadi(A, B, f, g, pA, pB, tol=P.tol)
    assert res.k == stored["k"]
    assert np.allclose(res.res_hist, stored["res_hist"], rtol=1e-10, atol=0)
    assert res.norm_fg == pytest.approx(stored["norm_fg"], rel=1e-13)
    assert np.array_equal(res.gammas, np.array(stored["gammas"]))
    fs, gs = OF.rescale_rhs(f, g)
    true = OF.lowrank_residual_norm(A, B, fs, gs, res.Z, res.D(), res.Y) / res.norm_fg
    assert true == pytest.approx(stored["true_rel_residual"], rel=1e-8)


@pytest.mark.gpu
def test_gpu_reproduces_stored_config1(stored):
    from paper_2312_02891_amd import lradi as L
    from gpu_util import say, to_dev
    say("golden config 1")
    P, A, B, f, g, pA, pB = _inputs()
    HA = L.convdiff(P.A.dim, P.A.N, P.A.omega)
    HB = L.convdiff(P.B.dim, P.B.N, P.B.omega)
    ctx = L.Context(0)
    try:
        o = L.default_opts(selection="relative", rho=1e-12, tol=P.tol)
        res = ctx.solve(HA, HB, to_dev(f), to_dev(g), pA, pB, o)
        assert res.status == L.OK
        assert res.k == stored["k"]
        h = res.history()
        assert np.allclose(h[:, 15], stored["res_hist"], rtol=1e-7, atol=0)
        assert np.array_equal(h[:, 14], np.array(stored["gammas"]))
        assert res.norm_fg == pytest.approx(stored["norm_fg"], rel=1e-12)
    finally:
        ctx.close()
