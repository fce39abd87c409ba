"""Writes the stored expected values under tests/golden/ by calling only the
oracle (and the shared seeded input generators).  Run from the repo root:
    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import fadi as OF  # noqa: E402
from oracle.convdiff import convdiff_matrix  # noqa: E402
from paper_2312_02891_amd import workloads as WL  # noqa: E402


def config1():
    P = WL.C1
    A = convdiff_matrix(P.A.dim, P.A.N, P.A.omega)
    B = convdiff_matrix(P.B.dim, P.B.N, P.B.omega)
    f, g = WL.rhs_factors(P.seed, P.A.n, P.B.n, P.r)
    pA, pB = WL.wachspress_shifts(P.A, P.B, P.nshifts)
    res = OF.fadi(A, B, f, g, pA, pB, tol=P.tol)
    fs, gs = OF.rescale_rhs(f, g)
    true = OF.lowrank_residual_norm(A, B, fs, gs, res.Z, res.D(), res.Y) / res.norm_fg
    return {
        "what": "oracle LR-ADI with direct solves on config 1 (2-D upwind N=20, "
                "omega_A=(10,5), omega_B=(-5,8), r=1, seed 1, 16 Wachspress shifts, tau=1e-8)",
        "k": res.k,
        "res_hist": res.res_hist,
        "true_rel_residual": true,
        "norm_fg": res.norm_fg,
        "gammas": res.gammas.tolist(),
        "pA": pA.tolist(),
        "pB": pB.tolist(),
    }


if __name__ == "__main__":
    out = os.path.join(HERE, "config1_oracle.json")
    with open(out, "w") as fh:
        json.dump(config1(), fh, indent=1)
    print("wrote", out)
