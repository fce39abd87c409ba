"""Writes tests/golden/config3_oracle_fingerprint.json: the oracle's
direct-solve LR-ADI (Algorithm 1 with exact inner solves) on the full 3-D
configuration (A: 3-D upwind convection-diffusion 64^3, omega (20,10,5);
B: 48^3, omega (-10,15,5); r = 8, seed 3, 24 Wachspress shifts, tau = 1e-8).

The factors (262144 x 8k and 110592 x 8k doubles) are too large to store, so
the file keeps a fingerprint of X = Z Gamma Y^T: the step count, the
computed residual history, ||f g^T||, the gammas, ||X||_F and the Gaussian
sketch P^T X Q (P: n x 16, Q: m x 16, drawn from numpy's default_rng with
SKETCH_SEED, P first), stored per step so that P^T X_k Q is available for
every k.  Each step factors its two shifted matrices with SuperLU
(MMD on A^T + A, factors discarded after the solve: every step uses a new
shift).  Calls only the oracle and the shared seeded input generators.
Run from the repo root (about an hour of one CPU core):
    python tests/golden/make_config3_fingerprint.py
"""
import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import fadi as OF  # noqa: E402
from oracle.convdiff import convdiff_matrix  # noqa: E402
from paper_2312_02891_amd import workloads as WL  # noqa: E402

SKETCH_SEED = 303
SKETCH_K = 16
OUT = os.path.join(HERE, "config3_oracle_fingerprint.json")


def sketch_mats(n, m, seed=SKETCH_SEED, k=SKETCH_K):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, k)), rng.standard_normal((m, k))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def main():
    P = WL.C3
    A = convdiff_matrix(P.A.dim, P.A.N, P.A.omega)
    B = convdiff_matrix(P.B.dim, P.B.N, P.B.omega)
    f, g = WL.rhs_factors(P.seed, P.A.n, P.B.n, P.r)
    pA, pB = WL.wachspress_shifts(P.A, P.B, P.nshifts)
    Bt = B.T.tocsr()
    times = {"A": [], "B": []}

    def timed(side, Op):
        # the oracle's own factor-solve-discard direct solve, timed per step
        def solve(k, shift, rhs):
            t = time.perf_counter()
            out = OF._direct_solver(Op, None, shift, None, "MMD_AT_PLUS_A")(rhs)
            times[side].append(time.perf_counter() - t)
            return out
        return solve

    t0 = time.perf_counter()

    def log(k, res):
        print(f"step {k}: ||w t^T||/||f g^T|| = {res:.3e}  A {times['A'][-1]:.0f} s, "
              f"B {times['B'][-1]:.0f} s ({time.perf_counter() - t0:.0f} s)", flush=True)

    res = OF.fadi(A, B, f, g, pA, pB, tol=P.tol, kmax=50, solve_A=timed("A", A),
                  solve_B=timed("B", Bt), log=log)
    wall = time.perf_counter() - t0
    Ps, Qs = sketch_mats(P.A.n, P.B.n)
    r = P.r
    PZ = Ps.T @ res.Z          # 16 x k r
    YQ = res.Y.T @ Qs          # k r x 16
    steps = []
    for j in range(res.k):
        sl = slice(j * r, (j + 1) * r)
        steps.append((res.gammas[j] * (PZ[:, sl] @ YQ[sl, :])).tolist())
    xfro = OF.lowrank_fro(res.Z, res.D(), res.Y)
    fs, gs = OF.rescale_rhs(f, g)
    true = OF.lowrank_residual_norm(A, B, fs, gs, res.Z, res.D(), res.Y) / res.norm_fg
    out = {
        "what": "oracle LR-ADI with direct (SuperLU) inner solves on the 3-D configuration: "
                "A 64^3 omega (20,10,5), B 48^3 omega (-10,15,5), r=8, seed 3, "
                "24 Wachspress shifts, tau=1e-8",
        "k": res.k,
        "res_hist": res.res_hist,
        "norm_fg": res.norm_fg,
        "gammas": res.gammas.tolist(),
        "x_fro": xfro,
        "true_rel_residual": true,
        "sketch_seed": SKETCH_SEED,
        "sketch_k": SKETCH_K,
        "sketch_steps": steps,
        "wall_s": wall,
        "step_s_A": times["A"],
        "step_s_B": times["B"],
        "host": {"cpu_count": os.cpu_count(), "cpu_model": cpu_model(),
                 "lu": "scipy SuperLU, MMD_AT_PLUS_A, factor-solve-discard per step"},
    }
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", OUT, f"k={res.k} true={true:.3e} wall={wall:.0f} s")


if __name__ == "__main__":
    main()
