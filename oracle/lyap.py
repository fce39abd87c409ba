"""Oracle (test infrastructure only): low-rank ADI for the (generalized)
Lyapunov equation

    A X M^T + M X A^T = -f f^T,

the special case B = A^T, C = M^T, g = f of the generalized Sylvester
equation (eq. (gsylv)) named among the related equations of Sec. 3.2.4.
With alpha_k = beta_k =: p_k (one shift per step, added to A) the B-side
system of eq. (lradi_g) is the A-side system, t_0 = w_0 = f, so y_k = z_k,
t_k = w_k and X_k = Z_k Gamma_k Z_k^T: one solve per step instead of two.
Written directly in the Lyapunov residual-factor form:

    z_k = (A + p_k M)^{-1} w_{k-1},   w_k = w_{k-1} - 2 p_k M z_k,
    gamma_k = -2 p_k,                 w_0 = f,

stopping once ||w_k w_k^T|| = ||w_k||^2 < tau ||f f^T|| = tau ||f||^2
(the while-condition of Algorithm 1 with t = w), with sparse-direct
("exact") solves.  Independent of the Sylvester oracle; tests compare the
two.  No rescaling: f and g are the same matrix.

Only tests/, the smoke check and the bench's CPU baseline use this module;
the product path never imports it.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _norm2(X: np.ndarray) -> float:
    """||X||_2 by a dense SVD."""
    if X.size == 0:
        return 0.0
    return float(np.linalg.svd(X, compute_uv=False)[0])


@dataclasses.dataclass
class LyapResult:
    Z: np.ndarray            # n x (k r)
    gammas: np.ndarray       # k
    W: np.ndarray            # final residual factor w_k
    res_hist: List[float]    # ||w_j||^2 / ||f||^2, j = 1..k
    norm_ff: float           # ||f f^T|| = ||f||^2
    k: int
    nMz: List[float]         # ||M z_j|| (||z_j|| for M = I)

    def D(self) -> np.ndarray:
        r = self.Z.shape[1] // max(self.k, 1) if self.k else 0
        return np.repeat(self.gammas, r)

    def X(self) -> np.ndarray:
        """Dense Z Gamma Z^T (small problems only)."""
        return (self.Z * self.D()) @ self.Z.T


def lyap_adi(A: sp.spmatrix, f: np.ndarray, p: np.ndarray, tol: float = 1e-8,
             kmax: int = 50, kfixed: Optional[int] = None, M=None) -> LyapResult:
    """Low-rank Lyapunov ADI with direct solves; p holds the shifts added to
    A (cycled), M = None means the identity; kfixed runs exactly that many
    steps."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    E = sp.identity(n, format="csr") if M is None else sp.csr_matrix(M)
    W = np.array(f, dtype=np.float64, copy=True)
    nff = _norm2(W) ** 2
    lus = {}
    Zs, gam, hist, nMz = [], [], [], []
    k = 0
    while nff > 0.0:
        if kfixed is not None:
            if k >= kfixed:
                break
        elif k >= kmax or _norm2(W) ** 2 < tol * nff:
            break
        pk = float(p[k % len(p)])
        if pk not in lus:
            lus[pk] = spla.splu((A + pk * E).tocsc())
        z = lus[pk].solve(W).reshape(W.shape)
        Mz = np.asarray(E @ z)
        W = W - 2.0 * pk * Mz
        Zs.append(z)
        gam.append(-2.0 * pk)
        nMz.append(_norm2(Mz))
        k += 1
        hist.append(_norm2(W) ** 2 / nff)
    Z = np.hstack(Zs) if Zs else np.zeros((n, 0))
    return LyapResult(Z, np.asarray(gam), W, hist, nff, k, nMz)
