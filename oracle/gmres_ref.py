"""Oracle (test infrastructure only): the block minimal-residual iterate that
block GMRES produces for the shifted inner systems of Algorithm 1,
eq. (gfadi_incsolves), written as its definition.

For S = A + p I and a block right-hand side W (n x r), after j block steps
from a zero initial guess block GMRES returns

    Z_j = argmin { ||W - S Z||_F : Z has columns in K_j(S, W) },
    K_j(S, W) = span[W, S W, ..., S^{j-1} W],

each column of W being fitted with the whole block space.  Here the space is
spanned by an orthonormal basis built with dense QR (orthogonalised twice)
and the minimiser is a dense least-squares solve; nothing is blocked, fused
or updated incrementally.

Only tests/ use this module.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def block_krylov_basis(S, W: np.ndarray, j: int) -> np.ndarray:
    """Orthonormal basis (n x j r) of K_j(S, W)."""
    Q, _ = np.linalg.qr(W)
    basis = [Q]
    cur = Q
    for _ in range(1, j):
        nxt = np.asarray(S @ cur)
        V = np.hstack(basis)
        for _ in range(2):
            nxt = nxt - V @ (V.T @ nxt)
        cur, _ = np.linalg.qr(nxt)
        basis.append(cur)
    return np.hstack(basis)


def block_gmres_iterate(A, shift: float, W: np.ndarray, j: int, precond=None, M=None) -> np.ndarray:
    """Z_j of block GMRES on (A + shift I) Z = W (or (A + shift M) Z = W)
    after j block steps.  With a right preconditioner (precond(X) = P X) the
    space is P K_j(S P, W) and the minimised residual is still ||W - S Z||_F."""
    n = W.shape[0]
    E = sp.identity(n, format="csr") if M is None else sp.csr_matrix(M)
    S = sp.csr_matrix(A) + shift * E
    if precond is None:
        V = block_krylov_basis(S, W, j)
        SV = np.asarray(S @ V)
        C, *_ = np.linalg.lstsq(SV, W, rcond=None)
        return V @ C

    class _SM:
        def __matmul__(self, X):
            return np.asarray(S @ precond(X))

    V = block_krylov_basis(_SM(), W, j)
    MV = precond(V)
    SMV = np.asarray(S @ MV)
    C, *_ = np.linalg.lstsq(SMV, W, rcond=None)
    return MV @ C
