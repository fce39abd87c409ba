"""Oracle (test infrastructure only): the right preconditioner of the inner
block GMRES solves.

The paper's inner Krylov solvers are preconditioned (Sec. 3.2.4 asks for
right preconditioning so that the solver's residual is the true inner
residual; Table 1 lists incomplete LU / Cholesky factorizations).  The
preconditioner here is an incomplete LU factorization with zero fill,
ILU(0), of S = A + s I in red-black order, for matrices whose sparsity graph
is bipartite (the 2-D five-point and 3-D seven-point stencils of the test
operators are).  Written as the block elimination it is:

    S = [[D_r, E], [F, D_b]]   (red rows first; D_r, D_b diagonal),
    y_r = v_r,                  y_b = v_b - F D_r^{-1} v_r,
    z_b ~ T^{-1} y_b,           z_r = D_r^{-1} (v_r - E z_b),

with T = D_b - F D_r^{-1} E the exact Schur complement on the black rows.
ILU(0) keeps only T's diagonal (T's off-diagonal entries are fill outside
S's pattern), so z_b = diag(T)^{-1} y_b; `sweeps` > 0 refines z_b by that
many Jacobi steps on T y = ... (z_b += diag(T)^{-1} (y_b - T z_b)), which
tends to the exact block solve (and M to S^{-1}) when Jacobi converges.

poly="chebyshev" replaces the Jacobi steps by the Chebyshev semi-iterative
method (Golub and Varga) on the same splitting, an acceleration that is not
in the paper.  With J = I - diag(T)^{-1} T and its spectrum assumed real and
inside [lo, hi] (bounds below), the extrapolated iteration
x <- G x + gamma c, G = gamma J + (1 - gamma) I, c = diag(T)^{-1} y_b,
gamma = 2 / (2 - lo - hi), has its spectrum in [-sigma, sigma],
sigma = (hi - lo) / (2 - lo - hi).  From x_0 = 0: x_1 = gamma c and, for
k >= 1, x_{k+1} = omega_{k+1} (G x_k + gamma c - x_{k-1}) + x_{k-1} with
omega_2 = 2 / (2 - sigma^2), omega_{k+1} = 1 / (1 - sigma^2 omega_k / 4): the
error after k steps is T_{k+1}(G / sigma) / T_{k+1}(1 / sigma) times the
initial one (T_k the Chebyshev polynomials).  The same number of products
with T as the Jacobi sweeps.  Bounds, each a Gershgorin argument that holds
when T is similar by a diagonal to a symmetric matrix (constant-coefficient
upwind stencils are): hi = max_i sum_{j != i} sqrt(|T_ij T_ji| / |T_ii T_jj|)
(row sums of the symmetrised J) and lo = -max(0, max_i P_ii / T_ii) with
P = F D_r^{-1} E, T = D_b - P (J's off-diagonal part is diag(T)^{-1} times
P's, whose symmetrised form is semidefinite).  hi >= 1 (no diagonal
dominance) falls back to the Jacobi steps.

For a pencil A + s M (the generalized equation) the preconditioner is built
from A + s diag(M 1), M replaced by its row sums (mass lumping): the same
bipartite pattern as A, while the Krylov solver still multiplies by the
true pencil.

Only tests/ and the bench's CPU baseline use this module.
"""
from __future__ import annotations

from collections import deque
from typing import Optional

import numpy as np
import scipy.sparse as sp


def two_coloring(A) -> Optional[np.ndarray]:
    """0/1 colour per row such that no off-diagonal entry of A or A^T joins
    two rows of one colour, the lowest-numbered row of every connected
    component coloured 0; None if the graph is not bipartite.  Breadth-first
    search over the symmetrised pattern."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    G = (abs(A) + abs(A.T)).tocsr()
    G.setdiag(0)
    G.eliminate_zeros()
    col = -np.ones(n, dtype=np.int64)
    for s in range(n):
        if col[s] >= 0:
            continue
        col[s] = 0
        q = deque([s])
        while q:
            u = q.popleft()
            for v in G.indices[G.indptr[u]:G.indptr[u + 1]]:
                if col[v] < 0:
                    col[v] = 1 - col[u]
                    q.append(v)
                elif col[v] == col[u]:
                    return None
    return col


def schur_poly_bounds(T, sdiag_b: np.ndarray):
    """(lo, hi): the interval the Chebyshev steps assume for the spectrum of
    J = I - diag(T)^{-1} T, from T and the black rows' diagonal of S (module
    docstring)."""
    T = sp.csr_matrix(T)
    td = T.diagonal()
    off = (T - sp.diags(td)).tocsr()
    prod = off.multiply(off.T).tocsr()
    prod.data = np.sqrt(np.abs(prod.data))
    rs = np.asarray((sp.diags(1.0 / np.sqrt(np.abs(td))) @ prod @ sp.diags(1.0 / np.sqrt(np.abs(td))))
                    .sum(axis=1)).ravel()
    hi = float(rs.max()) if rs.size else 0.0
    ratio = (sdiag_b - td) / td
    lo = -max(0.0, float(ratio.max()) if ratio.size else 0.0)
    return lo, hi


def chebyshev_coefficients(lo: float, hi: float, k: int):
    """(gamma, [omega_2, ..., omega_{k+1}]) of the Chebyshev steps for the
    interval [lo, hi]; None when hi >= 1 (module docstring)."""
    if not hi < 1.0:
        return None
    gamma = 2.0 / (2.0 - lo - hi)
    sigma = (hi - lo) / (2.0 - lo - hi)
    om = []
    for step in range(1, k + 1):
        om.append(2.0 / (2.0 - sigma * sigma) if step == 1 else 1.0 / (1.0 - sigma * sigma * om[-1] / 4.0))
    return gamma, om


def rb_precond_apply(A, shift: float, V: np.ndarray, sweeps: int = 0, mass=None,
                     poly: str = "jacobi") -> np.ndarray:
    """M V for the red-black ILU(0) of A + shift I, or of A + shift diag(mass 1)
    when a mass matrix is given (module docstring), with `sweeps` extra Jacobi
    steps on the Schur complement, or as many Chebyshev steps
    (poly="chebyshev")."""
    if poly not in ("jacobi", "chebyshev"):
        raise ValueError("poly must be 'jacobi' or 'chebyshev'")
    A = sp.csr_matrix(A)
    n = A.shape[0]
    col = two_coloring(A)
    if col is None:
        raise ValueError("sparsity graph is not bipartite")
    red = np.where(col == 0)[0]
    blk = np.where(col == 1)[0]
    if mass is None:
        S = (A + shift * sp.identity(n, format="csr")).tocsr()
    else:
        lump = np.asarray(sp.csr_matrix(mass).sum(axis=1)).ravel()
        S = (A + shift * sp.diags(lump)).tocsr()
    d = S.diagonal()
    E = S[red][:, blk]
    F = S[blk][:, red]
    dr, db = d[red], d[blk]
    V = np.asarray(V, dtype=np.float64)
    vr, vb = V[red], V[blk]
    yb = vb - F @ (vr / dr[:, None])
    # the exact Schur complement and its diagonal
    T = sp.diags(db) - F @ sp.diags(1.0 / dr) @ E
    tdiag = T.diagonal()
    zb = yb / tdiag[:, None]
    coef = None
    if poly == "chebyshev" and sweeps > 0:
        coef = chebyshev_coefficients(*schur_poly_bounds(T, db), sweeps)
    if coef is None:
        for _ in range(sweeps):
            zb = zb + (yb - T @ zb) / tdiag[:, None]
    else:
        gamma, om = coef
        prev = np.zeros_like(zb)
        zb = gamma * zb
        for w in om:
            g = zb + gamma * (yb - T @ zb) / tdiag[:, None]
            prev, zb = zb, w * (g - prev) + prev
    zr = (vr - E @ zb) / dr[:, None]
    Z = np.empty_like(V)
    Z[red] = zr
    Z[blk] = zb
    return Z


def ilu0_dense(S: np.ndarray):
    """Textbook ILU(0) (IKJ order) of a small dense-stored matrix: unit lower
    L and upper U with (L U)_ij = S_ij wherever S_ij != 0, no fill elsewhere.
    Pure loops, for pinning the block form on tiny inputs."""
    n = S.shape[0]
    nz = S != 0.0
    Wm = S.astype(np.float64).copy()
    for i in range(1, n):
        for k in range(i):
            if not nz[i, k]:
                continue
            Wm[i, k] = Wm[i, k] / Wm[k, k]
            for j in range(k + 1, n):
                if nz[i, j]:
                    Wm[i, j] -= Wm[i, k] * Wm[k, j]
    L = np.tril(Wm, -1) + np.eye(n)
    U = np.triu(Wm)
    return L, U
