"""Oracle (test infrastructure only): the low-rank factored ADI iteration for
A X + X B = -f g^T (eq. (sylv)) with sparse-direct ("exact") inner solves.

This follows Algorithm 1 (inexact LR-ADI) in the residual-factor form of
eq. (lradi_basic):

    z_k = (A + beta_k I)^{-1} w_{k-1},        w_k = w_{k-1} + gamma_k z_k,
    y_k = (B + alpha_k I)^{-*} t_{k-1},       t_k = t_{k-1} + conj(gamma_k) y_k,
    gamma_k = -(beta_k + alpha_k),            w_0 = f, t_0 = g,

and, given M and C, for the generalized equation A X C + M X B = -f g^T
(eq. (gsylv)) in the form of eq. (lradi_g):

    z_k = (A + beta_k M)^{-1} w_{k-1},        w_k = w_{k-1} + gamma_k M z_k,
    y_k = (B + alpha_k C)^{-*} t_{k-1},       t_k = t_{k-1} + conj(gamma_k) C^* y_k,

and returns Z_k, Gamma_k = diag(gamma_1 I_r, ..., gamma_k I_r), Y_k with
X ~ Z_k Gamma_k Y_k^*.  The loop runs while ||w_{k-1} t_{k-1}^*|| >= tau ||f g^T||
(the while-condition of Algorithm 1; spectral norm, Sec. 1.1).

Shift naming used throughout: pA[k] is the shift added to A (beta_k of
Algorithm 1), pB[k] the shift added to B^T = B^* (conj(alpha_k) for the real
B of every workload); so gamma_k = -(pA[k] + conj(pB[k])), which is
-(pA[k] + pB[k]) for real shifts.  Complex shifts run the complex form of the
iteration as printed (complex w_k, t_k, z_k, y_k, gamma_k; X ~ Z Gamma Y^*),
which Sec. 3.2.4 keeps for complex shift parameters.  Shift arrays are cycled
when the iteration runs longer than they are.

Only tests/, the smoke check and the bench's CPU baseline use this module;
the product path never imports it.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def spectral_norm(M: np.ndarray) -> float:
    """||M||_2 (largest singular value) by a dense SVD."""
    if M.size == 0:
        return 0.0
    return float(np.linalg.svd(M, compute_uv=False)[0])


def lowrank_product_norm(W: np.ndarray, T: np.ndarray) -> float:
    """||W T^*||_2 without forming the n x m product: with thin QR factors
    W = Q_w R_w and T = Q_t R_t, ||W T^*|| = ||R_w R_t^*|| (Sec. 2.1 uses this
    to evaluate the residual norm cheaply from the rank-r factors)."""
    Rw = np.linalg.qr(W, mode="r")
    Rt = np.linalg.qr(T, mode="r")
    return spectral_norm(Rw @ Rt.conj().T)


def rescale_rhs(f: np.ndarray, g: np.ndarray):
    """Scale f and g to equal spectral norm keeping f g^T unchanged (the
    experiments of Sec. 4 rescale the random factors so that ||f|| = ||g||)."""
    nf, ng = spectral_norm(f), spectral_norm(g)
    s = np.sqrt(ng / nf)
    return f * s, g / s


@dataclasses.dataclass
class FadiResult:
    Z: np.ndarray            # n x (k r)
    Y: np.ndarray            # m x (k r)
    gammas: np.ndarray       # k
    W: np.ndarray            # final residual factor w_k
    T: np.ndarray            # final residual factor t_k
    res_hist: List[float]    # ||w_j t_j^*|| / ||f g^T||, j = 1..k
    norm_fg: float
    k: int
    rA: List[np.ndarray]     # inner residuals r^A_j = w_{j-1} - (A + pA_j M) z_j
    rB: List[np.ndarray]     # inner residuals r^B_j = t_{j-1} - (B^T + pB_j C^T) y_j
    nMz: List[float] = dataclasses.field(default_factory=list)  # ||M z_j||
    nCy: List[float] = dataclasses.field(default_factory=list)  # ||C^T y_j||

    def D(self) -> np.ndarray:
        r = self.Z.shape[1] // max(self.k, 1) if self.k else 0
        return np.repeat(self.gammas, r)

    def X(self) -> np.ndarray:
        """Dense Z Gamma Y^* (small problems only)."""
        return (self.Z * self.D()) @ self.Y.conj().T


def _direct_solver(Op: sp.spmatrix, cache: Optional[dict], shift: float, mass=None,
                   permc_spec: Optional[str] = None) -> Callable:
    """LU of Op + shift * mass (mass = I when None), once per distinct shift
    (cache = None: factor for this one solve and discard).  permc_spec picks
    SuperLU's column ordering (None: its default); it changes the fill of
    the factors, not what is solved."""
    key = complex(shift) if np.iscomplexobj(shift) else float(shift)
    if cache is not None and key in cache:
        return cache[key].solve
    n = Op.shape[0]
    E = sp.identity(n, format="csr") if mass is None else mass
    kw = {} if permc_spec is None else {"permc_spec": permc_spec}
    lu = spla.splu((Op + shift * E).tocsc(), **kw)
    if cache is not None:
        cache[key] = lu
    return lu.solve


def fadi(A: sp.spmatrix, B: sp.spmatrix, f: np.ndarray, g: np.ndarray,
         pA: np.ndarray, pB: np.ndarray, tol: float = 1e-8, kmax: int = 50,
         rescale: bool = True, solve_A: Optional[Callable] = None,
         solve_B: Optional[Callable] = None, kfixed: Optional[int] = None,
         M=None, C=None, keep_factors: bool = True, permc_spec: Optional[str] = None,
         log: Optional[Callable] = None) -> FadiResult:
    """Algorithm 1 with direct inner solves (the "direct solves" rows of Table 2).

    solve_A(k, shift, rhs) / solve_B(k, shift, rhs) may replace the direct
    solves (used by tests that plant inexact solves); by default each distinct
    shift is LU-factorised once (SuperLU).  keep_factors = False factors per
    solve and discards (for large 3-D operators whose factors do not fit
    many at a time); permc_spec selects SuperLU's column ordering.  kfixed
    runs exactly that many steps ignoring tau.  M, C (None = identity) give
    the generalized equation (eq. (gsylv), iteration (lradi_g)).  log(k,
    res) is called after each step.  Returns the factors, the computed
    residual history and the inner residual blocks."""
    A = sp.csr_matrix(A)
    Bt = sp.csr_matrix(B).conj().T.tocsr()          # B^* (B^T for real B)
    Mm = None if M is None else sp.csr_matrix(M)
    Ct = None if C is None else sp.csr_matrix(C).conj().T.tocsr()
    f = np.array(f, dtype=np.result_type(f, np.float64), copy=True)
    g = np.array(g, dtype=np.result_type(g, np.float64), copy=True)
    if rescale:
        f, g = rescale_rhs(f, g)
    norm_fg = lowrank_product_norm(f, g)
    cacheA, cacheB = ({}, {}) if keep_factors else (None, None)
    W, T = f.copy(), g.copy()
    Zs, Ys, gam, hist, rA, rB, nMz, nCy = [], [], [], [], [], [], [], []
    J = len(pA)
    k = 0
    while True:
        if norm_fg == 0.0:
            break          # f g^T = 0: X = 0 is exact, nothing to iterate
        if kfixed is not None:
            if k >= kfixed:
                break
        else:
            if k >= kmax or lowrank_product_norm(W, T) < tol * norm_fg:
                break
        a, b = pA[k % J], pB[k % J]
        a = complex(a) if np.iscomplexobj(a) else float(a)
        b = complex(b) if np.iscomplexobj(b) else float(b)
        if solve_A is None:
            z = _direct_solver(A, cacheA, a, Mm, permc_spec)(W)
        else:
            z = solve_A(k, a, W)
        if solve_B is None:
            y = _direct_solver(Bt, cacheB, b, Ct, permc_spec)(T)
        else:
            y = solve_B(k, b, T)
        z = np.asarray(z).reshape(W.shape)
        y = np.asarray(y).reshape(T.shape)
        Mz = z if Mm is None else np.asarray(Mm @ z)
        Cy = y if Ct is None else np.asarray(Ct @ y)
        rA.append(W - (A @ z + a * Mz))
        rB.append(T - (Bt @ y + b * Cy))
        # gamma_k = -(beta_k + alpha_k) with pA = beta_k, pB = conj(alpha_k)
        gk = -(a + np.conj(b))
        W = W + gk * Mz
        T = T + np.conj(gk) * Cy
        nMz.append(spectral_norm(Mz))
        nCy.append(spectral_norm(Cy))
        Zs.append(z)
        Ys.append(y)
        gam.append(gk)
        k += 1
        hist.append(lowrank_product_norm(W, T) / norm_fg)
        if log is not None:
            log(k, hist[-1])
    n, r = f.shape
    m = g.shape[0]
    Z = np.hstack(Zs) if Zs else np.zeros((n, 0))
    Y = np.hstack(Ys) if Ys else np.zeros((m, 0))
    return FadiResult(Z, Y, np.asarray(gam), W, T, hist, norm_fg, k, rA, rB, nMz, nCy)


def true_residual_dense(A, B, f, g, X, M=None, C=None) -> np.ndarray:
    """Sylvester residual A X C + M X B + f g^T as a dense matrix (the sign
    that makes the k = 0 residual equal f g^T, eq. (adi_res_inexact));
    M, C = None mean identity."""
    A = sp.csr_matrix(A)
    B = sp.csr_matrix(B)
    AX = np.asarray(A @ X)
    AXC = AX if C is None else np.asarray((sp.csr_matrix(C).T @ AX.T).T)
    MX = X if M is None else np.asarray(sp.csr_matrix(M) @ X)
    return AXC + np.asarray((B.T @ MX.T).T) + f @ g.conj().T


def lowrank_residual_norm(A, B, f, g, Z, d, Y, M=None, C=None) -> float:
    """||A Z D Y^* C + M Z D Y^* B + f g^*||_2 exactly, without forming n x m
    matrices: the residual equals U V^* with U = [A Z, M Z, f] and
    V = [C^* Y D^*, B^* Y D^*, g]; with thin QRs U = Q_u R_u, V = Q_v R_v its
    norm is ||R_u R_v^*||_2.  d holds the diagonal of D; M, C = None mean
    identity (real matrices; Z, d, Y may be complex)."""
    A = sp.csr_matrix(A)
    Bt = sp.csr_matrix(B).conj().T.tocsr()
    YD = Y * np.conj(d)
    MZ = Z if M is None else np.asarray(sp.csr_matrix(M) @ Z)
    CtYD = YD if C is None else np.asarray(sp.csr_matrix(C).conj().T @ YD)
    U = np.hstack([np.asarray(A @ Z), MZ, f])
    V = np.hstack([CtYD, np.asarray(Bt @ YD), g])
    Ru = np.linalg.qr(U, mode="r")
    Rv = np.linalg.qr(V, mode="r")
    return spectral_norm(Ru @ Rv.conj().T)


def lowrank_diff_fro(Z1, d1, Y1, Z2, d2, Y2) -> float:
    """||Z1 D1 Y1^* - Z2 D2 Y2^*||_F without forming the n x m matrices."""
    L = np.hstack([Z1 * d1, -(Z2 * d2)])
    R = np.hstack([Y1, Y2])
    Rl = np.linalg.qr(L, mode="r")
    Rr = np.linalg.qr(R, mode="r")
    return float(np.linalg.norm(Rl @ Rr.conj().T, "fro"))


def lowrank_fro(Z, d, Y) -> float:
    """||Z D Y^*||_F without forming it."""
    Rl = np.linalg.qr(Z * d, mode="r")
    Rr = np.linalg.qr(Y, mode="r")
    return float(np.linalg.norm(Rl @ Rr.conj().T, "fro"))


def bartels_stewart(A, B, f, g) -> np.ndarray:
    """Dense reference solution of A X + X B = -f g^T (Bartels-Stewart via
    scipy.linalg.solve_sylvester); small n, m only."""
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A)
    Bd = B.toarray() if sp.issparse(B) else np.asarray(B)
    return sla.solve_sylvester(Ad, Bd, -f @ g.T)
