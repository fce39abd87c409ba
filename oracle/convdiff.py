"""Oracle (test infrastructure only): CSR of the upwind convection-diffusion
coefficient matrices of Sec. 4, eq. (ex:convdiff).

L(u) = -Lap u + omega^T grad u on the open unit square/cube, N interior grid
points per axis, mesh width h = 1/(N+1), homogeneous Dirichlet boundary
(neighbours outside the grid are dropped), lexicographic ordering with the
first axis fastest.  The first-order term is discretised upwind (backward
difference for omega_c > 0, forward for omega_c < 0).  The Sylvester
coefficient is A = -L_h, so that Lambda(A) lies in the open left half plane
as Sec. 2 assumes (Table 1 writes the preconditioners for -A).

Floating-point recipe, fixed so that an independent implementation can
reproduce every stored value bit for bit: with ih = N+1 and ih2 = ih*ih, the
coefficient of u at p - s_c is -ih2 - max(w_c,0)*ih, at p + s_c it is
-ih2 - max(-w_c,0)*ih, and the diagonal is the sum over c = 0..d-1 (starting
from 0.0) of 2*ih2 + |w_c|*ih, every product and sum rounded separately (no
fused multiply-add).  All values are then negated.  Columns ascend within a
row.

Only tests/, the smoke check and the bench's CPU baseline use this module.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def convdiff_csr(dim: int, N: int, omega, negate: bool = True, scheme: str = "upwind"):
    """Return (rowptr int32, colind int32, val float64) of A = -L_h (or L_h
    when negate=False).  scheme "central" discretises the first-order term by
    central differences, w_c (u_{p+s_c} - u_{p-s_c}) / (2h): neighbours
    -ih2 -+ (w_c ih)/2 (the product w_c ih halved, an exact scaling), diagonal
    the sum of 2 ih2; its spectrum is complex once |w_c| h / 2 > 1."""
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    if len(omega) != dim:
        raise ValueError("omega needs one component per axis")
    if scheme not in ("upwind", "central"):
        raise ValueError("scheme must be upwind or central")
    ih = float(N + 1)
    ih2 = ih * ih
    if scheme == "central":
        lo = [-ih2 - (float(w) * ih) * 0.5 for w in omega]
        hi = [-ih2 + (float(w) * ih) * 0.5 for w in omega]
        diag = 0.0
        for _ in omega:
            diag = diag + 2.0 * ih2
    else:
        lo = [-ih2 - max(float(w), 0.0) * ih for w in omega]     # coefficient of u_{p - s_c}
        hi = [-ih2 - max(-float(w), 0.0) * ih for w in omega]    # coefficient of u_{p + s_c}
        diag = 0.0
        for w in omega:
            diag = diag + (2.0 * ih2 + abs(float(w)) * ih)
    n = N ** dim
    p = np.arange(n, dtype=np.int64)
    stride = [N ** c for c in range(dim)]
    coord = [(p // stride[c]) % N for c in range(dim)]
    # candidate neighbours in ascending column order:
    # p - s_{d-1}, ..., p - s_0, p, p + s_0, ..., p + s_{d-1}
    cand_col, cand_val, cand_ok = [], [], []
    for c in reversed(range(dim)):
        cand_col.append(p - stride[c])
        cand_val.append(np.full(n, lo[c]))
        cand_ok.append(coord[c] > 0)
    cand_col.append(p)
    cand_val.append(np.full(n, diag))
    cand_ok.append(np.ones(n, dtype=bool))
    for c in range(dim):
        cand_col.append(p + stride[c])
        cand_val.append(np.full(n, hi[c]))
        cand_ok.append(coord[c] < N - 1)
    col = np.stack(cand_col, axis=1)
    val = np.stack(cand_val, axis=1)
    ok = np.stack(cand_ok, axis=1)
    counts = ok.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum(counts)
    colind = col[ok]                 # row-major traversal keeps rows and column order
    vals = val[ok]
    if negate:
        vals = -vals
    return (rowptr.astype(np.int32), colind.astype(np.int32), vals.astype(np.float64))


def convdiff_matrix(dim: int, N: int, omega, negate: bool = True, scheme: str = "upwind") -> sp.csr_matrix:
    """scipy CSR view of convdiff_csr."""
    rp, ci, v = convdiff_csr(dim, N, omega, negate, scheme)
    n = N ** dim
    return sp.csr_matrix((v, ci, rp), shape=(n, n))
