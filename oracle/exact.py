"""Plain definitions used to pin the oracle (test infrastructure).

r(M)B = omega_0 B + Re sum_j c_j (M - tau_j I)^{-1} B is the exact quantity
the iteration converges to (Section 2, eq. 2.5 with the conjugate pairs
folded); e^{M}B differs from it by the CF error.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .cf import cf_table


def rational_dense(M: np.ndarray, B: np.ndarray, table=None) -> np.ndarray:
    """r(M)B with one dense complex LU solve per pole."""
    tau, c, w0 = cf_table() if table is None else table
    n = M.shape[0]
    out = w0 * B.astype(np.float64)
    for tj, cj in zip(tau, c):
        Xj = np.linalg.solve(M - tj * np.eye(n), B.astype(complex))
        out = out + np.real(cj * Xj)
    return out


def rational_sparse(M: sp.spmatrix, B: np.ndarray, table=None) -> np.ndarray:
    """r(M)B with one sparse complex LU (SuperLU) per pole."""
    tau, c, w0 = cf_table() if table is None else table
    n = M.shape[0]
    Mc = sp.csc_matrix(M, dtype=complex)
    I = sp.identity(n, dtype=complex, format="csc")
    out = w0 * B.astype(np.float64)
    for tj, cj in zip(tau, c):
        lu = spla.splu(Mc - tj * I)
        out = out + np.real(cj * lu.solve(B.astype(complex)))
    return out


def expm_dense(M: np.ndarray, B: np.ndarray) -> np.ndarray:
    """e^{M}B by scipy's Pade scaling-and-squaring expm (n <= a few thousand)."""
    return sla.expm(M) @ B


def expm_eigh(M: np.ndarray, B: np.ndarray) -> np.ndarray:
    """e^{M}B for symmetric M through its eigendecomposition."""
    lam, Q = np.linalg.eigh(0.5 * (M + M.T))
    return Q @ (np.exp(lam)[:, None] * (Q.T @ B))
