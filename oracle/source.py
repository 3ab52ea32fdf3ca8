"""Linear ODE with an exponential source term (test infrastructure).

    u'(s) = A u(s) + e^{gamma s} b,   u(0) = u0,   solution at s = t.

Section 5, Example 5.3 evaluates it (gamma = -1) by variation of constants:
when A - gamma I is invertible, with w = (A - gamma I)^{-1} b,
    u(t) = e^{tA} (u0 + w) - e^{gamma t} w.
The rational form replaces both exponentials by the CF approximant r of
eq. 2.5 (M = tA, sigma = gamma t):
    u_r(t) = r(M) (u0 + w) - r(sigma) w = r(M) u0 + (r(M) - r(sigma)) w,
and the partial fractions of r turn (r(M) - r(sigma)) (M - sigma I)^{-1}
into sum_i omega_i (M - tau_i I)^{-1} / (tau_i - sigma), so
    u_r(t) = omega_0 u0 + sum_i omega_i (M - tau_i I)^{-1}
                               [u0 + t / (tau_i - sigma) b],
which needs no solve with A - gamma I (nor its invertibility).  Folding the
conjugate pairs as in eq. 2.5 (c_j = 2 omega_j over the poles with Im > 0):
    u_r(t) = omega_0 u0 + Re sum_j c_j (M - tau_j I)^{-1}
                               [u0 + t / (tau_j - sigma) b].
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .cf import cf_table, r_eval
from .exact import rational_dense


def exact_augmented(A: np.ndarray, u0: np.ndarray, b: np.ndarray, gamma: float,
                    t: float) -> np.ndarray:
    """u(t) by one dense exponential of the augmented system
    d/ds [u; v] = [[A, b], [0, gamma I_p]] [u; v], v(0) = I_p: then
    v(s) = e^{gamma s} I_p and u solves the ODE column by column."""
    n, p = u0.shape
    aug = np.zeros((n + p, n + p))
    aug[:n, :n] = A
    aug[:n, n:] = b
    aug[n:, n:] = gamma * np.eye(p)
    start = np.vstack([u0, np.eye(p)])
    return (sla.expm(t * aug) @ start)[:n]


def variation_of_constants(A: np.ndarray, u0: np.ndarray, b: np.ndarray, gamma: float,
                           t: float) -> np.ndarray:
    """The formula of Example 5.3 with dense expm and a dense solve for w."""
    n = A.shape[0]
    w = np.linalg.solve(A - gamma * np.eye(n), b)
    return sla.expm(t * A) @ (u0 + w) - np.exp(gamma * t) * w


def rational_via_w(A: np.ndarray, u0: np.ndarray, b: np.ndarray, gamma: float,
                   t: float) -> np.ndarray:
    """r(tA)(u0 + w) - r(gamma t) w with w = (A - gamma I)^{-1} b."""
    n = A.shape[0]
    w = np.linalg.solve(A - gamma * np.eye(n), b)
    r_sigma = float(np.real(r_eval(np.array([gamma * t]))[0]))
    return rational_dense(t * A, u0 + w) - r_sigma * w


def rational_dense_source(A: np.ndarray, u0: np.ndarray, b: np.ndarray, gamma: float,
                          t: float, table=None) -> np.ndarray:
    """u_r(t) by the partial-fraction form: one dense complex LU per pole."""
    tau, c, w0 = cf_table() if table is None else table
    n = A.shape[0]
    M = t * A
    sigma = gamma * t
    out = w0 * u0.astype(np.float64)
    for tj, cj in zip(tau, c):
        rhs = u0.astype(complex) + (t / (tj - sigma)) * b.astype(complex)
        Xj = np.linalg.solve(M - tj * np.eye(n), rhs)
        out = out + np.real(cj * Xj)
    return out
