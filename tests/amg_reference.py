"""Plain numpy V-cycle over a hierarchy exported by the library
(`HostAmg`), used by the tests to check the device V-cycle element by
element and the quality of the hierarchy.  The AMG preconditioner is not
part of the paper's method (it only accelerates the inner solve that
applies A^{-1}, Section 4.1), so this is a test helper, not oracle code.

V-cycle on level l with right-hand side b:
  x = S(b, 0)             Chebyshev smoothing from zero, `degree` steps
  x += P_l V(P_l^T (b - A_l x), l + 1)
  x = S(b, x)             the same smoothing polynomial
with the coarsest level solved exactly.  Chebyshev smoothing on D^{-1} A
over [lmax / ratio, lmax] (Saad, Algorithm 12.1), ratio 10 for two or more
steps and 11 for one (damped Jacobi with weight 2 / (lmax (1 + 1/11))), as the
library chooses them:
  step 0: d = (1/theta) D^{-1} (b - A x);  x += d
  step k: d = rho_k rho_{k-1} d + (2 rho_k / delta) D^{-1} (b - A x);  x += d
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

EIG_RATIO = 10.0
JACOBI_RATIO = 11.0


def chebyshev_coefficients(lmax: float, degree: int, ratio: float | None = None):
    if ratio is None:
        ratio = JACOBI_RATIO if degree == 1 else EIG_RATIO
    lmin = lmax / ratio
    theta, delta = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    sigma = theta / delta
    rho = 1.0 / sigma
    cd, ad = [0.0], [1.0 / theta]
    for _ in range(1, degree):
        rn = 1.0 / (2.0 * sigma - rho)
        cd.append(rn * rho)
        ad.append(2.0 * rn / delta)
        rho = rn
    return cd, ad


class VCycle:
    def __init__(self, levels, degree: int = 2, coarse_degree=None):
        # `degree` Chebyshev steps on the finest level, `coarse_degree` (default:
        # the same) on the levels below it
        cdeg = degree if coarse_degree is None else coarse_degree
        self.deg = [degree if l == 0 else cdeg for l in range(len(levels))]
        self.A, self.P, self.dinv, self.coef = [], [], [], []
        for lv in levels:
            rp, ci, v = lv["A"]
            A = sp.csr_matrix((v, ci, rp), shape=(lv["n"], lv["n"]))
            self.A.append(A)
            self.dinv.append(1.0 / A.diagonal())
            if lv["P"] is not None:
                prp, pci, pv, nc = lv["P"]
                self.P.append(sp.csr_matrix((pv, pci, prp), shape=(lv["n"], nc)))
            self.coef.append(chebyshev_coefficients(lv["lmax"], self.deg[len(self.coef)]))
        self.coarse = np.linalg.inv(self.A[-1].toarray())

    def smooth(self, l, b, x):
        cd, ad = self.coef[l]
        A, dinv = self.A[l], self.dinv[l][:, None]
        d = None
        for k in range(self.deg[l]):
            r = b - A @ x
            dn = ad[k] * dinv * r
            if k > 0:
                dn = dn + cd[k] * d
            x = x + dn
            d = dn
        return x

    def apply(self, b, l: int = 0):
        b = np.asarray(b, dtype=np.float64)
        if b.ndim == 1:
            return self.apply(b[:, None], l)[:, 0]
        if l == len(self.A) - 1:
            return self.coarse @ b
        x = self.smooth(l, b, np.zeros_like(b))
        r = b - self.A[l] @ x
        xc = self.apply(self.P[l].T @ r, l + 1)
        x = x + self.P[l] @ xc
        return self.smooth(l, b, x)


def pcg(A, b, M, tol=1e-12, maxit=500):
    """Preconditioned CG (one column); returns (x, iterations)."""
    x = np.zeros_like(b)
    r = b.copy()
    z = M(r)
    p = z.copy()
    rz = r @ z
    bn = np.linalg.norm(b)
    for it in range(1, maxit + 1):
        q = A @ p
        a = rz / (p @ q)
        x += a * p
        r -= a * q
        if np.linalg.norm(r) <= tol * bn:
            return x, it
        z = M(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, maxit
