"""Plain definitions used to pin the oracle and as GPU references (test
infrastructure).

r(M)B = omega_0 B + Re sum_j c_j (M - tau_j I)^{-1} B is the exact quantity
the iteration converges to (Section 2, eq. 2.5 with the conjugate pairs
folded); e^{M}B differs from it by the CF error.  Every function here forms
that sum from direct solves, one per pole; they differ only in how each
shifted system is solved.

Each sparse solve takes one step of fixed-precision iterative refinement
with its own factors (x <- x + LU^{-1}(b - (M - tau I) x), Higham, Accuracy
and Stability of Numerical Algorithms, 2nd ed., Section 12.2): the terms of
the sum are up to ~10^3 times larger than r(M)B on the operators used here,
so a solve accurate to 1e-12 alone would leave r(M)B accurate to 1e-9 only.
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


def _refined_solve(lu, S: sp.spmatrix, rhs: np.ndarray, trans: str = "N",
                   steps: int = 1) -> np.ndarray:
    """S^{-1} rhs (trans 'T': S^{-T} rhs) from the factors lu of S, followed
    by `steps` refinement steps with the residual formed in working
    precision."""
    op = S if trans == "N" else S.T
    x = lu.solve(rhs, trans=trans)
    for _ in range(steps):
        x = x + lu.solve(rhs - op @ x, trans=trans)
    return x


def rational_sparse(M: sp.spmatrix, B: np.ndarray, table=None, refine: int = 1) -> np.ndarray:
    """r(M)B with one sparse complex LU (SuperLU) per pole, each solve refined
    `refine` times."""
    tau, c, w0 = cf_table() if table is None else table
    n = M.shape[0]
    Mc = sp.csc_matrix(M, dtype=complex)
    I = sp.identity(n, dtype=complex, format="csc")
    out = w0 * B.astype(np.float64)
    Bc = B.astype(complex)
    for tj, cj in zip(tau, c):
        S = (Mc - tj * I).tocsc()
        lu = spla.splu(S)
        out = out + np.real(cj * _refined_solve(lu, S, Bc, steps=refine))
    return out


def rational_sparse_adjoint(M: sp.spmatrix, B: np.ndarray, G: np.ndarray, t: float,
                            table=None, refine: int = 1):
    """The forward result, the adjoint result and the t-derivative pairing of
    L = <G, r(tA)B> from one sparse complex LU of M - tau_j I per pole (M = tA):

        Z     = r(M) B      = omega_0 B + Re sum_j c_j X_j,   X_j = (M - tau_j I)^{-1} B
        gradB = r(M^T) G    = omega_0 G + Re sum_j c_j Y_j,   Y_j = (M - tau_j I)^{-T} G
        gt    = <G, A r(M) B> = (1/t) <G, M r(M) B>

    with M r(M) expanded by the partial fractions of x r(x) (x/(x - tau) =
    1 + tau/(x - tau)):  <G, M r(M) B> = omega_0 <G, M B> + Re(sum_j c_j) <G, B>
    + Re sum_j c_j tau_j <G, X_j>, so no operator is applied to a computed
    solution.  Y_j uses the transposed solve of the same factors (SuperLU
    trans='T', a plain transpose for complex data).  Every solve is refined
    `refine` times."""
    tau, c, w0 = cf_table() if table is None else table
    n = M.shape[0]
    Mc = sp.csc_matrix(M, dtype=complex)
    I = sp.identity(n, dtype=complex, format="csc")
    Z = w0 * B.astype(np.float64)
    gB = w0 * G.astype(np.float64)
    pair = w0 * float(np.sum(G * (sp.csr_matrix(M) @ B))) + float(np.real(np.sum(c))) * float(
        np.sum(G * B))
    Bc, Gc = B.astype(complex), G.astype(complex)
    for tj, cj in zip(tau, c):
        S = (Mc - tj * I).tocsc()
        lu = spla.splu(S)
        Xj = _refined_solve(lu, S, Bc, steps=refine)
        Z = Z + np.real(cj * Xj)
        pair += float(np.real(cj * tj * np.sum(G * Xj)))
        del Xj
        Yj = _refined_solve(lu, S, Gc, trans="T", steps=refine)
        gB = gB + np.real(cj * Yj)
        del Yj, lu, S
    return Z, gB, pair / t


def _tridiag_modes(a: float, b: float, c: float, N: int):
    """Eigen-decomposition of the N x N tridiagonal Toeplitz matrix with
    sub-diagonal a, diagonal b, super-diagonal c, a c > 0: with
    r = sqrt(a/c) and s_k(i) = sin((i+1)(k+1) pi/(N+1)),
    (T v)_i = a v_{i-1} + b v_i + c v_{i+1} for v_i = r^i s_k(i) gives
    r^i (sqrt(ac) sgn(a) (s_{i-1} + s_{i+1}) + b s_i), and
    s_{i-1} + s_{i+1} = 2 cos((k+1) pi/(N+1)) s_i, so
    lam_k = b + 2 sgn(a) sqrt(ac) cos((k+1) pi/(N+1)), V = diag(r^i) S with S the
    orthonormal (symmetric, involutory) DST-I matrix and V^{-1} = S diag(r^{-i})."""
    if not a * c > 0:
        raise ValueError("closed-form modes need a c > 0")
    i = np.arange(N)
    theta = (i + 1) * np.pi / (N + 1)
    lam = b + 2.0 * np.sign(a) * np.sqrt(a * c) * np.cos(theta)
    S = np.sqrt(2.0 / (N + 1)) * np.sin(np.outer(i + 1, i + 1) * np.pi / (N + 1))
    r = np.sqrt(a / c)
    V = (r ** i)[:, None] * S
    Vinv = S * (r ** (-i.astype(np.float64)))[None, :]
    return lam, V, Vinv


def rational_kron3_tridiag(N: int, coef, t: float, B: np.ndarray, table=None,
                           modes=None, refine: int = 1) -> np.ndarray:
    """r(M)B for M = -t K with K = T_x (+) T_y (+) T_z the Kronecker sum of three
    N x N tridiagonal Toeplitz matrices (coef[d] = (sub, diagonal, super) of
    T_d, axis d = 0, 1, 2 = x, y, z), unknowns ordered x fastest
    (index x + N y + N^2 z), B of shape (N^3, p).

    T_z is diagonalised in closed form (_tridiag_modes), so in the z-mode
    basis K splits into N two-dimensional operators K_xy + lam_k I.  Since V
    is real, Re commutes with it, and
        r(M) B = V_z [omega_0 Bh + Re sum_j c_j (-t (K_xy + lam_k I) - tau_j I)^{-1} Bh_k]
    with Bh = V_z^{-1} B taken along z; each 2-D shifted system is solved by a
    sparse complex LU (SuperLU), one per pole and z mode, refined `refine`
    times.  Only the z factor
    is diagonalised: cond(V_z) = r^{N-1} stays near e^{Pe v_z / 2} for the
    upwind operators used here (~5e2), where the x and y factors would be
    far worse conditioned.  `modes` (default: all) restricts the work to
    those z modes, the others contributing nothing: a bounded sample of the
    computation for timing (the result is then not r(M)B)."""
    tau, cc, w0 = cf_table() if table is None else table
    n2 = N * N
    p = B.shape[1]
    ax, bx, cx = coef[0]
    ay, by, cy = coef[1]
    Tx = sp.diags([np.full(N - 1, ax), np.full(N, bx), np.full(N - 1, cx)], [-1, 0, 1])
    Ty = sp.diags([np.full(N - 1, ay), np.full(N, by), np.full(N - 1, cy)], [-1, 0, 1])
    Iy = sp.identity(N)
    Kxy = (sp.kron(Iy, Tx) + sp.kron(Ty, sp.identity(N))).tocsc().astype(complex)
    lam, V, Vinv = _tridiag_modes(*coef[2], N)
    B3 = np.asarray(B, np.float64).reshape(N, n2, p)          # [z, xy, column]
    Bh = np.einsum("kz,zmp->kmp", Vinv, B3)
    Zh = w0 * Bh
    I2 = sp.identity(n2, dtype=complex, format="csc")
    base = (-t) * Kxy
    for k in (range(N) if modes is None else modes):
        rhs = Bh[k].astype(complex)
        acc = np.zeros((n2, p))
        for tj, cj in zip(tau, cc):
            S = (base - (t * lam[k] + tj) * I2).tocsc()
            lu = spla.splu(S)
            acc += np.real(cj * _refined_solve(lu, S, rhs, steps=refine))
        Zh[k] += acc
    return np.einsum("zk,kmp->zmp", V, Zh).reshape(N ** 3, p)


def expm_dense(M: np.ndarray, B: np.ndarray) -> np.ndarray:
    """e^{M}B by scipy's Pade scaling-and-squaring expm (n <= a few thousand)."""
    return sla.expm(M) @ B
