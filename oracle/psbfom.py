"""Shifted block FOM with deflated restarting, plain FP64 numpy (test
infrastructure, see the package docstring).

Algorithm 2 (PSBFOM-DR, Section 4.1) solves the nu/2 = 7 conjugate-pair
shifted systems (M - tau_j I) X_j = B, M = tA, all at once: with the
preconditioner A^{-1} the systems become (I - tau_j M^{-1}) Y_j = B,
X_j = M^{-1} Y_j (eq. 4.4), and one real block Krylov basis of M^{-1} serves
every shift (eq. 4.5, 4.6).  Algorithm 1 (SBFOM-DR, Section 3) is the same
loop on M itself (eq. 3.1-3.6).

Steps in the paper's order, with the readings used where the paper is silent:

 1-2. X_j = 0; V_1 R^ = B (QR with diag(R^) > 0); right-hand sides g_j = E_1 R^.
 3.   block Arnoldi with A. Ruhe's variant: one basis vector at a time,
      w = op(v_{i-p}), orthogonalised against every earlier vector (modified
      Gram-Schmidt, plus one re-orthogonalisation pass), h = ||w||.
 4.   projected systems (I - tau_j H_d) Z_j = g_j (eq. 4.7) [Alg. 1:
      (H_d - tau_j I) Z_j = g_j, eq. 3.4]; residual estimate (eq. 4.9)
      rho_j = |tau_j| ||H_{d+1,d} E^T Z_j||_F [Alg. 1: eq. 3.6].
      X_j += V_{d+p} (H~ Z_j), which is M^{-1} V_d Z_j by eq. 4.5, so no
      extra solve is needed [Alg. 1: X_j += V_d Z_j].
      Stop when the rule below holds.
 5.   eigenpairs of H_d; keep k of them: the k largest |theta| for
      Algorithm 2 (Remark 4.1: deflate the smallest |lambda(A)|, i.e. the
      largest Ritz values of A^{-1}), the k smallest for Algorithm 1; a
      complex pair is kept whole, so k_eff may be k+1.
 6.   P_k = orthonormalised [real parts, imaginary parts] of those vectors.
 7.   P_{k+p} = [[P_k; 0], [0; I_p]].
 8.   H~_new = P_{k+p}^T H~ P_k, V_new = V_{d+p} P_{k+p}.
 9.   continue Ruhe's Arnoldi from V_new for q = floor((mp - k_eff)/p) more
      blocks, d = k_eff + q p.  The residuals after a cycle are collinear:
      R_j = V_{d+1} S_j with S_j = tau_j H_{d+1,d} E^T Z_j (eq. 4.8), and the
      old V_{d+1} is the block of V_new right after the Ritz vectors, so the
      next right-hand side is g_j = [0; S_j; 0] with S_j at rows k_eff..k_eff+p.
 10.  Z~ = omega_0 B + Re sum_j c_j X_j (eq. 2.5 with the pairs folded).

Stopping rules ("stop_rule"):
  "paper": max_j rho_j <= tol * ||B||_F  (Step 4 with (4.9), relative form).
  "bound": sum_j |c_j| rho_j / delta_j <= tol * ||Z~||_F, delta_j the distance
           from tau_j to (-inf, 0]; for normal M this bounds
           ||Z~ - r(M)B||_F (||(M - tau I)^{-1}|| <= 1/delta).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .cf import cf_table


@dataclasses.dataclass
class Info:
    cycles: int = 0
    op_columns: int = 0            # number of columns op() was applied to
    converged: bool = False
    rho: list = dataclasses.field(default_factory=list)       # per cycle: array(7)
    bound: list = dataclasses.field(default_factory=list)     # per cycle: float
    znorm: list = dataclasses.field(default_factory=list)
    dims: list = dataclasses.field(default_factory=list)
    keff: list = dataclasses.field(default_factory=list)
    ritz: list = dataclasses.field(default_factory=list)
    history: list = dataclasses.field(default_factory=list)   # optional per-cycle Z~
    breakdown: bool = False


def _qr_positive(B):
    Q, R = np.linalg.qr(B)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :], R * s[:, None]


def _ruhe_extend(op, Vb, H, col_from, col_to, p, info, reorth=True, tiny=1e-13):
    """Ruhe's variant of block Arnoldi: generate basis columns col_from+p ..
    col_to+p-1 from the images of columns col_from .. col_to-1."""
    for kk in range(col_from, col_to):
        j = kk + p
        w = op(Vb[:, kk:kk + 1])[:, 0].copy()
        info.op_columns += 1
        wnorm0 = np.linalg.norm(w)
        for _pass in range(2 if reorth else 1):
            for i in range(j):
                hij = Vb[:, i] @ w
                H[i, kk] += hij
                w -= hij * Vb[:, i]
        hn = np.linalg.norm(w)
        if hn <= tiny * max(wnorm0, 1e-300):
            # (near) invariant subspace (the h = 0 stop of Ruhe's variant):
            # keep a zero column so every later block is empty too
            info.breakdown = True
            H[j, kk] = 0.0
            Vb[:, j] = 0.0
        else:
            H[j, kk] = hn
            Vb[:, j] = w / hn


def shifted_block_fom_dr(op, B, m, k, tol, *, preconditioned=True, table=None,
                         max_cycles=60, stop_rule="paper", keep_history=False,
                         reorth=True):
    """Core loop shared by Algorithm 1 (preconditioned=False, op = M) and
    Algorithm 2 (preconditioned=True, op = M^{-1}).  Returns (Z~, X, info)."""
    tau, c, omega0 = cf_table() if table is None else table
    nshift = len(tau)
    n, p = B.shape
    info = Info()
    D = (m + 1) * p + p + 2                     # room for k_eff + q p + p columns
    Vb = np.zeros((n, D))
    H = np.zeros((D, D))
    X = np.zeros((nshift, n, p), dtype=complex)
    V1, Rhat = _qr_positive(B)
    Vb[:, :p] = V1
    bnorm = np.linalg.norm(B)
    delta = np.where(tau.real >= 0, np.abs(tau), np.abs(tau.imag))
    # cycle 1: Arnoldi from block 1 for m blocks
    keff = 0
    d = m * p
    _ruhe_extend(op, Vb, H, 0, d, p, info, reorth)
    G = np.zeros((nshift, d, p), dtype=complex)
    G[:, :p, :] = Rhat[None, :, :]
    Zt = omega0 * B
    for cyc in range(max_cycles):
        info.cycles = cyc + 1
        info.dims.append(d)
        info.keff.append(keff)
        Hd = H[:d, :d]
        Hb = H[:d + p, :d]
        Hlast = H[d:d + p, :d]
        S = np.zeros((nshift, p, p), dtype=complex)
        rho = np.zeros(nshift)
        for jj in range(nshift):
            if preconditioned:
                Zj = np.linalg.solve(np.eye(d) - tau[jj] * Hd, G[jj])
                X[jj] += Vb[:, :d + p] @ (Hb @ Zj)
                S[jj] = tau[jj] * (Hlast @ Zj)
            else:
                Zj = np.linalg.solve(Hd - tau[jj] * np.eye(d), G[jj])
                X[jj] += Vb[:, :d] @ Zj
                S[jj] = -(Hlast @ Zj)
            rho[jj] = np.linalg.norm(S[jj])
        Zt = omega0 * B + np.real(np.einsum("j,jnp->np", c, X))
        znorm = np.linalg.norm(Zt)
        bound = float(np.sum(np.abs(c) * rho / delta))
        info.rho.append(rho)
        info.bound.append(bound)
        info.znorm.append(znorm)
        if keep_history:
            info.history.append(Zt.copy())
        if stop_rule == "paper":
            done = rho.max() <= tol * bnorm
        elif stop_rule == "bound":
            done = bound <= tol * znorm
        else:
            raise ValueError(stop_rule)
        if done or rho.max() == 0.0:
            info.converged = True
            break
        if cyc + 1 == max_cycles:
            break
        # Steps 5-8: deflated restart
        theta, Y = np.linalg.eig(Hd)
        order = np.argsort(-np.abs(theta)) if preconditioned else np.argsort(np.abs(theta))
        chosen = []
        cols = []
        for idx in order:
            if len(chosen) >= k:
                break
            if idx in chosen:
                continue
            th = theta[idx]
            if th.imag == 0.0:
                chosen.append(idx)
                cols.append(Y[:, idx].real)
            else:
                partner = [i for i in range(d) if i not in chosen and i != idx
                           and theta[i] == np.conj(th)]
                chosen.append(idx)
                if partner:
                    chosen.append(partner[0])
                cols.append(Y[:, idx].real)
                cols.append(Y[:, idx].imag)
        Pk, _ = np.linalg.qr(np.stack(cols, 1))
        keff_new = Pk.shape[1]
        info.ritz.append(theta[chosen])
        Pkp = np.zeros((d + p, keff_new + p))
        Pkp[:d, :keff_new] = Pk
        Pkp[d:, keff_new:] = np.eye(p)
        Hnew = Pkp.T @ Hb @ Pk                       # (keff+p) x keff
        Vnew = Vb[:, :d + p] @ Pkp
        Vb[:] = 0.0
        H[:] = 0.0
        Vb[:, :keff_new + p] = Vnew
        H[:keff_new + p, :keff_new] = Hnew
        keff = keff_new
        q = (m * p - keff) // p
        d = keff + q * p
        _ruhe_extend(op, Vb, H, keff, d, p, info, reorth)
        G = np.zeros((nshift, d, p), dtype=complex)
        G[:, keff:keff + p, :] = S
    return Zt, X, info


def psbfom_dr(apply_inv, B, m, k, tol, **kw):
    """Algorithm 2: apply_inv(V) returns M^{-1} V for an n x q block V."""
    return shifted_block_fom_dr(apply_inv, B, m, k, tol, preconditioned=True, **kw)


def sbfom_dr(apply_M, B, m, k, tol, **kw):
    """Algorithm 1 (unpreconditioned): apply_M(V) returns M V."""
    return shifted_block_fom_dr(apply_M, B, m, k, tol, preconditioned=False, **kw)
