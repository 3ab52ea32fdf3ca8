"""Caratheodory-Fejer (CF) rational approximation of e^x on (-inf, 0].

Test infrastructure (see the package docstring): not part of the product.

Paper, Section 2: the CF approximant of type (nu, nu) is built from the
singular value decomposition of a Hankel matrix of Chebyshev coefficients of
e^x transplanted from R^- to [-1, 1]; written in partial fractions it is

    r(x) = omega_0 + sum_{i=1}^{nu} omega_i / (x - tau_i)

and e^A B ~= omega_0 B + sum_i omega_i (A - tau_i I)^{-1} B       (eq. 2.5).
The poles come in conjugate pairs, so for real data only nu/2 systems are
needed: r(x) = omega_0 + Re sum_{j=1}^{nu/2} c_j / (x - tau_j) with
Im tau_j > 0 and c_j = 2 omega_j.

The paper defers the construction to Trefethen et al.; the steps below are
the classical CF construction written out from its mathematics:

 1. transplant x = s_c (s - 1)/(s + 1), s in [-1, 1] (s_c = 9 here);
 2. f(s) = exp(x(s)); on the unit circle s = (z + 1/z)/2 its Fourier
    coefficients a_k (k >= 0) are the halved Chebyshev coefficients;
 3. the Hankel matrix H_ij = a_{1+i+j} (i, j < K) is real symmetric; take the
    eigenpair (lam, v) whose |lam| is the (nu+1)-st largest singular value;
 4. the nu roots zeta of P(z) = sum_j v_j z^{K-1-j} with |zeta| > 1 are the
    poles in the z plane; tau = s_c (zeta - 1)^2 / (zeta + 1)^2;
 5. on |z| = 1 the extended approximant is R~(z) = G(z) - lam z v(z)/v(1/z)
    with G(z) = sum_{k<=K} a_k z^k; multiplying by q(z) = prod (z - zeta)
    and keeping powers 0..nu gives the numerator p (the negative powers are
    the terms the paper says are dropped), so R = p/q;
 6. the real approximant is 2 Re R(z) - a_0.  Its residue at tau in the x
    variable is res_z(p/q, zeta) * dx/dz = res_z * 4 s_c (zeta-1)/(zeta+1)^3,
    and omega_0 = r(-inf) = 2 Re R(-1) - a_0.

Pins (tests/test_oracle_cf.py): the max error on (-inf, 0] is of the order
10^-nu (Section 2), the error curve equioscillates at >= 2 nu + 2 points
(best-approximation characterisation; CF equals best to O(56^-nu),
Section 2), max |tau| ~= 18.9 (Remark 2.1), poles in conjugate pairs.
"""
from __future__ import annotations

import functools
import json
import os

import numpy as np

NU = 14
SCALE = 9.0
HANKEL_K = 75
_TABLE_JSON = os.path.join(os.path.dirname(__file__), "cf_nu14_oracle.json")


def _poles_from_vector_np(v: np.ndarray, nu: int) -> np.ndarray:
    roots = np.roots(v)                     # v[0] is the leading coefficient
    out = roots[np.abs(roots) > 1.0]
    if len(out) != nu:
        raise RuntimeError(f"CF: expected {nu} roots outside the disk, got {len(out)}")
    return out


def cf_table_mp(nu: int = NU, scale: float = SCALE, K: int = HANKEL_K,
                nfft: int = 1024, dps: int = 40):
    """High-precision CF table.  Returns (tau_up, c_up, omega0) as mpmath
    numbers: the nu/2 poles with Im tau > 0, c_j = 2 omega_j, and omega_0."""
    import mpmath as mp
    mp.mp.dps = dps
    sc = mp.mpf(scale)
    ths = [2 * mp.pi * j / nfft for j in range(nfft)]
    fvals = []
    for th in ths:
        s = mp.cos(th)
        fvals.append(mp.mpf(0) if s + 1 < mp.mpf(10) ** (-dps + 5)
                     else mp.exp(sc * (s - 1) / (s + 1)))
    a = [mp.fsum(fvals[j] * mp.cos(k * ths[j]) for j in range(nfft)) / nfft
         for k in range(2 * K + 1)]
    # eigenpair of the Hankel matrix: FP64 start, refined by inverse iteration
    Hf = np.array([[float(a[i + j + 1]) for j in range(K)] for i in range(K)])
    lam_f, Q = np.linalg.eigh(Hf)
    order = np.argsort(-np.abs(lam_f))
    H = mp.matrix(K, K)
    for i in range(K):
        for j in range(K):
            H[i, j] = a[i + j + 1]
    x = mp.matrix([mp.mpf(q) for q in Q[:, order[nu]]])
    lam = mp.mpf(lam_f[order[nu]])
    for _ in range(3):
        y = mp.lu_solve(H - lam * mp.eye(K), x)
        x = y / mp.norm(y)
        lam = (x.T * H * x)[0]
    v = [x[i] for i in range(K)]

    def horner_with_derivative(z):
        val = mp.mpc(0)
        der = mp.mpc(0)
        for coef in v:
            der = der * z + val
            val = val * z + coef
        return val, der

    zeta = []
    for z0 in _poles_from_vector_np(np.array([float(q) for q in v]), nu):
        z = mp.mpc(z0.real, z0.imag)
        for _ in range(10):
            pv, dv = horner_with_derivative(z)
            z = z - pv / dv
        zeta.append(z)

    def poly_up(coefs, z):      # sum coefs[k] z^k
        acc = mp.mpc(0)
        for coef in reversed(coefs):
            acc = acc * z + coef
        return acc

    def qval(z):
        acc = mp.mpc(1)
        for zz in zeta:
            acc *= (z - zz)
        return acc

    M = 512
    samples = []
    for j in range(M):
        w = mp.expjpi(2 * mp.mpf(j) / M)
        Rt = poly_up(a[:K + 1], w) - lam * w * poly_up(v, w) / poly_up(v, 1 / w)
        samples.append(Rt * qval(w))
    pcoef = [mp.fsum(samples[j] * mp.expjpi(-2 * mp.mpf(j * k) / M) for j in range(M)) / M
             for k in range(nu + 1)]
    taus, oms = [], []
    for i, z in enumerate(zeta):
        dq = mp.mpc(1)
        for jj, zz in enumerate(zeta):
            if jj != i:
                dq *= (z - zz)
        res_z = poly_up(pcoef, z) / dq
        oms.append(res_z * 4 * sc * (z - 1) / (z + 1) ** 3)
        taus.append(sc * (z - 1) ** 2 / (z + 1) ** 2)
    omega0 = 2 * (poly_up(pcoef, mp.mpf(-1)) / qval(mp.mpf(-1))).real - a[0]
    up = sorted([i for i in range(nu) if taus[i].imag > 0], key=lambda i: taus[i].real)
    tau_up = [taus[i] for i in up]
    c_up = [2 * oms[i] for i in up]
    return tau_up, c_up, omega0


def cf_table_np(nu: int = NU, scale: float = SCALE, K: int = HANKEL_K, nfft: int = 1024):
    """FP64 numpy twin of cf_table_mp (same steps, FP64 FFT and SVD).  Its
    residues carry ~1e-13 rounding noise; it is pinned against cf_table_mp
    as a function on (-inf, 0]."""
    th = 2 * np.pi * np.arange(nfft) / nfft
    w = np.exp(1j * th)
    s = w.real
    with np.errstate(divide="ignore", over="ignore", invalid="ignore"):
        f = np.exp(scale * (s - 1) / (s + 1))
    f[~np.isfinite(f)] = 0.0
    a = np.real(np.fft.fft(f)) / nfft
    H = np.array([[a[i + j + 1] for j in range(K)] for i in range(K)])
    lam, Q = np.linalg.eigh(H)
    idx = np.argsort(-np.abs(lam))[nu]
    lam, v = lam[idx], Q[:, idx]
    zeta = _poles_from_vector_np(v, nu)
    q = np.poly(zeta)
    G = np.polyval(a[:K + 1][::-1], w)
    Rt = G - lam * w * np.polyval(v[::-1], w) / np.polyval(v[::-1], 1 / w)
    pc = (np.fft.fft(Rt * np.polyval(q, w)) / nfft)[:nu + 1][::-1]
    res_z = np.polyval(pc, zeta) / np.polyval(np.polyder(q), zeta)
    omega = res_z * 4 * scale * (zeta - 1) / (zeta + 1) ** 3
    tau = scale * (zeta - 1) ** 2 / (zeta + 1) ** 2
    omega0 = 2 * (np.polyval(pc, -1.0) / np.polyval(q, -1.0)).real - a[0]
    up = np.where(tau.imag > 0)[0]
    up = up[np.argsort(tau[up].real)]
    return tau[up].copy(), 2 * omega[up], float(omega0)


@functools.lru_cache(maxsize=1)
def cf_table():
    """The FP64 CF table the oracle uses: (tau[7], c[7], omega0) as numpy
    arrays, read from cf_nu14_oracle.json (written by oracle/gen_cf_table.py
    from cf_table_mp) or computed on the fly when the file is absent."""
    if os.path.exists(_TABLE_JSON):
        with open(_TABLE_JSON) as fh:
            d = json.load(fh)
        tau = np.array(d["tau_re"]) + 1j * np.array(d["tau_im"])
        c = np.array(d["c_re"]) + 1j * np.array(d["c_im"])
        return tau, c, float(d["omega0"])
    tau, c, w0 = cf_table_mp()
    return (np.array([complex(t) for t in tau]), np.array([complex(x) for x in c]),
            float(w0))


def r_eval(x, tau=None, c=None, omega0=None):
    """Evaluate r(x) = omega0 + Re sum_j c_j/(x - tau_j) at real points x (the
    partial-fraction form of Section 2 with the conjugate pairs folded, which
    holds for real x only), numpy FP64."""
    if tau is None:
        tau, c, omega0 = cf_table()
    x = np.asarray(x)
    if np.iscomplexobj(x):
        raise TypeError("r_eval takes real points: the folded pair form is real-only")
    terms = c[None, :] / (x.reshape(-1, 1) - tau[None, :])
    return (omega0 + terms.sum(1).real).reshape(x.shape)
