"""Pins of the oracle's Caratheodory-Fejer table against facts the paper and
approximation theory fix (Section 2 and Remark 2.1), independent of the code:

 * the uniform error of the type (14, 14) approximant of e^x on (-inf, 0] is
   of the order 10^{-nu} (Section 2);
 * CF differs from the best approximation by O(56^{-nu}) (Section 2), and the
   best approximation's error curve equioscillates at >= 2 nu + 2 points
   (Chebyshev alternation theorem for type (nu, nu));
 * max |tau_i| ~= 18.9 for nu = 14 (Remark 2.1);
 * the poles come in conjugate pairs, so nu/2 = 7 systems suffice (Section 2);
 * r(-inf) = omega_0 and r(0) ~= 1 are both at the error level.
"""
import mpmath as mp
import numpy as np
import pytest

from oracle.cf import cf_table, cf_table_np, r_eval


def _err_curve(tau, c, w0, npts=2400):
    mp.mp.dps = 30
    conv = lambda z: z if isinstance(z, mp.mpc) else mp.mpc(complex(z).real, complex(z).imag)
    T = [conv(t) for t in tau]
    Cc = [conv(x) for x in c]
    xs = [-mp.mpf(10) ** (mp.mpf(e) / 200) for e in range(-1400, 1001)] + [mp.mpf(0)]
    return [(w0 if isinstance(w0, mp.mpf) else mp.mpf(w0)) + mp.fsum([(Cc[i] / (x - T[i])).real for i in range(len(T))]) - mp.exp(x)
            for x in xs]


def _sign_changes(e):
    s = [1 if v > 0 else -1 for v in e]
    return sum(1 for i in range(1, len(s)) if s[i] != s[i - 1])


def test_cf_error_level_and_equioscillation(cf_mp):
    tau, c, w0 = cf_mp
    e = _err_curve(tau, c, w0)
    emax = float(max(abs(v) for v in e))
    # "about 10^{-nu}" for nu = 14
    assert 1e-15 < emax < 5e-14, emax
    # >= 2 nu + 2 = 30 alternation points  <=> >= 29 sign changes
    assert _sign_changes(e) >= 29
    # near-equal amplitude of the extrema (best-approximation characterisation)
    ext = []
    cur = [e[0]]
    for v in e[1:]:
        if (v > 0) == (cur[-1] > 0):
            cur.append(v)
        else:
            ext.append(max(abs(x) for x in cur))
            cur = [v]
    ext.append(max(abs(x) for x in cur))
    big = [float(x) for x in ext if x > 0.5 * emax]
    assert len(big) >= 28
    assert min(big) > 0.9 * emax


def test_cf_fp64_table_keeps_the_error_level():
    tau, c, w0 = cf_table()
    e = _err_curve(tau, c, w0)
    assert float(max(abs(v) for v in e)) < 2.5e-14
    assert _sign_changes(e) >= 29


def test_cf_poles_remark_2_1_and_pairs(cf_mp):
    tau, c, w0 = cf_mp
    assert len(tau) == 7                        # nu/2 poles with Im > 0
    mags = [abs(complex(t)) for t in tau]
    assert abs(max(mags) - 18.9) < 0.05         # Remark 2.1
    assert min(complex(t).imag for t in tau) > 1.0   # no real pole: 7 full pairs
    # r(0) = 1 and omega_0 = r(-inf) to the error level
    r0 = float(w0) + sum((complex(x) / (-complex(t))).real for t, x in zip(tau, c))
    assert abs(r0 - 1.0) < 3e-14
    assert abs(float(w0)) < 3e-14


def test_cf_numpy_twin_agrees_as_a_function():
    t2, c2, w2 = cf_table_np()
    x = -np.logspace(-6, 5, 4000)
    # the FP64 twin's residues carry FFT rounding noise (measured 1.7e-11)
    assert np.max(np.abs(r_eval(x, t2, c2, w2) - r_eval(x))) < 1e-10


def test_planted_mistake_in_residues_is_caught():
    # a plausible slip -- conjugating one residue -- must break the error pin
    tau, c, w0 = cf_table()
    bad = c.copy()
    bad[3] = np.conj(bad[3])
    x = -np.logspace(-4, 4, 2000)
    err = np.max(np.abs(r_eval(x, tau, bad, w0) - np.exp(x)))
    assert err > 1e-3
