"""Pins of the oracle's Toeplitz pieces: the circulant-embedding product
against the dense Toeplitz matrix, the Gohberg-Semencul inverse (Section 4.1)
against a dense solve, and PSBFOM-DR with that inverse against direct
per-pole solves."""
import numpy as np
import scipy.linalg as sla

import workloads as wl
from oracle import exact, inverses, psbfom


def test_toeplitz_generator_is_spd_and_matvec_is_exact():
    c = wl.toeplitz_column(600, 203)
    T = sla.toeplitz(c)
    lam = np.linalg.eigvalsh(T)
    assert lam.min() > 0
    # the symbol bound used to scale t bounds the spectrum
    assert lam.max() <= wl.toeplitz_symbol_max(c) * (1 + 1e-12)
    V = np.random.default_rng(1).standard_normal((600, 3))
    assert np.max(np.abs(inverses.toeplitz_matvec(c, V) - T @ V)) < 1e-13 * np.abs(T @ V).max()


def test_gohberg_semencul_matches_dense_solve():
    n = 700
    c = wl.toeplitz_column(n, 203)
    V = np.random.default_rng(2).standard_normal((n, 4))
    Y = inverses.gohberg_semencul_inverse(c, 2.5)(V)
    ref = np.linalg.solve(2.5 * sla.toeplitz(c), V)
    assert np.linalg.norm(Y - ref) / np.linalg.norm(ref) < 1e-12


def test_psbfom_toeplitz_matches_direct_rational():
    W = wl.c3(n=1024, p=4, m=8)
    T = sla.toeplitz(W.col)
    # t lambda_min = 0.73 as at n = 2^20 (the 1e3-norm scaling would make Z
    # vanish at this size)
    W.t = 0.73 / np.linalg.eigvalsh(T)[0]
    M = -W.t * T
    inv = inverses.gohberg_semencul_inverse(W.col, -W.t)
    Z, X, info = psbfom.psbfom_dr(inv, W.B, W.m, W.k, 1e-11, stop_rule="bound")
    ref = exact.rational_dense(M, W.B)
    assert np.linalg.norm(Z - ref) / np.linalg.norm(ref) < 1e-10


# ---------------------------------------------------------------------------
# nonsymmetric Toeplitz: the fractional diffusion matrix of the large-n
# Toeplitz experiment (Section 5) and the general Gohberg-Semencul formula

def _grunwald_dense(n, beta, d1, d2):
    """h^{-beta} (d1 G + d2 G^T) assembled entry by entry from its definition
    (G_ij = g_{i-j+1} for j <= i + 1, g_k = (-1)^k binom(beta, k))."""
    from scipy.special import binom
    G = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            k = i - j + 1
            if k >= 0:
                G[i, j] = (-1.0) ** k * binom(beta, k)
    return (n + 1.0) ** beta * (d1 * G + d2 * G.T)


def test_fractional_generator_matches_definition_and_is_negative_definite():
    n = 60
    col, row = wl.fractional_toeplitz(n)
    T = sla.toeplitz(col, row)
    A = _grunwald_dense(n, 1.8, 1.0, 3.0)
    assert np.allclose(-T, A, rtol=1e-13, atol=0)
    assert not np.allclose(T, T.T)
    # negative definite symmetric part of A; weights: sum -> 0, g_k >= 0 for k >= 2
    assert np.linalg.eigvalsh(-(A + A.T) / 2).min() > 0
    g = wl.grunwald_weights(1.8, 2000)
    assert abs(g[1] + 1.8) < 1e-15 and np.all(g[2:] > 0) and abs(g.sum()) < 1e-3
    # lambda_min(-A) ~ 27.6 independently of n (fixes t = 0.1 -> t lambda_min = 2.76)
    ev = np.linalg.eigvals(T)
    assert 26.5 < ev.real.min() < 28.5


def test_general_toeplitz_product_and_gohberg_semencul():
    rng = np.random.default_rng(9)
    for col, row in (wl.fractional_toeplitz(257),
                     (np.concatenate([[5.0], rng.standard_normal(199) / np.arange(2, 201)]),
                      np.concatenate([[5.0], rng.standard_normal(199) / np.arange(2, 201) ** 1.3]))):
        n = len(col)
        T = sla.toeplitz(col, row)
        V = rng.standard_normal((n, 3))
        assert np.abs(inverses.toeplitz_matvec_general(col, row, V) - T @ V).max() \
            < 1e-12 * np.abs(T @ V).max()
        inv = inverses.gohberg_semencul_general(col, row, 2.0)
        ref = np.linalg.solve(2.0 * T, V)
        assert np.linalg.norm(inv(V) - ref) < 1e-9 * np.linalg.norm(ref)
    # symmetric special case coincides with the symmetric formula
    c = wl.toeplitz_column(300, 203)
    V = rng.standard_normal((300, 2))
    a = inverses.gohberg_semencul_general(c, c, 1.5)(V)
    b = inverses.gohberg_semencul_inverse(c, 1.5)(V)
    assert np.linalg.norm(a - b) < 1e-12 * np.linalg.norm(b)


def test_planted_mistake_in_general_gohberg_semencul_is_caught(monkeypatch):
    """Dropping the reversal of y (using L(y)^T for L(J y)^T) must be detected."""
    col, row = wl.fractional_toeplitz(100)
    T = sla.toeplitz(col, row)
    V = np.random.default_rng(2).standard_normal((100, 2))
    orig = sla.solve_toeplitz
    calls = {"k": 0}

    def wrong(cr, b):
        out = orig(cr, b)
        calls["k"] += 1
        return out[::-1] if calls["k"] == 2 else out      # corrupt y
    monkeypatch.setattr(sla, "solve_toeplitz", wrong)
    bad = inverses.gohberg_semencul_general(col, row, 1.0)(V)
    assert np.linalg.norm(bad - np.linalg.solve(T, V)) > 1e-3 * np.linalg.norm(np.linalg.solve(T, V))
