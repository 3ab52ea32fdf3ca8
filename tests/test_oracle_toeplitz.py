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
