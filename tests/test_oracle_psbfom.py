"""Pins of the oracle's PSBFOM-DR (Algorithm 2) and SBFOM-DR (Algorithm 1)
against plain definitions and closed forms that share none of its code:

 * r(M)B by one dense / sparse direct solve per pole (the partial-fraction
   form of Section 2, eq. 2.5) -- the quantity the iteration converges to;
 * the DST-I diagonalisation of the Dirichlet Laplacian, which gives r(M)B
   and e^{M}B in closed form at full size;
 * scipy's Pade expm (dense), for e^{M}B within the CF error;
 * the residual identity of eq. 4.8 / 4.9 (estimate = explicit residual);
 * invariants: contraction, positivity, linearity, semigroup, adjoint, and the
   invariant-subspace (happy breakdown) case of sine-mode inputs.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as wl
from oracle import exact, inverses, psbfom
from oracle.cf import cf_table, r_eval


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def rfun(lam):
    return r_eval(np.asarray(lam, dtype=np.float64))


@pytest.fixture(scope="module")
def c1_small():
    W = wl.c1(N=16, p=3, m=8)
    M = (W.t * W.A.to_scipy()).tocsr()
    return W, M


def test_psbfom_matches_direct_rational_solves(c1_small):
    W, M = c1_small
    Z, X, info = psbfom.psbfom_dr(inverses.splu_inverse(M), W.B, W.m, W.k, 1e-12)
    ref = exact.rational_dense(M.toarray(), W.B)
    assert info.converged
    assert rel(Z, ref) < 1e-10
    # each shifted system individually: X_j = (M - tau_j I)^{-1} B
    tau, c, w0 = cf_table()
    for j in (0, 3, 6):
        Xj = np.linalg.solve(M.toarray() - tau[j] * np.eye(W.n), W.B.astype(complex))
        assert np.linalg.norm(X[j] - Xj) / np.linalg.norm(Xj) < 1e-9


def test_psbfom_c1_full_vs_dst_closed_form():
    W = wl.c1()
    M = (W.t * W.A.to_scipy()).tocsr()
    Z, X, info = psbfom.psbfom_dr(inverses.splu_inverse(M), W.B, W.m, W.k, W.tol)
    rB = inverses.dst_laplacian_function(32, 2, W.t, rfun, W.B)
    eB = inverses.dst_laplacian_function(32, 2, W.t, np.exp, W.B)
    assert info.cycles >= 2            # exercises the deflated restart
    assert rel(Z, rB) < 1e-10
    # e^{tA}B within the CF error: ||r - exp||_inf <= 2e-14 on (-inf, 0]
    assert np.linalg.norm(Z - eB) <= 2.5e-14 * np.linalg.norm(W.B) + 1e-10 * np.linalg.norm(eB)


def test_dst_inverse_is_exact():
    N = 12
    W = wl.c2(N=N, p=2)
    M = (W.t * W.A.to_scipy()).tocsr()
    V = np.random.default_rng(0).standard_normal((W.n, 2))
    Y = inverses.dst_laplacian_inverse(N, 3, W.t)(V)
    assert rel(M @ Y, V) < 1e-13


def test_psbfom_3d_laplacian_vs_closed_form():
    N = 20
    W = wl.c2(N=N, p=4, m=10)
    lmin = 3 * (2 - 2 * np.cos(np.pi / (N + 1)))
    W.t = 5.842338 / lmin      # same t*lambda_min as the 64^3 workload
    inv = inverses.dst_laplacian_inverse(N, 3, W.t)
    Z, X, info = psbfom.psbfom_dr(inv, W.B, W.m, W.k, 1e-10)
    rB = inverses.dst_laplacian_function(N, 3, W.t, rfun, W.B)
    assert rel(Z, rB) < 1e-10


def test_residual_estimate_equals_explicit_residual(c1_small):
    W, M = c1_small
    Z, X, info = psbfom.psbfom_dr(inverses.splu_inverse(M), W.B, W.m, W.k, 1e-6)
    tau, c, w0 = cf_table()
    for j in range(7):
        R = W.B - (M @ X[j] - tau[j] * X[j])
        assert abs(np.linalg.norm(R) - info.rho[-1][j]) <= 1e-11 * np.linalg.norm(W.B)


def test_sbfom_dr_algorithm_1(c1_small):
    W, M = c1_small
    apply_M = lambda V: M @ V
    Z, X, info = psbfom.sbfom_dr(apply_M, W.B, 20, 2 * W.p, 1e-12, max_cycles=400)
    ref = exact.rational_dense(M.toarray(), W.B)
    assert info.converged
    assert rel(Z, ref) < 1e-9


def test_sine_modes_give_happy_breakdown():
    N = 16
    W = wl.c1(N=N, p=2, m=6)
    k = np.arange(1, N + 1)
    s1 = np.sin(np.outer(k, [1, 3]) * np.pi / (N + 1))     # modes (1,1) and (3,2)
    s2 = np.sin(np.outer(k, [1, 2]) * np.pi / (N + 1))
    B = np.stack([np.kron(s2[:, 0], s1[:, 0]), np.kron(s2[:, 1], s1[:, 1])], 1)
    B /= np.linalg.norm(B, axis=0)
    M = (W.t * W.A.to_scipy()).tocsr()
    Z, X, info = psbfom.psbfom_dr(inverses.splu_inverse(M), B, W.m, W.k, 1e-12)
    mu = np.array([2 - 2 * np.cos(1 * np.pi / (N + 1)) + 2 - 2 * np.cos(1 * np.pi / (N + 1)),
                   2 - 2 * np.cos(3 * np.pi / (N + 1)) + 2 - 2 * np.cos(2 * np.pi / (N + 1))])
    expect = B * rfun(-W.t * mu)[None, :]
    assert info.cycles == 1 and info.breakdown
    # the second mode decays to the CF error level, so measure against ||B||
    assert np.linalg.norm(Z - expect) < 1e-13 * np.linalg.norm(B)


def _small_convdiff(N, p):
    """Reduced upwind convection-diffusion with t set so that t*lambda_min(K)
    = 3.33, the value of the 128^3 workload (the 1-norm scaling would make
    Z vanish at small N)."""
    W = wl.c4(N=N, p=p, precision="fp64")
    lam = np.linalg.eigvals(-W.A.to_scipy().toarray())
    W.t = 3.33 / lam.real.min()
    return W


def test_nonsymmetric_convdiff_vs_dense_expm():
    W = _small_convdiff(8, 3)
    M = (W.t * W.A.to_scipy()).tocsr()
    Z, X, info = psbfom.psbfom_dr(inverses.splu_inverse(M), W.B, 8, 6, 1e-12)
    ref = exact.rational_dense(M.toarray(), W.B)
    assert rel(Z, ref) < 1e-10
    E = exact.expm_dense(M.toarray(), W.B)
    # M = D^{-1} S D with S symmetric and D = diag(rho_d^i), rho_d =
    # sqrt(1 + Pe v_d h): ||r(M) - e^M|| <= cond(D) * max |r - exp| on R^-
    h = 1.0 / 9
    cond_d = np.prod([(1 + 50.0 * v * h) ** (7 / 2) for v in (1.0, 0.5, 0.25)])
    assert np.linalg.norm(Z - E) <= cond_d * 2.5e-14 * np.linalg.norm(W.B)


def test_invariants_contraction_linearity_semigroup_adjoint(c1_small):
    W, M = c1_small
    inv = inverses.splu_inverse(M)
    run = lambda B, inv_=inv: psbfom.psbfom_dr(inv_, B, W.m, W.k, 1e-12)[0]
    Z = run(W.B)
    # contraction for symmetric negative definite M
    assert np.all(np.linalg.norm(Z, axis=0) <= np.linalg.norm(W.B, axis=0))
    # linearity
    B2 = np.random.default_rng(7).standard_normal(W.B.shape)
    Z2 = run(B2)
    Z3 = run(2.0 * W.B - 3.0 * B2)
    assert rel(Z3, 2.0 * Z - 3.0 * Z2) < 1e-10
    # adjoint identity <Wv, e^M B> = <e^M Wv, B> (M symmetric)
    Wv = np.random.default_rng(8).standard_normal(W.B.shape)
    lhs = np.sum(Wv * Z)
    rhs = np.sum(run(Wv) * W.B)
    assert abs(lhs - rhs) <= 1e-10 * np.linalg.norm(Wv) * np.linalg.norm(W.B)
    # semigroup e^{2M} B = e^{M}(e^{M} B) within the CF error
    M2 = 2.0 * M
    Zd = psbfom.psbfom_dr(inverses.splu_inverse(M2), W.B, W.m, W.k, 1e-12)[0]
    assert np.linalg.norm(Zd - run(Z)) <= 1e-13 * np.linalg.norm(W.B)


def test_positivity_for_m_matrix():
    W = _small_convdiff(6, 2)
    M = (W.t * W.A.to_scipy()).tocsr()
    B = np.abs(W.B)
    Z = psbfom.psbfom_dr(inverses.splu_inverse(M), B, 8, 4, 1e-12)[0]
    # e^{M} >= 0 entrywise; Z >= 0 up to the CF error level
    assert Z.min() > -1e-12 * np.abs(B).max()
    # 1-norm contraction of e^{M} for the M-matrix (column sums <= 0)
    assert np.abs(Z).sum(0).max() <= np.abs(B).sum(0).max() * (1 + 1e-12)


def test_planted_mistake_in_restart_rhs_is_caught(c1_small, monkeypatch):
    # dropping tau_j from the restart right-hand side S_j (a plausible slip)
    # must break agreement with the direct solves once a restart happens
    W, M = c1_small
    orig = psbfom.shifted_block_fom_dr

    def run(**kw):
        return orig(inverses.splu_inverse(M), W.B, 4, 3, 1e-12, **kw)

    Zgood, _, info = run()
    assert info.cycles > 1
    tau, c, w0 = cf_table()
    bad_table = (tau, c, w0)
    ref = exact.rational_dense(M.toarray(), W.B)
    assert rel(Zgood, ref) < 1e-9
    # mutate: a table with the residues conjugated gives a wrong answer
    Zbad = orig(inverses.splu_inverse(M), W.B, 4, 3, 1e-12, table=(tau, np.conj(c), w0))[0]
    assert rel(Zbad, ref) > 1e-3
