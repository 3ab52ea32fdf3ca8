"""Pins of the oracle's direct references (oracle/exact.py) and of the
conjugate-gradient generator of the Gohberg-Semencul inverse, each against a
route that shares none of its code:

 * rational_sparse (one sparse LU per pole) against rational_dense (one dense
   LU per pole) on symmetric and nonsymmetric operators, and against the
   DST-I closed form S diag(r(-t mu)) S^T B of the Dirichlet Laplacian;
 * rational_sparse_adjoint: its three outputs against the dense per-pole
   solves with M and M^T, the plain pairing <G, A Z>, and the closed form
   S diag(-mu r(-t mu)) S^T of A r(tA) on the Laplacian;
 * rational_kron3_tridiag: its closed-form tridiagonal modes against the
   dense matrix, and the whole result against rational_sparse on the 3D
   convection-diffusion operator and against the DST-I closed form of the
   3D Laplacian;
 * cg_first_column against Levinson's recursion (scipy).
Each group also plants a plausible slip and checks that a pin catches it.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as wl
from oracle import exact, inverses
from oracle.cf import cf_table, r_eval


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rfun(lam):
    return r_eval(np.asarray(lam, dtype=np.float64))


def _convdiff_small(N, p, seed=1):
    A = wl.convdiff_3d(N)
    # t lambda_min = 3.33 as on the 128^3 workload; lambda_min of the
    # Kronecker sum of the 1-D upwind factors (sub a, diagonal b, super c,
    # a c > 0) is sum_d (b_d - 2 sqrt(a_d c_d) cos(pi/(N+1)))
    lmin = sum(b - 2.0 * np.sqrt(a * c) * np.cos(np.pi / (N + 1))
               for a, b, c in _convdiff_coef(N))
    t = 3.33 / lmin
    B = np.random.default_rng(seed).standard_normal((N ** 3, p))
    return A, t, B


def _lap2d_small(N, p):
    """Reduced 2D Laplacian with t lambda_min = 2.2692, the value of the 32^2
    workload (its ||tA|| = 1e3 scaling would make Z vanish at small N)."""
    W = wl.c1(N=N, p=p)
    W.t = 2.2692 / (2 * (2 - 2 * np.cos(np.pi / (N + 1))))
    return W


def _convdiff_coef(N, pe=50.0, vel=(1.0, 0.5, 0.25)):
    h = 1.0 / (N + 1)
    return [(-1.0 / h ** 2 - pe * v / h, 2.0 / h ** 2 + pe * v / h, -1.0 / h ** 2) for v in vel]


# --------------------------------------------------------------------------- rational_sparse

def test_rational_sparse_matches_dense_solves_symmetric_and_not():
    W = _lap2d_small(12, 3)
    M = (W.t * W.A.to_scipy()).tocsr()
    assert rel(exact.rational_sparse(M, W.B), exact.rational_dense(M.toarray(), W.B)) < 1e-12
    A, t, B = _convdiff_small(6, 2)
    M = (t * A.to_scipy()).tocsr()
    Md = M.toarray()
    assert rel(exact.rational_sparse(M, B), exact.rational_dense(Md, B)) < 1e-12
    MT = M.T.tocsr()
    assert rel(exact.rational_sparse(MT, B), exact.rational_dense(Md.T, B)) < 1e-12
    # the operator is far from symmetric: M and M^T give different results
    assert rel(exact.rational_sparse(MT, B), exact.rational_sparse(M, B)) > 1e-3


def test_rational_sparse_matches_dst_closed_form_full_2d():
    W = wl.c1()   # 2D Laplacian 32^2, ||tA||_2 = 1e3
    M = (W.t * W.A.to_scipy()).tocsr()
    ref = inverses.dst_laplacian_function(32, 2, W.t, rfun, W.B)
    assert rel(exact.rational_sparse(M, W.B), ref) < 1e-12


def test_rational_sparse_planted_mistakes_are_caught():
    """A sign slip on the shift (conjugated poles) or a dropped real part
    before the c_j weighting must move the result far from the closed form."""
    W = _lap2d_small(16, 2)
    M = (W.t * W.A.to_scipy()).tocsr()
    ref = inverses.dst_laplacian_function(16, 2, W.t, rfun, W.B)
    tau, c, w0 = cf_table()
    assert rel(exact.rational_sparse(M, W.B, table=(np.conj(tau), c, w0)), ref) > 1e-3
    assert rel(exact.rational_sparse(M, W.B, table=(tau, np.conj(c), w0)), ref) > 1e-3


# --------------------------------------------------------------------------- adjoint triple

def test_rational_sparse_adjoint_nonsymmetric():
    A, t, B = _convdiff_small(6, 3, seed=2)
    G = np.random.default_rng(3).standard_normal(B.shape)
    M = (t * A.to_scipy()).tocsr()
    Md = M.toarray()
    Z, gB, gt = exact.rational_sparse_adjoint(M, B, G, t)
    Zd = exact.rational_dense(Md, B)
    assert rel(Z, Zd) < 1e-12
    assert rel(gB, exact.rational_dense(Md.T, G)) < 1e-12
    # the plain definition <G, A Z> (no amplification at this size)
    plain = float(np.sum(G * (A.to_scipy() @ Zd)))
    assert abs(gt - plain) <= 1e-10 * abs(plain)
    # adjoint identity <G, r(M) B> = <r(M^T) G, B>
    assert abs(np.sum(G * Z) - np.sum(gB * B)) <= 1e-12 * np.linalg.norm(G) * np.linalg.norm(B)


def test_rational_sparse_adjoint_laplacian_closed_form():
    N = 20
    W = _lap2d_small(N, 2)
    G = np.random.default_rng(4).standard_normal(W.B.shape)
    M = (W.t * W.A.to_scipy()).tocsr()
    Z, gB, gt = exact.rational_sparse_adjoint(M, W.B, G, W.t)
    assert rel(Z, inverses.dst_laplacian_function(N, 2, W.t, rfun, W.B)) < 5e-12
    assert rel(gB, inverses.dst_laplacian_function(N, 2, W.t, rfun, G)) < 5e-12
    # A r(tA) = S diag(lam r(lam) / t) S^T with lam = -t mu
    AZ = inverses.dst_laplacian_function(N, 2, W.t, lambda lam: lam * rfun(lam) / W.t, W.B)
    ref = float(np.sum(G * AZ))
    assert abs(gt - ref) <= 1e-11 * abs(ref)
    # planted slip: conjugated poles (a sign slip on the shift) are caught
    tau, c, w0 = cf_table()
    _, _, bad = exact.rational_sparse_adjoint(M, W.B, G, W.t, table=(np.conj(tau), c, w0))
    assert abs(bad - ref) > 1e-3 * abs(ref)


# --------------------------------------------------------------------------- z-mode solve

@pytest.mark.parametrize("a,b,c", [(-3.0, 7.0, -1.5), (2.0, -1.0, 0.5), (-1.0, 2.0, -1.0)])
def test_tridiagonal_modes_diagonalise_the_matrix(a, b, c):
    N = 17
    T = np.diag(np.full(N - 1, a), -1) + np.diag(np.full(N, b)) + np.diag(np.full(N - 1, c), 1)
    lam, V, Vinv = exact._tridiag_modes(a, b, c, N)
    cond = max(a / c, c / a) ** ((N - 1) / 2)      # cond(diag(r^i)), r = sqrt(a / c)
    assert np.max(np.abs(Vinv @ V - np.eye(N))) < 1e-14 * cond
    assert np.max(np.abs(V @ np.diag(lam) @ Vinv - T)) < 1e-14 * cond * np.abs(T).max()
    assert np.max(np.abs(np.sort(lam) - np.sort(np.linalg.eigvals(T).real))) < 1e-11 * abs(b)


def test_tridiagonal_modes_planted_mistake():
    """Using r = sqrt(c/a) instead of sqrt(a/c) (the transposed matrix's
    modes) must fail to diagonalise T."""
    N, a, b, c = 12, -3.0, 7.0, -1.5
    T = np.diag(np.full(N - 1, a), -1) + np.diag(np.full(N, b)) + np.diag(np.full(N - 1, c), 1)
    lam, V, Vinv = exact._tridiag_modes(c, b, a, N)
    assert np.max(np.abs(V @ np.diag(lam) @ Vinv - T)) > 1e-3


@pytest.mark.parametrize("N", [8, 12])
def test_kron_zmode_solve_matches_sparse_lu_convdiff(N):
    A, t, B = _convdiff_small(N, 3)
    M = (t * A.to_scipy()).tocsr()
    got = exact.rational_kron3_tridiag(N, _convdiff_coef(N), t, B)
    ref = exact.rational_sparse(M, B)
    assert rel(got, ref) < 5e-12
    assert np.abs(got - ref).max() < 5e-12 * np.abs(ref).max()


def test_kron_zmode_solve_matches_dst_closed_form_laplacian():
    N = 10
    W = wl.c2(N=N, p=2)
    W.t = 5.842338 / (3 * (2 - 2 * np.cos(np.pi / (N + 1))))
    coef = [(-1.0, 2.0, -1.0)] * 3          # K = L_3, A = -L_3
    got = exact.rational_kron3_tridiag(N, coef, W.t, W.B)
    ref = inverses.dst_laplacian_function(N, 3, W.t, rfun, W.B)
    # both routes sum O(||B||) partial fractions: rounding floor ~eps ||B||
    floor = 50 * np.finfo(float).eps * np.linalg.norm(W.B) / np.linalg.norm(ref)
    assert rel(got, ref) < max(1e-12, floor)


def test_kron_zmode_solve_axis_order_is_checked():
    """Swapping the x and z factors (a plausible slip in the index order)
    must break agreement with the sparse solve of the real operator."""
    N = 8
    A, t, B = _convdiff_small(N, 2)
    M = (t * A.to_scipy()).tocsr()
    coef = _convdiff_coef(N)
    got = exact.rational_kron3_tridiag(N, [coef[2], coef[1], coef[0]], t, B)
    assert rel(got, exact.rational_sparse(M, B)) > 1e-3


# --------------------------------------------------------------------------- CG generator

@pytest.mark.parametrize("n", [1000, 4096])
def test_cg_first_column_matches_levinson(n):
    c = wl.toeplitz_column(n, 203)
    x = inverses.cg_first_column(c)
    assert rel(x, inverses.levinson_first_column(c)) < 1e-12
    V = np.random.default_rng(n).standard_normal((n, 3))
    Y = inverses.gohberg_semencul_inverse(c, 2.0, x=x)(V)
    assert rel(Y, np.linalg.solve(2.0 * sla.toeplitz(c), V)) < 1e-12


def test_gohberg_semencul_with_a_wrong_generator_is_caught():
    n = 600
    c = wl.toeplitz_column(n, 203)
    x = inverses.cg_first_column(c, rtol=1e-4)      # stopped far too early
    V = np.random.default_rng(1).standard_normal((n, 2))
    Y = inverses.gohberg_semencul_inverse(c, 1.0, x=x)(V)
    assert rel(Y, np.linalg.solve(sla.toeplitz(c), V)) > 1e-8
