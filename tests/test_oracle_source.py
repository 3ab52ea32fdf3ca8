"""Pins of the source-term oracle (oracle/source.py) against what the
mathematics fixes: an ODE integrator, the exact solution of the PDE of
Section 5, Example 5.3, the spectral closed form of the divided difference
for symmetric A, the plain exponential when the source vanishes, and planted
mistakes that each pin must catch."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import workloads as wl
from oracle import exact, inverses, source
from oracle.cf import r_eval


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rf(x):
    return np.real(r_eval(np.asarray(x, dtype=np.float64)))


def test_augmented_exponential_matches_ode_integrator():
    P = wl.fractional_source(20)
    A = P.dense_A()
    f = lambda s, u: A @ u + np.exp(P.gamma * s) * P.b[:, 0]
    sol = solve_ivp(f, (0.0, P.t), P.u0[:, 0], method="Radau", rtol=1e-12, atol=1e-14, jac=A)
    u = source.exact_augmented(A, P.u0, P.b, P.gamma, P.t)[:, 0]
    assert np.linalg.norm(sol.y[:, -1] - u) <= 1e-9 * np.linalg.norm(u)


@pytest.mark.parametrize("n", [100, 200])
def test_variation_of_constants_matches_augmented(n):
    P = wl.fractional_source(n)
    A = P.dense_A()
    ex = source.exact_augmented(A, P.u0, P.b, P.gamma, P.t)
    assert rel(source.variation_of_constants(A, P.u0, P.b, P.gamma, P.t), ex) < 1e-12


def test_semidiscrete_solution_converges_to_pde_solution():
    """Example 5.3's PDE has the exact solution e^{-t} x^3; the shifted
    Gruenwald scheme is first order, so the error halves with h.  A dropped
    boundary term, a wrong d(x) or a wrong source fails this."""
    errs = []
    for n in (100, 200, 400):
        P = wl.fractional_source(n)
        u = source.exact_augmented(P.dense_A(), P.u0, P.b, P.gamma, P.t)
        errs.append(rel(u, np.exp(-P.t) * P.x[:, None] ** 3))
    assert errs[0] < 2e-3
    assert 0.4 < errs[1] / errs[0] < 0.6 and 0.4 < errs[2] / errs[1] < 0.6, errs


def test_generator_matches_the_grunwald_definition():
    n, beta = 9, 1.7
    P = wl.fractional_source(n, beta)
    h = 1.0 / (n + 1)
    G = np.zeros((n, n))
    g = [1.0]
    for k in range(1, n + 1):
        g.append(g[-1] * (k - 1 - beta) / k)     # (-1)^k binom(beta, k)
    for i in range(n):
        for j in range(n):
            if j <= i + 1:
                G[i, j] = g[i - j + 1]
    A = h ** (-beta) * np.diag(P.d) @ G
    assert np.allclose(P.dense_A(), A, rtol=1e-14, atol=0)


@pytest.mark.parametrize("gamma", [-1.0, 0.0, -7.5])
def test_rational_form_matches_spectral_closed_form(gamma):
    """Symmetric A = -L (1D Laplacian): u_r = Q r(t lam) Q^T u0 +
    Q [t (r(t lam) - r(gamma t)) / (t lam - gamma t)] Q^T b, with the scalar
    r and no solve; the partial-fraction oracle must agree."""
    N, t = 60, 0.02
    A = -(2 * np.eye(N) - np.eye(N, k=1) - np.eye(N, k=-1)) * (N + 1) ** 2
    rng = np.random.default_rng(3)
    u0, b = rng.standard_normal((N, 2)), rng.standard_normal((N, 2))
    lam, Q = np.linalg.eigh(A)
    x, sigma = t * lam, gamma * t
    dd = t * (rf(x) - rf([sigma])[0]) / (x - sigma)
    ref = Q @ (rf(x)[:, None] * (Q.T @ u0)) + Q @ (dd[:, None] * (Q.T @ b))
    assert rel(source.rational_dense_source(A, u0, b, gamma, t), ref) < 1e-12


@pytest.mark.parametrize("n", [100, 200])
def test_rational_form_two_routes_and_cf_error(n):
    """Partial fractions against r(tA)(u0 + w) - r(gamma t) w with w solved,
    and both within the CF error of the exact solution."""
    P = wl.fractional_source(n)
    A = P.dense_A()
    ra = source.rational_dense_source(A, P.u0, P.b, P.gamma, P.t)
    assert rel(ra, source.rational_via_w(A, P.u0, P.b, P.gamma, P.t)) < 1e-11
    assert rel(ra, source.exact_augmented(A, P.u0, P.b, P.gamma, P.t)) < 1e-11


def test_zero_source_is_the_plain_exponential():
    W = wl.c1(N=12, p=3)
    A = W.A.to_scipy().toarray()
    ra = source.rational_dense_source(A, W.B, np.zeros_like(W.B), -1.0, W.t)
    assert rel(ra, exact.rational_dense(W.t * A, W.B)) < 1e-14


def test_laplacian_closed_form_through_dst():
    """The DST-I route of the library's full-size checks: f1 = r on the
    eigenvalues of M = tA, f2 = t (r(x) - r(sigma)) / (x - sigma)."""
    N, gamma = 12, -3.0
    W = wl.c1(N=N, p=2)
    W.t = 2.0 / (2 * (2 - 2 * np.cos(np.pi / (N + 1))))   # t lambda_min = 2
    A = W.A.to_scipy().toarray()
    sigma = gamma * W.t
    b = np.random.default_rng(8).standard_normal((N * N, 2))
    f2 = lambda x: W.t * (rf(x) - rf([sigma])[0]) / (x - sigma)
    ref = (inverses.dst_laplacian_function(N, 2, W.t, rf, W.B)
           + inverses.dst_laplacian_function(N, 2, W.t, f2, b))
    assert rel(source.rational_dense_source(A, W.B, b, gamma, W.t), ref) < 1e-12


def test_planted_mistakes_are_caught():
    """A source coefficient without its factor t, or a sign error in the
    shift, breaks the spectral closed form."""
    N, t, gamma = 40, 0.05, -2.0
    A = -(2 * np.eye(N) - np.eye(N, k=1) - np.eye(N, k=-1)) * (N + 1) ** 2
    rng = np.random.default_rng(4)
    u0, b = rng.standard_normal((N, 1)), rng.standard_normal((N, 1))
    lam, Q = np.linalg.eigh(A)
    x, sigma = t * lam, gamma * t
    ref = (Q @ (rf(x)[:, None] * (Q.T @ u0))
           + Q @ ((t * (rf(x) - rf([sigma])[0]) / (x - sigma))[:, None] * (Q.T @ b)))

    def no_t(A, u0, b, gamma, t, table=None):
        tau, c, w0 = source.cf_table()
        out = w0 * u0
        for tj, cj in zip(tau, c):
            rhs = u0 + (1.0 / (tj - gamma * t)) * b
            out = out + np.real(cj * np.linalg.solve(t * A - tj * np.eye(len(A)), rhs))
        return out

    def wrong_sign(A, u0, b, gamma, t, table=None):
        tau, c, w0 = source.cf_table()
        out = w0 * u0
        for tj, cj in zip(tau, c):
            rhs = u0 + (t / (tj + gamma * t)) * b
            out = out + np.real(cj * np.linalg.solve(t * A - tj * np.eye(len(A)), rhs))
        return out

    assert rel(source.rational_dense_source(A, u0, b, gamma, t), ref) < 1e-12
    assert rel(no_t(A, u0, b, gamma, t), ref) > 1e-3
    assert rel(wrong_sign(A, u0, b, gamma, t), ref) > 1e-3
