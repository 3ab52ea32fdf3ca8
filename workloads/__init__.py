"""Seeded synthetic inputs for e^{tA}B, shared by the oracle and the library's
tests and benchmark.

This module builds matrices, blocks and scalars only; it holds none of the
method's arithmetic (no rational approximation, no Krylov step, no solve).

Every generator is deterministic: random numbers come from
numpy.random.default_rng(seed) (PCG64).  Grids are lexicographic with x
fastest, interior nodes only, zero Dirichlet boundary, h = 1/(N+1).

The exponent matrix is M = t*A with A given in CSR (int32 row pointers and
column indices, FP64 values) and t > 0 chosen as each workload states; A is
negative definite, as the paper's problem statement requires (Section 1).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class CSR:
    n: int
    rowptr: np.ndarray      # int32, n+1
    colind: np.ndarray      # int32, nnz
    val: np.ndarray         # float64, nnz

    @property
    def nnz(self) -> int:
        return int(self.val.shape[0])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.colind, self.rowptr), shape=(self.n, self.n))

    @staticmethod
    def from_scipy(m) -> "CSR":
        m = sp.csr_matrix(m)
        m.sort_indices()
        return CSR(m.shape[0], m.indptr.astype(np.int32), m.indices.astype(np.int32),
                   m.data.astype(np.float64))


def _lap1d(N: int) -> sp.csr_matrix:
    e = np.ones(N)
    return sp.diags([-e[:-1], 2 * e, -e[:-1]], [-1, 0, 1], format="csr")


def laplacian_2d(N: int) -> CSR:
    """-L for the 2D 5-point Laplacian with stencil (4, -1) on an N x N grid."""
    I = sp.identity(N, format="csr")
    T = _lap1d(N)
    L = sp.kron(I, T) + sp.kron(T, I)
    return CSR.from_scipy(-L)


def laplacian_3d(N: int) -> CSR:
    """-L for the 3D 7-point Laplacian with stencil (6, -1) on N^3."""
    I = sp.identity(N, format="csr")
    T = _lap1d(N)
    L = (sp.kron(sp.kron(I, I), T) + sp.kron(sp.kron(I, T), I) + sp.kron(sp.kron(T, I), I))
    return CSR.from_scipy(-L)


def lap_lambda_max(N: int, dim: int) -> float:
    """Largest eigenvalue of the unscaled dim-D Laplacian: dim*(2 + 2cos(pi/(N+1)))."""
    return dim * (2.0 + 2.0 * math.cos(math.pi / (N + 1)))


def convdiff_3d(N: int, pe: float = 50.0, vel=(1.0, 0.5, 0.25)) -> CSR:
    """-K with K = -Delta_h + Pe * (v . grad_h), first-order upwind (backward
    differences for v > 0), on N^3 interior nodes, h = 1/(N+1).  K is a
    nonsymmetric M-matrix."""
    h = 1.0 / (N + 1)
    I = sp.identity(N, format="csr")
    e = np.ones(N)
    T = sp.diags([-e[:-1], 2 * e, -e[:-1]], [-1, 0, 1], format="csr") / h ** 2
    D = sp.diags([-e[:-1], e], [-1, 0], format="csr") / h        # backward difference
    ops = []
    for axis in range(3):
        one = T + pe * vel[axis] * D
        mats = [I, I, I]
        mats[axis] = one
        # lexicographic with x fastest: kron(z, kron(y, x))
        ops.append(sp.kron(mats[2], sp.kron(mats[1], mats[0])))
    K = ops[0] + ops[1] + ops[2]
    return CSR.from_scipy(-K)


def vardiff_2d(N: int, seed: int = 205, sigma: float = 1.0) -> CSR:
    """-K for -div(kappa grad u) on N x N interior nodes, kappa log-normal
    (i.i.d. exp(sigma*N(0,1)) at all (N+2)^2 nodes), face coefficient = harmonic
    mean of its two nodes; K_ii = sum of face coefficients / h^2, K_ij = -kappa_f/h^2."""
    h = 1.0 / (N + 1)
    rng = np.random.default_rng(seed)
    kap = np.exp(sigma * rng.standard_normal((N + 2, N + 2)))     # [y, x] incl. boundary
    hm = lambda a, b: 2.0 * a * b / (a + b)
    kx = hm(kap[1:-1, :-1], kap[1:-1, 1:])     # faces between x-neighbours, (N, N+1)
    ky = hm(kap[:-1, 1:-1], kap[1:, 1:-1])     # faces between y-neighbours, (N+1, N)
    idx = np.arange(N * N).reshape(N, N)       # [y, x], x fastest
    diag = (kx[:, :-1] + kx[:, 1:] + ky[:-1, :] + ky[1:, :]) / h ** 2
    rows = [idx.ravel()]
    cols = [idx.ravel()]
    vals = [-diag.ravel()]
    # x-neighbours
    a = kx[:, 1:-1] / h ** 2                   # face between (y,x) and (y,x+1), x=0..N-2
    rows += [idx[:, :-1].ravel(), idx[:, 1:].ravel()]
    cols += [idx[:, 1:].ravel(), idx[:, :-1].ravel()]
    vals += [a.ravel(), a.ravel()]
    b = ky[1:-1, :] / h ** 2
    rows += [idx[:-1, :].ravel(), idx[1:, :].ravel()]
    cols += [idx[1:, :].ravel(), idx[:-1, :].ravel()]
    vals += [b.ravel(), b.ravel()]
    m = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N * N, N * N)).tocsr()
    return CSR.from_scipy(m)


def toeplitz_column(n: int, seed: int = 203) -> np.ndarray:
    """First column of a symmetric positive definite Toeplitz T:
    c_0 = 2, c_k = -(k+1)^{-1.5} (1 + 0.1 s_k) / S for k >= 1, s_k = +-1 seeded,
    S normalising sum_{k>=1} |c_k| = 1.  The symbol 2 - 2 sum |c_k| cos(k theta)
    is >= 0 and vanishes only at theta = 0 in the limit, so every finite
    section is SPD with lambda_min ~ n^{-1/2}.  Returns c (T = toeplitz(c));
    the exponent matrix is t * (-T)."""
    rng = np.random.default_rng(seed)
    s = rng.choice(np.array([-1.0, 1.0]), size=n - 1)
    k = np.arange(1, n, dtype=np.float64)
    raw = (k + 1.0) ** -1.5 * (1.0 + 0.1 * s)
    c = np.empty(n)
    c[0] = 2.0
    c[1:] = -raw / raw.sum()
    return c


def toeplitz_symbol_max(c: np.ndarray) -> float:
    """max over theta of 2*c_0... the symbol c_0 + 2 sum c_k cos(k theta) on a
    grid of 2n angles: an upper estimate of ||T||_2 used to scale t."""
    n = len(c)
    v = np.zeros(4 * n)
    v[0] = c[0]
    v[1:n] = c[1:]
    v[-(n - 1):] = c[1:][::-1]
    return float(np.max(np.fft.rfft(v).real))


def grunwald_weights(beta: float, count: int) -> np.ndarray:
    """g_k = (-1)^k binom(beta, k), k = 0..count-1, by g_k = g_{k-1} (1 - (beta+1)/k)."""
    g = np.empty(count)
    g[0] = 1.0
    for k in range(1, count):
        g[k] = g[k - 1] * (1.0 - (beta + 1.0) / k)
    return g


def fractional_toeplitz(n: int, beta: float = 1.8, d1: float = 1.0, d2: float = 3.0):
    """Two-sided space-fractional diffusion d1 D_+^beta + d2 D_-^beta on (0, 1),
    zero Dirichlet data, shifted Gruenwald formula, h = 1/(n+1):
    A = h^{-beta} (d1 G + d2 G^T), G the lower Hessenberg Toeplitz matrix with
    G_ij = g_{i-j+1} (j <= i + 1).  A is a nonsymmetric Toeplitz matrix with a
    negative definite symmetric part.  Returns (col, row): first column and
    first row of T = -A (the exponent matrix is t * (-T))."""
    g = grunwald_weights(beta, n + 2)
    col = np.zeros(n)
    row = np.zeros(n)
    col[0] = row[0] = (d1 + d2) * g[1]
    if n > 1:
        col[1] = d1 * g[2] + d2 * g[0]
        row[1] = d1 * g[0] + d2 * g[2]
    if n > 2:
        col[2:] = d1 * g[3:n + 1]
        row[2:] = d2 * g[3:n + 1]
    scale = (n + 1.0) ** beta
    return -col * scale, -row * scale


@dataclasses.dataclass
class SourceProblem:
    """u'(s) = A u(s) + e^{gamma s} b, u(0) = u0, with A = -diag(d) T and T
    the Toeplitz matrix given by its first column and first row."""
    n: int
    col: np.ndarray
    row: np.ndarray
    d: np.ndarray
    u0: np.ndarray       # n x p
    b: np.ndarray        # n x p
    gamma: float
    t: float
    x: np.ndarray        # interior nodes

    def dense_A(self) -> np.ndarray:
        import scipy.linalg as sla
        return -self.d[:, None] * sla.toeplitz(self.col, self.row)


def fractional_source(n: int, beta: float = 1.7, t: float = 1.0) -> SourceProblem:
    """One-sided fractional diffusion with a source (Section 5, Example 5.3):
    u_t = d(x) D_+^beta u + q(x, t) on (0, 1), u(0, t) = 0, u(1, t) = e^{-t},
    u(x, 0) = x^3, d(x) = Gamma(4 - beta)/6 x^{1+beta},
    q(x, t) = -(1 + x) e^{-t} x^3 (exact solution e^{-t} x^3).
    Shifted Gruenwald formula on the nodes x_i = i h, h = 1/(n+1):
    (D_+^beta u)(x_i) ~ h^{-beta} sum_{k=0}^{i+1} g_k u_{i-k+1}, so
    A = h^{-beta} diag(d) G with G_ij = g_{i-j+1} (lower Hessenberg), and the
    source is e^{-s} b with b_i = -(1 + x_i) x_i^3, plus the boundary value
    u_{n+1} = e^{-s} entering row n as d(x_n) h^{-beta} g_0.
    Returned as A = -diag(d) T with T = -h^{-beta} G (col, row: T's first
    column and row), gamma = -1."""
    g = grunwald_weights(beta, n + 1)
    h = 1.0 / (n + 1)
    hb = h ** (-beta)
    x = h * np.arange(1, n + 1)
    d = math.gamma(4.0 - beta) / 6.0 * x ** (1.0 + beta)
    col = -hb * g[1:n + 1]
    row = np.zeros(n)
    row[0] = -hb * g[1]
    if n > 1:
        row[1] = -hb * g[0]
    b = -(1.0 + x) * x ** 3
    b[-1] += d[-1] * hb * g[0]
    return SourceProblem(n, col, row, d, (x ** 3)[:, None].copy(), b[:, None].copy(), -1.0, t, x)


def gaussian_block(n: int, p: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal((n, p))


@dataclasses.dataclass
class Workload:
    name: str
    kind: str                 # "csr" or "toeplitz"
    n: int
    p: int
    t: float
    m: int
    k: int
    tol: float
    B: np.ndarray
    A: CSR | None = None      # A (not tA) for kind == "csr"
    col: np.ndarray | None = None   # first column of T for kind == "toeplitz" (A = -T)
    row: np.ndarray | None = None   # first row of T when T is not symmetric
    symmetric: bool = True
    precision: str = "fp64"
    note: str = ""


def c1(N: int = 32, p: int = 4, m: int = 10) -> Workload:
    """2D 5-point Dirichlet Laplacian on N^2, ||tA||_2 = 1e3 exactly."""
    A = laplacian_2d(N)
    t = 1e3 / lap_lambda_max(N, 2)
    return Workload("lap2d", "csr", N * N, p, t, m, p * (m // 3), 1e-10,
                    gaussian_block(N * N, p, 1), A=A, note=f"2D Laplacian {N}^2")


def c2(N: int = 64, p: int = 8, m: int = 15) -> Workload:
    """3D 7-point Laplacian on N^3, ||tA||_2 = 1e4 exactly."""
    A = laplacian_3d(N)
    t = 1e4 / lap_lambda_max(N, 3)
    return Workload("lap3d", "csr", N ** 3, p, t, m, p * (m // 3), 1e-10,
                    gaussian_block(N ** 3, p, 2), A=A, note=f"3D Laplacian {N}^3")


def c3(n: int = 1 << 20, p: int = 16, m: int = 17) -> Workload:
    """Symmetric positive definite Toeplitz T, A = -T, ||tA||_2 ~= 1e3.  m = 17
    (k = 80) converges in one cycle of 17 block steps; m = 10 needed two
    cycles and the same 17 applications of the inverse, 20 two cycles and
    20 applications."""
    col = toeplitz_column(n, 203)
    t = 1e3 / toeplitz_symbol_max(col)
    return Workload("toeplitz", "toeplitz", n, p, t, m, p * (m // 3), 1e-10,
                    gaussian_block(n, p, 3), col=col, note=f"SPD Toeplitz n={n}")


def c6(n: int = 1 << 17, p: int = 2, m: int = 30, t: float = 0.1) -> Workload:
    """Nonsymmetric Toeplitz: fractional diffusion, beta = 1.8, d1 = 1, d2 = 3
    (the large-n Toeplitz experiment of Section 5), A = -T, B Gaussian n x 2.
    t = 0.1 puts t lambda_min at 2.76 (lambda_min(-A) = 27.6 for every n)."""
    col, row = fractional_toeplitz(n)
    return Workload("fractional", "toeplitz", n, p, t, m, p * (m // 3), 1e-10,
                    gaussian_block(n, p, 6), col=col, row=row, symmetric=False,
                    note=f"fractional diffusion Toeplitz n={n}, beta=1.8, d1=1, d2=3")


def c4(N: int = 128, p: int = 16, m: int = 10, precision: str = "mixed") -> Workload:
    """3D upwind convection-diffusion on N^3 (nonsymmetric), ||tA||_1 = 1e3."""
    A = convdiff_3d(N)
    colsum = np.abs(A.to_scipy()).sum(axis=0).max()
    t = 1e3 / float(colsum)
    return Workload("convdiff3d", "csr", N ** 3, p, t, m, p * (m // 3),
                    1e-5 if precision == "mixed" else 1e-10,
                    gaussian_block(N ** 3, p, 4), A=A, symmetric=False, precision=precision,
                    note=f"3D upwind convection-diffusion {N}^3, Pe=50")


def c5(N: int = 1024, p: int = 32, m: int = 10, precision: str = "mixed") -> Workload:
    """2D log-normal variable-coefficient diffusion on N^2, t = 0.1."""
    A = vardiff_2d(N, 205)
    return Workload("vardiff2d", "csr", N * N, p, 0.1, m, p * (m // 3),
                    1e-5 if precision == "mixed" else 1e-10,
                    gaussian_block(N * N, p, 5), A=A, precision=precision,
                    note=f"2D log-normal diffusion {N}^2")


def c5_weights(N: int = 1024, p: int = 32) -> np.ndarray:
    return gaussian_block(N * N, p, 105)
