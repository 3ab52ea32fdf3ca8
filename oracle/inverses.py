"""Ways to apply M^{-1} (M = tA) for the oracle (test infrastructure).

Section 4.1: for moderate n the paper factors A once by sparse LU and applies
U \\ (L \\ w); for Toeplitz A it uses the Gohberg-Semencul formula.  Each
function returns a callable V -> M^{-1} V.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def splu_inverse(M: sp.spmatrix):
    """Sparse LU of M once, then two triangular solves per column (Section 4.1)."""
    lu = spla.splu(sp.csc_matrix(M))
    return lambda V: lu.solve(np.asarray(V, dtype=np.float64))


def laplacian_eigs(N: int, dim: int) -> np.ndarray:
    """Eigenvalues of the unscaled dim-D Dirichlet Laplacian on N^dim, as an
    array of shape (N,)*dim indexed like the grid (axis order z, y, x)."""
    mu1 = 2.0 - 2.0 * np.cos(np.pi * np.arange(1, N + 1) / (N + 1))
    grids = np.meshgrid(*([mu1] * dim), indexing="ij")
    return sum(grids)


def _dst_apply(V, N, dim, diag):
    """S diag S^T V with S the orthonormal DST-I on each grid axis."""
    n, q = V.shape
    shp = (N,) * dim
    out = np.empty_like(V)
    axes = tuple(range(dim))
    for j in range(q):
        u = V[:, j].reshape(shp)
        u = sfft.dstn(u, type=1, axes=axes, norm="ortho")
        u *= diag
        u = sfft.idstn(u, type=1, axes=axes, norm="ortho")
        out[:, j] = u.ravel()
    return out


def dst_laplacian_inverse(N: int, dim: int, t: float):
    """M = -t L exactly diagonalised by the DST-I: M^{-1} = S diag(-1/(t mu)) S."""
    mu = laplacian_eigs(N, dim)
    diag = -1.0 / (t * mu)
    return lambda V: _dst_apply(np.asarray(V, np.float64), N, dim, diag)


def dst_laplacian_function(N: int, dim: int, t: float, f, V):
    """f(M) V for M = -t L, f applied to the exact eigenvalues -t mu."""
    mu = laplacian_eigs(N, dim)
    lam = -t * mu
    vals = f(lam.ravel()).reshape(lam.shape)
    return _dst_apply(np.asarray(V, np.float64), N, dim, vals)


# ---- Toeplitz -----------------------------------------------------------------

def toeplitz_matvec(col: np.ndarray, V: np.ndarray) -> np.ndarray:
    """T V for symmetric Toeplitz T = toeplitz(col) via circulant embedding of
    size 2n (Section 2 remark on fast Toeplitz products)."""
    n = len(col)
    emb = np.concatenate([col, [0.0], col[1:][::-1]])
    sym = sfft.rfft(emb)
    W = sfft.irfft(sym[:, None] * sfft.rfft(V, n=2 * n, axis=0), n=2 * n, axis=0)
    return W[:n]


def levinson_first_column(col: np.ndarray) -> np.ndarray:
    """x = T^{-1} e_1 for symmetric positive definite Toeplitz T (scipy's
    Levinson-Durbin solver)."""
    e1 = np.zeros(len(col))
    e1[0] = 1.0
    return sla.solve_toeplitz(col, e1)


def cg_first_column(col: np.ndarray, rtol: float = 1e-15, maxiter: int = 100000) -> np.ndarray:
    """x = T^{-1} e_1 for symmetric positive definite Toeplitz T = toeplitz(col)
    by plain conjugate gradients with the circulant-embedding product
    (toeplitz_matvec): O(n log n) per step where Levinson's recursion costs
    O(n^2).  Iterates until ||e_1 - T x||_2 <= rtol (||e_1|| = 1) or the
    residual stops decreasing for 50 steps; the true residual is recomputed
    every 50 steps so the recurrence cannot drift."""
    n = len(col)
    b = np.zeros(n)
    b[0] = 1.0
    T = lambda v: toeplitz_matvec(col, v[:, None])[:, 0]
    x = np.zeros(n)
    r = b.copy()
    d = r.copy()
    rr = r @ r
    best, stall = np.inf, 0
    for it in range(maxiter):
        q = T(d)
        alpha = rr / (d @ q)
        x += alpha * d
        if (it + 1) % 50 == 0:
            r = b - T(x)
        else:
            r -= alpha * q
        rr_new = r @ r
        rn = np.sqrt(rr_new)
        if rn <= rtol:
            break
        if rn < 0.5 * best:
            best, stall = rn, 0
        else:
            stall += 1
            if stall >= 50:
                break
        d = r + (rr_new / rr) * d
        rr = rr_new
    return x


def gohberg_semencul_inverse(col: np.ndarray, scale: float, x: np.ndarray | None = None):
    """(scale*T)^{-1} V for symmetric positive definite Toeplitz T by the
    Gohberg-Semencul formula (Section 4.1): with x = T^{-1} e_1,
        T^{-1} = (1/x_0) (L(x) L(x)^T - L(Z x~) L(Z x~)^T),
    L(y) the lower-triangular Toeplitz matrix with first column y, x~ the
    reversal of x and Z the down-shift.  Each lower/upper triangular Toeplitz
    product is a length-2n FFT convolution.  x defaults to Levinson's solve
    (levinson_first_column); for large n pass cg_first_column(col)."""
    n = len(col)
    if x is None:
        x = levinson_first_column(col)
    xr = x[::-1]
    y = np.concatenate([[0.0], xr[:-1]])      # Z x~

    def lower(vec_col, V):                    # L(vec) V
        F = sfft.rfft(vec_col, n=2 * n)
        return sfft.irfft(F[:, None] * sfft.rfft(V, n=2 * n, axis=0), n=2 * n, axis=0)[:n]

    def upper(vec_col, V):                    # L(vec)^T V = reverse(L(vec) reverse(V))
        return lower(vec_col, V[::-1])[::-1]

    def apply(V):
        V = np.asarray(V, np.float64)
        W = lower(x, upper(x, V)) - lower(y, upper(y, V))
        return W / (x[0] * scale)
    return apply


def toeplitz_matvec_general(col: np.ndarray, row: np.ndarray, V: np.ndarray) -> np.ndarray:
    """T V for Toeplitz T with first column col and first row row (row[0] =
    col[0]) via the circulant of size 2n whose first column is
    [col, 0, row[n-1], ..., row[1]]."""
    n = len(col)
    emb = np.concatenate([col, [0.0], row[1:][::-1]])
    F = sfft.fft(emb)
    W = sfft.ifft(F[:, None] * sfft.fft(np.asarray(V, np.float64), n=2 * n, axis=0), axis=0)
    return W[:n].real


def gohberg_semencul_general(col: np.ndarray, row: np.ndarray, scale: float):
    """(scale*T)^{-1} V for a nonsymmetric Toeplitz T (first column col, first
    row row) by the Gohberg-Semencul formula (Section 4.1 and the Toeplitz
    experiment of Section 5): with x = T^{-1} e_1, y = T^{-1} e_n (Levinson
    solves, scipy) and x_0 = x[0] != 0,
        T^{-1} = (1/x_0) (L(x) L(J y)^T - L(Z y) L(Z J x)^T),
    L(v) lower-triangular Toeplitz with first column v, J the reversal, Z the
    down-shift; for symmetric T (y = J x) this is the symmetric formula."""
    n = len(col)
    e1 = np.zeros(n)
    e1[0] = 1.0
    en = np.zeros(n)
    en[-1] = 1.0
    x = sla.solve_toeplitz((col, row), e1)
    y = sla.solve_toeplitz((col, row), en)
    shift = lambda v: np.concatenate([[0.0], v[:-1]])   # Z v

    def lower(vec_col, V):                    # L(vec) V
        F = sfft.rfft(vec_col, n=2 * n)
        return sfft.irfft(F[:, None] * sfft.rfft(V, n=2 * n, axis=0), n=2 * n, axis=0)[:n]

    def upper(vec_col, V):                    # L(vec)^T V = J L(vec) J V
        return lower(vec_col, V[::-1])[::-1]

    def apply(V):
        V = np.asarray(V, np.float64)
        W = lower(x, upper(y[::-1], V)) - lower(shift(y), upper(shift(x[::-1]), V))
        return W / (x[0] * scale)
    return apply
