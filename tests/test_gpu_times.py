"""GPU parity of the several-times driver (expmv_execute_times): Z_q =
e^{t_q A} B for a t-sweep on one shared Krylov basis, each block against the
plain definition r(t_q A) B (closed form or direct per-pole solves) and
against the one-time solve of the same plan."""
import numpy as np
import pytest
import scipy.linalg as sla
import torch

import workloads as wl
from oracle import exact, inverses
from oracle.cf import r_eval
from paper_1405_0707_amd import Plan, _lib
from paper_1405_0707_amd._lib import ExpmvError

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def announce(name):
    print(f"[gpu-test] {name}", flush=True)


def rfun(lam):
    return r_eval(np.asarray(lam, dtype=np.float64))


@pytest.mark.parametrize("inner", ["jacobi", "amg"])
def test_laplacian_sweep_matches_closed_form(inner):
    """2D Laplacian 70^2 (n = 4900), p = 4, four times spanning 8x."""
    announce(f"times 2D 70^2 {inner}")
    N = 70
    A = wl.laplacian_2d(N)
    t0 = 2.2692 / (2 * (2 - 2 * np.cos(np.pi / (N + 1))))   # t lambda_min as the 32^2 case
    times = [0.25 * t0, 0.5 * t0, t0, 2.0 * t0]
    B = np.random.default_rng(31).standard_normal((A.n, 4))
    pl = Plan.csr(A.rowptr, A.colind, A.val, t0, device=DEV, m=12, k=16, inner_precond=inner)
    Z, info = pl.execute_times(times, torch.from_numpy(B), tol=1e-11)
    Z = Z.cpu().numpy()
    for q, tq in enumerate(times):
        ref = inverses.dst_laplacian_function(N, 2, tq, rfun, B)
        assert rel(Z[q], ref) < 1e-10, (q, rel(Z[q], ref))
    Z1, _ = pl.execute(torch.from_numpy(B), tol=1e-11)
    assert rel(Z[2], Z1.cpu().numpy()) < 1e-10
    assert info.err_bound <= 1e-11


def test_3d_sweep_with_amg_and_restarts():
    """Times t0/3 .. 1.25 t0 (t lambda_min up to 7.3).  Much larger times are
    not a relative-error case: Z = omega_0 B + Re sum c_j X_j is a sum of
    O(|B|) terms, so its rounding floor is ~1e-15 |B| whatever the solver
    (at t lambda_min = 17.5, |Z| ~ 2.5e-8 |B| and that floor is 3e-7 of |Z|)."""
    announce("times 3D 24^3 AMG, restarted")
    N = 24
    W = wl.c2(N=N)
    t0 = 5.842338 / (3 * (2 - 2 * np.cos(np.pi / (N + 1))))
    times = [t0 / 3, t0, 1.25 * t0]
    pl = Plan.csr(W.A.rowptr, W.A.colind, W.A.val, t0, device=DEV, m=6, k=16)
    Z, info = pl.execute_times(times, torch.from_numpy(W.B), tol=1e-11)
    assert info.cycles >= 2
    for q, tq in enumerate(times):
        ref = inverses.dst_laplacian_function(N, 3, tq, rfun, W.B)
        assert rel(Z[q].cpu().numpy(), ref) < 1e-10


def test_nonsymmetric_sweep_matches_direct_rational():
    announce("times convdiff 12^3")
    A = wl.convdiff_3d(12, 50.0)
    import scipy.sparse.linalg as spla
    lam = spla.eigs((-A.to_scipy()).tocsc(), k=1, sigma=0, return_eigenvectors=False)
    t0 = 3.33 / float(lam.real.min())
    times = [0.5 * t0, t0, 1.7 * t0]
    B = np.random.default_rng(12).standard_normal((A.n, 3))
    pl = Plan.csr(A.rowptr, A.colind, A.val, t0, device=DEV, m=10, k=12, max_cycles=200)
    Z, _ = pl.execute_times(times, torch.from_numpy(B), tol=1e-11)
    for q, tq in enumerate(times):
        ref = exact.rational_sparse((tq * A.to_scipy()).tocsc(), B)
        assert rel(Z[q].cpu().numpy(), ref) < 1e-10
    Zt, _ = pl.execute_times(times, torch.from_numpy(B), tol=1e-11, transpose=True)
    for q, tq in enumerate(times):
        ref = exact.rational_sparse((tq * A.to_scipy()).T.tocsc(), B)
        assert rel(Zt[q].cpu().numpy(), ref) < 1e-10


def test_toeplitz_sweep_matches_dense_rational():
    announce("times toeplitz n=1000")
    W = wl.c3(n=1000, p=3, m=8)
    T = sla.toeplitz(W.col)
    t0 = 0.73 / np.linalg.eigvalsh(T)[0]
    times = [0.5 * t0, t0, 1.5 * t0]
    pl = Plan.toeplitz(torch.from_numpy(W.col), t0, device=DEV, m=8, k=W.k)
    Z, _ = pl.execute_times(times, torch.from_numpy(W.B), tol=1e-11)
    for q, tq in enumerate(times):
        ref = exact.rational_dense(-tq * T, W.B)
        assert rel(Z[q].cpu().numpy(), ref) < 1e-10


def test_mixed_sweep_within_1e5():
    announce("times mixed 3D 24^3")
    N = 24
    W = wl.c2(N=N)
    t0 = 5.842338 / (3 * (2 - 2 * np.cos(np.pi / (N + 1))))
    times = [0.5 * t0, t0, 1.25 * t0]
    pl = Plan.csr(W.A.rowptr, W.A.colind, W.A.val, t0, device=DEV, m=W.m, k=W.k,
                  precision="mixed")
    Z, _ = pl.execute_times(times, torch.from_numpy(W.B), tol=1e-6)
    for q, tq in enumerate(times):
        ref = inverses.dst_laplacian_function(N, 3, tq, rfun, W.B)
        assert rel(Z[q].cpu().numpy(), ref) < 1e-5


def test_times_errors():
    announce("times errors")
    W = wl.c1(N=16, p=2)
    pl = Plan.csr(W.A.rowptr, W.A.colind, W.A.val, W.t, device=DEV)
    B = torch.from_numpy(W.B)
    with pytest.raises(ExpmvError) as e:
        pl.execute_times([W.t, -W.t], B)
    assert e.value.status == _lib.ENOTNEG
    with pytest.raises(ExpmvError) as e:
        pl.execute_times([W.t, float("nan")], B)
    assert e.value.status == _lib.EINVAL
    with pytest.raises(ExpmvError) as e:
        pl.execute_times([], B)
    assert e.value.status == _lib.EINVAL
