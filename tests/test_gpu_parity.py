"""GPU parity: the HIP path (through the C ABI) against the oracle and the
plain definitions, element by element, on seeded inputs.

Tolerance (FP64 form): 1e-10 relative in the Frobenius norm against the
rational form r(tA)B, the bar the target sets for FP64; it is measured
against r(tA)B and not e^{tA}B because the CF error (~2e-14 ||B||) is
amplified by ||B||/||Z|| (up to 2e5 on the 3D Laplacian).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import workloads as wl
from oracle import exact, inverses, psbfom
from oracle.cf import r_eval
from paper_1405_0707_amd import Plan, _lib

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rfun(lam):
    return r_eval(np.asarray(lam, dtype=np.float64))


def plan_for(W, **opts):
    return Plan.csr(W.A.rowptr, W.A.colind, W.A.val, W.t, device=DEV, **opts)


def announce(name):
    print(f"[gpu-test] {name}", flush=True)


@pytest.mark.parametrize("N,p", [(7, 1), (16, 3), (27, 4), (32, 8), (17, 16), (12, 32)])
def test_operator_matches_scipy(N, p):
    announce(f"operator N={N} p={p}")
    W = wl.c1(N=N, p=p)
    pl = plan_for(W)
    X = np.random.default_rng(p).standard_normal((W.n, p))
    Y = pl.apply_operator(torch.from_numpy(X)).cpu().numpy()
    ref = (W.t * W.A.to_scipy()) @ X
    assert np.max(np.abs(Y - ref)) <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("p", [2, 5, 8])
def test_inverse_matches_splu(p):
    announce(f"inverse p={p}")
    W = wl.c1(N=32, p=p)
    pl = plan_for(W, inner_tol=1e-13)
    X = np.random.default_rng(10 + p).standard_normal((W.n, p))
    Y, iters = pl.apply_inverse(torch.from_numpy(X))
    M = (W.t * W.A.to_scipy()).tocsr()
    ref = inverses.splu_inverse(M)(X)
    assert iters > 0
    assert rel(Y.cpu().numpy(), ref) < 1e-10


def test_c1_full_matches_oracle_and_closed_form():
    announce("execute C1 32^2 p=4 m=10")
    W = wl.c1()
    pl = plan_for(W, m=W.m, k=W.k)
    Z, info = pl.execute(torch.from_numpy(W.B), tol=W.tol)
    Z = Z.cpu().numpy()
    rB = inverses.dst_laplacian_function(32, 2, W.t, rfun, W.B)
    M = (W.t * W.A.to_scipy()).tocsr()
    Zo, _, oinfo = psbfom.psbfom_dr(inverses.splu_inverse(M), W.B, W.m, W.k, W.tol,
                                    stop_rule="bound")
    assert info.cycles >= 2, info.cycles          # the restart is exercised
    assert rel(Z, rB) < 1e-10
    assert rel(Z, Zo) < 1e-10


def test_wide_block_projected_solves_both_back_substitutions():
    """p = 32, m = 6: the projected systems reach d = 192 (d p = 6144), past
    the LDS back substitution of the projected solves (d p <= 4096), which
    the residual estimates at d = 64 and 128 still take."""
    announce("execute C1 32^2 p=32 m=6")
    W = wl.c1(N=32, p=32, m=6)
    pl = plan_for(W, m=W.m, k=W.k)
    Z, info = pl.execute(torch.from_numpy(W.B), tol=1e-10)
    rB = inverses.dst_laplacian_function(32, 2, W.t, rfun, W.B)
    assert rel(Z.cpu().numpy(), rB) < 1e-10


def test_ragged_sizes_match_dense_rational():
    announce("execute ragged 2D N=27 p=3")
    W = wl.c1(N=27, p=3, m=8)
    pl = plan_for(W, m=8, k=6)
    Z, info = pl.execute(torch.from_numpy(W.B), tol=1e-11)
    M = (W.t * W.A.to_scipy()).toarray()
    ref = exact.rational_dense(M, W.B)
    assert rel(Z.cpu().numpy(), ref) < 1e-10


def test_3d_laplacian_reduced_matches_closed_form():
    announce("execute 3D N=24 p=8 m=15")
    N = 24
    W = wl.c2(N=N)
    W.t = 5.842338 / (3 * (2 - 2 * np.cos(np.pi / (N + 1))))
    pl = plan_for(W, m=W.m, k=W.k)
    Z, info = pl.execute(torch.from_numpy(W.B), tol=W.tol)
    rB = inverses.dst_laplacian_function(N, 3, W.t, rfun, W.B)
    assert rel(Z.cpu().numpy(), rB) < 1e-10


def test_c2_full_size_matches_closed_form():
    """The benchmark workload (64^3, p = 8, m = 15) in the benchmark's launch
    configuration, against the DST-I closed form of r(tA)B at full size."""
    announce("execute C2 64^3 p=8 m=15")
    W = wl.c2()
    pl = plan_for(W, m=W.m, k=W.k)
    Z, info = pl.execute(torch.from_numpy(W.B), tol=W.tol)
    rB = inverses.dst_laplacian_function(64, 3, W.t, rfun, W.B)
    e = rel(Z.cpu().numpy(), rB)
    print(f"C2 rel err {e:.3e} cycles {info.cycles} inner {info.inner_iters}")
    assert e < 1e-10


def test_sine_modes_happy_breakdown():
    announce("sine-mode breakdown")
    N = 16
    W = wl.c1(N=N, p=2, m=6)
    k = np.arange(1, N + 1)
    s = lambda j: np.sin(k * j * np.pi / (N + 1))
    B = np.stack([np.kron(s(1), s(1)), np.kron(s(2), s(3))], 1)
    B /= np.linalg.norm(B, axis=0)
    pl = plan_for(W, m=6, k=2)
    Z, info = pl.execute(torch.from_numpy(B), tol=1e-12)
    mu = np.array([2 * (2 - 2 * np.cos(np.pi / (N + 1))),
                   (2 - 2 * np.cos(2 * np.pi / (N + 1))) + (2 - 2 * np.cos(3 * np.pi / (N + 1)))])
    expect = B * rfun(-W.t * mu)[None, :]
    assert info.cycles == 1 and info.breakdown == 1
    assert np.linalg.norm(Z.cpu().numpy() - expect) < 1e-12 * np.linalg.norm(B)


@pytest.mark.parametrize("eps", [1e-9, 1e-11])
def test_nearly_collinear_block_uses_shifted_cholesky_qr(eps):
    """B = [v, v + eps w]: its Gram matrix is singular to rounding, so plain
    Cholesky QR cannot factor the first block; the shifted factor and a
    third pass must give a basis on which the solve still converges to the
    closed form (before the fallback this block ended in EBREAKDOWN)."""
    announce(f"nearly collinear block eps={eps}")
    N = 24
    W = wl.c1(N=N, p=2)
    W.t = 2.2692 / (2 * (2 - 2 * np.cos(np.pi / (N + 1))))
    rng = np.random.default_rng(24)
    v, w = rng.standard_normal(N * N), rng.standard_normal(N * N)
    B = np.stack([v, v + eps * w], 1)
    pl = plan_for(W, m=10, k=12)
    Z, info = pl.execute(torch.from_numpy(B), tol=1e-11)
    Z = Z.cpu().numpy()
    ref = inverses.dst_laplacian_function(N, 2, W.t, rfun, B)
    assert rel(Z, ref) < 1e-10


def test_algorithm_1_unpreconditioned():
    announce("SBFOM-DR")
    W = wl.c1(N=16, p=3)
    pl = plan_for(W, m=20, k=6, preconditioned=0, max_cycles=400)
    Z, info = pl.execute(torch.from_numpy(W.B), tol=1e-12)
    ref = exact.rational_dense((W.t * W.A.to_scipy()).toarray(), W.B)
    assert rel(Z.cpu().numpy(), ref) < 1e-10


def test_grad_t_matches_definition():
    announce("grad_t")
    W = wl.c1(N=20, p=3)
    pl = plan_for(W)
    G = np.random.default_rng(3).standard_normal(W.B.shape)
    Zt = np.random.default_rng(4).standard_normal(W.B.shape)
    g = pl.grad_t(torch.from_numpy(G), torch.from_numpy(Zt))
    ref = float(np.sum(G * (W.A.to_scipy() @ Zt)))
    assert abs(g - ref) <= 1e-12 * abs(ref) + 1e-12


def test_deterministic_bitwise():
    announce("determinism")
    W = wl.c1(N=24, p=4)
    pl = plan_for(W)
    Z1, _ = pl.execute(torch.from_numpy(W.B), tol=1e-10)
    Z2, _ = pl.execute(torch.from_numpy(W.B), tol=1e-10)
    assert torch.equal(Z1, Z2)


def test_error_statuses():
    announce("error statuses")
    W = wl.c1(N=8, p=2)
    pl = plan_for(W)
    B = torch.from_numpy(W.B)
    with pytest.raises(_lib.ExpmvError) as e:
        pl.execute(B, tol=0.0)
    assert e.value.status == _lib.EINVAL
    with pytest.raises(_lib.ExpmvError) as e:
        pl.execute(torch.zeros((W.n, 40), dtype=torch.float64), tol=1e-8)
    assert e.value.status == _lib.EINVAL
    # tA not negative definite: flip the sign of A
    with pytest.raises(_lib.ExpmvError) as e:
        Plan.csr(W.A.rowptr, W.A.colind, -W.A.val, W.t, device=DEV)
    assert e.value.status == _lib.ENOTNEG
    # a basis too wide for the block Gram-Schmidt (m = 20 at p = 32) is
    # refused by the call and by the workspace size; m = 17 runs
    W32 = wl.c1(N=32, p=32)
    wide = plan_for(W32, m=20, k=32)
    with pytest.raises(_lib.ExpmvError) as e:
        wide.workspace_size(32)
    assert e.value.status == _lib.EINVAL
    with pytest.raises(_lib.ExpmvError) as e:
        wide.execute(torch.from_numpy(W32.B), tol=1e-8)
    assert e.value.status == _lib.EINVAL
    Z32, _ = plan_for(W32, m=17, k=32).execute(torch.from_numpy(W32.B), tol=1e-8)
    assert bool(torch.isfinite(Z32).all())
    # max_cycles = 1 on a problem that needs two cycles
    W1 = wl.c1()
    pl1 = plan_for(W1, m=4, k=4, max_cycles=1)
    Z, info = pl1.execute(torch.from_numpy(W1.B), tol=1e-12, allow=(_lib.ENOCONV,))
    assert info.cycles == 1


# ---------------------------------------------------------------------------
# nonsymmetric operator (upwind convection-diffusion): BiCGStab inner solver,
# general restart eigenproblem with complex Ritz pairs, transpose

def small_convdiff(N, p):
    """Reduced upwind convection-diffusion with t set so that t lambda_min(K)
    = 3.33, the value of the 128^3 workload."""
    W = wl.c4(N=N, p=p, precision="fp64")
    lam = np.linalg.eigvals(-W.A.to_scipy().toarray()) if W.n <= 4096 else None
    if lam is not None:
        W.t = 3.33 / lam.real.min()
    return W


def test_nonsymmetric_inverse_matches_splu():
    announce("BiCGStab inverse")
    W = small_convdiff(12, 4)
    pl = plan_for(W, inner_tol=1e-13)
    X = np.random.default_rng(21).standard_normal((W.n, 4))
    Y, iters = pl.apply_inverse(torch.from_numpy(X))
    M = (W.t * W.A.to_scipy()).tocsr()
    assert rel(Y.cpu().numpy(), inverses.splu_inverse(M)(X)) < 1e-10
    Yt, _ = pl.apply_inverse(torch.from_numpy(X), transpose=True)
    assert rel(Yt.cpu().numpy(), inverses.splu_inverse(M.T.tocsr())(X)) < 1e-10


@pytest.mark.parametrize("m,k", [(10, 12), (4, 4)])
def test_nonsymmetric_matches_direct_rational(m, k):
    announce(f"convdiff N=12 m={m} k={k}")
    W = small_convdiff(12, 4)
    pl = plan_for(W, m=m, k=k, max_cycles=200)
    Z, info = pl.execute(torch.from_numpy(W.B), tol=1e-11)
    M = (W.t * W.A.to_scipy()).tocsr()
    ref = exact.rational_sparse(M, W.B)
    if m == 4:
        assert info.cycles > 2        # restarts with the general eigensolver
    assert rel(Z.cpu().numpy(), ref) < 1e-10


def test_nonsymmetric_transpose_execute():
    announce("convdiff transpose")
    W = small_convdiff(10, 3)
    pl = plan_for(W, m=8, k=6)
    G = np.random.default_rng(5).standard_normal(W.B.shape)
    Zt, _ = pl.execute(torch.from_numpy(G), tol=1e-11, transpose=True)
    M = (W.t * W.A.to_scipy()).tocsr()
    ref = exact.rational_sparse(M.T.tocsr(), G)
    assert rel(Zt.cpu().numpy(), ref) < 1e-10


# ---------------------------------------------------------------------------
# mixed precision: FP32 inner solver and basis, FP64 small side, X and sums

def test_mixed_3d_laplacian_within_1e5():
    announce("mixed 3D N=24")
    N = 24
    W = wl.c2(N=N)
    W.t = 5.842338 / (3 * (2 - 2 * np.cos(np.pi / (N + 1))))
    pl = plan_for(W, m=W.m, k=W.k, precision="mixed")
    Z, info = pl.execute(torch.from_numpy(W.B), tol=1e-6)
    rB = inverses.dst_laplacian_function(N, 3, W.t, rfun, W.B)
    e = rel(Z.cpu().numpy(), rB)
    print(f"mixed 3D rel err {e:.2e}")
    assert e < 1e-5


def test_mixed_convdiff_within_1e5():
    announce("mixed convdiff N=16")
    W = small_convdiff(16, 4)
    pl = plan_for(W, m=10, k=12, precision="mixed")
    Z, info = pl.execute(torch.from_numpy(W.B), tol=1e-6)
    M = (W.t * W.A.to_scipy()).tocsr()
    ref = exact.rational_sparse(M, W.B)
    e = rel(Z.cpu().numpy(), ref)
    print(f"mixed convdiff rel err {e:.2e}")
    assert e < 1e-5


# ---------------------------------------------------------------------------
# Toeplitz operator: FFT circulant embedding and Gohberg-Semencul inverse

import scipy.linalg as sla  # noqa: E402


def small_toeplitz(n, p, m=8):
    W = wl.c3(n=n, p=p, m=m)
    W.t = 0.73 / np.linalg.eigvalsh(sla.toeplitz(W.col))[0]   # t lambda_min as at n = 2^20
    return W


def toe_plan(W, **opts):
    return Plan.toeplitz(torch.from_numpy(W.col), W.t, device=DEV, **opts)


@pytest.mark.parametrize("n,p", [(1000, 3), (1024, 4), (4096, 16), (1001, 3)])
def test_toeplitz_operator_and_inverse(n, p):
    """n with prime factors up to 5: the length-n circulant / skew-circulant
    form of the Gohberg-Semencul inverse; n = 1001 = 7 11 13: the triangular
    factors through the length-2048 embedding."""
    announce(f"toeplitz operator n={n} p={p}")
    W = wl.c3(n=n, p=p)
    pl = toe_plan(W)
    X = np.random.default_rng(n + p).standard_normal((n, p))
    T = sla.toeplitz(W.col)
    Y = pl.apply_operator(torch.from_numpy(X)).cpu().numpy()
    ref = -W.t * (T @ X)
    assert np.max(np.abs(Y - ref)) <= 1e-12 * np.abs(ref).max()
    Yi, _ = pl.apply_inverse(torch.from_numpy(X))
    refi = np.linalg.solve(-W.t * T, X)
    assert rel(Yi.cpu().numpy(), refi) < 1e-11


@pytest.mark.parametrize("n,p", [(1000, 3), (4096, 4)])
def test_toeplitz_execute_matches_direct_rational(n, p):
    announce(f"toeplitz execute n={n} p={p}")
    W = small_toeplitz(n, p)
    pl = toe_plan(W, m=W.m, k=W.k)
    Z, info = pl.execute(torch.from_numpy(W.B), tol=1e-11)
    ref = exact.rational_dense(-W.t * sla.toeplitz(W.col), W.B)
    assert rel(Z.cpu().numpy(), ref) < 1e-10
    assert max(info.true_res) < 1e-8 * np.linalg.norm(W.B)


def test_toeplitz_full_size_properties():
    """n = 2^20, p = 16, m = 17 (the full Toeplitz workload): properties that
    hold at any size, contraction and the symmetric adjoint identity (the
    oracle parity at this size is test_gpu_full_size.py's
    test_toeplitz2p20_matches_oracle)."""
    announce("toeplitz 2^20 p=16")
    W = wl.c3()
    pl = toe_plan(W, m=W.m, k=W.k)
    B = torch.from_numpy(W.B).to(DEV)
    Z, info = pl.execute(B, tol=W.tol)
    print(f"toeplitz full: cycles {info.cycles} err_bound {info.err_bound:.2e} "
          f"ms {info.ms_total:.1f}")
    zn = torch.linalg.norm(Z, dim=0)
    bn = torch.linalg.norm(B, dim=0)
    assert bool(torch.all(zn <= bn))
    Wt = torch.from_numpy(np.random.default_rng(77).standard_normal((W.n, W.p))).to(DEV)
    ZW, _ = pl.execute(Wt, tol=W.tol)
    lhs = float(torch.sum(Wt * Z))
    rhs = float(torch.sum(ZW * B))
    assert abs(lhs - rhs) <= 1e-9 * abs(lhs)


@pytest.mark.parametrize("precision,bar,inner", [("fp64", 1e-11, "jacobi"),
                                                 ("mixed", 1e-5, "jacobi"),
                                                 ("fp64", 1e-11, "amg"),
                                                 ("mixed", 1e-5, "amg")])
def test_bicgstab_wide_block_full_grid(precision, bar, inner):
    """p = 16 on 32^3 launches the inner solver's full 512-workgroup grid;
    regression test for the scalars of one iteration being overwritten while
    other workgroups of the same kernel still read them."""
    announce(f"BiCGStab 32^3 p=16 {precision} {inner}")
    W = wl.c4(N=32, p=16, precision="fp64")
    pl = plan_for(W, precision=precision, inner_maxit=2000, inner_precond=inner)
    Y, iters = pl.apply_inverse(torch.from_numpy(W.B))
    M = (W.t * W.A.to_scipy()).tocsr()
    res = np.linalg.norm(M @ Y.cpu().numpy() - W.B) / np.linalg.norm(W.B)
    assert iters < 200 and res < bar


# ---------------------------------------------------------------------------
# the caller's workspace, the status of a capped inner solve, and the FP64
# true residuals of the restart refinement

import ctypes as C  # noqa: E402


def test_workspace_is_checked_through_the_c_abi():
    """Every per-call device array comes from the caller's buffer: a missing,
    too small or misaligned one is refused with EINVAL before any device
    work, and the exact size runs."""
    announce("workspace checks")
    W = wl.c1(N=12, p=2)
    pl = plan_for(W)
    L = _lib.lib()
    need = pl.workspace_size(2)
    assert need > 0 and pl.workspace_size(4) > need
    assert pl.workspace_size(2, "times", 3) > need
    assert pl.workspace_size(2, "source") >= pl.workspace_size(4)
    work = torch.empty(need + 1024, dtype=torch.uint8, device=DEV)
    B = torch.from_numpy(W.B).to(DEV)
    Z = torch.full_like(B, 7.0)
    info = _lib.Info()
    for ptr, nb in ((work.data_ptr(), need - 1), (work.data_ptr() + 8, need), (None, need)):
        st = L.expmv_execute(pl._h, 0, B.data_ptr(), 2, 1e-10, ptr, nb, Z.data_ptr(),
                             C.byref(info))
        assert st == _lib.EINVAL
    torch.cuda.synchronize()
    assert bool(torch.all(Z == 7.0))          # nothing was written
    st = L.expmv_execute(pl._h, 0, B.data_ptr(), 2, 1e-10, work.data_ptr(), need, Z.data_ptr(),
                         C.byref(info))
    assert st == _lib.OK
    Zb, _ = pl.execute(B, tol=1e-10)
    assert torch.equal(Z, Zb)


def test_capped_inner_solve_is_reported():
    """An inner solve stopped by inner_maxit leaves the Arnoldi relation
    inexact: EINNER, even on the cycle whose estimates converge."""
    announce("inner cap status")
    W = wl.c1(N=16, p=2)
    pl = plan_for(W, m=4, k=2, inner_maxit=1, inner_precond="jacobi")
    with pytest.raises(_lib.ExpmvError) as e:
        pl.execute(torch.from_numpy(W.B), tol=1e-2)
    assert e.value.status == _lib.EINNER


@pytest.mark.parametrize("cycles", [1, 2])
def test_true_residuals_match_oracle_explicit_residuals(cycles):
    """After one and two cycles (max_cycles stops the run) the iterate of
    the shifted systems is unique, so the library's FP64 true residual norms
    ||B - (M - tau_j I) X_j|| must match the oracle's explicit residuals of
    its own X_j, shift by shift; with near-exact inner solves the residuals
    are collinear (eq. 4.8), so the part outside the last block is tiny."""
    announce(f"true residuals after {cycles} cycles")
    N = 16
    W = wl.c1(N=N, p=3)
    W.t = 2.2692 / (2 * (2 - 2 * np.cos(np.pi / (N + 1))))
    M = (W.t * W.A.to_scipy()).tocsr()
    pl = plan_for(W, m=6, k=6, max_cycles=cycles, inner_tol=1e-14, inner_relax=0,
                  inner_precond="jacobi")
    Z, info = pl.execute(torch.from_numpy(W.B), tol=1e-14, allow=(_lib.ENOCONV,))
    Zo, Xo, oinfo = psbfom.psbfom_dr(inverses.splu_inverse(M), W.B, 6, 6, 1e-14,
                                     max_cycles=cycles, stop_rule="bound")
    assert info.cycles == oinfo.cycles == cycles
    from oracle.cf import cf_table
    tau, _, _ = cf_table()
    bn = float(np.linalg.norm(W.B))
    for j in range(7):
        Rj = W.B - (M @ Xo[j] - tau[j] * Xo[j])
        r = float(np.linalg.norm(Rj))
        # the residuals are differences of O(||B||) terms: each side carries
        # ~1e-13 ||B|| of rounding, the floor of the comparisons below
        floor = 1e-12 * bn
        assert abs(info.true_res[j] - r) <= 1e-6 * r + floor, (j, info.true_res[j], r)
        assert info.noncollinear[j] <= 1e-8 * r + floor, (j, info.noncollinear[j], r)
        assert abs(info.est[j] - r) <= 1e-6 * r + floor
    assert rel(Z.cpu().numpy(), Zo) < 1e-9


@pytest.mark.parametrize("refine", [0, 1])
def test_restart_refinement_on_and_off_match_oracle(refine):
    announce(f"restart refinement {refine}")
    W = wl.c1()
    pl = plan_for(W, m=W.m, k=W.k, restart_refine=refine)
    Z, info = pl.execute(torch.from_numpy(W.B), tol=W.tol)
    rB = inverses.dst_laplacian_function(32, 2, W.t, rfun, W.B)
    assert info.cycles >= 2
    assert info.refined_restarts == (info.cycles - 1 if refine else 0)
    assert rel(Z.cpu().numpy(), rB) < 1e-10
