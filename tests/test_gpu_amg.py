"""GPU checks of the AMG-preconditioned inner solver (through the C ABI):
the device V-cycle against the numpy V-cycle over the same host hierarchy
(element by element), the inner solve against a sparse LU solve, and whole
solves against the closed form, with AMG and with Jacobi."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import inverses
from oracle.cf import r_eval
from paper_1405_0707_amd import HostAmg, Plan

from amg_reference import VCycle

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def announce(name):
    print(f"[gpu-test] {name}", flush=True)


def _workload(name):
    if name == "lap3d20":
        A, t = wl.laplacian_3d(20), 5.842338 / (3 * (2 - 2 * np.cos(np.pi / 21)))
    elif name == "lap3d40":   # four levels: a sparse fused restriction on level 1
        A, t = wl.laplacian_3d(40), 5.842338 / (3 * (2 - 2 * np.cos(np.pi / 41)))
    elif name == "lap2d40":   # two levels: the finest level restricts into the dense solve
        A, t = wl.laplacian_2d(40), 30.0
    elif name == "vardiff96":
        A, t = wl.vardiff_2d(96, 205), 0.1
    else:
        A, t = wl.laplacian_2d(70), 30.0
    return A, t


def _host_vcycle(A, t, degree):
    """The numpy V-cycle with the library's default coarse degree,
    max(1, degree - 1)."""
    K = A.val * (-t)   # the plan's K = -tA, rounded the same way
    return VCycle(HostAmg(A.rowptr, A.colind, K).levels(), degree, max(1, degree - 1))


@pytest.mark.parametrize("name,p,degree", [("lap3d20", 8, 2), ("lap3d20", 3, 1),
                                           ("vardiff96", 32, 2), ("lap2d70", 1, 3),
                                           ("vardiff96", 16, 4), ("lap3d40", 8, 2),
                                           ("lap3d40", 5, 1), ("lap2d40", 4, 2),
                                           ("vardiff96", 12, 2), ("lap3d20", 20, 2)])
def test_device_vcycle_matches_numpy_vcycle(name, p, degree):
    announce(f"V-cycle {name} p={p} degree={degree}")
    A, t = _workload(name)
    pl = Plan.csr(A.rowptr, A.colind, A.val, t, device=DEV, inner_precond="amg",
                  amg_degree=degree, amg_fp32=0)
    X = np.random.default_rng(p).standard_normal((A.n, p))
    Y = pl.apply_preconditioner(torch.from_numpy(X)).cpu().numpy()
    ref = _host_vcycle(A, t, degree).apply(X)
    assert rel(Y, ref) < 1e-12
    # the preconditioner is symmetric: <P x, y> = <x, P y>
    Xs = X[:, :1]
    Ys = np.random.default_rng(99).standard_normal((A.n, 1))
    Px = pl.apply_preconditioner(torch.from_numpy(Xs)).cpu().numpy()
    Py = pl.apply_preconditioner(torch.from_numpy(Ys)).cpu().numpy()
    a, b = float(Px[:, 0] @ Ys[:, 0]), float(Xs[:, 0] @ Py[:, 0])
    assert abs(a - b) <= 1e-12 * abs(a)


@pytest.mark.parametrize("form,p", [("mixed", 8), ("fp64_fp32_vcycle", 8), ("mixed", 12),
                                    ("fp64_fp32_vcycle", 20), ("mixed", 16), ("mixed", 24),
                                    ("mixed", 32), ("fp64_fp32_vcycle", 32)])
def test_device_fp32_vcycle(form, p):
    """The FP32 V-cycle (FP32 values and vectors, FP64 sums) of the mixed
    form and, by default, of the FP64 form's CG, against the numpy V-cycle
    in FP64; symmetric to FP32 rounding."""
    announce(f"V-cycle FP32 ({form}) p={p}")
    A, t = _workload("vardiff96")
    kw = {"precision": "mixed"} if form == "mixed" else {"amg_fp32": 1}
    pl = Plan.csr(A.rowptr, A.colind, A.val, t, device=DEV, inner_precond="amg", **kw)
    X = np.random.default_rng(4).standard_normal((A.n, p))
    Y = pl.apply_preconditioner(torch.from_numpy(X)).cpu().numpy()
    assert rel(Y, _host_vcycle(A, t, 2).apply(X)) < 1e-5
    Px = pl.apply_preconditioner(torch.from_numpy(X[:, :1])).cpu().numpy()[:, 0]
    Py = pl.apply_preconditioner(torch.from_numpy(X[:, 1:2])).cpu().numpy()[:, 0]
    a, b = float(Px @ X[:, 1]), float(X[:, 0] @ Py)
    assert abs(a - b) <= 1e-5 * np.linalg.norm(Px) * np.linalg.norm(X[:, 1])


@pytest.mark.parametrize("p", [12, 16, 20, 24, 32])
def test_mixed_amg_inverse_wide_blocks(p):
    """The FP32 inner CG and V-cycle of the mixed form against a sparse LU
    solve: four columns per lane with masked lanes (p = 12, 20), eight
    columns per lane (p = 16, 32, the 128^3 and 1024^2 workloads' widths) and
    eight with one of four lanes masked (p = 24)."""
    announce(f"mixed AMG inverse vardiff96 p={p}")
    A, t = _workload("vardiff96")
    X = np.random.default_rng(7).standard_normal((A.n, p))
    M = (t * A.to_scipy()).tocsr()
    ref = inverses.splu_inverse(M)(X)
    pl = Plan.csr(A.rowptr, A.colind, A.val, t, device=DEV, inner_precond="amg",
                  precision="mixed", inner_tol=1e-6)
    Y, it = pl.apply_inverse(torch.from_numpy(X))
    assert rel(Y.cpu().numpy(), ref) < 1e-5
    assert 0 < it <= 40


@pytest.mark.parametrize("name,p", [("lap3d20", 8), ("vardiff96", 5), ("lap3d20", 12),
                                    ("vardiff96", 20)])
def test_amg_inverse_matches_splu_in_few_iterations(name, p):
    announce(f"AMG inverse {name} p={p}")
    A, t = _workload(name)
    X = np.random.default_rng(3).standard_normal((A.n, p))
    M = (t * A.to_scipy()).tocsr()
    ref = inverses.splu_inverse(M)(X)
    amg = Plan.csr(A.rowptr, A.colind, A.val, t, device=DEV, inner_precond="amg",
                   inner_tol=1e-13)
    jac = Plan.csr(A.rowptr, A.colind, A.val, t, device=DEV, inner_precond="jacobi",
                   inner_tol=1e-13)
    Ya, ita = amg.apply_inverse(torch.from_numpy(X))
    Yj, itj = jac.apply_inverse(torch.from_numpy(X))
    assert rel(Ya.cpu().numpy(), ref) < 1e-10
    assert rel(Yj.cpu().numpy(), ref) < 1e-10
    assert 0 < ita <= 40 and itj >= 5 * ita, (ita, itj)


@pytest.mark.parametrize("precond", ["amg", "jacobi"])
def test_solve_with_each_preconditioner_matches_closed_form(precond):
    announce(f"execute 3D N=24 p=8 m=15 inner={precond}")
    N = 24
    W = wl.c2(N=N)
    W.t = 5.842338 / (3 * (2 - 2 * np.cos(np.pi / (N + 1))))
    pl = Plan.csr(W.A.rowptr, W.A.colind, W.A.val, W.t, device=DEV, m=W.m, k=W.k,
                  inner_precond=precond)
    Z, info = pl.execute(torch.from_numpy(W.B), tol=W.tol)
    rB = inverses.dst_laplacian_function(N, 3, W.t, lambda x: r_eval(np.asarray(x)), W.B)
    assert rel(Z.cpu().numpy(), rB) < 1e-10
    assert (info.amg_levels > 1) == (precond == "amg")


def test_amg_vardiff_matches_direct_rational():
    """Variable coefficients (log-normal, sigma = 1), 64^2, p = 4: AMG-PCG
    inner solves inside the whole method against per-pole sparse solves."""
    announce("execute vardiff 64^2 AMG")
    A = wl.vardiff_2d(64, 205)
    t = 0.1
    B = np.random.default_rng(5).standard_normal((A.n, 4))
    pl = Plan.csr(A.rowptr, A.colind, A.val, t, device=DEV, m=10, inner_precond="amg")
    Z, info = pl.execute(torch.from_numpy(B), tol=1e-11)
    from oracle import exact
    ref = exact.rational_sparse((t * A.to_scipy()).tocsc(), B)
    assert rel(Z.cpu().numpy(), ref) < 1e-10
    assert info.amg_levels >= 2


# ---------------------------------------------------------------------------
# nonsymmetric operator: AMG-preconditioned BiCGStab, hierarchies of K and K^T

def _convdiff(N):
    """Upwind convection-diffusion on N^3 with t lambda_min = 3.33, as on 128^3."""
    import scipy.sparse.linalg as spla
    A = wl.convdiff_3d(N, 50.0)
    lam = spla.eigs((-A.to_scipy()).tocsc(), k=1, sigma=0, return_eigenvectors=False)
    return A, 3.33 / float(lam.real.min())


@pytest.mark.parametrize("N,p,transpose", [(20, 4, False), (20, 4, True), (20, 16, False),
                                           (40, 4, True)])
def test_device_vcycle_nonsymmetric_matches_numpy(N, p, transpose):
    announce(f"V-cycle convdiff {N}^3 p={p} transpose={transpose}")
    A, t = _convdiff(N)
    pl = Plan.csr(A.rowptr, A.colind, A.val, t, device=DEV, inner_precond="amg")
    X = np.random.default_rng(p).standard_normal((A.n, p))
    Y = pl.apply_preconditioner(torch.from_numpy(X), transpose=transpose).cpu().numpy()
    K = (A.to_scipy() * (-t)).tocsr()
    if transpose:
        K = K.T.tocsr()
        K.sort_indices()
    V = VCycle(HostAmg(K.indptr, K.indices, K.data, symmetric=False).levels(), 1)
    assert rel(Y, V.apply(X)) < 1e-12


def _convdiff27(N):
    """The upwind operator plus a symmetric M-matrix part with 27-point rows,
    0.2 mean(diag K) (I - S (x) S (x) S), S = tridiag(1, 1, 1) / 3: operator
    rows longer than one pipelined step of the inner SpMM (8 entries), and
    fused transfer operators whose rows outgrow one step of the V-cycle
    kernels (restriction rows of 200 to 335 entries)."""
    import scipy.sparse as sp
    A, t = _convdiff(N)
    S = sp.diags([1.0, 1.0, 1.0], [-1, 0, 1], shape=(N, N)) / 3.0
    K7 = -A.to_scipy()
    K = (K7 + 0.2 * K7.diagonal().mean() * (sp.identity(A.n) - sp.kron(S, sp.kron(S, S)))).tocsr()
    K.sort_indices()
    return wl.CSR.from_scipy(-K), t


@pytest.mark.parametrize("p,transpose", [(16, False), (6, True)])
def test_long_rows_vcycle_and_inverse(p, transpose):
    announce(f"27-point convdiff 16^3 p={p} transpose={transpose}: V-cycle and inverse")
    A, t = _convdiff27(16)
    pl = Plan.csr(A.rowptr, A.colind, A.val, t, device=DEV, inner_precond="amg",
                  inner_tol=1e-13)
    X = np.random.default_rng(p).standard_normal((A.n, p))
    Y = pl.apply_preconditioner(torch.from_numpy(X), transpose=transpose).cpu().numpy()
    K = (A.to_scipy() * (-t)).tocsr()
    if transpose:
        K = K.T.tocsr()
        K.sort_indices()
    H = HostAmg(K.indptr, K.indices, K.data, symmetric=False)
    rf = np.diff(H.fused(0, "restriction", 0.5, 0.0)[0])
    assert rf.mean() >= 32 and rf.max() > 80
    assert rel(Y, VCycle(H.levels(), 1).apply(X)) < 1e-12
    M = (t * A.to_scipy()).tocsr()
    ref = inverses.splu_inverse(M.T.tocsr() if transpose else M)(X)
    Yi, its = pl.apply_inverse(torch.from_numpy(X), transpose=transpose)
    assert rel(Yi.cpu().numpy(), ref) < 1e-10, its


@pytest.mark.parametrize("transpose", [False, True])
def test_amg_bicgstab_inverse_matches_splu(transpose):
    announce(f"AMG BiCGStab inverse convdiff 24^3 transpose={transpose}")
    A, t = _convdiff(24)
    X = np.random.default_rng(8).standard_normal((A.n, 4))
    M = (t * A.to_scipy()).tocsr()
    ref = inverses.splu_inverse(M.T.tocsr() if transpose else M)(X)
    amg = Plan.csr(A.rowptr, A.colind, A.val, t, device=DEV, inner_precond="amg",
                   inner_tol=1e-13)
    jac = Plan.csr(A.rowptr, A.colind, A.val, t, device=DEV, inner_precond="jacobi",
                   inner_tol=1e-13)
    Ya, ita = amg.apply_inverse(torch.from_numpy(X), transpose=transpose)
    Yj, itj = jac.apply_inverse(torch.from_numpy(X), transpose=transpose)
    assert rel(Ya.cpu().numpy(), ref) < 1e-10
    assert rel(Yj.cpu().numpy(), ref) < 1e-10
    assert 0 < ita <= 40 and itj > 2 * ita, (ita, itj)


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_amg_convdiff_solve_matches_direct_rational(precision, bar):
    announce(f"execute convdiff 16^3 AMG {precision}")
    A, t = _convdiff(16)
    B = np.random.default_rng(6).standard_normal((A.n, 4))
    pl = Plan.csr(A.rowptr, A.colind, A.val, t, device=DEV, m=10, k=12, inner_precond="amg",
                  precision=precision)
    Z, info = pl.execute(torch.from_numpy(B), tol=1e-11 if precision == "fp64" else 1e-6)
    from oracle import exact
    ref = exact.rational_sparse((t * A.to_scipy()).tocsc(), B)
    assert rel(Z.cpu().numpy(), ref) < bar
    assert info.amg_levels >= 2


# ---------------------------------------------------------------------------
# relaxed inner solves (inner_relax): inner tolerance grows like ||B|| / rho

@pytest.mark.parametrize("inner", ["amg", "jacobi"])
def test_relaxed_inner_solves_keep_accuracy(inner):
    announce(f"relaxed inner solves 3D 24^3 {inner}")
    N = 24
    W = wl.c2(N=N)
    W.t = 5.842338 / (3 * (2 - 2 * np.cos(np.pi / (N + 1))))
    rB = inverses.dst_laplacian_function(N, 3, W.t, lambda x: r_eval(np.asarray(x)), W.B)
    its = {}
    for relax in (0, 8):
        pl = Plan.csr(W.A.rowptr, W.A.colind, W.A.val, W.t, device=DEV, m=6, k=16,
                      inner_precond=inner, inner_relax=relax)
        Z, info = pl.execute(torch.from_numpy(W.B), tol=1e-10)
        assert rel(Z.cpu().numpy(), rB) < 1e-10
        its[relax] = info.inner_iters
    assert its[8] < 0.9 * its[0], its
