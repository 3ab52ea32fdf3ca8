"""Gradients of L = sum(W * e^{tA} B) through paper_1405_0707_amd.expmv
(torch.autograd.Function over the C ABI):
grad_B = e^{tA^T} W (the same solver on A^T), grad_t = <W, A e^{tA} B>.
Checked against the oracle's direct rational solves with A^T, an exact
directional derivative in B (L is linear in B), and central differences in t.
"""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import exact
from paper_1405_0707_amd import expmv

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def announce(name):
    print(f"[gpu-test] {name}", flush=True)


def vardiff_small(N=48, p=4):
    """Reduced 2D log-normal diffusion (seed 205) with t = 0.1 as at 1024^2."""
    return wl.c5(N=N, p=p, precision="fp64")


def csr_tuple(W):
    return (torch.from_numpy(W.A.rowptr), torch.from_numpy(W.A.colind), torch.from_numpy(W.A.val))


@pytest.mark.parametrize("precision,tol_b,tol_t", [("fp64", 1e-10, 1e-10), ("mixed", 1e-5, 1e-5)])
def test_grad_b_and_t(precision, tol_b, tol_t):
    announce(f"autograd vardiff {precision}")
    W = vardiff_small()
    Wt = np.random.default_rng(105).standard_normal(W.B.shape)
    B = torch.from_numpy(W.B).to(DEV).requires_grad_(True)
    t = torch.tensor(W.t, dtype=torch.float64, requires_grad=True)
    Z = expmv(csr_tuple(W), B, t, tol=1e-11 if precision == "fp64" else 1e-7, precision=precision)
    Lv = torch.sum(torch.from_numpy(Wt).to(DEV) * Z)
    Lv.backward()
    M = (W.t * W.A.to_scipy()).tocsr()
    gB_ref = exact.rational_sparse(M.T.tocsr(), Wt)
    eb = rel(B.grad.cpu().numpy(), gB_ref)
    # grad_t = <W, A r(tA) B> from the oracle's direct solves (partial
    # fractions of x r(x), so no operator multiplies a computed solution)
    _, _, gt_ref = exact.rational_sparse_adjoint(M, W.B, Wt, W.t)
    et = abs(float(t.grad) - gt_ref) / abs(gt_ref)
    print(f"{precision}: grad_B rel err {eb:.2e}, grad_t rel err {et:.2e}")
    assert eb < tol_b
    assert et < tol_t


def test_grad_t_central_difference():
    announce("grad_t central difference")
    W = vardiff_small(N=40, p=3)
    Wt = torch.from_numpy(np.random.default_rng(6).standard_normal(W.B.shape)).to(DEV)
    B = torch.from_numpy(W.B).to(DEV)
    A = csr_tuple(W)
    t = torch.tensor(W.t, dtype=torch.float64, requires_grad=True)
    L = torch.sum(Wt * expmv(A, B, t, tol=1e-12))
    L.backward()
    h = 1e-4 * W.t
    Lp = float(torch.sum(Wt * expmv(A, B, W.t + h, tol=1e-12)))
    Lm = float(torch.sum(Wt * expmv(A, B, W.t - h, tol=1e-12)))
    fd = (Lp - Lm) / (2 * h)
    print(f"grad_t {float(t.grad):.10e} fd {fd:.10e}")
    assert abs(float(t.grad) - fd) <= 1e-6 * abs(fd)


def test_grad_b_directional_is_exact():
    announce("grad_B directional")
    W = vardiff_small(N=40, p=3)
    Wt = torch.from_numpy(np.random.default_rng(7).standard_normal(W.B.shape)).to(DEV)
    A = csr_tuple(W)
    B = torch.from_numpy(W.B).to(DEV).requires_grad_(True)
    L = torch.sum(Wt * expmv(A, B, W.t, tol=1e-12))
    L.backward()
    dB = torch.from_numpy(np.random.default_rng(8).standard_normal(W.B.shape)).to(DEV)
    L2 = torch.sum(Wt * expmv(A, B.detach() + dB, W.t, tol=1e-12))
    lhs = float(L2 - L)
    rhs = float(torch.sum(B.grad * dB))
    assert abs(lhs - rhs) <= 1e-9 * abs(lhs)


def test_nonsymmetric_grad_b_uses_transpose():
    announce("autograd convdiff")
    Wc = wl.c4(N=10, p=3, precision="fp64")
    lam = np.linalg.eigvals(-Wc.A.to_scipy().toarray())
    Wc.t = 3.33 / lam.real.min()
    G = np.random.default_rng(9).standard_normal(Wc.B.shape)
    B = torch.from_numpy(Wc.B).to(DEV).requires_grad_(True)
    Z = expmv(csr_tuple(Wc), B, Wc.t, tol=1e-11)
    torch.sum(torch.from_numpy(G).to(DEV) * Z).backward()
    M = (Wc.t * Wc.A.to_scipy()).tocsr()
    assert rel(B.grad.cpu().numpy(), exact.rational_sparse(M.T.tocsr(), G)) < 1e-10


def test_vector_input_and_reused_plan():
    """A vector B gives a vector Z and a vector grad_B; a plan made once is
    reused for another B; a plan for another t is refused."""
    announce("autograd vector B, reused plan")
    from paper_1405_0707_amd import Plan
    W = vardiff_small(N=24, p=1)
    A = csr_tuple(W)
    pl = Plan.csr(*A, W.t, device=DEV)
    g = np.random.default_rng(11).standard_normal(W.A.n)
    b = torch.from_numpy(W.B[:, 0].copy()).to(DEV).requires_grad_(True)
    z = expmv(A, b, W.t, tol=1e-11, plan=pl)
    assert z.shape == b.shape
    torch.sum(torch.from_numpy(g).to(DEV) * z).backward()
    assert b.grad.shape == b.shape
    M = (W.t * W.A.to_scipy()).tocsr()
    assert rel(z.detach().cpu().numpy(), exact.rational_sparse(M, W.B[:, :1])[:, 0]) < 1e-10
    assert rel(b.grad.cpu().numpy(), exact.rational_sparse(M.T.tocsr(), g[:, None])[:, 0]) < 1e-10
    z2 = expmv(A, 2.0 * b.detach(), W.t, tol=1e-11, plan=pl)
    assert rel(z2.cpu().numpy(), 2.0 * z.detach().cpu().numpy()) < 1e-10
    with pytest.raises(ValueError):
        expmv(A, b, 2.0 * W.t, plan=pl)


def test_calls_from_another_stream_are_ordered():
    """A plan made on the default stream, used from a side stream whose
    pending work produces the input and whose next work reads the output:
    the binding orders the library's stream after and before it."""
    announce("side stream ordering")
    from paper_1405_0707_amd import Plan
    W = vardiff_small(N=32, p=2)
    A = csr_tuple(W)
    pl = Plan.csr(*A, W.t, device=DEV)
    ref, _ = pl.execute(torch.from_numpy(W.B).to(DEV), tol=1e-11)
    side = torch.cuda.Stream(device=DEV)
    base = torch.from_numpy(W.B).to(DEV)
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        big = torch.ones(4096, 4096, dtype=torch.float64, device=DEV)
        for _ in range(4):
            big = big @ big * (1.0 / 4096)       # keeps the side stream busy
        B = base * big[0, 0]                     # = base, ready only after the products
        Z, _ = pl.execute(B, tol=1e-11)
        Z2 = Z * 1.0                             # read on the side stream
    torch.cuda.synchronize()
    assert rel(Z2.cpu().numpy(), ref.cpu().numpy()) < 1e-12
