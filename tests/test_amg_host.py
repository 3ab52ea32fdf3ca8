"""CPU checks of the AMG hierarchy the library builds on the host for its
inner preconditioner (exported as expmv_host_amg_*): aggregation, smoothed
prolongator, Galerkin operators, eigenvalue bound, coarse inverse, and the
symmetry, definiteness and effect of the V-cycle assembled from them."""
from __future__ import annotations

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as wl
from paper_1405_0707_amd import HostAmg
from paper_1405_0707_amd._lib import ExpmvError

from amg_reference import VCycle, pcg


def _pos(A: wl.CSR):
    """K = -A (positive definite) as CSR arrays and scipy."""
    K = -A.to_scipy()
    K.eliminate_zeros()
    K.sort_indices()
    return K


def _levels(K, symmetric=True, **kw):
    h = HostAmg(K.indptr, K.indices, K.data, symmetric=symmetric, **kw)
    return h, h.levels()


def _csr(lv):
    rp, ci, v = lv["A"]
    return sp.csr_matrix((v, ci, rp), shape=(lv["n"], lv["n"]))


def _prolong(lv):
    prp, pci, pv, nc = lv["P"]
    return sp.csr_matrix((pv, pci, prp), shape=(lv["n"], nc))


@pytest.mark.parametrize("name", ["lap3d16", "vardiff64", "lap2d32"])
def test_hierarchy_structure_and_galerkin(name):
    A = {"lap3d16": lambda: wl.laplacian_3d(16), "vardiff64": lambda: wl.vardiff_2d(64, 205),
         "lap2d32": lambda: wl.laplacian_2d(32)}[name]()
    K = _pos(A)
    _, lvs = _levels(K, max_coarse=100)
    assert len(lvs) >= 2
    assert abs(_csr(lvs[0]) - K).max() == 0.0
    for l in range(len(lvs) - 1):
        Al, P = _csr(lvs[l]), _prolong(lvs[l])
        nc = P.shape[1]
        agg = lvs[l]["agg"]
        # aggregates partition the unknowns, none empty, real coarsening
        assert agg.min() == 0 and agg.max() == nc - 1
        assert np.all(np.bincount(agg, minlength=nc) > 0)
        assert nc < 0.85 * lvs[l]["n"]
        # P = (I - omega D^{-1} A) T, T piecewise constant with unit columns
        size = np.bincount(agg)
        T = sp.csr_matrix((1.0 / np.sqrt(size[agg]), (np.arange(lvs[l]["n"]), agg)),
                          shape=(lvs[l]["n"], nc))
        assert np.allclose((T.T @ T).toarray(), np.eye(nc), atol=1e-14)
        omega = (4.0 / 3.0) / lvs[l]["lmax"]
        Pref = T - omega * sp.diags(1.0 / Al.diagonal()) @ Al @ T
        assert abs(P - Pref).max() <= 1e-14 * abs(Pref).max()
        # Galerkin coarse operator
        Ac = _csr(lvs[l + 1])
        Gal = P.T @ Al @ P
        assert abs(Ac - Gal).max() <= 1e-12 * abs(Gal).max()
        assert lvs[l + 1]["n"] == nc
    assert lvs[-1]["n"] <= 100


@pytest.mark.parametrize("symmetric", [True, False])
def test_lambda_max_bound(symmetric):
    """lmax is an upper bound of the spectral radius of D^{-1} A, never above
    the Gershgorin bound, and for symmetric A within 10% of the radius
    (Lanczos estimate times 1.1; the power estimate of a non-normal D^{-1} A
    can exceed the radius)."""
    A = wl.laplacian_3d(8) if symmetric else wl.convdiff_3d(8, 50.0)
    K = _pos(A)
    _, lvs = _levels(K, symmetric=symmetric, max_coarse=20)
    for lv in lvs:
        Al = _csr(lv).toarray()
        rad = np.abs(np.linalg.eigvals(Al / np.diag(Al)[:, None])).max()
        gersh = (np.abs(Al).sum(axis=1) / np.diag(Al)).max()
        assert lv["lmax"] >= rad * (1 - 1e-12)
        assert lv["lmax"] <= gersh * (1 + 1e-12)
        if symmetric:
            assert lv["lmax"] <= 1.1 * rad * (1 + 1e-12)


def test_coarse_inverse():
    K = _pos(wl.vardiff_2d(32, 205))
    h, lvs = _levels(K, max_coarse=200)
    Ac = _csr(lvs[-1]).toarray()
    inv = h.coarse_inverse()
    assert np.abs(inv @ Ac - np.eye(Ac.shape[0])).max() < 1e-10


@pytest.mark.parametrize("degree", [1, 2, 3])
def test_vcycle_symmetric_positive_definite(degree):
    K = _pos(wl.laplacian_3d(8))
    _, lvs = _levels(K, max_coarse=30)
    V = VCycle(lvs, degree)
    M = V.apply(np.eye(K.shape[0]))
    assert np.abs(M - M.T).max() <= 1e-12 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0.0
    # a convergent two-sided method: spectrum of M K within (0, 2)
    ev = np.linalg.eigvals(M @ K.toarray()).real
    assert ev.min() > 0.0 and ev.max() < 2.0


@pytest.mark.parametrize("name,maxit", [("lap3d24", 25), ("vardiff128", 30)])
def test_vcycle_cuts_pcg_iterations(name, maxit):
    A = wl.laplacian_3d(24) if name == "lap3d24" else wl.vardiff_2d(128, 205)
    K = _pos(A)
    _, lvs = _levels(K)
    V = VCycle(lvs, 2)
    b = np.random.default_rng(7).standard_normal(K.shape[0])
    x, it = pcg(K, b, V.apply, tol=1e-12)
    assert np.linalg.norm(b - K @ x) <= 1e-12 * np.linalg.norm(b)
    assert it <= maxit
    _, itj = pcg(K, b, lambda r: r / K.diagonal(), tol=1e-12, maxit=20000)
    assert itj >= 5 * it


def test_nonpositive_diagonal_is_rejected():
    K = _pos(wl.laplacian_2d(8)).tolil()
    K[3, 3] = 0.0
    K = K.tocsr()
    with pytest.raises(ExpmvError):
        HostAmg(K.indptr, K.indices, K.data)


@pytest.mark.parametrize("name,symmetric", [("vardiff", True), ("convdiff", False)])
def test_fused_transfer_operators(name, symmetric):
    """The fused operators of the device V-cycle against their definition
    with scipy products: the restriction of the pre-smoothed residual
    R (I - A D^{-1}(alpha I - beta A D^{-1})) for one step (beta = 0) and for
    two Chebyshev steps (beta != 0), and the prolongation followed by one
    smoothing step (I - s D^{-1} A) P, on every level above the coarsest.
    A planted mistake (the wrong side of D^{-1}) fails the comparison."""
    # variable diagonals, so that D^{-1} A and A D^{-1} differ
    A = wl.vardiff_2d(48, 205) if name == "vardiff" else wl.convdiff_3d(12, 50.0)
    K = _pos(A)
    h, lvs = _levels(K, symmetric=symmetric, max_coarse=60)
    assert len(lvs) >= 3
    planted = 0
    for level, lv in enumerate(lvs[:-1]):
        Al = _csr(lv)
        # the planted mistake shows where the diagonal is not constant
        varies = np.ptp(Al.diagonal()) > 1e-9 * abs(Al.diagonal()).max()
        planted += int(varies)
        P = _prolong(lv)
        R = P.T.tocsr()
        Dinv = sp.diags(1.0 / Al.diagonal())
        I = sp.identity(Al.shape[0], format="csr")
        s0 = 0.7 / lv["lmax"]
        for alpha, beta in ((s0, 0.0), (1.9 * s0, 0.4 * s0 * s0)):
            rp, ci, v, shape = h.fused(level, "restriction", alpha, beta)
            F = sp.csr_matrix((v, ci, rp), shape=shape)
            ref = R @ (I - Al @ Dinv @ (alpha * I - beta * Al @ Dinv))
            assert shape == ref.shape
            assert abs(F - ref).max() <= 1e-14 * abs(ref).max()
            wrong = R @ (I - Dinv @ Al @ (alpha * I - beta * Dinv @ Al))
            assert not varies or abs(F - wrong).max() > 1e-6 * abs(ref).max()
        rp, ci, v, shape = h.fused(level, "prolongation", s0)
        F = sp.csr_matrix((v, ci, rp), shape=shape)
        ref = (I - s0 * Dinv @ Al) @ P
        assert abs(F - ref).max() <= 1e-14 * abs(ref).max()
        wrong = (I - s0 * Al @ Dinv) @ P
        assert not varies or abs(F - wrong).max() > 1e-6 * abs(ref).max()
    assert planted >= 1
    with pytest.raises(ExpmvError):
        h.fused(len(lvs) - 1, "restriction", 1.0)
