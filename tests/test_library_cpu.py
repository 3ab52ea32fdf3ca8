"""Host-side checks of libexpmv.so that need no GPU: it loads, exports every
symbol include/expmv.h declares, its CF table agrees with the oracle's as a
function on (-inf, 0], and its host eigensolvers (restart step) are right."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1405_0707_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "expmv.h")).read()
    return sorted(set(re.findall(r"\b(expmv_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    names = header_symbols()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name


def test_cf_table_matches_oracle_as_function():
    from oracle.cf import r_eval, cf_table
    from paper_1405_0707_amd.api import cf_table as lib_table
    tau, c, w0 = lib_table()
    x = -np.logspace(-6, 6, 6000)
    r_lib = r_eval(x, np.array(tau), np.array(c), w0)
    r_orc = r_eval(x)
    assert np.max(np.abs(r_lib - r_orc)) < 2e-14
    # same poles (both are the CF poles; FP64 rounding apart)
    t_o, c_o, w_o = cf_table()
    assert np.max(np.abs(np.array(tau) - t_o)) < 1e-12


def _sym(n, seed):
    A = np.random.default_rng(seed).standard_normal((n, n))
    return A + A.T


@pytest.mark.parametrize("n", [1, 2, 7, 40, 120])
def test_host_symmetric_eig(n):
    A = _sym(n, n)
    w = np.zeros(n)
    Q = np.zeros((n, n))
    st = _lib.lib().expmv_host_eig_sym(n, A.ctypes.data, w.ctypes.data, Q.ctypes.data)
    assert st == 0
    ref = np.linalg.eigvalsh(A)
    assert np.max(np.abs(np.sort(w) - ref)) < 1e-12 * max(1.0, np.abs(ref).max())
    assert np.max(np.abs(Q.T @ Q - np.eye(n))) < 1e-12
    assert np.max(np.abs(A @ Q - Q * w[None, :])) < 1e-11 * max(1.0, np.abs(ref).max())


def _general_case(kind, n):
    rng = np.random.default_rng(100 + n)
    if kind == "gauss":
        return rng.standard_normal((n, n))
    if kind == "graded":       # the restart's shape: a spread spectrum, weak coupling
        return np.diag(1.0 / (1.0 + np.arange(n))) + 0.3 * rng.standard_normal((n, n)) / np.sqrt(n)
    if kind == "cyclic":       # roots of unity: the unshifted QR iteration stalls on it
        return np.roll(np.eye(n), 1, axis=0)
    if kind == "companion":
        return np.ascontiguousarray(np.vstack([np.eye(n)[1:], -rng.standard_normal(n)]).T)
    if kind == "upper":        # already triangular: every step deflates at once
        return np.triu(rng.standard_normal((n, n)))
    raise ValueError(kind)


@pytest.mark.parametrize("kind,n", [("gauss", 3), ("gauss", 10), ("gauss", 60), ("gauss", 320),
                                    ("graded", 320), ("cyclic", 9), ("companion", 12),
                                    ("upper", 15)])
def test_host_general_eig(kind, n):
    A = _general_case(kind, n)
    wr, wi = np.zeros(n), np.zeros(n)
    Vr, Vi = np.zeros((n, n)), np.zeros((n, n))
    st = _lib.lib().expmv_host_eig_general(n, A.ctypes.data, wr.ctypes.data, wi.ctypes.data,
                                           Vr.ctypes.data, Vi.ctypes.data)
    assert st == 0
    ev = wr + 1j * wi
    ref = np.linalg.eigvals(A)
    # every eigenvalue matched (as a multiset) and every pair exactly conjugate
    for e in ref:
        assert np.min(np.abs(ev - e)) < 1e-9 * np.abs(ref).max()
    for e in ev[np.abs(wi) > 0]:
        assert np.min(np.abs(ev - np.conj(e))) == 0.0
    V = Vr + 1j * Vi
    res = np.abs(A @ V - V * ev[None, :]).max()
    assert res < 1e-9 * np.abs(ref).max()


def test_host_eig_reports_non_finite_input():
    """A NaN entry cannot converge: both eigensolvers return EXPMV_ENOCONV
    (the restart step turns that into EXPMV_EBREAKDOWN)."""
    n = 6
    A = _sym(n, 3)
    A[2, 4] = A[4, 2] = np.nan
    w, Q = np.zeros(n), np.zeros((n, n))
    assert _lib.lib().expmv_host_eig_sym(n, A.ctypes.data, w.ctypes.data,
                                         Q.ctypes.data) == _lib.ENOCONV
    wr, wi = np.zeros(n), np.zeros(n)
    Vr, Vi = np.zeros((n, n)), np.zeros((n, n))
    assert _lib.lib().expmv_host_eig_general(n, A.ctypes.data, wr.ctypes.data, wi.ctypes.data,
                                             Vr.ctypes.data, Vi.ctypes.data) == _lib.ENOCONV


def test_default_options_and_range_checks():
    """expmv_default_opts fills the documented defaults; expmv_plan_csr
    rejects an out-of-range option with EINVAL before it touches a device
    (the pointers below are never dereferenced)."""
    import ctypes as C

    import numpy as np

    from paper_1405_0707_amd import _lib
    o = _lib.Opts()
    assert _lib.lib().expmv_default_opts(C.byref(o)) == 0
    assert (o.m, o.inner_relax, o.amg_fp32, o.amg_coarse_degree, o.inner_precond) == (10, 8, 0, 0, -1)
    dummy = np.zeros(4)
    ptr = dummy.ctypes.data
    bad = [("amg_fp32", 2), ("amg_coarse_degree", 5), ("amg_coarse_degree", -1), ("amg_degree", -1),
           ("inner_relax", 11), ("m", 1), ("m", 65), ("inner_precond", 2), ("precision", 7)]
    for field, value in bad:
        q = _lib.Opts()
        _lib.lib().expmv_default_opts(C.byref(q))
        setattr(q, field, value)
        h = C.c_void_p()
        st = _lib.lib().expmv_plan_csr(2, 2, ptr, ptr, ptr, 1.0, C.byref(q), None, C.byref(h))
        assert st == _lib.EINVAL, (field, value, st)
        assert not h.value


def test_binding_refuses_blocks_of_the_wrong_height():
    """The C entry points read n rows through each block pointer, so the
    binding checks every block's shape before it calls them.  A plan object
    with no library handle on the CPU shows that the checks come first."""
    import torch

    from paper_1405_0707_amd.api import Plan, expmv
    pl = Plan(None, 10, torch.device("cpu"), 0.5)
    good = torch.zeros(10, 2, dtype=torch.float64)
    for bad in (torch.zeros(9, 2), torch.zeros(11), torch.zeros(10, 0), torch.zeros(2, 10, 1)):
        with pytest.raises(ValueError):
            pl.execute(bad)
        with pytest.raises(ValueError):
            pl.apply_operator(bad)
        with pytest.raises(ValueError):
            pl.apply_inverse(bad)
        with pytest.raises(ValueError):
            pl.apply_preconditioner(bad)
        with pytest.raises(ValueError):
            pl.execute_times([1.0], bad)
        with pytest.raises(ValueError):
            pl.execute_source(good, bad, -1.0)
        with pytest.raises(ValueError):
            pl.adjoint(good, bad)
        with pytest.raises(ValueError):
            pl.grad_t(bad, good)
    with pytest.raises(ValueError):
        pl.adjoint(good, torch.zeros(10, 3))
    for out in (torch.zeros(10, 3, dtype=torch.float64), torch.zeros(10, 2, dtype=torch.float32),
                torch.zeros(2, 10, dtype=torch.float64).t()):
        with pytest.raises(ValueError):
            pl.execute(good, out=out)
    with pytest.raises(ValueError):   # output aliasing the input
        pl.execute(good, out=good)
    with pytest.raises(ValueError):   # a plan made for another t
        expmv(None, good, 0.25, plan=pl)
