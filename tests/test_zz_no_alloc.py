"""The no-allocation entry point expmv_execute_noalloc (static device
workspace) through the C ABI, against expmv_execute with a caller workspace
on the same inputs, on two calls in a row (the second with a smaller
problem and block), and its refusal of a problem whose workspace exceeds
the static array."""
import ctypes as C
import os
import re

import numpy as np
import pytest
import torch

import workloads as wl
from paper_1405_0707_amd import Plan, _lib

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def static_bytes():
    txt = open(os.path.join(ROOT, "include", "expmv.h")).read()
    m = re.search(r"#define EXPMV_STATIC_WORKSPACE_BYTES \(\(size_t\)(\d+) << (\d+)\)", txt)
    return int(m.group(1)) << int(m.group(2))


def small_lap2d(N, p):
    W = wl.c1(N=N, p=p)
    W.t = 2.2692 / (2 * (2 - 2 * np.cos(np.pi / (N + 1))))
    return W


def test_noalloc_matches_execute_on_two_calls_then_refuses_too_large():
    L = _lib.lib()
    cap = static_bytes()
    # call 1: 32^2, p = 4, two cycles; call 2: 16^2, p = 2 (smaller)
    for N, p, m, k in ((32, 4, 10, 12), (16, 2, 6, 4)):
        print(f"[gpu-test] noalloc N={N} p={p}", flush=True)
        W = small_lap2d(N, p)
        pl = Plan.csr(W.A.rowptr, W.A.colind, W.A.val, W.t, device=DEV, m=m, k=k)
        assert pl.workspace_size(p) <= cap
        B = torch.from_numpy(W.B).to(DEV)
        Zref, iref = pl.execute(B, tol=1e-11)
        Z = torch.full_like(B, np.nan)
        info = _lib.Info()
        st = L.expmv_execute_noalloc(pl._h, 0, B.data_ptr(), p, 1e-11, Z.data_ptr(),
                                     C.byref(info))
        assert st == _lib.OK
        assert info.cycles == iref.cycles and info.inner_iters == iref.inner_iters
        e = float(torch.linalg.norm(Z - Zref) / torch.linalg.norm(Zref))
        assert e < 1e-13, e
    # a problem whose workspace exceeds the static array: EINVAL, Z untouched
    W = wl.c2(N=64, p=8)
    pl = Plan.csr(W.A.rowptr, W.A.colind, W.A.val, W.t, device=DEV, m=15, k=40)
    assert pl.workspace_size(8) > cap
    B = torch.from_numpy(W.B).to(DEV)
    Z = torch.full_like(B, 3.0)
    st = L.expmv_execute_noalloc(pl._h, 0, B.data_ptr(), 8, 1e-10, Z.data_ptr(), None)
    assert st == _lib.EINVAL
    assert b"needs" in L.expmv_last_error_detail()
    torch.cuda.synchronize()
    assert bool(torch.all(Z == 3.0))
