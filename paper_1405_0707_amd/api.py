"""Torch-facing API over the C ABI (argument marshalling only; every step of
the computation runs in libexpmv.so).

    plan = Plan.csr(rowptr, colind, val, t, m=15)       # device tensors
    Z, info = plan.execute(B, tol=1e-10)                 # Z = e^{tA} B
    Z = expmv(A, B, t)                                   # autograd-aware

`expmv` is a torch.autograd.Function: grad_B = e^{tA^T} G (the same solver on
A^T) and grad_t = <G, A r(tA) B> from the shifted solutions of that same
solve (expmv_adjoint); the forward Krylov basis is not stored (only B), the
backward solve rebuilds its own.
"""
from __future__ import annotations

import ctypes as C
import dataclasses

import torch

from . import _lib
from ._lib import Info, Opts, check, lib


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().expmv_default_opts(C.byref(o))
    for key, v in kw.items():
        if key == "precision" and isinstance(v, str):
            v = {"fp64": _lib.FP64, "mixed": _lib.MIXED, "mixed_inner": _lib.MIXED_INNER}[v]
        if key == "stop_rule" and isinstance(v, str):
            v = {"paper": _lib.STOP_PAPER, "bound": _lib.STOP_BOUND}[v]
        if key == "inner_precond" and isinstance(v, str):
            v = {"jacobi": _lib.JACOBI, "amg": _lib.AMG, "auto": _lib.AUTO}[v]
        if not hasattr(o, key):
            raise TypeError(f"unknown option {key}")
        setattr(o, key, v)
    return o


def _stream_ptr(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _dev_f64(x, device) -> torch.Tensor:
    x = torch.as_tensor(x)
    return x.to(device=device, dtype=torch.float64).contiguous()


@dataclasses.dataclass
class Toeplitz:
    """Toeplitz T given by its first column (and first row when T is not
    symmetric), optionally with a positive row scaling d; the exponent is
    t * (-diag(d) T)."""
    col0: torch.Tensor
    row0: torch.Tensor | None = None
    diag: torch.Tensor | None = None


class Plan:
    """Owns an expmv_plan (K = -tA and its workspace on one device)."""

    def __init__(self, handle, n: int, device, t: float, keepalive=()):
        self._h = handle
        self.n = n
        self.device = device
        self.t = t
        self._keep = keepalive
        # the stream the library runs this plan's work on (torch's current
        # stream when the plan was made)
        self._stream = (torch.cuda.current_stream(device)
                        if torch.device(device).type == "cuda" else None)
        self._work = {}   # (kind, p, nt) -> uint8 device tensor (the call's workspace)

    def workspace_size(self, p: int, kind: str = "execute", nt: int = 1) -> int:
        """Bytes of device workspace a call with block width p needs (kind:
        "execute" for execute / adjoint / grad_t / apply_*, "times" for
        execute_times with nt times, "source" for execute_source)."""
        b = C.c_size_t()
        if kind == "times":
            st = lib().expmv_workspace_size_times(self._h, int(p), int(nt), C.byref(b))
        elif kind == "source":
            st = lib().expmv_workspace_size_source(self._h, int(p), C.byref(b))
        else:
            st = lib().expmv_workspace_size(self._h, int(p), C.byref(b))
        check(st, "expmv_workspace_size")
        return b.value

    def _ws(self, p: int, kind: str = "execute", nt: int = 1):
        """(pointer, bytes) of a workspace for the call, allocated by torch on
        the plan's device and kept for later calls of the same shape."""
        key = (kind, int(p), int(nt))
        t = self._work.get(key)
        if t is None:
            nbytes = self.workspace_size(p, kind, nt)
            t = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=self.device)
            self._work[key] = t
        return t.data_ptr(), t.numel()

    def _run(self, call):
        """Run a library call on the plan's stream, ordered after the work
        queued on the caller's current stream (which produced the inputs) and
        before what the caller queues next (which reads the outputs)."""
        cur = torch.cuda.current_stream(self.device) if self._stream is not None else None
        other = cur is not None and cur != self._stream
        if other:
            self._stream.wait_stream(cur)
        st = call()
        if other:
            cur.wait_stream(self._stream)
        return st

    @classmethod
    def csr(cls, rowptr, colind, val, t: float, device="cuda", **opts):
        rowptr = torch.as_tensor(rowptr).to(device=device, dtype=torch.int32).contiguous()
        colind = torch.as_tensor(colind).to(device=device, dtype=torch.int32).contiguous()
        val = _dev_f64(val, device)
        n = rowptr.numel() - 1
        o = default_opts(**opts)
        h = C.c_void_p()
        st = lib().expmv_plan_csr(n, val.numel(), rowptr.data_ptr(), colind.data_ptr(),
                                  val.data_ptr(), float(t), C.byref(o), _stream_ptr(rowptr.device),
                                  C.byref(h))
        check(st, "expmv_plan_csr")
        return cls(h, n, rowptr.device, float(t))

    @classmethod
    def toeplitz(cls, col0, t: float, device="cuda", row0=None, diag=None, **opts):
        """A = -diag(d) T with T Toeplitz: first column col0, first row row0
        (None: T symmetric), d = diag (None: d = 1)."""
        col0 = _dev_f64(col0, device)
        o = default_opts(**opts)
        h = C.c_void_p()
        if row0 is None and diag is None:
            st = lib().expmv_plan_toeplitz(col0.numel(), col0.data_ptr(), float(t), C.byref(o),
                                           _stream_ptr(col0.device), C.byref(h))
            check(st, "expmv_plan_toeplitz")
            return cls(h, col0.numel(), col0.device, float(t))
        row0 = None if row0 is None else _dev_f64(row0, device)
        diag = None if diag is None else _dev_f64(diag, device)
        st = lib().expmv_plan_toeplitz_general(col0.numel(), col0.data_ptr(),
                                               None if row0 is None else row0.data_ptr(),
                                               None if diag is None else diag.data_ptr(),
                                               float(t), C.byref(o), _stream_ptr(col0.device),
                                               C.byref(h))
        check(st, "expmv_plan_toeplitz_general")
        return cls(h, col0.numel(), col0.device, float(t))

    def _block(self, x, name: str) -> torch.Tensor:
        """x as a contiguous FP64 n x p block on the plan's device (a vector
        becomes one column).  The library reads n rows through the pointer,
        so a block of any other height is refused here."""
        x = _dev_f64(x, self.device)
        if x.dim() == 1:
            x = x[:, None]
        if x.dim() != 2 or x.shape[0] != self.n or x.shape[1] < 1:
            raise ValueError(f"{name} must be an n x p block with n = {self.n}, "
                             f"got shape {tuple(x.shape)}")
        return x

    def _out(self, out, like: torch.Tensor, name: str) -> torch.Tensor:
        if out is None:
            return torch.empty_like(like)
        if (out.dtype != torch.float64 or out.device != like.device or not out.is_contiguous()
                or tuple(out.shape) != tuple(like.shape)):
            raise ValueError(f"{name} must be a contiguous float64 tensor of shape "
                             f"{tuple(like.shape)} on {like.device}")
        nb = like.numel() * 8
        if out.data_ptr() < like.data_ptr() + nb and like.data_ptr() < out.data_ptr() + nb:
            raise ValueError(f"{name} may not overlap the input block")
        return out

    def release_workspaces(self):
        """Drop the cached workspaces (torch frees them)."""
        self._work = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().expmv_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    def execute(self, B: torch.Tensor, tol: float = 1e-10, transpose: bool = False,
                out: torch.Tensor | None = None, allow=()):
        B = self._block(B, "B")
        Z = self._out(out, B, "out")
        info = Info()
        wp, wb = self._ws(B.shape[1])
        st = self._run(lambda: lib().expmv_execute(
            self._h, int(transpose), B.data_ptr(), B.shape[1], float(tol), wp, wb, Z.data_ptr(),
            C.byref(info)))
        check(st, "expmv_execute", allow)
        return Z, info

    def execute_times(self, times, B: torch.Tensor, tol: float = 1e-10, transpose: bool = False,
                      allow=()):
        """Z[q] = e^{t_q A} B for every t_q in `times` on one shared Krylov
        basis (A = the plan's matrix); returns (Z of shape (nt, n, p), info)."""
        B = self._block(B, "B")
        ts = (C.c_double * len(times))(*[float(x) for x in times])
        Z = torch.empty((len(times),) + tuple(B.shape), dtype=torch.float64, device=self.device)
        info = Info()
        wp, wb = self._ws(B.shape[1], "times", len(times))
        st = self._run(lambda: lib().expmv_execute_times(
            self._h, int(transpose), ts, len(times), B.data_ptr(), B.shape[1], float(tol),
            wp, wb, Z.data_ptr(), C.byref(info)))
        check(st, "expmv_execute_times", allow)
        return Z, info

    def execute_source(self, U0: torch.Tensor, S: torch.Tensor, gamma: float,
                       tol: float = 1e-10, transpose: bool = False, allow=()):
        """U = solution at the plan's t of u' = A u + e^{gamma s} S, u(0) = U0,
        with both exponentials in the CF form (one solve on [U0 | S])."""
        U0 = self._block(U0, "U0")
        S = self._block(S, "S")
        if U0.shape != S.shape:
            raise ValueError("U0 and S must have the same shape")
        U = torch.empty_like(U0)
        info = Info()
        wp, wb = self._ws(U0.shape[1], "source")
        st = self._run(lambda: lib().expmv_execute_source(
            self._h, int(transpose), U0.data_ptr(), S.data_ptr(), U0.shape[1], float(gamma),
            float(tol), wp, wb, U.data_ptr(), C.byref(info)))
        check(st, "expmv_execute_source", allow)
        return U, info

    def grad_t(self, G: torch.Tensor, Z: torch.Tensor) -> float:
        G = self._block(G, "G")
        Z = self._block(Z, "Z")
        if G.shape != Z.shape:
            raise ValueError("G and Z must have the same shape")
        out = C.c_double()
        wp, wb = self._ws(G.shape[1])
        check(self._run(lambda: lib().expmv_grad_t(
            self._h, G.data_ptr(), Z.data_ptr(), G.shape[1], wp, wb, C.byref(out))),
            "expmv_grad_t")
        return out.value

    def adjoint(self, G: torch.Tensor, B: torch.Tensor, tol: float = 1e-10, allow=()):
        """(e^{tA^T} G, <G, A r(tA) B>, info) from one transposed solve."""
        G = self._block(G, "G")
        B = self._block(B, "B")
        if G.shape != B.shape:
            raise ValueError("G and B must have the same shape")
        gB = torch.empty_like(G)
        gt = C.c_double()
        info = Info()
        wp, wb = self._ws(G.shape[1])
        st = self._run(lambda: lib().expmv_adjoint(
            self._h, G.data_ptr(), B.data_ptr(), G.shape[1], float(tol), wp, wb, gB.data_ptr(),
            C.byref(gt), C.byref(info)))
        check(st, "expmv_adjoint", allow)
        return gB, gt.value, info

    def apply_operator(self, X: torch.Tensor, transpose: bool = False) -> torch.Tensor:
        X = self._block(X, "X")
        Y = torch.empty_like(X)
        wp, wb = self._ws(X.shape[1])
        check(self._run(lambda: lib().expmv_apply_operator(
            self._h, int(transpose), X.data_ptr(), X.shape[1], wp, wb, Y.data_ptr())),
            "expmv_apply_operator")
        return Y

    def apply_preconditioner(self, X: torch.Tensor, transpose: bool = False) -> torch.Tensor:
        """One application of the inner solver's preconditioner for K = -tA
        (Jacobi D^{-1}, or one AMG V-cycle): Y ~= K^{-1} X."""
        X = self._block(X, "X")
        Y = torch.empty_like(X)
        wp, wb = self._ws(X.shape[1])
        check(self._run(lambda: lib().expmv_apply_preconditioner(
            self._h, int(transpose), X.data_ptr(), X.shape[1], wp, wb, Y.data_ptr())),
            "expmv_apply_preconditioner")
        return Y

    def apply_inverse(self, X: torch.Tensor, transpose: bool = False):
        X = self._block(X, "X")
        Y = torch.empty_like(X)
        it = C.c_longlong()
        wp, wb = self._ws(X.shape[1])
        check(self._run(lambda: lib().expmv_apply_inverse(
            self._h, int(transpose), X.data_ptr(), X.shape[1], wp, wb, Y.data_ptr(),
            C.byref(it))), "expmv_apply_inverse")
        return Y, it.value


class HostAmg:
    """The library's AMG hierarchy of a host CSR matrix (numpy arrays), for
    inspection: levels()[l] = dict(A=(rowptr, colind, val), P=(...) or None,
    agg, lmax, n); coarse_inverse() the dense inverse of the coarsest A."""

    def __init__(self, rowptr, colind, val, symmetric=True, theta=0.08, max_coarse=500):
        import numpy as np
        self._np = np
        rp = np.ascontiguousarray(rowptr, dtype=np.int32)
        ci = np.ascontiguousarray(colind, dtype=np.int32)
        v = np.ascontiguousarray(val, dtype=np.float64)
        h = C.c_void_p()
        check(lib().expmv_host_amg_build(rp.size - 1, rp.ctypes.data, ci.ctypes.data, v.ctypes.data,
                                         int(bool(symmetric)), float(theta), int(max_coarse),
                                         C.byref(h)), "expmv_host_amg_build")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().expmv_host_amg_destroy(h)
            except Exception:
                pass
            self._h = None

    def fused(self, level: int, which: str, alpha: float, beta: float = 0.0):
        """The device V-cycle's fused transfer operator of `level` as
        (rowptr, colind, val, shape): which = "restriction" gives
        R (I - A D^{-1}(alpha I - beta A D^{-1})), "prolongation" gives
        (I - alpha D^{-1} A) P."""
        np = self._np
        w = {"restriction": 0, "prolongation": 1}[which]
        dims = np.zeros(3, dtype=np.int64)
        check(lib().expmv_host_amg_fused(self._h, level, w, float(alpha), float(beta),
                                         dims.ctypes.data, None, None, None), "expmv_host_amg_fused")
        rows, cols, nnz = (int(x) for x in dims)
        rp = np.zeros(rows + 1, np.int32)
        ci = np.zeros(nnz, np.int32)
        v = np.zeros(nnz, np.float64)
        check(lib().expmv_host_amg_fused(self._h, level, w, float(alpha), float(beta),
                                         dims.ctypes.data, rp.ctypes.data, ci.ctypes.data,
                                         v.ctypes.data), "expmv_host_amg_fused")
        return rp, ci, v, (rows, cols)

    def levels(self):
        np = self._np
        out = []
        for lv in range(lib().expmv_host_amg_levels(self._h)):
            dims = np.zeros(4, dtype=np.int64)
            lmax = C.c_double()
            check(lib().expmv_host_amg_level(self._h, lv, dims.ctypes.data, C.byref(lmax), None,
                                             None, None, None, None, None, None),
                  "expmv_host_amg_level")
            n, nnz_a, nc, nnz_p = (int(x) for x in dims)
            arp = np.zeros(n + 1, np.int32)
            aci = np.zeros(nnz_a, np.int32)
            av = np.zeros(nnz_a, np.float64)
            prp = np.zeros(n + 1, np.int32)
            pci = np.zeros(nnz_p, np.int32)
            pv = np.zeros(nnz_p, np.float64)
            agg = np.zeros(n, np.int32)
            check(lib().expmv_host_amg_level(self._h, lv, dims.ctypes.data, C.byref(lmax),
                                             arp.ctypes.data, aci.ctypes.data, av.ctypes.data,
                                             prp.ctypes.data, pci.ctypes.data, pv.ctypes.data,
                                             agg.ctypes.data), "expmv_host_amg_level")
            out.append({"n": n, "A": (arp, aci, av), "lmax": lmax.value,
                        "P": (prp, pci, pv, nc) if nc > 0 else None,
                        "agg": agg if nc > 0 else None})
        return out

    def coarse_inverse(self):
        np = self._np
        nc = self.levels()[-1]["n"]
        inv = np.zeros((nc, nc), np.float64)
        check(lib().expmv_host_amg_coarse_inverse(self._h, inv.ctypes.data),
              "expmv_host_amg_coarse_inverse")
        return inv


def cf_table():
    """The library's CF table: (tau[7], c[7], omega0) as Python complex/float."""
    a = [(C.c_double * 7)() for _ in range(4)]
    w0 = C.c_double()
    lib().expmv_cf_table(a[0], a[1], a[2], a[3], C.byref(w0))
    tau = [complex(a[0][i], a[1][i]) for i in range(7)]
    c = [complex(a[2][i], a[3][i]) for i in range(7)]
    return tau, c, w0.value


def _make_plan(A, t, device, opts):
    if isinstance(A, Toeplitz):
        return Plan.toeplitz(A.col0, t, device=device, row0=A.row0, diag=A.diag, **opts)
    if isinstance(A, torch.Tensor) and A.layout == torch.sparse_csr:
        return Plan.csr(A.crow_indices(), A.col_indices(), A.values(), t, device=device, **opts)
    rowptr, colind, val = A
    return Plan.csr(rowptr, colind, val, t, device=device, **opts)


class _ExpmvFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, B, t, plan, tol, t_float):
        Bd = B.detach()
        Z, info = plan.execute(Bd, tol=tol)
        ctx.plan = plan
        ctx.tol = tol
        ctx.save_for_backward(Bd)
        ctx.info = info
        return Z.view(B.shape)   # a vector B gives a vector Z

    @staticmethod
    def backward(ctx, G):
        (B,) = ctx.saved_tensors
        gB, gt, _ = ctx.plan.adjoint(G.contiguous(), B, tol=ctx.tol)
        gB = gB.view(B.shape)
        gt_t = torch.tensor(gt, dtype=torch.float64, device=gB.device)
        return (gB if ctx.needs_input_grad[0] else None,
                gt_t if ctx.needs_input_grad[1] else None, None, None, None)


def expmv(A, B: torch.Tensor, t, tol: float = 1e-10, plan: Plan | None = None, **opts):
    """Z = e^{tA} B with gradients for B and t (not A).  A is a CSR tuple
    (rowptr, colind, val), a torch sparse CSR tensor or a Toeplitz; t is a
    float or a 0-dim tensor."""
    t_t = t if isinstance(t, torch.Tensor) else torch.tensor(float(t), dtype=torch.float64)
    t_float = float(t_t.detach())
    if plan is None:
        plan = _make_plan(A, t_float, B.device, opts)
    elif plan.t != t_float:
        raise ValueError(f"the plan was made for t = {plan.t}, not t = {t_float}")
    return _ExpmvFn.apply(B, t_t, plan, tol, t_float)
