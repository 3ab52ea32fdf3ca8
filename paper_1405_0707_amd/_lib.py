"""ctypes binding of libexpmv.so (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libexpmv.so")

OK, EINVAL, ENOTNEG, ENOMEM, ENOCONV, EBREAKDOWN, EHIP, EINNER = range(8)
JACOBI, AMG, AUTO = 0, 1, -1
FP64, MIXED, MIXED_INNER = 0, 1, 2
STOP_PAPER, STOP_BOUND = 0, 1
# expmv_kernel_class (timed kernel classes, opts.profile > 0)
KT_NAMES = ["cg_spmm", "cg_resid", "cg_dir", "bcg_spmm1", "bcg_spmm2", "bcg_u1", "bcg_u2",
            "bcg_u3", "amg_smooth", "amg_restrict", "amg_prolong", "amg_coarse", "orth"]
KT_COUNT = 16


class Opts(C.Structure):
    _fields_ = [("m", C.c_int), ("k", C.c_int), ("max_cycles", C.c_int),
                ("precision", C.c_int), ("stop_rule", C.c_int), ("inner_tol", C.c_double),
                ("inner_maxit", C.c_int), ("symmetric", C.c_int), ("preconditioned", C.c_int),
                ("profile", C.c_int), ("inner_refine", C.c_int), ("inner_precond", C.c_int),
                ("amg_degree", C.c_int), ("inner_relax", C.c_int), ("amg_fp32", C.c_int),
                ("amg_coarse_degree", C.c_int), ("restart_refine", C.c_int)]


class Info(C.Structure):
    _fields_ = [("cycles", C.c_int), ("block_apps", C.c_int), ("inner_iters", C.c_longlong),
                ("inner_maxit_hit", C.c_int), ("est", C.c_double * 7),
                ("true_res", C.c_double * 7), ("err_bound", C.c_double),
                ("bnorm", C.c_double), ("znorm", C.c_double), ("ms_total", C.c_double),
                ("ms_apply", C.c_double), ("ms_orth", C.c_double), ("ms_small", C.c_double),
                ("ms_update", C.c_double), ("breakdown", C.c_int), ("amg_levels", C.c_int),
                ("kern_launches", C.c_int * KT_COUNT), ("kern_ms", C.c_double * KT_COUNT),
                ("kern_bytes", C.c_double * KT_COUNT), ("noncollinear", C.c_double * 7),
                ("true_bound", C.c_double), ("noncollinear_bound", C.c_double),
                ("refined_restarts", C.c_int)]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if isinstance(v, C.Array) else v
        return d


EXPORTS = [
    "expmv_default_opts", "expmv_plan_csr", "expmv_plan_toeplitz", "expmv_execute",
    "expmv_grad_t", "expmv_adjoint", "expmv_apply_operator", "expmv_apply_inverse", "expmv_cf_table",
    "expmv_host_eig_sym", "expmv_host_eig_general", "expmv_plan_destroy",
    "expmv_status_string", "expmv_block_csr", "expmv_block_toeplitz",
    "expmv_apply_preconditioner", "expmv_host_amg_build", "expmv_host_amg_levels",
    "expmv_host_amg_level", "expmv_host_amg_coarse_inverse", "expmv_host_amg_destroy",
    "expmv_host_amg_fused",
    "expmv_execute_times", "expmv_last_error_detail", "expmv_plan_toeplitz_general",
    "expmv_execute_source", "expmv_workspace_size", "expmv_workspace_size_times",
    "expmv_workspace_size_source", "expmv_execute_noalloc",
]

_lib = None


def lib():
    """Load libexpmv.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libexpmv.so not found at {LIB_PATH}: build it with "
                           "`python -m paper_1405_0707_amd.build` (there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    vp, i64, dbl, i32 = C.c_void_p, C.c_int64, C.c_double, C.c_int
    L.expmv_default_opts.argtypes = [C.POINTER(Opts)]
    L.expmv_plan_csr.argtypes = [i64, i64, vp, vp, vp, dbl, C.POINTER(Opts), vp, C.POINTER(vp)]
    L.expmv_plan_toeplitz.argtypes = [i64, vp, dbl, C.POINTER(Opts), vp, C.POINTER(vp)]
    L.expmv_plan_toeplitz_general.argtypes = [i64, vp, vp, vp, dbl, C.POINTER(Opts), vp,
                                              C.POINTER(vp)]
    sz = C.c_size_t
    L.expmv_workspace_size.argtypes = [vp, i64, C.POINTER(sz)]
    L.expmv_workspace_size_times.argtypes = [vp, i64, i32, C.POINTER(sz)]
    L.expmv_workspace_size_source.argtypes = [vp, i64, C.POINTER(sz)]
    L.expmv_execute.argtypes = [vp, i32, vp, i64, dbl, vp, sz, vp, C.POINTER(Info)]
    L.expmv_execute_noalloc.argtypes = [vp, i32, vp, i64, dbl, vp, C.POINTER(Info)]
    L.expmv_grad_t.argtypes = [vp, vp, vp, i64, vp, sz, C.POINTER(dbl)]
    L.expmv_adjoint.argtypes = [vp, vp, vp, i64, dbl, vp, sz, vp, C.POINTER(dbl),
                                C.POINTER(Info)]
    L.expmv_apply_operator.argtypes = [vp, i32, vp, i64, vp, sz, vp]
    L.expmv_apply_inverse.argtypes = [vp, i32, vp, i64, vp, sz, vp, C.POINTER(C.c_longlong)]
    L.expmv_cf_table.argtypes = [vp, vp, vp, vp, vp]
    L.expmv_host_eig_sym.argtypes = [i32, vp, vp, vp]
    L.expmv_host_eig_general.argtypes = [i32, vp, vp, vp, vp, vp]
    L.expmv_plan_destroy.argtypes = [vp]
    L.expmv_plan_destroy.restype = None
    L.expmv_status_string.argtypes = [i32]
    L.expmv_status_string.restype = C.c_char_p
    L.expmv_last_error_detail.argtypes = []
    L.expmv_last_error_detail.restype = C.c_char_p
    L.expmv_block_csr.argtypes = [i64, i64, vp, vp, vp, vp, i64, dbl, dbl, vp, vp]
    L.expmv_block_toeplitz.argtypes = [i64, vp, vp, i64, dbl, dbl, vp, vp]
    L.expmv_apply_preconditioner.argtypes = [vp, i32, vp, i64, vp, sz, vp]
    L.expmv_execute_times.argtypes = [vp, i32, vp, i32, vp, i64, dbl, vp, sz, vp,
                                      C.POINTER(Info)]
    L.expmv_execute_source.argtypes = [vp, i32, vp, vp, i64, dbl, dbl, vp, sz, vp,
                                       C.POINTER(Info)]
    L.expmv_host_amg_build.argtypes = [i64, vp, vp, vp, i32, dbl, i32, C.POINTER(vp)]
    L.expmv_host_amg_levels.argtypes = [vp]
    L.expmv_host_amg_level.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.expmv_host_amg_fused.argtypes = [vp, i32, i32, dbl, dbl, vp, vp, vp, vp]
    L.expmv_host_amg_coarse_inverse.argtypes = [vp, vp]
    L.expmv_host_amg_destroy.argtypes = [vp]
    L.expmv_host_amg_destroy.restype = None
    for name in EXPORTS:
        if name not in ("expmv_plan_destroy", "expmv_status_string", "expmv_host_amg_destroy",
                        "expmv_last_error_detail"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


class ExpmvError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = lib().expmv_status_string(status).decode()
        detail = lib().expmv_last_error_detail().decode()
        super().__init__(f"{where}: {msg} (status {status})" + (f" [{detail}]" if detail else ""))
        self.status = status


def check(status: int, where: str, allow=()):
    if status != OK and status not in allow:
        raise ExpmvError(status, where)
    return status
