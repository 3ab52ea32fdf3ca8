"""MI355X-native e^{tA}B by the preconditioned, restarted and shifted block
FOM with deflation (PSBFOM-DR; Wu, Pang, Sun, arXiv:1405.0707).

The computation runs in libexpmv.so (hand-written HIP for gfx950, C ABI in
include/expmv.h); this package only marshals torch tensors to it.
"""
from .api import HostAmg, Plan, Toeplitz, expmv, cf_table, default_opts  # noqa: F401
