"""Write the full-size reference samples under tests/golden/ (run on a CPU;
calls only the oracle and the seeded input generators).

The three large workloads are too big for the oracle to finish within a test
step, so their references are computed once here and a seeded sample of rows
is stored with the norms of the whole result:

  convdiff128.npz  3D upwind convection-diffusion 128^3, p = 16, ||tA||_1 = 1e3:
                   r(tA)B by the oracle's z-mode semi-direct solve
                   (exact.rational_kron3_tridiag), a direct solve per pole
                   and z mode with one refinement step.
  vardiff1024.npz  2D log-normal diffusion 1024^2, p = 32, t = 0.1, weights W:
                   r(tA)B, r(tA^T)W and <W, A r(tA)B> by one sparse LU per pole
                   with one refinement step per solve
                   (exact.rational_sparse_adjoint).
  toeplitz2p20.npz SPD Toeplitz n = 2^20, p = 16, ||tA||_2 ~= 1e3: the oracle's
                   PSBFOM-DR (Algorithm 2) with the Gohberg-Semencul inverse
                   whose generator T^{-1} e_1 comes from conjugate gradients,
                   stopped at the error bound 1e-12 (no direct solve fits).

Each file holds `rows` (sorted sample of row indices), `Z` (those rows of the
result), `fro` and `maxabs` (Frobenius norm and largest |entry| of the whole
result), and a JSON `meta` string.  Usage:

    python tests/golden/make_full_size_references.py convdiff vardiff toeplitz
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle import exact, inverses, psbfom  # noqa: E402

SAMPLE_SEED = 9001


def sample_rows(n: int, count: int, salt: int) -> np.ndarray:
    rng = np.random.default_rng(SAMPLE_SEED + salt)
    return np.sort(rng.choice(n, size=count, replace=False)).astype(np.int64)


def log(msg):
    print(f"[golden] {msg}", flush=True)


def convdiff(N=128, pe=50.0, vel=(1.0, 0.5, 0.25)):
    W = wl.c4(N=N, precision="fp64")
    h = 1.0 / (N + 1)
    # the 1-D factors of K = -A: second difference plus Pe v_d times the
    # backward difference (first-order upwind for v_d > 0)
    coef = [(-1.0 / h ** 2 - pe * v / h, 2.0 / h ** 2 + pe * v / h, -1.0 / h ** 2) for v in vel]
    t0 = time.perf_counter()
    Z = exact.rational_kron3_tridiag(N, coef, W.t, W.B)
    el = time.perf_counter() - t0
    rows = sample_rows(W.n, 2048, 4)
    meta = {"workload": f"convdiff3d N={N} Pe={pe} v={vel}", "n": W.n, "p": W.p, "t": W.t,
            "seed_B": 4,
            "reference": "r(tA)B, z-mode semi-direct solve per pole, one refinement step",
            "oracle_s": round(el, 1)}
    np.savez(os.path.join(HERE, "convdiff128.npz"), rows=rows, Z=Z[rows],
             fro=np.linalg.norm(Z), maxabs=np.abs(Z).max(), bfro=np.linalg.norm(W.B),
             meta=json.dumps(meta))
    log(f"convdiff {N}^3: {el:.1f} s, ||Z||/||B|| = {np.linalg.norm(Z) / np.linalg.norm(W.B):.3e}")


def vardiff(N=1024):
    W = wl.c5(N=N, precision="fp64")
    G = wl.c5_weights(N, W.p)
    M = (W.t * W.A.to_scipy()).tocsr()
    t0 = time.perf_counter()
    Z, gB, gt = exact.rational_sparse_adjoint(M, W.B, G, W.t)
    el = time.perf_counter() - t0
    rows = sample_rows(W.n, 1024, 5)
    meta = {"workload": f"vardiff2d N={N} seed 205", "n": W.n, "p": W.p, "t": W.t,
            "seed_B": 5, "seed_W": 105,
            "reference": "r(tA)B, r(tA^T)W, <W, A r(tA)B> from one sparse LU per pole, "
                         "one refinement step per solve",
            "oracle_s": round(el, 1)}
    np.savez(os.path.join(HERE, "vardiff1024.npz"), rows=rows, Z=Z[rows], fro=np.linalg.norm(Z),
             maxabs=np.abs(Z).max(), G=gB[rows], gfro=np.linalg.norm(gB),
             gmaxabs=np.abs(gB).max(), grad_t=gt, bfro=np.linalg.norm(W.B),
             meta=json.dumps(meta))
    log(f"vardiff {N}^2: {el:.1f} s, grad_t = {gt:.12e}")


def toeplitz(n=1 << 20, tol=1e-12):
    W = wl.c3(n=n)
    t0 = time.perf_counter()
    x = inverses.cg_first_column(W.col)
    log(f"toeplitz generator by CG: {time.perf_counter() - t0:.1f} s")
    inv = inverses.gohberg_semencul_inverse(W.col, -W.t, x=x)
    Z, _, info = psbfom.psbfom_dr(inv, W.B, W.m, W.k, tol, stop_rule="bound")
    el = time.perf_counter() - t0
    if not info.converged:
        raise RuntimeError("oracle did not converge")
    rows = sample_rows(W.n, 2048, 3)
    meta = {"workload": f"SPD Toeplitz n={n} seed 203", "n": W.n, "p": W.p, "t": W.t,
            "seed_B": 3, "m": W.m, "k": W.k,
            "reference": f"oracle PSBFOM-DR, Gohberg-Semencul inverse, bound rule tol {tol}",
            "cycles": info.cycles, "oracle_s": round(el, 1)}
    np.savez(os.path.join(HERE, "toeplitz2p20.npz"), rows=rows, Z=Z[rows],
             fro=np.linalg.norm(Z), maxabs=np.abs(Z).max(), bfro=np.linalg.norm(W.B),
             meta=json.dumps(meta))
    log(f"toeplitz 2^20: {el:.1f} s, {info.cycles} cycles")


if __name__ == "__main__":
    todo = sys.argv[1:] or ["convdiff", "vardiff", "toeplitz"]
    for name in todo:
        {"convdiff": convdiff, "vardiff": vardiff, "toeplitz": toeplitz}[name]()
