#!/usr/bin/env python
"""Benchmark: time of one e^{tA}B solve (PSBFOM-DR, FP64) on one MI355X.

Workload (default): 3D 7-point Dirichlet Laplacian on 64^3 (n = 262,144,
1.81M nonzeros), ||tA||_2 = 1e4, B = 262,144 x 8 Gaussian (seed 2), block
Arnoldi length m = 15, k = 40, tol = 1e-10 on the error bound.  One "step"
is one full solve (every cycle, inner solve, orthogonalisation, projected
solve, update and the final combination) with A's plan and B already in
HBM.  Prints one JSON line.

Also reported:
  roofline      the dominant kernel of the inner solve (largest device time
                per inner iteration among the CG's SpMM, residual update,
                direction update and, with AMG, the finest level's
                smoothing-step kernel), timed with HIP events on the
                solver's stream during the timed steps (every 4th
                iteration); achieved = algorithmic bytes per launch / mean
                duration; traffic = counter bytes per launch when the
                kernel sources are the ones the counters were taken on.
  cpu_baseline  the oracle (plain numpy FP64, one thread) on a bounded
                sample of the same workload, scaled to one solve.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the dominant kernels from two rocprofv3 --pmc runs
# (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, calibrated on a 256 MiB device copy;
# early-exit launches excluded), valid while the kernel sources hash to the
# recorded value; any change to them makes `traffic` null until re-measured.
MEASURED_TRAFFIC = {
    "S": {"bytes": 100.7e6, "sources": ("amg.hpp", "kernels.hpp"),
          "sha256": "841ed70e9cb9439da49da9f743bf7c1b7f4b6475c95831105e1ba6ffa305e34f"},
}


def sources_hash(names) -> str:
    import hashlib
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_1405_0707_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(key):
    rec = MEASURED_TRAFFIC.get(key)
    if rec is None:
        return None
    try:
        ok = sources_hash(rec["sources"]) == rec["sha256"]
    except OSError:
        ok = False
    return rec["bytes"] if ok else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the solve, copy a 256 MiB buffer 3 times (a plain copy kernel "
                         "of known size, used to scale HBM byte counters)")
    ap.add_argument("--suite", action="store_true",
                    help="also time the Toeplitz, convection-diffusion (FP64 and mixed) and "
                         "variable-coefficient (forward + adjoint) workloads; reported under "
                         "'suite'")
    ap.add_argument("--vardiff-n", type=int, default=256,
                    help="grid side of the variable-coefficient workload in --suite")
    ap.add_argument("--suite-parts", default=",".join(SUITE_PARTS),
                    help="comma-separated parts of --suite: " + ", ".join(SUITE_PARTS))
    ap.add_argument("--profile-every", type=int, default=4,
                    help="sample every N-th inner iteration with HIP events (0 = off)")
    ap.add_argument("--inner", choices=["auto", "amg", "jacobi"], default="auto",
                    help="preconditioner of the inner CG (auto = AMG at this size)")
    ap.add_argument("--amg-fp32", action="store_true",
                    help="run the AMG V-cycle in FP32 under the FP64 CG (default: FP64)")
    return ap.parse_args()


def cg_kernel_bytes(n: int, nnz: int, p: int, precond: str = "jacobi") -> dict:
    """Algorithmic HBM bytes per launch of the inner CG's three kernels
    (FP64 values, int32 indices; precond "jacobi", "amg64" or "amg32", the
    V-cycle's precision):
      A  q = K p (CSR SpMM) + partial (p, q): rowptr 4(n+1), colind and
         values 12 nnz, read p and write q 16 n p;
      B  r -= alpha q + partials: read r, q and write r 24 n p (+ dinv 8 n
         for Jacobi's (r, D^{-1} r); + 4 n p writing the FP32 copy of r);
      C  x += alpha p_old, p_new = z + beta p_old: read p_old, x and write
         p_new, x 32 n p, and z = D^{-1} r (dinv 8 n + r 8 n p) or the
         V-cycle's z (8 n p, or 4 n p in FP32)."""
    return {"A": 4 * (n + 1) + 12 * nnz + 16 * n * p,
            "B": 24 * n * p + {"jacobi": 8 * n, "amg64": 0, "amg32": 4 * n * p}[precond],
            "C": 32 * n * p + {"jacobi": 8 * n + 8 * n * p, "amg64": 8 * n * p,
                               "amg32": 4 * n * p}[precond]}


def smooth_kernel_bytes(n: int, nnz: int, p: int, degree: int, es: int = 8,
                        fused: bool = False) -> float:
    """Mean algorithmic HBM bytes per launch of the finest AMG level's
    smoothing-step kernel k_amg_step over its launches in one V-cycle (2 *
    degree; the degree post-steps alone when the level is fused, i.e. its
    pre-smoothing, residual and restriction run as one restriction of b),
    with es-byte values and vectors (8: FP64 V-cycle, 4: FP32) and int32
    indices, A = 4(n+1) + (4 + es) nnz for the CSR operator:
      first pre-step (iterate s0 D^{-1} b implicit): A + es n + 3 es np
      later pre-steps: A + es n + 5 es np
      residual: A + 3 es np (A + es n + 2 es np when degree = 1)
      post-steps: A + es n + 3 es np (+ es np for the direction d unless the
      step is the last one, + es np for reading d after the first)."""
    A = 4 * (n + 1) + (4 + es) * nnz
    launches = []
    if not fused:
        for st in range(1, degree):
            launches.append(A + es * n + (3 if st == 1 else 5) * es * n * p)
        launches.append(A + 3 * es * n * p if degree > 1 else A + es * n + 2 * es * n * p)
    for st in range(degree):
        b = A + es * n + 3 * es * n * p
        if st > 0:
            b += es * n * p
        if st + 1 < degree:
            b += es * n * p
        launches.append(b)
    return sum(launches) / len(launches)


def cpu_baseline(W):
    """Oracle PSBFOM-DR on the same workload with m = 6 (48 of the 120
    A^{-1} column applications of one solve, one cycle), DST-I inverse,
    one thread; scaled by the A^{-1} column count to one solve."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import inverses, psbfom
    m_s = 6
    N = round(W.n ** (1 / 3))
    inv = inverses.dst_laplacian_inverse(N, 3, W.t)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        _, _, info = psbfom.psbfom_dr(inv, W.B, m_s, W.k, W.tol, max_cycles=1)
        el = time.perf_counter() - t0
    full_cols = W.m * W.p
    scale = full_cols / info.op_columns
    return {"value": el * scale, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle PSBFOM-DR, same 64^3 workload, m={m_s} (1 cycle, "
                       f"{info.op_columns} of {full_cols} A^-1 column applications), "
                       f"{el:.2f} s measured, scaled x{scale:.1f} by A^-1 applications; "
                       "MGS cost grows faster than linearly, so this underestimates")}


SUITE_PARTS = ("toeplitz", "fractional", "example53", "convdiff", "vardiff")


def run_suite(dev, vardiff_n, parts=SUITE_PARTS):
    """Secondary measurements: one timed solve each (the Toeplitz one after a
    warm-up; the large ones cold, their first-call setup being negligible);
    `parts` selects among SUITE_PARTS."""
    import numpy as np
    import torch

    import workloads as wl
    from paper_1405_0707_amd import Plan

    def timed(fn, name, warm=True):
        if warm:
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            print(f"[suite] {name}: warm-up {time.perf_counter() - t0:.2f} s", file=sys.stderr,
                  flush=True)
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        print(f"[suite] {name}: {el:.2f} s", file=sys.stderr, flush=True)
        return el, out

    res = {}
    if "toeplitz" in parts:
        _suite_toeplitz(dev, timed, res)
    if "fractional" in parts:
        _suite_fractional(dev, timed, res)
    if "example53" in parts:
        _suite_example53(dev, timed, res)
    if "convdiff" in parts:
        _suite_convdiff(dev, timed, res)
    if "vardiff" in parts:
        _suite_vardiff(dev, timed, res, vardiff_n)
    return res


def _suite_toeplitz(dev, timed, res):
    import torch

    import workloads as wl
    from paper_1405_0707_amd import Plan
    # Toeplitz 2^20, p = 16, FP64
    W = wl.c3()
    pl = Plan.toeplitz(torch.from_numpy(W.col), W.t, device=dev, m=W.m, k=W.k)
    B = torch.from_numpy(W.B).to(dev)
    el, (Z, info) = timed(lambda: pl.execute(B, tol=W.tol), "toeplitz")
    res["toeplitz_2^20_p16_fp64"] = {"s": round(el, 4), "cycles": info.cycles,
                                     "err_bound": info.err_bound}
    del pl, B, Z


def _suite_fractional(dev, timed, res):
    import torch

    import workloads as wl
    from paper_1405_0707_amd import Plan
    # nonsymmetric fractional-diffusion Toeplitz 2^17, p = 2, m = 30: forward
    # and adjoint (e^{tA^T} G and grad_t), FP64
    W = wl.c6()
    pl = Plan.toeplitz(torch.from_numpy(W.col), W.t, device=dev, row0=torch.from_numpy(W.row),
                       m=W.m, k=W.k)
    B = torch.from_numpy(W.B).to(dev)
    G = torch.from_numpy(wl.gaussian_block(W.n, W.p, 106)).to(dev)
    el_f, (Z, info_f) = timed(lambda: pl.execute(B, tol=W.tol), "fractional toeplitz fwd")
    el_b, (gB, gt, info_b) = timed(lambda: pl.adjoint(G, B, tol=W.tol),
                                   "fractional toeplitz adjoint")
    res["fractional_toeplitz_2^17_p2_fp64"] = {"forward_s": round(el_f, 4),
                                               "adjoint_s": round(el_b, 4),
                                               "cycles_fwd": info_f.cycles,
                                               "cycles_adj": info_b.cycles,
                                               "err_bound": info_f.err_bound}
    del pl, B, G, Z, gB


def _suite_example53(dev, timed, res):
    import numpy as np
    import torch

    import workloads as wl
    from paper_1405_0707_amd import Plan
    # Example 5.3: one-sided fractional diffusion with a source, A = -diag(d) T,
    # u(1) from the source-term driver on [u0 | b], m = 40, FP64
    for n in (1000, 2000, 3000):
        P = wl.fractional_source(n)
        t0 = time.perf_counter()
        pl = Plan.toeplitz(torch.from_numpy(P.col), P.t, device=dev, row0=torch.from_numpy(P.row),
                           diag=torch.from_numpy(P.d), m=40)
        torch.cuda.synchronize()
        el_plan = time.perf_counter() - t0
        U0 = torch.from_numpy(P.u0).to(dev)
        S = torch.from_numpy(P.b).to(dev)
        el, (U, info) = timed(lambda: pl.execute_source(U0, S, P.gamma, tol=1e-10),
                              f"example 5.3 n={n}")
        exact_pde = np.exp(-P.t) * P.x[:, None] ** 3
        res[f"example5.3_n{n}_fp64"] = {
            "s": round(el, 4), "plan_s": round(el_plan, 4), "cycles": info.cycles,
            "err_bound": info.err_bound,
            "rel_err_vs_pde_solution": float(np.linalg.norm(U.cpu().numpy() - exact_pde)
                                             / np.linalg.norm(exact_pde))}
        del pl, U0, S, U


def _suite_convdiff(dev, timed, res):
    import torch

    import workloads as wl
    from paper_1405_0707_amd import Plan
    # convection-diffusion 128^3, p = 16: FP64 (tol 1e-10) and mixed (tol 1e-6)
    W = wl.c4()
    print("[suite] convection-diffusion 128^3 built", file=sys.stderr, flush=True)
    B = torch.from_numpy(W.B).to(dev)
    Zs = {}
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-6)):
        pl = Plan.csr(W.A.rowptr, W.A.colind, W.A.val, W.t, device=dev, m=W.m, k=W.k,
                      precision=prec)
        el, (Z, info) = timed(lambda: pl.execute(B, tol=tol, allow=(4,)), f"convdiff {prec}",
                              warm=False)
        Zs[prec] = Z
        res[f"convdiff_128^3_p16_{prec}"] = {"s": round(el, 4), "cycles": info.cycles,
                                             "inner_iters": int(info.inner_iters),
                                             "err_bound": info.err_bound}
        del pl
    res["convdiff_mixed_vs_fp64_rel_diff"] = float(torch.linalg.norm(Zs["mixed"] - Zs["fp64"])
                                                   / torch.linalg.norm(Zs["fp64"]))
    del Zs, B


def _suite_vardiff(dev, timed, res, vardiff_n):
    import torch

    import workloads as wl
    from paper_1405_0707_amd import Plan
    # variable-coefficient diffusion, forward + adjoint, mixed and FP64
    N = vardiff_n
    W = wl.c5(N=N)
    G = torch.from_numpy(wl.gaussian_block(N * N, W.p, 105)).to(dev)
    B = torch.from_numpy(W.B).to(dev)
    outs = {}
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-6)):
        pl = Plan.csr(W.A.rowptr, W.A.colind, W.A.val, W.t, device=dev, m=W.m, k=W.k,
                      precision=prec, inner_maxit=200000)
        el_f, (Z, info_f) = timed(lambda: pl.execute(B, tol=tol, allow=(4,)),
                                  f"vardiff fwd {prec}", warm=False)
        el_b, (gB, gt, info_b) = timed(lambda: pl.adjoint(G, B, tol=tol, allow=(4,)),
                                       f"vardiff adjoint {prec}", warm=False)
        outs[prec] = (Z, gB, gt)
        res[f"vardiff_{N}^2_p32_{prec}"] = {"forward_s": round(el_f, 4),
                                            "adjoint_s": round(el_b, 4),
                                            "cycles_fwd": info_f.cycles,
                                            "inner_iters_fwd": int(info_f.inner_iters)}
        del pl
    z64, g64, t64 = outs["fp64"]
    zm, gm, tm = outs["mixed"]
    res["vardiff_mixed_vs_fp64"] = {
        "Z_rel_diff": float(torch.linalg.norm(zm - z64) / torch.linalg.norm(z64)),
        "gradB_rel_diff": float(torch.linalg.norm(gm - g64) / torch.linalg.norm(g64)),
        "gradt_rel_diff": abs(tm - t64) / abs(t64)}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; --gpus must be 1 "
                          "(sharding over several GPUs is not implemented)"}))
        sys.exit(2)
    import numpy as np
    import torch

    import workloads as wl
    from paper_1405_0707_amd import Plan

    dev = "cuda:0"
    W = wl.c2()
    t0 = time.perf_counter()
    plan = Plan.csr(W.A.rowptr, W.A.colind, W.A.val, W.t, device=dev, m=W.m, k=W.k,
                    profile=max(0, args.profile_every), inner_precond=args.inner,
                    amg_fp32=1 if args.amg_fp32 else 0)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    B = torch.from_numpy(W.B).to(dev)
    Z = torch.empty_like(B)
    for _ in range(args.warmup):
        plan.execute(B, tol=W.tol, out=Z)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, info = plan.execute(B, tol=W.tol, out=Z)
        infos.append(info)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = 1000.0 * el / args.steps
    info = infos[-1]

    # accuracy against the DST-I closed form of r(tA)B (oracle, CPU)
    from oracle import inverses
    from oracle.cf import r_eval
    rB = inverses.dst_laplacian_function(64, 3, W.t, lambda lam: r_eval(np.asarray(lam)), W.B)
    Zh = Z.cpu().numpy()
    rel_err = float(np.linalg.norm(Zh - rB) / np.linalg.norm(rB))

    samples = sum(i.kern_samples for i in infos)
    roof = None
    kernels = None
    if samples:
        mean = {key: sum(getattr(i, "kern_ms_" + key.lower()) * i.kern_samples for i in infos)
                / samples for key in ("A", "B", "C")}
        precond = ("jacobi" if not info.amg_levels else ("amg32" if args.amg_fp32 else "amg64"))
        byt = cg_kernel_bytes(W.n, W.A.nnz, W.p, precond)
        names = {"A": "k_cg_a (CSR SpMM q = K p of the inner CG)",
                 "B": "k_cg_b (inner CG residual update)",
                 "C": "k_cg_c (inner CG direction and iterate update)"}
        per_iter = dict(mean)          # device time per inner iteration
        sm_launches = sum(i.kern_smooth_launches for i in infos)
        if sm_launches:
            # default degree 2 on the finest level; with more than two levels
            # the library fuses its pre-smoothing, residual and restriction
            degree = 2
            fused = info.amg_levels > 2
            mean["S"] = sum(i.kern_ms_smooth * i.kern_smooth_launches for i in infos) / sm_launches
            byt["S"] = smooth_kernel_bytes(W.n, W.A.nnz, W.p, degree, 4 if args.amg_fp32 else 8,
                                           fused)
            names["S"] = ("k_amg_step, finest level (AMG V-cycle post-smoothing steps, "
                          "CSR SpMM fused with the Chebyshev update)" if fused else
                          "k_amg_step, finest level (AMG V-cycle smoothing steps and residual, "
                          "CSR SpMM fused with the Chebyshev update)")
            per_iter["S"] = mean["S"] * sm_launches / samples
        kernels = {key: {"kernel": names[key], "mean_launch_ms": round(mean[key], 5),
                         "bytes_per_launch": int(byt[key]),
                         "achieved_GBs": round(byt[key] / (mean[key] * 1e-3) / 1e9, 1),
                         "ms_per_inner_iteration": round(per_iter[key], 5)}
                   for key in mean}
        dom = max(per_iter, key=lambda key: per_iter[key])
        ach = byt[dom] / (mean[dom] * 1e-3) / 1e9
        ol = sum(i.kern_orth_launches for i in infos)
        if ol:
            oms = sum(i.kern_ms_orth * i.kern_orth_launches for i in infos) / ol
            oby = sum(i.kern_orth_bytes * i.kern_orth_launches for i in infos) / ol
            kernels["orth"] = {
                "kernel": "k_orth_mma (block Gram-Schmidt / CholQR passes, FP64 MFMA)",
                "mean_launch_ms": round(oms, 5), "bytes_per_launch": int(oby),
                "achieved_GBs": round(oby / (oms * 1e-3) / 1e9, 1),
                "launches": ol}
        roof = {"bound": "hbm", "kernel": names[dom], "achieved": round(ach, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(dom), "bytes_per_launch": int(byt[dom]),
                "mean_launch_ms": round(mean[dom], 5),
                "samples": sm_launches if dom == "S" else samples}

    if args.copy_calibration:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    parts = tuple(x for x in args.suite_parts.split(",") if x)
    suite = run_suite(dev, args.vardiff_n, parts) if args.suite else None

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(W)

    out = {
        "metric": "e^{tA}B time per solve (FP64, 3D Laplacian 64^3, p=8)",
        "value": round(ms / 1000.0, 6), "unit": "s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 3), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "3D 7-point Laplacian 64^3 (n=262144, nnz=1810432), "
                               "||tA||_2=1e4, B n x 8 Gaussian seed 2, m=15, k=40, tol=1e-10",
                   "n": W.n, "p": W.p, "m": W.m, "k": W.k, "tol": W.tol},
        "rel_err_vs_rational_closed_form": rel_err,
        "inner_preconditioner": (f"AMG ({info.amg_levels} levels, "
                                 f"{'FP32' if args.amg_fp32 else 'FP64'} V-cycle)"
                                 if info.amg_levels else "Jacobi"),
        "cycles": info.cycles, "block_apps": info.block_apps,
        "inner_iters": int(info.inner_iters), "err_bound": info.err_bound,
        "phase_ms": {"apply": round(info.ms_apply, 2), "orth": round(info.ms_orth, 2),
                     "small": round(info.ms_small, 2), "update": round(info.ms_update, 2)},
        "plan_setup_s": round(plan_s, 3),
        "roofline": roof,
        "inner_kernels": kernels,
        "cpu_baseline": cpu,
    }
    if suite is not None:
        out["suite"] = suite
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
