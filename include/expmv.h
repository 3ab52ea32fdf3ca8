/* expmv.h -- C ABI of the MI355X library computing Z = e^{tA} B by the
 * preconditioned, restarted and shifted block FOM with deflation
 * (PSBFOM-DR; Wu, Pang, Sun, arXiv:1405.0707).
 *
 * Problem (paper, Section 1, eq. 1.1): t is a real scalar, tA is an n x n
 * large sparse negative definite matrix with ||tA|| >> 1, B is n x p with
 * 1 <= p << n.  e^{tA} is replaced by the degree-14 Caratheodory-Fejer
 * rational form omega_0 B + sum_i omega_i (tA - tau_i I)^{-1} B (Section 2,
 * eq. 2.5); its 7 conjugate-pair shifted systems are solved on one shared
 * real block Krylov basis of (tA)^{-1} (Section 4.1, eq. 4.4-4.9), restarted
 * with deflation (Algorithm 2).
 *
 * Conventions for every entry point:
 *  - Array arguments are DEVICE pointers (memory from hipMalloc or a torch
 *    CUDA tensor) unless the comment says "host".
 *  - Blocks (B, Z, G, X, Y) are n x p, row-major, contiguous: element (i, j)
 *    is at [i * p + j].  Values are FP64 at the boundary in every precision
 *    mode.
 *  - CSR matrices use int32 row pointers (n + 1 entries, rowptr[0] = 0) and
 *    int32 column indices (nnz entries), FP64 values; column indices in a row
 *    need not be sorted.
 *  - The caller owns every array it passes and keeps it alive for the call,
 *    including the device workspace `work` (work_bytes bytes, 256-byte
 *    aligned, contents ignored on entry) that every call doing device work
 *    takes; expmv_workspace_size* give the bytes a call needs, and a smaller
 *    or misaligned buffer is refused with EINVAL before any device work.  A
 *    plan copies what it needs from A at creation (the caller may free A
 *    afterwards) and owns only what its creation set up (K, its transpose,
 *    the AMG hierarchy, the Toeplitz spectra, the CF table), released by
 *    expmv_plan_destroy: the library allocates device memory at plan
 *    creation only (and in the one-shot forms, which create a plan).  Two
 *    calls must not share one workspace while both can be running.
 *  - All device work is ordered on the stream given at plan creation
 *    (NULL = the default stream).  Entry points that return host values
 *    synchronise that stream before returning.
 *  - No C++ exception crosses the ABI; a plan must not be used by two host
 *    threads at once.
 */
#ifndef EXPMV_H
#define EXPMV_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EXPMV_OK = 0,
  EXPMV_EINVAL = 1,      /* bad argument: n < 1, p < 1 or p > n, p > 32, t = 0 or not
                            finite, tol not in (0, 1), m or k out of range, NULL pointer */
  EXPMV_ENOTNEG = 2,     /* some diagonal entry of tA is >= 0: tA is not negative definite */
  EXPMV_ENOMEM = 3,      /* device or host allocation failed */
  EXPMV_ENOCONV = 4,     /* max_cycles reached; Z holds the last iterate, info is filled */
  EXPMV_EBREAKDOWN = 5,  /* a block of the Krylov basis became rank deficient without the
                            space becoming invariant; Z holds the last iterate */
  EXPMV_EHIP = 6,        /* a HIP runtime call failed */
  EXPMV_EINNER = 7       /* an inner solve for (tA)^{-1} V hit inner_maxit; Z holds the
                            iterate of the cycle where it happened */
} expmv_status;

typedef enum {
  EXPMV_FP64 = 0,         /* everything in FP64 */
  EXPMV_MIXED = 1,        /* FP32 inner solver, SpMM vectors, Krylov basis and its
                             Gram-Schmidt traffic; FP64 operator values, projections,
                             Gram/Cholesky, H, projected solves, X, combination */
  EXPMV_MIXED_INNER = 2   /* FP32 inner solver only (the dominant cost); Krylov basis
                             and everything else FP64 */
} expmv_precision;

typedef enum {
  EXPMV_STOP_PAPER = 0,  /* max_j rho_j <= tol * ||B||_F, rho_j the residual norm of
                            eq. 4.9 (Algorithm 2, Step 4) */
  EXPMV_STOP_BOUND = 1   /* sum_j |c_j| rho_j / delta_j <= tol * ||Z~||_F, delta_j the
                            distance of tau_j to (-inf, 0]: a bound on the error
                            against the rational form when tA is normal */
} expmv_stop_rule;

typedef struct {
  int m;               /* block Arnoldi steps per cycle, 2..64; a call whose basis of
                          m + 1 blocks of p columns is wider than the block
                          Gram-Schmidt takes ((m + 1) p <= 512 for p <= 32, else
                          (m + 1) p^2 doubles within 150 KB: m <= 17 at p = 32)
                          returns EXPMV_EINVAL, also from the workspace sizes   */
  int k;               /* Ritz vectors kept at a restart (multiple of p, k < m*p;
                          0 = p * floor(m / 3))                                          */
  int max_cycles;      /* restart cycles before EXPMV_ENOCONV                           */
  int precision;       /* expmv_precision                                                */
  int stop_rule;       /* expmv_stop_rule                                                */
  double inner_tol;    /* relative residual of each inner solve (0 = 1e-12 in FP64,
                          1e-6 in the FP32 inner solver of the mixed form)               */
  int inner_maxit;     /* iteration cap of each inner solve                             */
  int symmetric;       /* 1: A symmetric (CG inner solver, symmetric Ritz step),
                          0: general (BiCGStab, general Ritz step), -1: detect          */
  int preconditioned;  /* 1: Algorithm 2 (Krylov space of (tA)^{-1}), 0: Algorithm 1
                          (Krylov space of tA, no inner solve)                            */
  int profile;         /* 0: off; N > 0: time every N-th inner-solver iteration's
                          kernels with HIP events (results in expmv_info.kern_*)          */
  int inner_refine;    /* mixed forms: rounds of FP64 iterative refinement of each FP32
                          inner solve (FP64 residual with the exact operator, FP32
                          correction solve); -1 = 1 for nonsymmetric A, 0 otherwise      */
  int inner_precond;   /* preconditioner of the CSR inner solver (the solve that applies
                          (tA)^{-1}, Section 4.1): 0 Jacobi (diagonal scaling),
                          1 smoothed-aggregation AMG V-cycle (CG for symmetric A,
                          BiCGStab for general A with a second hierarchy for A^T; A
                          with n <= 500 has no coarse level and keeps Jacobi),
                          -1 auto = AMG for n >= 4096, else Jacobi                       */
  int amg_degree;      /* Chebyshev smoothing steps before and after each coarse
                          correction (1..4; 0 = 2 for symmetric A, 1 otherwise)          */
  int inner_relax;     /* c in 0..10, relaxed inner solves (CSR plans, Algorithm 2):
                          the inner tolerance of block j is inner_tol * min(cap,
                          ||B||_F / rho_{j-1}), rho_{j-1} the largest residual estimate
                          (eq. 4.9) over the shifts after block j-1, cap = 10^c (at
                          most 10^2 in the mixed forms); the estimates cost one
                          projected solve per block.  0: fixed inner tolerance        */
  int amg_fp32;        /* FP64 form, symmetric A with the AMG-preconditioned CG: 1 runs
                          the V-cycle in FP32 (FP32 operator values and vectors, FP64
                          sums); the CG, its SpMM, its recurrences and its stopping
                          test stay FP64, so the result's accuracy is unchanged and
                          only the iteration count can move.  0 (default): FP64
                          V-cycle.  The mixed forms always use FP32.                  */
  int amg_coarse_degree; /* Chebyshev smoothing steps on the levels below the finest
                          (1..4; 0 = one less than the finest level's, at least 1).
                          Every level uses one polynomial before and after its coarse
                          correction, so the V-cycle stays symmetric.                 */
  int restart_refine;  /* after every cycle the true residuals R_j = B - (tA - tau_j I) X_j
                          are recomputed in FP64 from X_j (reported in expmv_info).
                          1: the next cycle's right-hand sides are their coordinates
                          S_j = V_{d+1}^T R_j on the block after the basis (refinement
                          of the collinear residuals of eq. 4.8); 0 (default): the
                          coordinates tau_j H_{d+1,d} E^T Z_j of eq. 4.8 themselves  */
} expmv_opts;

/* Kernel classes timed when opts.profile = N > 0: the launches of every N-th
 * iteration of each inner solve and every orthogonalisation pass get HIP
 * start/stop events on the plan's stream (launches that return at once
 * because their solve has finished are not counted).  Index into
 * expmv_info.kern_launches / kern_ms / kern_bytes. */
typedef enum {
  EXPMV_KT_CG_SPMM = 0,    /* inner CG: q = K p and the (p, q) partials (k_cg_a)           */
  EXPMV_KT_CG_RESID = 1,   /* inner CG: r -= alpha q (k_cg_b)                              */
  EXPMV_KT_CG_DIR = 2,     /* inner CG: x, p updates (k_cg_c)                              */
  EXPMV_KT_BCG_SPMM1 = 3,  /* inner BiCGStab: v = K (M^{-1} p) (k_bcg_s)                   */
  EXPMV_KT_BCG_SPMM2 = 4,  /* inner BiCGStab: t = K (M^{-1} s) (k_bcg_s)                   */
  EXPMV_KT_BCG_U1 = 5,     /* inner BiCGStab: p = r + beta (p - omega v) (k_bcg_u1)        */
  EXPMV_KT_BCG_U2 = 6,     /* inner BiCGStab: s = r - alpha v (k_bcg_u2)                   */
  EXPMV_KT_BCG_U3 = 7,     /* inner BiCGStab: x, r updates and partials (k_bcg_u3)         */
  EXPMV_KT_AMG_SMOOTH = 8, /* AMG finest level: smoothing steps (k_amg_step)               */
  EXPMV_KT_AMG_RESTRICT = 9,  /* AMG finest level: restriction (k_amg_restrict / dense)    */
  EXPMV_KT_AMG_PROLONG = 10,  /* AMG finest level: prolongation (+ smoothing step)
                                 (k_amg_affine_pair / k_amg_prolong)                      */
  EXPMV_KT_AMG_COARSE = 11,   /* every launch of the AMG levels below the finest          */
  EXPMV_KT_ORTH = 12,         /* block Gram-Schmidt / CholQR passes (k_orth_mma, k_orth)   */
  EXPMV_KT_COUNT = 16
} expmv_kernel_class;

typedef struct {                  /* host struct, filled by expmv_execute */
  int cycles;                     /* restart cycles run                               */
  int block_apps;                 /* operator applications to an n x p block          */
  long long inner_iters;          /* inner solver iterations, summed over blocks      */
  int inner_maxit_hit;            /* inner solves that stopped at inner_maxit         */
  double est[7];                  /* rho_j of the last cycle (eq. 4.9)                */
  double true_res[7];             /* ||R_j||_F, R_j = B - (tA - tau_j I) X_j in FP64,
                                     after the last cycle                             */
  double err_bound;               /* sum_j |c_j| rho_j / delta_j / ||Z~||_F           */
  double bnorm, znorm;            /* ||B||_F, ||Z~||_F                                 */
  double ms_total, ms_apply, ms_orth, ms_small, ms_update;  /* host wall times      */
  int breakdown;                  /* 1 when the Krylov space became invariant          */
  int amg_levels;                 /* levels of the AMG hierarchy of the inner solver
                                     (0: Jacobi preconditioning)                      */
  int kern_launches[EXPMV_KT_COUNT];  /* timed launches of each kernel class
                                         (expmv_kernel_class; opts.profile > 0)      */
  double kern_ms[EXPMV_KT_COUNT];     /* their mean device time, ms                  */
  double kern_bytes[EXPMV_KT_COUNT];  /* their mean algorithmic HBM bytes per launch:
                                         operands each read or written once (CSR:
                                         4 (rows + 1) + 12 nnz), 8 bytes per FP64
                                         and 4 per FP32 value                        */
  double noncollinear[7];         /* ||R_j - V_{d+1} V_{d+1}^T R_j||_F after the last
                                     cycle: the part of the true residual outside the
                                     block the restart carries (0 in exact arithmetic,
                                     Section 3)                                       */
  double true_bound;              /* sum_j |c_j| ||R_j||_F / delta_j / ||Z~||_F        */
  double noncollinear_bound;      /* the same sum over the remainders                 */
  int refined_restarts;           /* restarts whose right-hand sides were refined     */
} expmv_info;

typedef struct expmv_plan_s* expmv_plan;

/* Fill *o with the defaults: m = 10, k = 0 (auto), max_cycles = 50, FP64,
 * EXPMV_STOP_BOUND, inner_tol = 0 (auto), inner_maxit = 50000, symmetric = -1,
 * preconditioned = 1, profile = 0, inner_refine = -1, inner_precond = -1,
 * amg_degree = 0, inner_relax = 8, amg_fp32 = 0, amg_coarse_degree = 0,
 * restart_refine = 0.  o is a host pointer. */
expmv_status expmv_default_opts(expmv_opts* o);

/* Plan for Z = e^{tA} B with A in CSR (device arrays, see conventions).
 * The plan stores K = -tA (FP64 values in both forms), the Jacobi scaling
 * 1/diag(K), the transpose of K when A is not symmetric, the CF table, and,
 * with the AMG inner preconditioner, the hierarchy built on the host from K
 * (levels, prolongators, Galerkin operators, dense inverse of the coarsest
 * operator).  opts may be NULL (defaults).  *out receives the plan.
 * Errors: EINVAL (also: inner_precond = 1 and an AMG hierarchy that cannot
 * be built), ENOTNEG (a diagonal entry of tA >= 0, or
 * missing), ENOMEM, EHIP. */
expmv_status expmv_plan_csr(int64_t n, int64_t nnz, const int32_t* rowptr,
                            const int32_t* colind, const double* val, double t,
                            const expmv_opts* opts, hipStream_t stream, expmv_plan* out);

/* Plan for A = -T with T symmetric positive definite Toeplitz given by its
 * first column col0 (device, n values), so tA = -t T with t > 0 (Section 5,
 * Example 5.4 setting).  Products with T use a length-2n circulant embedding
 * and FFTs; (tA)^{-1} uses the Gohberg-Semencul formula (Section 4.1) with
 * x = T^{-1} e_1 solved once at plan creation.  Errors as expmv_plan_csr. */
expmv_status expmv_plan_toeplitz(int64_t n, const double* col0, double t,
                                 const expmv_opts* opts, hipStream_t stream, expmv_plan* out);

/* Plan for A = -diag(d) T with T a general (nonsymmetric) Toeplitz matrix
 * given by its first column col0 and first row row0 (device, n values each;
 * row0[0] is ignored, row0 = NULL means T symmetric) and d = diag (device, n
 * positive values; NULL means d = 1), tA = -t diag(d) T with t > 0.  T's
 * symmetric part should be positive definite: the space-fractional diffusion
 * matrices of Section 5 (Example 5.4: d = 1; Example 5.3: a variable
 * diffusion coefficient d(x) times a one-sided Gruenwald matrix).  Products
 * with T and T^T use length-2n circulant embeddings, scaled by d on the
 * output (input, transposed); (tA)^{-1} = -(1/t) T^{-1} diag(1/d) and its
 * transpose use the Gohberg-Semencul formula with x = T^{-1} e_1 and
 * y = T^{-1} e_n, solved once at plan creation (CG for symmetric T, else
 * BiCGStab with the FFT product, preconditioned by T's Strang circulant when
 * n is a power of two).  The plan copies col0, row0 and diag.  Errors as
 * expmv_plan_csr (ENOTNEG also for a d_i <= 0); ENOCONV if those set-up
 * solves do not reach a relative residual of 1e-10. */
expmv_status expmv_plan_toeplitz_general(int64_t n, const double* col0, const double* row0,
                                         const double* diag, double t, const expmv_opts* opts,
                                         hipStream_t stream, expmv_plan* out);

/* *bytes (host) = the device workspace expmv_execute, expmv_adjoint,
 * expmv_grad_t and the expmv_apply_* calls need for a block of p columns
 * (1 <= p <= 32, p <= n): the Krylov basis (two copies of (m+1) n p values),
 * the inner solver's and the V-cycle's vectors, X (n x 14p FP64), the true
 * residuals (n x 14p FP64), the projected systems and the reductions (and,
 * for Toeplitz plans, the FFT arrays).  Errors: EINVAL. */
expmv_status expmv_workspace_size(expmv_plan plan, int64_t p, size_t* bytes);
/* The same for expmv_execute_times with nt times (1 <= nt <= 32). */
expmv_status expmv_workspace_size_times(expmv_plan plan, int64_t p, int nt, size_t* bytes);
/* The same for expmv_execute_source with n x p blocks U0 and S (2p <= 32). */
expmv_status expmv_workspace_size_source(expmv_plan plan, int64_t p, size_t* bytes);

/* Z = e^{tA} B (transpose = 0) or Z = e^{tA^T} B (transpose = 1), p = block
 * width (1 <= p <= 32, p <= n), tol = stopping tolerance of opts.stop_rule,
 * work = device workspace of work_bytes >= expmv_workspace_size(plan, p).
 * B and Z are device n x p blocks and may not overlap (nor the workspace).
 * info (host) may be NULL.  Returns OK, EINVAL (also: workspace missing, too
 * small or not 256-byte aligned), ENOCONV, EBREAKDOWN (also: a singular
 * projected system or a non-finite estimate), EINNER, ENOMEM or EHIP; after
 * ENOCONV, EBREAKDOWN and EINNER Z holds the last iterate. */
expmv_status expmv_execute(expmv_plan plan, int transpose, const double* B, int64_t p,
                           double tol, void* work, size_t work_bytes, double* Z,
                           expmv_info* info);

/* expmv_execute for callers that cannot allocate device memory or bring a
 * workspace (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc).  It allocates nothing: its workspace is a static
 * device array of EXPMV_STATIC_WORKSPACE_BYTES, one copy on every GPU the
 * library runs on, held until the process ends.  A call whose
 * expmv_workspace_size(plan, p) exceeds that size returns EINVAL (with a
 * detail); so does a call made while another device than the plan's is
 * current.  All such calls on one GPU share the array and it keeps the last
 * call's contents (every array the method needs zeroed is cleared by the
 * call itself): calls from one process are serialised by a host lock, and
 * each call has finished its device work when it returns, so calls must not
 * overlap in any other way (e.g. the same array used from device work that
 * is still queued).  Arguments, results and statuses as expmv_execute. */
#define EXPMV_STATIC_WORKSPACE_BYTES ((size_t)32 << 20)
expmv_status expmv_execute_noalloc(expmv_plan plan, int transpose, const double* B, int64_t p,
                                   double tol, double* Z, expmv_info* info);

/* Several times at once: Z_q = e^{t_q A} B for q = 0..nt-1 (times: host
 * array, 1 <= nt <= 32; Z: device, nt consecutive n x p blocks, block q at
 * Z + q n p).  A is the plan's matrix (the plan holds t_0 A for its own t_0);
 * every t_q must have the sign of t_0 so that t_q A is negative definite
 * (ENOTNEG otherwise).  Since t_q A = s_q (t_0 A) with s_q = t_q / t_0 and
 * r(s M) B = omega_0 B + Re sum_j (c_j / s)(M - (tau_j / s) I)^{-1} B, all 7 nt
 * shifted systems are solved on one Krylov basis of (t_0 A)^{-1}: the inner
 * solves, Gram-Schmidt passes and restarts are shared, and the stopping rule
 * must hold for every time.  info as expmv_execute (err_bound: the largest
 * over the times; true_res[j]: the largest over the times; znorm, est: time
 * 0).  Statuses as expmv_execute. */
expmv_status expmv_execute_times(expmv_plan plan, int transpose, const double* times, int nt,
                                 const double* B, int64_t p, double tol, void* work,
                                 size_t work_bytes, double* Z, expmv_info* info);

/* Linear ODE with an exponential source (Section 5, Example 5.3, gamma = -1):
 * U = the solution at time t (the plan's t) of u' = A u + e^{gamma s} S,
 * u(0) = U0, with both exponentials of its variation-of-constants form
 * e^{tA}(U0 + W) - e^{gamma t} W, W = (A - gamma I)^{-1} S, taken in the CF
 * form r of eq. 2.5:
 *   U = r(tA) U0 + (r(tA) - r(gamma t) I) (A - gamma I)^{-1} S
 *     = omega_0 U0 + Re sum_j c_j (tA - tau_j I)^{-1} (U0 + t / (tau_j - gamma t) S)
 * (partial fractions of r), so no solve with A - gamma I is made and
 * A - gamma I need not be invertible.  One run of the method on the joined
 * n x 2p block [U0 | S] (the 7 shifted systems share one Krylov basis),
 * which must have full column rank unless U0 or S is entirely zero (S = 0:
 * the plain e^{tA} U0; U0 = 0: one run on S alone; otherwise rank loss ends
 * in EBREAKDOWN); opts.k counts columns of the block the method runs on.  transpose = 1 uses A^T.  U0, S, U:
 * device n x p blocks, 1 <= p <= 16, 2p <= n; U may not overlap U0 or S.
 * tol bounds the estimated error of U relative to ||U||_F (opts.stop_rule
 * as in expmv_execute, the paper rule on the joined block).  info as
 * expmv_execute (znorm = ||U||_F; est and true_res refer to the joined
 * block).  EINVAL for a non-finite gamma, U0 = S = 0 or bad sizes; other
 * statuses as expmv_execute. */
expmv_status expmv_execute_source(expmv_plan plan, int transpose, const double* U0,
                                  const double* S, int64_t p, double gamma, double tol,
                                  void* work, size_t work_bytes, double* U, expmv_info* info);

/* *out (host) = <G, A Z> = sum_ij G_ij (A Z)_ij: the derivative of
 * <G, e^{tA}B> with respect to t when Z = e^{tA}B (d/dt e^{tA}B = A e^{tA}B).
 * G, Z device n x p; work as expmv_execute. */
expmv_status expmv_grad_t(expmv_plan plan, const double* G, const double* Z, int64_t p,
                          void* work, size_t work_bytes, double* out);

/* Adjoint of Z = e^{tA}B for a loss L with dL/dZ = G: one solve with A^T
 * gives gradB = e^{tA^T} G (n x p, device), and *grad_t (host) =
 * <G, A r(tA) B> evaluated, with M = tA and Y_j = (M^T - tau_j I)^{-1} G the
 * shifted solutions of that same solve, as
 *   (1/t) [omega_0 <G, M B> + Re(sum_j c_j) <G, B> + Re sum_j c_j tau_j <Y_j, B>]
 * (partial fractions of x r(x)), which applies no operator to a computed
 * iterate.  tol and info as in expmv_execute; returns its statuses. */
expmv_status expmv_adjoint(expmv_plan plan, const double* G, const double* B, int64_t p,
                           double tol, void* work, size_t work_bytes, double* gradB,
                           double* grad_t, expmv_info* info);

/* Y = tA X (transpose = 0) or (tA)^T X (transpose = 1), X, Y device n x p;
 * work as expmv_execute. */
expmv_status expmv_apply_operator(expmv_plan plan, int transpose, const double* X,
                                  int64_t p, void* work, size_t work_bytes, double* Y);

/* Y ~= (tA)^{-1} X by the plan's preconditioner application (inner solve to
 * relative residual inner_tol, or Gohberg-Semencul for Toeplitz plans);
 * *iters (host, may be NULL) receives the largest inner iteration count. */
expmv_status expmv_apply_inverse(expmv_plan plan, int transpose, const double* X,
                                 int64_t p, void* work, size_t work_bytes, double* Y,
                                 long long* iters);

/* Y = P X, one application of the CSR inner solver's preconditioner P for
 * K = -tA (or K^T when transpose = 1): P = D^{-1} (Jacobi) or one AMG
 * V-cycle, so that Y ~= K^{-1} X = -(tA)^{-1} X.  X, Y device n x p
 * (1 <= p <= 32), not overlapping.  Errors: EINVAL (Toeplitz plan, bad
 * arguments), EHIP. */
expmv_status expmv_apply_preconditioner(expmv_plan plan, int transpose, const double* X,
                                        int64_t p, void* work, size_t work_bytes, double* Y);

/* Copy the library's CF table to host arrays of 7 entries (poles with
 * Im tau > 0, c_j = 2 omega_j) and *omega0.  Any pointer may be NULL. */
expmv_status expmv_cf_table(double* tau_re, double* tau_im, double* c_re, double* c_im,
                            double* omega0);

/* Host eigensolvers of the restart step (Algorithm 2, Step 5), exported so
 * they can be checked without a GPU.  A is a host n x n row-major matrix.
 * sym: eigenvalues w (n) and orthonormal eigenvectors in the columns of Q
 * (n x n row-major) of (A + A^T)/2.  general: eigenvalues wr + i wi and unit
 * eigenvectors Vr + i Vi (columns), complex ones in exact conjugate pairs.
 * Return EINVAL on bad arguments, ENOCONV if the QR iteration does not
 * converge or the input or result is not finite. */
expmv_status expmv_host_eig_sym(int n, const double* A, double* w, double* Q);
expmv_status expmv_host_eig_general(int n, const double* A, double* wr, double* wi, double* Vr,
                                    double* Vi);

/* Host-side AMG hierarchy of a CSR matrix (all pointers host), the same
 * construction a plan uses for its inner preconditioner, exported so it can
 * be inspected without a GPU.  A is n x n CSR (int32 rowptr/colind, FP64
 * values) with a positive diagonal; symmetric selects the eigenvalue
 * estimate (Lanczos or power iteration); theta is the strength threshold of
 * the finest level (halved per level); max_coarse the coarsest size.
 * Errors: EINVAL (bad arguments, non-positive diagonal, coarsest operator
 * singular or larger than 4096), ENOMEM. */
typedef struct expmv_amg_s* expmv_amg;
expmv_status expmv_host_amg_build(int64_t n, const int32_t* rowptr, const int32_t* colind,
                                  const double* val, int symmetric, double theta,
                                  int max_coarse, expmv_amg* out);
/* Number of levels (>= 1; the last is the coarsest). */
int expmv_host_amg_levels(expmv_amg h);
/* Level `level`: dims[0] = n_l, dims[1] = nnz(A_l), dims[2] = n_{l+1} (0 on
 * the coarsest), dims[3] = nnz(P_l); *lmax = the smoother's upper estimate
 * of lambda_max(D_l^{-1} A_l).  Any array pointer may be NULL; otherwise it
 * receives A_l (a_rowptr n_l + 1, a_colind and a_val nnz(A_l)), the
 * prolongator P_l (n_l x n_{l+1}: p_rowptr n_l + 1, p_colind and p_val
 * nnz(P_l)) and the aggregate of each unknown (agg, n_l). */
expmv_status expmv_host_amg_level(expmv_amg h, int level, int64_t* dims, double* lmax,
                                  int32_t* a_rowptr, int32_t* a_colind, double* a_val,
                                  int32_t* p_rowptr, int32_t* p_colind, double* p_val,
                                  int32_t* agg);
/* Dense row-major inverse of the coarsest operator (n_c x n_c doubles). */
expmv_status expmv_host_amg_coarse_inverse(expmv_amg h, double* inv);
/* The fused transfer operators the device V-cycle uses on level `level`
 * (not the coarsest), host CSR.  which = 0: the restriction of the residual
 * of the pre-smoothed iterate x1 = D^{-1}(alpha b - beta A D^{-1} b),
 * Rf = R (I - A D^{-1} (alpha I - beta A D^{-1})), n_{l+1} x n_l (one smoothing
 * step from zero: alpha = s0, beta = 0); which = 1: the prolongation followed
 * by one smoothing step x += alpha D^{-1}(b - A x), Pf = (I - alpha D^{-1} A) P,
 * n_l x n_{l+1} (beta ignored).  dims receives rows, columns, nnz; the
 * arrays (rowptr rows + 1, colind and val nnz; NULL: sizes only) receive the
 * matrix.  Errors: EINVAL (no such level, the coarsest, which not 0 or 1,
 * alpha or beta not finite), ENOMEM. */
expmv_status expmv_host_amg_fused(expmv_amg h, int level, int which, double alpha, double beta,
                                  int64_t* dims, int32_t* rowptr, int32_t* colind, double* val);
void expmv_host_amg_destroy(expmv_amg h);

void expmv_plan_destroy(expmv_plan plan);

const char* expmv_status_string(expmv_status s);

/* Detail of the last EHIP / ENOMEM returned on this host thread (the failing
 * runtime call's source line and message), "" if none.  Host string owned by
 * the library. */
const char* expmv_last_error_detail(void);

/* One-shot forms of the problem statement: plan, execute, destroy, with the
 * default options and a given tol. */
expmv_status expmv_block_csr(int64_t n, int64_t nnz, const int32_t* rowptr,
                             const int32_t* colind, const double* val, const double* B,
                             int64_t p, double t, double tol, double* Z, hipStream_t stream);
expmv_status expmv_block_toeplitz(int64_t n, const double* col0, const double* B, int64_t p,
                                  double t, double tol, double* Z, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* EXPMV_H */
