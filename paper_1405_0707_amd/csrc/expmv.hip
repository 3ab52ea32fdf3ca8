// expmv: Z = e^{tA} B by the preconditioned, restarted and shifted block FOM
// with deflation (PSBFOM-DR, Wu-Pang-Sun, Algorithm 2), on one MI355X.
//
// Host driver: plan creation, the restart-cycle loop and the C ABI.  Every
// n-sized operation runs in the kernels of kernels.hpp / kernels_dense.hpp /
// toeplitz.hpp; the host only moves the small projected matrices (H, the
// pole residuals, the restart rotation) and decides convergence.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <future>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <type_traits>
#include <vector>

#include "amg.hpp"
#include "amg_host.hpp"
#include "eig_host.hpp"
#include "expmv.h"
#include "kernels.hpp"
#include "kernels_dense.hpp"
#include "orth_mfma.hpp"
#include "residual.hpp"
#include "toeplitz.hpp"

#include "cf_nu14.inc"

namespace expmv {

struct HipError {
  hipError_t err;
  int line;
};
struct StatusError {
  expmv_status st;
};

// Detail of the last EHIP / ENOMEM / EINVAL from a check inside a call.
thread_local char g_error_detail[256] = "";

#define HIPCHK(call)                                             \
  do {                                                           \
    hipError_t e_ = (call);                                      \
    if (e_ != hipSuccess) throw ::expmv::HipError{e_, __LINE__}; \
  } while (0)

template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void alloc(size_t count) {
    if (count <= n && p) return;
    release();
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&p), count * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      throw StatusError{EXPMV_ENOMEM};
    }
    n = count;
  }
};

static int pow2_lanes(int p) {
  int pp = 1;
  while (pp < p) pp <<= 1;
  return pp;
}

// Work arrays of one call, carved out of the caller's workspace buffer
// (expmv_workspace_size gives its size).  The basis, W and the inner
// solver's vectors hold the working type of the plan (FP64, or FP32 in the
// mixed form); everything else is FP64.
struct Workspace {
  char* V[2] = {};              // basis panels, (m+1) * n * p elements each
  char *W = nullptr, *Wt = nullptr;          // n x p (basis type)
  char *Win = nullptr, *Wout = nullptr;      // n x p (inner-solver type, when it differs)
  char *Rin = nullptr, *Din = nullptr;       // n x p (inner-solver type, refinement)
  char *kr = nullptr, *kpa = nullptr, *kpb = nullptr, *kq = nullptr, *kv = nullptr,
       *ks = nullptr, *kt = nullptr, *krh = nullptr;   // inner-solver vectors, n x p
  char *kz = nullptr, *kph = nullptr, *ksh = nullptr;  // AMG-preconditioned vectors
  float *kr32 = nullptr, *kz32 = nullptr;   // FP32 V-cycle input / output (n x p)
  double* X = nullptr;                      // n x 14p nt
  double* partial = nullptr;                // reductions of the dense kernels
  double *hcoef = nullptr, *gram = nullptr, *R1 = nullptr, *R2 = nullptr, *Rinv = nullptr,
         *w0 = nullptr;                     // small orth buffers
  double* H = nullptr;                      // ldh x ldh
  double* Rhat = nullptr;                   // p x p
  cplx *G = nullptr, *Zs = nullptr, *Ascr = nullptr, *S = nullptr;
  double *Cr = nullptr, *Crot = nullptr, *rho = nullptr;
  int *flags = nullptr, *singular = nullptr;
  CgState* cgst = nullptr;
  BcgState* bcgst = nullptr;
  double *part_rr = nullptr, *part_sig = nullptr;   // inner-solver partials
  double *taus = nullptr, *coefs = nullptr;         // poles and coefficients of all shifts
  cplx* S2 = nullptr;
  int* singular2 = nullptr;
  KrylovCtl* ctl = nullptr;
  double* Rres = nullptr;               // n x 14p: true residuals of one time block (also
                                        // K X of a Toeplitz plan, K B of the adjoint)
  double* projC = nullptr;              // p x 14p coordinates V_last^T R
  double* rpart = nullptr;              // residual and remainder partial norms
  cplx* Sref = nullptr;                 // restart coordinates when not refining
  cplx* fb[4] = {};                     // Toeplitz FFT work arrays, L x fq complex
  int fq = 0;
  double* srcB = nullptr;               // n x 2p joined block [U0 | S] (source-term solves)
};

// Hands out 256-byte aligned pieces of one buffer in a fixed order; with
// base == nullptr it only adds up the sizes.
struct Carver {
  char* base = nullptr;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* ptr = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += std::max<size_t>(count, 1) * sizeof(T);
    return ptr;
  }
};

constexpr int kAmgMaxDeg = 4;
// Chebyshev interval [lmax / ratio, lmax] of two or more smoothing steps:
// the 1024^2 variable-coefficient solve (AMG-CG, degree 2) needed 244 inner
// iterations at ratio 6, 8 and 10, 253 at 20 and 256 at 30
constexpr double kAmgEigRatio = 10.0;
// one smoothing step (damped Jacobi, weight 2 / (lmax (1 + 1/ratio))): with
// the nonsymmetric prolongator weight 1.6 / lmax the 128^3
// convection-diffusion solve needed 964 BiCGStab iterations at ratio 6, 942
// at 8, 926 at 11 (weight 1.83 / lmax), 979 at 14 and 1,043 at 20
constexpr double kAmgJacobiRatio = 11.0;
constexpr int64_t kAmgFuseGrowth = 16;  // fused operators: at most this many times nnz(A) + nnz(P)
constexpr int kKtSlots = 4096;   // timed launches between two collections (opts.profile > 0)

// Kernel timing (opts.profile > 0): event pairs from a pool, each with the
// launch's kernel class, the inner iteration it belongs to (-1: none) and
// its algorithmic bytes; summed per class by kt_collect.
struct KernelTimer {
  std::vector<hipEvent_t> ev;   // 2 per slot
  std::vector<int> cls, iter;
  std::vector<double> bytes;
  int used = 0;
  int cur_iter = -1;            // inner iteration being launched, -1 outside inner solves
  bool sampling = false;        // that iteration is timed
  double ms[EXPMV_KT_COUNT] = {}, by[EXPMV_KT_COUNT] = {};
  int cnt[EXPMV_KT_COUNT] = {};
};

// One level of the AMG hierarchy on the device.  Level 0 borrows the plan's
// CSR operator and Jacobi scaling; coarser levels own their Galerkin
// operators.  P/R connect the level to the next one.  Vectors (n_l x p,
// inner-solver type): b (right-hand side, levels >= 1), u/v (iterates),
// d (Chebyshev direction), r (residual), o (the level's output, levels >= 1).
struct AmgDevLevel {
  int64_t n = 0;
  const int32_t* arp = nullptr;
  const int32_t* aci = nullptr;
  const double* av = nullptr;
  const double* dinv64 = nullptr;
  const float* dinv32 = nullptr;
  DevBuf<int32_t> Arp, Aci, Prp, Pci, Rrp, Rci;
  DevBuf<double> Av, Pv, Rv, dinv;
  DevBuf<float> dinvf;
  DevBuf<float> Av32, Pv32, Rv32;   // FP32 copies of the values (FP32 V-cycles)
  double cd[kAmgMaxDeg] = {}, ad[kAmgMaxDeg] = {};   // Chebyshev step coefficients
  int degree = 2;                                    // smoothing steps before / after
  double avg_a = 0.0, avg_p = 0.0, avg_r = 0.0;      // mean nonzeros per row of A, P, R
  int64_t nnz_a = 0, nnz_p = 0, nnz_r = 0, nnz_rf = 0, nnz_pf = 0;   // (timing byte counts)
  // A level below the finest smoothed by one step (degree 1, x0 = s0 D^{-1} b):
  // the pre-smoothing step, the residual and the restriction are one operator
  // Rf = R (I - s0 A D^{-1}), and the prolongation and the post-smoothing step
  // give out = s0 D^{-1} (2 b - s0 A D^{-1} b) + Pf xc with
  // Pf = (I - s0 D^{-1} A) P: two launches per level instead of four, the
  // same linear map up to rounding.
  // The finest level at degree 2 (fused likewise): its pre-smoothed iterate
  // x1 = D^{-1} (alpha b - beta A D^{-1} b) is recomputed where the
  // prolongation needs it, and the two pre-smoothing steps, the residual and
  // the restriction are one operator Rf = R (I - A D^{-1} (alpha I - beta A D^{-1})).
  double alpha = 0.0, beta = 0.0;
  bool fused = false;
  DevBuf<int32_t> Rfrp, Rfci, Pfrp, Pfci;
  DevBuf<double> Rfv, Pfv;
  // values of A D^{-1} (a_ij dinv[j], FP64) for the FP64 prolongation-plus-
  // smoothing pass of a fused degree-1 level: its sum over A needs no
  // gather of dinv
  DevBuf<double> ADv;
  DevBuf<float> Rfv32, Pfv32;
  double avg_rf = 0.0, avg_pf = 0.0;
  char *vb = nullptr, *vu = nullptr, *vv = nullptr, *vd = nullptr, *vr = nullptr,
       *vo = nullptr;   // carved from the call's workspace
};

// Sub-lanes per row for a matrix with `avg` nonzeros per row: the largest
// power of two with at least 4 nonzeros per sub-lane, PP * G <= 64.
inline int row_split(double avg, int PP) {
  int G = 1;
  while (2 * G * PP <= 64 && avg >= 4.0 * 2 * G) G *= 2;
  return G;
}

struct AmgDev {
  std::vector<std::unique_ptr<AmgDevLevel>> lv;
  DevBuf<double> cinv;   // dense inverse of the coarsest operator
  // Inv R of the level above the coarsest (restriction and coarsest solve as
  // one dense product), when it is small enough (kAmgFusedMax entries); on a
  // fused level (AmgDevLevel::fused) Inv Rf, which also takes in the level's
  // pre-smoothing step and residual
  DevBuf<double> cinvR;
  int degree = 2;
};

}  // namespace expmv

using namespace expmv;

struct expmv_plan_s {
  int kind = 0;                 // 0 CSR, 1 Toeplitz
  int64_t n = 0, nnz = 0;
  double t = 0.0;
  int device = 0;               // the device current when the plan was made
  expmv_opts opts{};
  hipStream_t stream = nullptr;
  bool symmetric = true;
  // K = -tA in CSR (FP64) and its transpose (nonsymmetric only)
  DevBuf<int32_t> rowptr, colind, rowptrT, colindT;
  DevBuf<double> val, valT, dinv, dinvT;
  DevBuf<float> dinvf, dinvTf;   // FP32 Jacobi scaling (mixed forms)
  bool mixed = false;            // FP32 inner solver
  bool basis32 = false;          // FP32 Krylov basis (EXPMV_MIXED)
  // Toeplitz operator: L = 2n circulant embedding; spectra of the embedded
  // first column (chat), of x = T^{-1} e_1 and of Z x~ (Gohberg-Semencul)
  int64_t L = 0;
  double x0 = 0.0;
  std::vector<int> radices;
  DevBuf<cplx> chat, xhat, yhat;
  // nonsymmetric T: spectrum of the embedding of T^T, and of the generators
  // J y, Z y (y = T^{-1} e_n) beside x and Z J x (xhat, yhat)
  DevBuf<cplx> chatT, jyhat, zyhat;
  // length-n Gohberg-Semencul form (n with no prime factor above 5): the
  // radices of n and the spectra F x, F (Z_1 y), F D (J y), F D (Z_{-1} J x)
  bool gsf_n = false;
  std::vector<int> radices_n;
  DevBuf<cplx> ncx, ncz, nsj, nsz;
  bool tsym = true;              // T symmetric (A = -diag(d) T symmetric needs d = 1 too)
  DevBuf<double> tdiag, tdinv;   // d and 1/d of A = -diag(d) T (empty: d = 1)
  DevBuf<cplx> setup_fb[3];      // L x 1 work arrays of the plan's own set-up transforms
  // CF table on the device
  DevBuf<double> tau_re, tau_im, c_re, c_im;
  Workspace ws;
  int* host_flags = nullptr;    // pinned, 2 slots x 4 ints
  hipEvent_t ev[2]{};
  int ldh = 0;
  int last_inner_iters = 0;       // iterations of the previous inner solve
  double relax_scale = 1.0;       // inner tolerance factor (opts.inner_relax)
  KernelTimer kt;                 // opts.profile > 0
  // AMG preconditioner of the CSR inner solver: hierarchy of K and, for a
  // nonsymmetric K, of K^T (transposed solves)
  std::unique_ptr<AmgDev> amg, amgT;
};

namespace expmv {
namespace {

constexpr int kCgGrid = 512;   // workgroups of the inner-solver kernels
constexpr int kOrthGrid = 768; // most workgroups (partial sums) of an orthogonalisation pass
constexpr int kCUs = 256;
constexpr size_t kLdsPerCU = 160 * 1024;
constexpr int64_t kAmgFusedMax = int64_t(1) << 21;   // entries of the fused Inv R (16 MB)
constexpr int kMaxTimes = 32;  // times of one expmv_execute_times call

int grid_for(int64_t rows, int PP, int cap = 1024) {
  const int64_t wgs = (rows * PP + kThreads - 1) / kThreads;
  return int(std::max<int64_t>(1, std::min<int64_t>(cap, wgs)));
}

// Grid of an AMG gather kernel (256 threads, `lanes` per row): up to 4096
// workgroups, a multiple of 8 from 8 on, so that RowRange keeps each
// workgroup's rows inside the eighth of the level its XCD works on.
int grid_amg(int64_t rows, int lanes) {
  const int g = grid_for(rows, lanes, 4096);
  return g < 8 ? g : (g + 7) / 8 * 8;
}

#define DISPATCH_PP(PP, ...)                         \
  switch (PP) {                                      \
    case 1: { constexpr int P_ = 1; __VA_ARGS__; } break;   \
    case 2: { constexpr int P_ = 2; __VA_ARGS__; } break;   \
    case 4: { constexpr int P_ = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int P_ = 8; __VA_ARGS__; } break;   \
    case 16: { constexpr int P_ = 16; __VA_ARGS__; } break; \
    default: { constexpr int P_ = 32; __VA_ARGS__; } break; \
  }

// Four adjacent columns per lane (16-byte FP32 or 32-byte FP64 accesses per
// lane) pay for FP32 blocks and for FP64 blocks of 16 or more columns; at
// p = 8 in FP64, two lanes per row with two double2 loads each measured
// slower than four lanes with one (59.4 against 57.7 ms per solve on the
// 64^3 benchmark; 0.61 against 0.67 s at p = 32).
template <typename T, int PP>
constexpr bool kWide4 = PP >= 4 && (sizeof(T) == 4 || PP >= 16);
// eight FP32 columns per lane (two 16-byte accesses) from 16 columns
// (measured: 32 bytes per lane pays for FP32 at p = 16 and 32; at p = 8, one
// lane per row, it changes nothing)
template <typename T, int PP>
constexpr bool kWide8 = sizeof(T) == 4 && PP >= 16;

// Lane width of the inner solvers' SpMMs (k_cg_a, k_bcg_s): two adjacent
// columns per lane for even p (one otherwise), so that the eight gathers of a
// pipelined row step (spmm_unroll) fit in the registers of a 1024-thread
// workgroup with FP32 and FP64 blocks alike (four FP32 columns spilled).
// Only the columns a lane owns change with the width: the rows of each
// workgroup, and so the partial sums, do not.
#define SPMM_DISPATCH(T, PP, p, ...)                                         \
  do {                                                                       \
    if constexpr (PP >= 2) {                                                 \
      if ((p) % 2 == 0) {                                                    \
        constexpr int PPL_ = PP / 2, VW_ = 2;                                \
        __VA_ARGS__;                                                         \
        break;                                                               \
      }                                                                      \
    }                                                                        \
    {                                                                        \
      constexpr int PPL_ = PP, VW_ = 1;                                      \
      __VA_ARGS__;                                                           \
    }                                                                        \
  } while (0)

// Lane width of the BiCGStab vector updates (k_bcg_u1/u2/u3): four FP64
// columns per lane (two 16-byte accesses) for blocks of 16 or more columns
// with p a multiple of 4, else as the SpMMs.  On the 128^3 workload u1 and u3
// took 0.247 / 0.472 ms at two columns and 0.228 / 0.450 ms at four, while
// the SpMMs lost at four (0.309 against 0.293 ms).
#define UPD_DISPATCH(T, PP, p, ...)                                          \
  do {                                                                       \
    if constexpr (PP >= 16 && sizeof(T) == 8) {                              \
      if ((p) % 4 == 0) {                                                    \
        constexpr int PPL_ = PP / 4, VW_ = 4;                                \
        __VA_ARGS__;                                                         \
        break;                                                               \
      }                                                                      \
    }                                                                        \
    SPMM_DISPATCH(T, PP, p, __VA_ARGS__);                                    \
  } while (0)

// CG kernels (working type T): PPL_ lanes per row with VW_ adjacent columns
// each, PPL_ VW_ = PP: VW_ = 8 for FP32 blocks of 16 or more columns with p a
// multiple of 8 (kWide8), else 4 when p is a multiple of 4 and the block is
// FP32 or at least 16 wide (kWide4), else 2 for even p
#define CG_CASE(PPV, p, ...)                                                \
  case PPV:                                                                 \
    if constexpr (kWide8<T, PPV>) {                                         \
      if ((p) % 8 == 0) {                                                   \
        constexpr int PPL_ = PPV / 8, VW_ = 8;                              \
        __VA_ARGS__;                                                        \
        break;                                                              \
      }                                                                     \
    }                                                                       \
    if constexpr (kWide4<T, PPV>) {                                         \
      if ((p) % 4 == 0) {                                                   \
        constexpr int PPL_ = PPV / 4, VW_ = 4;                              \
        __VA_ARGS__;                                                        \
        break;                                                              \
      }                                                                     \
    }                                                                       \
    if (PPV >= 2 && (p) % 2 == 0) {                                         \
      constexpr int PPL_ = (PPV >= 2 ? PPV / 2 : 1), VW_ = (PPV >= 2 ? 2 : 1); \
      __VA_ARGS__;                                                          \
    } else {                                                                \
      constexpr int PPL_ = PPV, VW_ = 1;                                    \
      __VA_ARGS__;                                                          \
    }                                                                       \
    break;
#define DISPATCH_CG(PP, p, ...)                                                       \
  switch (PP) {                                                                       \
    CG_CASE(1, p, __VA_ARGS__) CG_CASE(2, p, __VA_ARGS__) CG_CASE(4, p, __VA_ARGS__)  \
    CG_CASE(8, p, __VA_ARGS__) CG_CASE(16, p, __VA_ARGS__) CG_CASE(32, p, __VA_ARGS__) \
  }

// Lay out the call's workspace in `work` (nullptr: size only) and return its
// size in bytes.  p = width of the block the method runs on (the joined
// block's in source mode), nt = times, joined = source mode (the joined
// block itself is kept in the workspace).  All per-call device arrays come
// from here: the basis, the inner solver's and the V-cycle's vectors, X,
// the projected systems, the reductions and the Toeplitz FFT arrays.  The
// plan holds only what its creation set up.
// Whether the block Gram-Schmidt passes (orth_pass) can project a block of
// p columns against npan panels: the matrix-core path takes up to 24 column
// blocks of 16 for p <= 32; the other path keeps a workgroup's npan p x p
// projection partials and one row of the panels in LDS (150 KB).
bool basis_fits(int npan, int p, size_t elem) {
  if (p <= 32 && (npan * p + 15) / 16 <= 32) return true;
  const size_t O = size_t(npan) * p * p + p;
  return O * 8 + (size_t(npan) * p + 2 * size_t(p)) * elem <= 150 * 1024;
}

size_t layout_workspace(expmv_plan_s* pl, int p, int nt, bool joined, char* work) {
  Carver c{work};
  Workspace w;
  const int64_t n = pl->n;
  const int m = pl->opts.m;
  const int npan_max = m + 1;
  const int ldh = (m + 1) * p;
  const int ns = kNShift * nt;
  const size_t elb = pl->basis32 ? sizeof(float) : sizeof(double);   // basis
  if (!basis_fits(npan_max, p, elb)) {
    std::snprintf(g_error_detail, sizeof(g_error_detail),
                  "a basis of m + 1 = %d blocks of %d columns is wider than the block "
                  "Gram-Schmidt passes take: lower m or p",
                  npan_max, p);
    throw StatusError{EXPMV_EINVAL};
  }
  const size_t el = pl->mixed ? sizeof(float) : sizeof(double);      // inner solver
  const size_t blk = size_t(n) * p;
  const bool csr = pl->kind == 0;
  w.V[0] = c.take<char>(blk * npan_max * elb);
  w.V[1] = c.take<char>(blk * npan_max * elb);
  w.W = c.take<char>(blk * std::max(elb, el));
  w.Wt = c.take<char>(blk * std::max(elb, el));
  w.Win = c.take<char>(blk * el);
  w.Wout = c.take<char>(blk * el);
  if (pl->mixed && csr) {
    w.Rin = c.take<char>(blk * el);
    w.Din = c.take<char>(blk * el);
  }
  if (csr) {
    w.kr = c.take<char>(blk * el);
    w.kpa = c.take<char>(blk * el);
    w.kpb = c.take<char>(blk * el);
    w.kq = c.take<char>(blk * el);
    if (pl->amg) w.kz = c.take<char>(blk * el);
    if (pl->amg && !pl->symmetric) {
      w.kph = c.take<char>(blk * el);
      w.ksh = c.take<char>(blk * el);
    }
    if (!pl->symmetric) {
      w.kv = c.take<char>(blk * el);
      w.ks = c.take<char>(blk * el);
      w.kt = c.take<char>(blk * el);
      w.krh = c.take<char>(blk * el);
    }
    if (pl->amg && !pl->mixed && pl->opts.amg_fp32) {
      w.kr32 = c.take<float>(blk);
      w.kz32 = c.take<float>(blk);
    }
  }
  w.X = c.take<double>(blk * 2 * ns);
  const size_t O = size_t(npan_max) * p * p + p;
  const int Wres = 2 * kNShift * p;
  w.partial = c.take<double>(std::max({O * kOrthGrid, size_t(512) * std::max(nt, 16),
                                       size_t(kResGrid) * p * Wres, size_t(4096)}));
  w.hcoef = c.take<double>(O);
  w.gram = c.take<double>(size_t(p) * p);
  w.R1 = c.take<double>(size_t(p) * p);
  w.R2 = c.take<double>(size_t(p) * p);
  w.Rinv = c.take<double>(size_t(p) * p);
  w.w0 = c.take<double>(O);
  w.H = c.take<double>(size_t(ldh) * ldh);
  w.Rhat = c.take<double>(size_t(p) * p);
  const int dmax = m * p;
  w.G = c.take<cplx>(size_t(ns) * dmax * p);
  w.Zs = c.take<cplx>(size_t(ns) * dmax * p);
  w.Ascr = c.take<cplx>(size_t(ns) * dmax * dmax);
  w.S = c.take<cplx>(size_t(ns) * p * p);
  w.Cr = c.take<double>(size_t(ldh) * 2 * ns * p);
  w.Crot = c.take<double>(size_t(dmax) * dmax);
  w.rho = c.take<double>(ns);
  w.flags = c.take<int>(4);
  w.singular = c.take<int>(ns);
  w.cgst = c.take<CgState>(1);
  w.bcgst = c.take<BcgState>(1);
  w.part_rr = c.take<double>(size_t(kCgGrid) * 2 * kMaxP);
  w.part_sig = c.take<double>(size_t(kCgGrid) * 2 * kMaxP);
  w.taus = c.take<double>(2 * size_t(ns));
  w.coefs = c.take<double>(4 * size_t(ns));
  w.S2 = c.take<cplx>(size_t(ns) * p * p);
  w.singular2 = c.take<int>(ns);
  w.ctl = c.take<KrylovCtl>(1);
  w.Rres = c.take<double>(blk * 2 * kNShift);
  w.projC = c.take<double>(size_t(p) * Wres);
  w.rpart = c.take<double>(size_t(512 + kResGrid) * kNShift);
  w.Sref = c.take<cplx>(size_t(ns) * p * p);
  if (!csr) {
    w.fq = p;   // the residual transforms 2p real columns as p complex ones
    for (auto& b : w.fb) b = c.take<cplx>(size_t(pl->L) * w.fq);
  }
  if (joined) w.srcB = c.take<double>(blk);
  // V-cycle vectors of the hierarchy of K and of K^T: one call uses one of
  // them, so both share one region
  size_t amg_base = 0, amg_end = 0;
  for (AmgDev* Hd : {pl->amg.get(), pl->amgT.get()}) {
    if (!Hd) continue;
    Carver h{nullptr, 0};
    const size_t start = (c.off + 255) & ~size_t(255);
    if (amg_base == 0) amg_base = start;
    h.off = amg_base;
    h.base = work;
    for (size_t l = 0; l < Hd->lv.size(); ++l) {
      AmgDevLevel& L = *Hd->lv[l];
      const size_t bytes = size_t(L.n) * p * sizeof(double);
      char *vu = nullptr, *vv = nullptr, *vd = nullptr, *vr = nullptr, *vb = nullptr, *vo = nullptr;
      if (l + 1 < Hd->lv.size()) {
        vu = h.take<char>(bytes);
        vv = h.take<char>(bytes);
        vd = h.take<char>(bytes);
        vr = h.take<char>(bytes);
      }
      if (l > 0) {
        vb = h.take<char>(bytes);
        vo = h.take<char>(bytes);
      }
      if (work) {
        L.vu = vu;
        L.vv = vv;
        L.vd = vd;
        L.vr = vr;
        L.vb = vb;
        L.vo = vo;
      }
    }
    amg_end = std::max(amg_end, h.off);
  }
  if (amg_end > c.off) c.off = amg_end;
  if (work) {
    pl->ws = w;
    pl->ldh = ldh;
  }
  return c.off;
}

// Bind the call's workspace; EINVAL (with a detail) when `work` is missing
// or smaller than layout_workspace asks for.
void bind_workspace(expmv_plan_s* pl, int p, int nt, bool joined, void* work, size_t bytes);

// ------------------------------------------------------------------------
// operator data of the working type

template <typename T>
struct Csr {
  const int32_t* rowptr;
  const int32_t* colind;
  const double* val;   // FP64 in both forms
  const T* dinv;       // Jacobi scaling in the working type
};

template <typename T>
Csr<T> csr_of(expmv_plan_s* pl, int transpose);

template <>
Csr<double> csr_of<double>(expmv_plan_s* pl, int transpose) {
  const bool tr = transpose && !pl->symmetric;
  return tr ? Csr<double>{pl->rowptrT.p, pl->colindT.p, pl->valT.p, pl->dinvT.p}
            : Csr<double>{pl->rowptr.p, pl->colind.p, pl->val.p, pl->dinv.p};
}

template <>
Csr<float> csr_of<float>(expmv_plan_s* pl, int transpose) {
  const bool tr = transpose && !pl->symmetric;
  return tr ? Csr<float>{pl->rowptrT.p, pl->colindT.p, pl->valT.p, pl->dinvTf.p}
            : Csr<float>{pl->rowptr.p, pl->colind.p, pl->val.p, pl->dinvf.p};
}

// Y = K X (K = -tA, or its transpose) for n x p blocks of type T.
template <typename T>
void toeplitz_apply(expmv_plan_s* pl, const T* X, int64_t ldx, T* Y, int64_t ldy, int p,
                    double scale, int accumulate, int transpose = 0, bool with_diag = true);
template <typename T>
void toeplitz_gsf(expmv_plan_s* pl, int transpose, const T* V, T* W, int p, double scale);

template <typename T>
void apply_K(expmv_plan_s* pl, int transpose, const T* X, T* Y, int p) {
  if (pl->kind == 1) {   // K = t T (or t T^T)
    toeplitz_apply<T>(pl, X, p, Y, p, p, pl->t, 0, transpose);
    return;
  }
  Csr<T> A = csr_of<T>(pl, transpose);
  const int PP = pow2_lanes(p);
  const int grid = grid_for(pl->n, PP, 4096);
  DISPATCH_PP(PP, hipLaunchKernelGGL((k_spmm<T, P_>), dim3(grid), dim3(kThreads), 0, pl->stream,
                                     int(pl->n), p, A.rowptr, A.colind, A.val, X, Y));
}

struct KtEv {
  hipEvent_t e0 = nullptr, e1 = nullptr;
};

// Start/stop events for one launch of kernel class `cls` moving `bytes`
// algorithmic bytes, or none when it is not timed (profile off, an inner
// iteration that is not sampled, or the pool is full until the next
// collection).
KtEv kt_take(expmv_plan_s* pl, int cls, double bytes) {
  KernelTimer& k = pl->kt;
  if (pl->opts.profile <= 0 || (k.cur_iter >= 0 && !k.sampling) || k.used >= kKtSlots) return {};
  const int u = k.used++;
  k.cls[u] = cls;
  k.iter[u] = k.cur_iter;
  k.bytes[u] = bytes;
  return {k.ev[2 * u], k.ev[2 * u + 1]};
}

// Add the timed launches to the per-class sums.  Launches of inner
// iterations at or after kexec (the iterations the solve ran) returned at
// once and are dropped.
void kt_collect(expmv_plan_s* pl, int kexec) {
  KernelTimer& k = pl->kt;
  if (k.used == 0) return;
  HIPCHK(hipEventSynchronize(k.ev[2 * (k.used - 1) + 1]));
  for (int u = 0; u < k.used; ++u) {
    if (k.iter[u] >= 0 && k.iter[u] >= kexec) continue;
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, k.ev[2 * u], k.ev[2 * u + 1]));
    k.ms[k.cls[u]] += ms;
    k.by[k.cls[u]] += k.bytes[u];
    k.cnt[k.cls[u]] += 1;
  }
  k.used = 0;
}

// CSR bytes of an operator with `rows` rows and `nnz` nonzeros (int32
// indices, FP64 values)
inline double csr_bytes(int64_t rows, int64_t nnz) {
  return 4.0 * double(rows + 1) + 12.0 * double(nnz);
}

struct InnerResult {
  int iters;
  int hit_cap;
};

int cg_grid(int64_t n, int PP) {
  return int(std::max<int64_t>(
      1, std::min<int64_t>(kCgGrid, (n * PP + kCgThreads - 1) / kCgThreads)));
}

double inner_tol_of(expmv_plan_s* pl) {
  const double base = pl->opts.inner_tol > 0.0 ? pl->opts.inner_tol : (pl->mixed ? 1e-6 : 1e-12);
  return base * pl->relax_scale;
}

// Poll the inner solver's control word every `chunk` iterations, one chunk
// ahead of the device; returns when a chunk has seen every column stop.
// The first chunk may be larger (first_chunk, e.g. a few iterations short
// of what the previous inner solve needed).
template <typename LaunchChunk>
InnerResult run_inner_loop(expmv_plan_s* pl, int maxit, LaunchChunk&& launch_chunk,
                           int chunk = 16, int first_chunk = 0) {
  Workspace& w = pl->ws;
  hipStream_t s = pl->stream;
  int launched = 0;
  int pending = -1, slot = 0;
  bool done = false;
  while (!done) {
    const int c = (launched == 0 && first_chunk > chunk) ? std::min(first_chunk, maxit) : chunk;
    launch_chunk(launched, c);
    launched += c;
    HIPCHK(hipMemcpyAsync(pl->host_flags + 4 * slot, w.ctl, sizeof(KrylovCtl),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipEventRecord(pl->ev[slot], s));
    if (pending >= 0) {
      HIPCHK(hipEventSynchronize(pl->ev[pending]));
      const KrylovCtl* c = reinterpret_cast<const KrylovCtl*>(pl->host_flags + 4 * pending);
      if (c->done >= 0) done = true;
    }
    pending = slot;
    slot ^= 1;
    if (launched > maxit + 4 * chunk) break;  // the cap stops every column before this
  }
  HIPCHK(hipEventSynchronize(pl->ev[pending]));
  const KrylovCtl* c = reinterpret_cast<const KrylovCtl*>(pl->host_flags + 4 * pending);
  return {c->iters_max, c->hit_cap};
}

// ------------------------------------------------------------------------
// AMG V-cycle (preconditioner of the inner CG)

// operator values of a level in the V-cycle's precision
template <typename T>
struct LevelVals {
  const T *a, *p, *r, *pf, *rf;
};
LevelVals<double> vals_of(const AmgDevLevel& L, double) {
  return {L.av, L.Pv.p, L.Rv.p, L.Pfv.p, L.Rfv.p};
}
LevelVals<float> vals_of(const AmgDevLevel& L, float) {
  return {L.Av32.p, L.Pv32.p, L.Rv32.p, L.Pfv32.p, L.Rfv32.p};
}

template <typename T>
const T* dinv_of(const AmgDevLevel& L);
template <>
const double* dinv_of<double>(const AmgDevLevel& L) { return L.dinv64; }
template <>
const float* dinv_of<float>(const AmgDevLevel& L) { return L.dinv32; }

// out = V-cycle(b) on level l (level 0: the inner solver's launch shape,
// and with part_rz the (b, out) partials of the last smoothing step).  The
// kernels take VW columns per lane and PPL = PP / VW lanes per row; the finest
// level keeps the inner solver's grid (its partials are re-summed by the CG
// kernels over that many workgroups).
template <typename T, int PP>
void amg_level(expmv_plan_s* pl, AmgDev& H, int l, int p, const T* b, T* out, int k,
               const KrylovCtl* ctl, double* part_rz);

template <typename T, int PPL, int VW>
void amg_level_vw(expmv_plan_s* pl, AmgDev& H, int l, int p, const T* b, T* out, int k,
                  const KrylovCtl* ctl, double* part_rz) {
  constexpr int PP = PPL * VW;
  AmgDevLevel& L = *H.lv[l];
  hipStream_t s = pl->stream;
  const int n = int(L.n);
  const bool fine = (l == 0);
  // timing: class of this level's launches and the bytes of their operands
  const double es = double(sizeof(T));
  const double blk = es * double(n) * p;
  auto csr = [&](int64_t rows, int64_t nnz) {
    return 4.0 * double(rows + 1) + (4.0 + es) * double(nnz);
  };
  const int c_smooth = fine ? EXPMV_KT_AMG_SMOOTH : EXPMV_KT_AMG_COARSE;
  const int c_restr = fine ? EXPMV_KT_AMG_RESTRICT : EXPMV_KT_AMG_COARSE;
  const int c_prol = fine ? EXPMV_KT_AMG_PROLONG : EXPMV_KT_AMG_COARSE;
  if (l + 1 == int(H.lv.size())) {
    const int grid = std::max(1, std::min(n, 1024));
    const KtEv e = kt_take(pl, EXPMV_KT_AMG_COARSE, 8.0 * double(n) * n + 2 * blk);
    hipExtLaunchKernelGGL((k_amg_dense<T, PP>), dim3(grid), dim3(1024), 0, s, e.e0, e.e1, 0, k,
                          ctl, n, n, p, H.cinv.p, b, out);
    return;
  }
  const T* dinv = dinv_of<T>(L);
  const LevelVals<T> lv = vals_of(L, T());
  AmgDevLevel& C = *H.lv[l + 1];
  const int nc = int(C.n);
  const double cblk = es * double(nc) * p;
  // restriction of b by a fused operator Rf (sparse), or Inv Rf (dense) into
  // the coarsest level
  auto restrict_fused = [&](T* bc, T* xc, bool dense) {
    if (dense) {
      const KtEv e = kt_take(pl, c_restr, 8.0 * double(nc) * n + blk + cblk);
      hipExtLaunchKernelGGL((k_amg_dense<T, PP>), dim3(std::max(1, std::min(nc, 1024))),
                            dim3(1024), 0, s, e.e0, e.e1, 0, k, ctl, nc, n, p, H.cinvR.p, b, xc);
      return;
    }
    const int GR = row_split(L.avg_rf, PPL);
    const KtEv e = kt_take(pl, c_restr, csr(nc, L.nnz_rf) + blk + cblk);
    hipExtLaunchKernelGGL((k_amg_restrict<T, PPL, VW, kThreads, false>),
                          dim3(grid_amg(nc, PPL * GR)), dim3(kThreads), 0, s, e.e0, e.e1, 0,
                          k, ctl, nc, p, GR, L.Rfrp.p, L.Rfci.p, lv.rf, b, bc);
    amg_level<T, PPL * VW>(pl, H, l + 1, p, bc, xc, k, ctl, nullptr);
  };
  // the prolongation-plus-smoothing pass (256-thread workgroups over the
  // XCD's eighth of the rows); in FP64 at four columns per lane its sum over
  // A reads A D^{-1}
  auto launch_pair = [&](int G, const KtEv& e, const T* xc) {
    if constexpr (std::is_same<T, double>::value && VW == 4) {
      if (L.ADv.p && PPL == 4) {
        const int nx = int(H.lv[l + 1]->n);
        hipExtLaunchKernelGGL((k_amg_affine_pair_q<T, VW, kThreads>),
                              dim3(grid_amg(n, PPL * G)), dim3(kThreads), 0, s, e.e0, e.e1, 0, k,
                              ctl, n, p, G, L.arp, L.aci, L.ADv.p, dinv, b, L.Pfrp.p, L.Pfci.p,
                              lv.pf, xc, nx, L.alpha, L.beta, out);
        return;
      }
      if (L.ADv.p) {
        hipExtLaunchKernelGGL((k_amg_affine_pair_ad<T, PPL, VW, kThreads, false>),
                              dim3(grid_amg(n, PPL * G)), dim3(kThreads), 0, s, e.e0, e.e1, 0, k,
                              ctl, n, p, G, L.arp, L.aci, L.ADv.p, dinv, b, L.Pfrp.p, L.Pfci.p,
                              lv.pf, xc, L.alpha, L.beta, out);
        return;
      }
    }
    hipExtLaunchKernelGGL((k_amg_affine_pair<T, PPL, VW, kThreads, false>),
                          dim3(grid_amg(n, PPL * G)), dim3(kThreads), 0, s, e.e0, e.e1, 0, k, ctl,
                          n, p, G, L.arp, L.aci, lv.a, dinv, b, L.Pfrp.p, L.Pfci.p, lv.pf, xc,
                          L.alpha, L.beta, out);
  };
  // prolongation plus the post-smoothing step in one pass (fused levels)
  const double pair_bytes = csr(n, L.nnz_a) + es * n + blk + csr(n, L.nnz_pf) + cblk + blk;
  if (!fine && L.fused) {
    T* xc = reinterpret_cast<T*>(C.vo);
    restrict_fused(reinterpret_cast<T*>(C.vb), xc, l + 2 == int(H.lv.size()) && H.cinvR.p);
    const int G = std::max(row_split(L.avg_a, PPL), row_split(L.avg_pf, PPL));
    const KtEv e = kt_take(pl, c_prol, pair_bytes);
    launch_pair(G, e, xc);
    return;
  }
  const int gfine = cg_grid(n, PP);
  const int GA = row_split(L.avg_a, PPL), GP = row_split(L.avg_p, PPL);
  const int gcoarse_a = grid_amg(n, PPL * GA), gcoarse_p = grid_amg(n, PPL * GP);
  // one smoothing step: reads A, D^{-1}, b and the iterate (unless it is the
  // implicit first one), the direction when HasD; writes the output and the
  // direction when WriteD (the residual step writes r only)
  auto step = [&](int mode, const T* x, T* o, double cd, double ad, double* part) {
    T* d = reinterpret_cast<T*>(L.vd);
    double bytes = csr(n, L.nnz_a) + es * n + 2 * blk;   // A, D^{-1}, b, output
    if (!(mode & kAmgX0)) bytes += blk;
    if (mode & kAmgHasD) bytes += blk;
    if (mode & kAmgWriteD) bytes += blk;
    const KtEv e = kt_take(pl, c_smooth, bytes);
    if (fine)
      hipExtLaunchKernelGGL((k_amg_step<T, PPL, VW, kCgThreads, true>), dim3(gfine),
                            dim3(kCgThreads), 0, s, e.e0, e.e1, 0, k, ctl, n, p, GA, L.arp, L.aci,
                            lv.a, dinv, b, x, d, o, L.ad[0], cd, ad, mode, part);
    else
      hipExtLaunchKernelGGL((k_amg_step<T, PPL, VW, kThreads, false>), dim3(gcoarse_a),
                            dim3(kThreads), 0, s, e.e0, e.e1, 0, k, ctl, n, p, GA, L.arp, L.aci,
                            lv.a, dinv, b, x, d, o, L.ad[0], cd, ad, mode, part);
  };
  T* x = reinterpret_cast<T*>(L.vu);
  T* y = reinterpret_cast<T*>(L.vv);
  if (fine && L.fused && L.degree == 1 && part_rz == nullptr && sizeof(T) == 8) {
    // one step (nonsymmetric K): Rf b, the coarse correction, then the
    // prolongation and the post-smoothing step in one pass (FP64 V-cycles:
    // in FP32 the unfused launches measured faster, 4.45 against 4.77 s on
    // the 128^3 convection-diffusion workload)
    T* xc = reinterpret_cast<T*>(C.vo);
    restrict_fused(reinterpret_cast<T*>(C.vb), xc, false);
    const int G = std::max(GA, row_split(L.avg_pf, PPL));
    const KtEv e = kt_take(pl, c_prol, pair_bytes);
    // 256-thread workgroups over the XCD's eighth of the rows, as on the
    // coarse levels (this kernel writes no partial sums, so it need not
    // keep the inner solver's launch shape): 0.467 against 0.493 ms per
    // launch on the 128^3 workload in 1024-thread row segments
    launch_pair(G, e, xc);
    return;
  }
  if (fine && L.fused && L.degree == 2) {
    // bc = Rf b, the coarse correction, then x = x1 + P xc (x1, the
    // pre-smoothed iterate, recomputed from b)
    T* xc = reinterpret_cast<T*>(C.vo);
    restrict_fused(reinterpret_cast<T*>(C.vb), xc, false);
    const KtEv e = kt_take(pl, c_prol, csr(n, L.nnz_a) + es * n + blk + csr(n, L.nnz_p) + cblk +
                                           blk);
    hipExtLaunchKernelGGL((k_amg_affine_pair<T, PPL, VW, kCgThreads, true>), dim3(gfine),
                          dim3(kCgThreads), 0, s, e.e0, e.e1, 0, k, ctl, n, p, std::max(GA, GP),
                          L.arp, L.aci, lv.a, dinv, b, L.Prp.p, L.Pci.p, lv.p, xc, L.alpha, L.beta,
                          x);
  } else {
    // pre-smoothing from zero: the first step's iterate s0 D^{-1} b stays implicit
    bool implicit = true;
    for (int st = 1; st < L.degree; ++st) {
      step(kAmgHasD | kAmgWriteD | (implicit ? kAmgX0 : 0), x, y, L.cd[st], L.ad[st], nullptr);
      implicit = false;
      std::swap(x, y);
    }
    T* r = reinterpret_cast<T*>(L.vr);
    step(kAmgResid | (implicit ? kAmgX0 : 0), x, r, 0.0, 0.0, nullptr);
    T* bc = reinterpret_cast<T*>(C.vb);
    T* xc = reinterpret_cast<T*>(C.vo);
    if (l + 2 == int(H.lv.size()) && H.cinvR.p) {
      // coarsest correction in one dense product: xc = (Inv R) r
      const KtEv e = kt_take(pl, c_restr, 8.0 * double(nc) * n + blk + cblk);
      hipExtLaunchKernelGGL((k_amg_dense<T, PP>), dim3(std::max(1, std::min(nc, 1024))),
                            dim3(1024), 0, s, e.e0, e.e1, 0, k, ctl, nc, n, p, H.cinvR.p, r, xc);
    } else {
      const int GR = row_split(L.avg_r, PPL);
      const KtEv e = kt_take(pl, c_restr, csr(nc, L.nnz_r) + blk + cblk);
      hipExtLaunchKernelGGL((k_amg_restrict<T, PPL, VW, kThreads, false>),
                            dim3(grid_amg(nc, PPL * GR)), dim3(kThreads), 0, s, e.e0, e.e1,
                            0, k, ctl, nc, p, GR, L.Rrp.p, L.Rci.p, lv.r, r, bc);
      amg_level<T, PPL * VW>(pl, H, l + 1, p, bc, xc, k, ctl, nullptr);
    }
    const int pmode = implicit ? kAmgX0 : 0;
    // x (+)= P xc (with the implicit iterate from b and D^{-1} when pmode)
    const double pb = csr(n, L.nnz_p) + cblk + blk + (implicit ? es * n + blk : blk);
    const KtEv e = kt_take(pl, c_prol, pb);
    if (fine)
      hipExtLaunchKernelGGL((k_amg_prolong<T, PPL, VW, kCgThreads, true>), dim3(gfine),
                            dim3(kCgThreads), 0, s, e.e0, e.e1, 0, k, ctl, n, p, GP, L.Prp.p,
                            L.Pci.p, lv.p, xc, dinv, b, L.ad[0], pmode, x);
    else
      hipExtLaunchKernelGGL((k_amg_prolong<T, PPL, VW, kThreads, false>), dim3(gcoarse_p),
                            dim3(kThreads), 0, s, e.e0, e.e1, 0, k, ctl, n, p, GP, L.Prp.p,
                            L.Pci.p, lv.p, xc, dinv, b, L.ad[0], pmode, x);
  }
  // post-smoothing from x, the same polynomial (symmetric V-cycle)
  for (int st = 0; st < L.degree; ++st) {
    const bool last = (st + 1 == L.degree);
    T* o = last ? out : y;
    const int mode = (st > 0 ? kAmgHasD : 0) | (last ? 0 : kAmgWriteD) |
                     (last && part_rz ? kAmgRz : 0);
    step(mode, x, o, L.cd[st], L.ad[st], last ? part_rz : nullptr);
    if (!last) std::swap(x, y);
  }
}

// two adjacent columns per lane when p is even, four when p is a multiple of
// 4 and kWide4, and on the levels below the finest (their longer Galerkin
// rows: 0.7% on the 64^3 benchmark); each level picks its own layout
template <typename T, int PP>
void amg_level(expmv_plan_s* pl, AmgDev& H, int l, int p, const T* b, T* out, int k,
               const KrylovCtl* ctl, double* part_rz) {
  if constexpr (kWide8<T, PP>) {
    if (p % 8 == 0) {
      amg_level_vw<T, PP / 8, 8>(pl, H, l, p, b, out, k, ctl, part_rz);
      return;
    }
  }
  if constexpr (PP >= 4) {
    if (p % 4 == 0 && (kWide4<T, PP> || l > 0)) {
      amg_level_vw<T, PP / 4, 4>(pl, H, l, p, b, out, k, ctl, part_rz);
      return;
    }
  }
  if constexpr (PP >= 2) {
    if (p % 2 == 0) {
      amg_level_vw<T, PP / 2, 2>(pl, H, l, p, b, out, k, ctl, part_rz);
      return;
    }
  }
  amg_level_vw<T, PP, 1>(pl, H, l, p, b, out, k, ctl, part_rz);
}

// The hierarchy for K (transpose = 0) or K^T; NULL without AMG.
AmgDev* amg_for(expmv_plan_s* pl, int transpose) {
  if (transpose && !pl->symmetric) return pl->amgT.get();
  return pl->amg.get();
}

// One V-cycle of hierarchy H.
template <typename T>
void amg_vcycle(expmv_plan_s* pl, AmgDev& H, int p, const T* b, T* out, int k,
                const KrylovCtl* ctl, double* part_rz) {
  const int PP = pow2_lanes(p);
  DISPATCH_PP(PP, amg_level<T, P_>(pl, H, 0, p, b, out, k, ctl, part_rz));
}

// out = K^{-1} (sign * src) by batched Jacobi-PCG (K SPD); out is the iterate.
template <typename T>
InnerResult inner_cg(expmv_plan_s* pl, const T* src, double sign, T* out, int p) {
  Workspace& w = pl->ws;
  hipStream_t s = pl->stream;
  const int64_t n = pl->n;
  const int PP = pow2_lanes(p);
  const int grid = cg_grid(n, PP);
  const double tol = inner_tol_of(pl);
  const double tol2 = tol * tol;
  const int maxit = pl->opts.inner_maxit;
  Csr<T> A = csr_of<T>(pl, 0);
  T* r = reinterpret_cast<T*>(w.kr);
  T* q = reinterpret_cast<T*>(w.kq);
  T* P[2] = {reinterpret_cast<T*>(w.kpa), reinterpret_cast<T*>(w.kpb)};
  AmgDev* H = amg_for(pl, 0);
  const bool amg = H != nullptr;
  T* z = amg ? reinterpret_cast<T*>(w.kz) : nullptr;
  // FP32 V-cycle under the FP64 CG (opts.amg_fp32): k_cg_init / k_cg_b write an
  // FP32 copy of r, the V-cycle maps it to an FP32 z that k_cg_c reads
  const bool v32 = amg && !std::is_same<T, float>::value && pl->opts.amg_fp32 != 0;
  float* r32 = nullptr;
  float* z32 = nullptr;
  if (v32) {
    r32 = w.kr32;
    z32 = w.kz32;
  }
  DISPATCH_CG(PP, p, hipLaunchKernelGGL((k_cg_init<T, T, PPL_, VW_>), dim3(grid), dim3(kCgThreads), 0, s,
                                     int(n), p, sign, src, A.dinv, out, r, P[0], w.ctl,
                                     w.part_rr, r32));
  auto vcycle = [&](int k) {
    if (v32)
      amg_vcycle<float>(pl, *H, p, r32, z32, k, w.ctl, w.part_rr);
    else
      amg_vcycle<T>(pl, *H, p, r, z, k, w.ctl, w.part_rr);
  };
  if (amg) vcycle(0);
  // timed bytes per launch: A q = K p (CSR, p gathered, q written);
  // B r -= alpha q (+ D^{-1} for Jacobi's (r, D^{-1} r), + the FP32 copy of r);
  // C x += alpha p_old, p_new = z + beta p_old (z = D^{-1} r for Jacobi)
  const double es = double(sizeof(T)), blk = es * double(n) * p;
  const double by_a = csr_bytes(n, pl->nnz) + 2 * blk;
  const double by_b = 3 * blk + (amg ? 0.0 : es * n) + (v32 ? 4.0 * n * p : 0.0);
  const double by_c = 4 * blk + (amg ? (v32 ? 4.0 : es) * n * p : es * n + blk);
  KernelTimer& kt = pl->kt;
  InnerResult res = run_inner_loop(pl, maxit, [&](int launched, int chunk) {
    for (int it = 0; it < chunk; ++it) {
      const int k = launched + it;
      T* pold = P[k & 1];
      T* pnew = P[(k + 1) & 1];
      kt.cur_iter = k;
      kt.sampling = pl->opts.profile > 0 && ((k + 1) % pl->opts.profile) == 0;
      const KtEv ec = kt_take(pl, EXPMV_KT_CG_DIR, by_c);
      if (v32) {
        DISPATCH_CG(PP, p, hipExtLaunchKernelGGL((k_cg_c<T, float, PPL_, VW_>), dim3(grid),
                                                 dim3(kCgThreads), 0, s, ec.e0, ec.e1, 0, k,
                                                 int(n), p, A.dinv, r, z32, pold, pnew, out,
                                                 w.cgst, w.ctl, w.part_rr, tol2, maxit));
      } else {
        DISPATCH_CG(PP, p, hipExtLaunchKernelGGL((k_cg_c<T, T, PPL_, VW_>), dim3(grid),
                                                 dim3(kCgThreads), 0, s, ec.e0, ec.e1, 0, k,
                                                 int(n), p, A.dinv, r, z, pold, pnew, out,
                                                 w.cgst, w.ctl, w.part_rr, tol2, maxit));
      }
      const KtEv ea = kt_take(pl, EXPMV_KT_CG_SPMM, by_a);
      DISPATCH_PP(PP, SPMM_DISPATCH(T, P_, p,
                                    hipExtLaunchKernelGGL((k_cg_a<T, PPL_, VW_>), dim3(grid),
                                                          dim3(kCgThreads), 0, s, ea.e0, ea.e1, 0,
                                                          k, int(n), p, A.rowptr, A.colind, A.val,
                                                          pnew, q, w.ctl, w.part_sig)));
      const KtEv eb = kt_take(pl, EXPMV_KT_CG_RESID, by_b);
      DISPATCH_CG(PP, p, hipExtLaunchKernelGGL((k_cg_b<T, PPL_, VW_>), dim3(grid),
                                               dim3(kCgThreads), 0, s, eb.e0, eb.e1, 0, k, int(n),
                                               p, A.dinv, r, q, w.cgst, w.ctl, w.part_sig,
                                               w.part_rr, amg ? 0 : 1, r32));
      if (amg) vcycle(k);
    }
    kt.cur_iter = -1;
    kt.sampling = false;
  }, amg ? 1 : 16, amg ? pl->last_inner_iters - 2 : 0);
  kt_collect(pl, res.iters);
  pl->last_inner_iters = res.iters;
  return res;
}

template <typename T, int PP, int NV>
void bcg_spmm(hipStream_t s, KtEv e, int grid, int i, int n, int p, const int32_t* rowptr,
              const int32_t* colind, const double* val, const T* dinv, const T* in, const T* a,
              T* out, const KrylovCtl* ctl, double* part) {
  SPMM_DISPATCH(T, PP, p,
                hipExtLaunchKernelGGL((k_bcg_s<T, PPL_, VW_, NV>), dim3(grid), dim3(kCgThreads),
                                      0, s, e.e0, e.e1, 0, i, n, p, rowptr, colind, val, dinv,
                                      in, a, out, ctl, part));
}

// out = K^{-1} (sign * src) (or K^{-T}) by batched BiCGStab with right
// Jacobi preconditioning (K nonsymmetric).
template <typename T>
InnerResult inner_bicgstab(expmv_plan_s* pl, int transpose, const T* src, double sign, T* out,
                           int p) {
  Workspace& w = pl->ws;
  hipStream_t s = pl->stream;
  const int64_t n = pl->n;
  const int PP = pow2_lanes(p);
  const int grid = cg_grid(n, PP);
  const double tol = inner_tol_of(pl);
  const double tol2 = tol * tol;
  const int maxit = pl->opts.inner_maxit;
  Csr<T> A = csr_of<T>(pl, transpose);
  T* r = reinterpret_cast<T*>(w.kr);
  T* pv = reinterpret_cast<T*>(w.kpa);
  T* v = reinterpret_cast<T*>(w.kv);
  T* sv = reinterpret_cast<T*>(w.ks);
  T* tv = reinterpret_cast<T*>(w.kt);
  T* rh = reinterpret_cast<T*>(w.krh);
  AmgDev* H = amg_for(pl, transpose);
  T* ph = H ? reinterpret_cast<T*>(w.kph) : nullptr;   // M^{-1} p
  T* sh = H ? reinterpret_cast<T*>(w.ksh) : nullptr;   // M^{-1} s
  const T* dscale = H ? nullptr : A.dinv;
  DISPATCH_PP(PP, hipLaunchKernelGGL((k_bcg_init<T, T, P_>), dim3(grid), dim3(kCgThreads), 0, s,
                                     int(n), p, sign, src, out, r, rh, w.ctl, w.part_rr));
  // timed bytes per launch: each SpMM reads K (CSR), its input (gathered)
  // and the vector its partials pair with, and writes its output (+ D^{-1}
  // for Jacobi); u1 reads r, p, v and writes p (reads r only at i = 0);
  // u2 reads r, v, writes s; u3 reads p^ and s^ (Jacobi: p and D^{-1}), s,
  // t, r~ and x, writes x and r
  const double es = double(sizeof(T)), blk = es * double(n) * p;
  const double by_s = csr_bytes(n, pl->nnz) + 3 * blk + (H ? 0.0 : es * n);
  const double by_u3 = H ? 8 * blk : 7 * blk + es * n;
  KernelTimer& kt = pl->kt;
  InnerResult res = run_inner_loop(pl, maxit, [&](int launched, int chunk) {
    for (int it = 0; it < chunk; ++it) {
      const int i = launched + it;
      kt.cur_iter = i;
      kt.sampling = pl->opts.profile > 0 && ((i + 1) % pl->opts.profile) == 0;
      DISPATCH_PP(PP, {
        const KtEv e1 = kt_take(pl, EXPMV_KT_BCG_U1, (i == 0 ? 2 : 4) * blk);
        UPD_DISPATCH(T, P_, p,
                      hipExtLaunchKernelGGL((k_bcg_u1<T, PPL_, VW_>), dim3(grid),
                                            dim3(kCgThreads), 0, s, e1.e0, e1.e1, 0, i, int(n),
                                            p, r, pv, v, w.bcgst, w.ctl, w.part_rr, tol2, maxit));
        if (H) amg_vcycle<T>(pl, *H, p, pv, ph, i, w.ctl, nullptr);
        bcg_spmm<T, P_, 1>(s, kt_take(pl, EXPMV_KT_BCG_SPMM1, by_s), grid, i, int(n), p, A.rowptr,
                           A.colind, A.val, dscale, H ? ph : pv, rh, v, w.ctl, w.part_sig);
        const KtEv e2 = kt_take(pl, EXPMV_KT_BCG_U2, 3 * blk);
        UPD_DISPATCH(T, P_, p,
                      hipExtLaunchKernelGGL((k_bcg_u2<T, PPL_, VW_>), dim3(grid),
                                            dim3(kCgThreads), 0, s, e2.e0, e2.e1, 0, i, int(n),
                                            p, r, v, sv, w.bcgst, w.ctl, w.part_sig));
        if (H) amg_vcycle<T>(pl, *H, p, sv, sh, i, w.ctl, nullptr);
        bcg_spmm<T, P_, 2>(s, kt_take(pl, EXPMV_KT_BCG_SPMM2, by_s), grid, i, int(n), p, A.rowptr,
                           A.colind, A.val, dscale, H ? sh : sv, sv, tv, w.ctl, w.part_sig);
        const KtEv e3 = kt_take(pl, EXPMV_KT_BCG_U3, by_u3);
        UPD_DISPATCH(T, P_, p,
                      hipExtLaunchKernelGGL((k_bcg_u3<T, PPL_, VW_>), dim3(grid),
                                            dim3(kCgThreads), 0, s, e3.e0, e3.e1, 0, i, int(n),
                                            p, A.dinv, pv, sv, tv, rh, ph, sh, out, r, w.bcgst,
                                            w.ctl, w.part_sig, w.part_rr));
      });
    }
    kt.cur_iter = -1;
    kt.sampling = false;
  }, H ? 1 : 16, H ? pl->last_inner_iters - 2 : 0);
  kt_collect(pl, res.iters);
  pl->last_inner_iters = res.iters;
  return res;
}

// W ~= M^{-1} V = -(K^{-1} V), M = tA.
template <typename T>
InnerResult apply_inverse(expmv_plan_s* pl, int transpose, const T* V, T* Wout, int p) {
  if (pl->kind == 1) {   // M^{-1} = -(1/t) T^{-1} (or T^{-T}), Gohberg-Semencul
    toeplitz_gsf<T>(pl, transpose, V, Wout, p, -1.0 / pl->t);
    return {0, 0};
  }
  if (pl->symmetric) return inner_cg<T>(pl, V, -1.0, Wout, p);
  return inner_bicgstab<T>(pl, transpose, V, -1.0, Wout, p);
}

// -------------------------------------------------------------------------
// Toeplitz operator (FFT circulant embedding) and Gohberg-Semencul inverse

// Radices of a length-L transform: 512s and 64s (one pass doing three or
// two radix-8 stages in LDS), 8s, then 4 or 2 for the rest of the power of
// two, then 5s and 3s; empty when L has another prime factor.
std::vector<int> fft_radices(int64_t L) {
  std::vector<int> r;
  for (int R : {512, 64, 8, 4, 2, 5, 3})
    while (L % R == 0) {
      r.push_back(R);
      L /= R;
    }
  if (L != 1) r.clear();
  return r;
}

int stream_grid(int64_t items) {
  return int(std::max<int64_t>(1, std::min<int64_t>(4096, (items + kThreads - 1) / kThreads)));
}

// out = DFT(in) over L rows for q columns (sign -1 forward, +1 inverse,
// unnormalised); in, out and tmp distinct; L = the product of radices.
void fft_len(expmv_plan_s* pl, int64_t L, const std::vector<int>& radices, const cplx* in,
             cplx* out, cplx* tmp, int q, double sign) {
  const int np = int(radices.size());
  const cplx* src = in;
  int64_t Ns = 1;
  for (int i = 0; i < np; ++i) {
    cplx* dst = ((np - 1 - i) % 2 == 0) ? out : tmp;
    const int R = radices[i];
    const int grid = stream_grid((L / R) * q);
    if (R == 512)
      hipLaunchKernelGGL(k_fft_pass512, dim3(int(std::min<int64_t>(16384, ((L / 512) * q + 7) / 8))),
                         dim3(kFft512Threads), 0, pl->stream, L, q, Ns, src, dst, sign);
    else if (R == 64)
      hipLaunchKernelGGL(k_fft_pass64, dim3(int(std::min<int64_t>(8192, ((L / 64) * q + 63) / 64))),
                         dim3(kFft64Threads), 0, pl->stream, L, q, Ns, src, dst, sign);
    else if (R == 8)
      hipLaunchKernelGGL(k_fft_pass<8>, dim3(grid), dim3(kThreads), 0, pl->stream, L, q, Ns, src, dst, sign);
    else if (R == 4)
      hipLaunchKernelGGL(k_fft_pass<4>, dim3(grid), dim3(kThreads), 0, pl->stream, L, q, Ns, src, dst, sign);
    else if (R == 5)
      hipLaunchKernelGGL(k_fft_pass<5>, dim3(grid), dim3(kThreads), 0, pl->stream, L, q, Ns, src, dst, sign);
    else if (R == 3)
      hipLaunchKernelGGL(k_fft_pass<3>, dim3(grid), dim3(kThreads), 0, pl->stream, L, q, Ns, src, dst, sign);
    else
      hipLaunchKernelGGL(k_fft_pass<2>, dim3(grid), dim3(kThreads), 0, pl->stream, L, q, Ns, src, dst, sign);
    src = dst;
    Ns *= R;
  }
}

// the embedding's transform, length pl->L
void fft(expmv_plan_s* pl, const cplx* in, cplx* out, cplx* tmp, int q, double sign) {
  fft_len(pl, pl->L, pl->radices, in, out, tmp, q, sign);
}

// the call's FFT work arrays must hold q complex columns
void check_fft_buffers(expmv_plan_s* pl, int q) {
  if (q > pl->ws.fq) throw StatusError{EXPMV_EINVAL};
}

// Y (n x p, ld) (+)= scale * (K / t) X through the circulant embedding, K / t
// = diag(d) T, or T^T diag(d) when transposed (with_diag = false: T, T^T)
template <typename T>
void toeplitz_apply(expmv_plan_s* pl, const T* X, int64_t ldx, T* Y, int64_t ldy, int p,
                    double scale, int accumulate, int transpose, bool with_diag) {
  const cplx* sym = (transpose && !pl->tsym) ? pl->chatT.p : pl->chat.p;
  const double* dg = with_diag ? pl->tdiag.p : nullptr;
  const int q = (p + 1) / 2;
  check_fft_buffers(pl, q);
  const int64_t L = pl->L, n = pl->n;
  cplx *A = pl->ws.fb[0], *Bf = pl->ws.fb[1], *C = pl->ws.fb[2];
  hipStream_t s = pl->stream;
  hipLaunchKernelGGL((k_pack<T>), dim3(stream_grid(L * q)), dim3(kThreads), 0, s, n, p, ldx, q, L,
                     X, A, 0, 1.0, transpose ? dg : nullptr);
  fft(pl, A, Bf, C, q, -1.0);
  hipLaunchKernelGGL(k_spec_mul, dim3(stream_grid(L * q)), dim3(kThreads), 0, s, L, q, Bf, sym,
                     scale / double(L));
  fft(pl, Bf, A, C, q, +1.0);
  hipLaunchKernelGGL((k_unpack<T>), dim3(stream_grid(n * p)), dim3(kThreads), 0, s, n, p, ldy, q, A,
                     Y, 0, 1.0, accumulate, transpose ? nullptr : dg);
}

// W = scale * T^{-1} V (or T^{-T} V) in the length-n form of the
// Gohberg-Semencul formula.  T^{-1} - Z_1 T^{-1} Z_{-1}^T = (x (Jy)^T -
// (Z_1 y)(Z_{-1} J x)^T) / x0, with Z_1 the cyclic and Z_{-1} the skew-cyclic
// down-shift, so (the displacement of T^{-1} by a circulant and a
// skew-circulant shift determines it)
//   T^{-1} = (1/(2 x0)) (C(x) S(Jy)^T - C(Z_1 y) S(Z_{-1} J x)^T),
//   T^{-T} = (1/(2 x0)) (S(Jy) C(x)^T - S(Z_{-1} J x) C(Z_1 y)^T),
// C(g) the circulant and S(h) the skew-circulant with first column g, h;
// x = T^{-1} e_1, y = T^{-1} e_n (the remark on fast Toeplitz inverses in
// Section 2).  With F the DFT, D = diag(exp(i pi k / n)):
//   C(g) u = F^{-1} (F g . F u),        C(g)^T u = F^{-1} (rev(F g) . F u),
//   S(h) u = D^{-1} F^{-1} (F D h . F D u),
//   S(h)^T u = D F^{-1} (rev(F D h) . F D^{-1} u),   rev(s)_k = s_{-k mod n}.
// Six length-n FFTs per block (two real columns per complex column: every
// factor is a real matrix, so it maps a + i b to its images of a and b).
template <typename T>
void toeplitz_gsf_n(expmv_plan_s* pl, int transpose, const T* V, T* W, int p, double scale) {
  const bool tr = transpose && !pl->tsym;
  const double* di = pl->tdinv.p;
  const int q = (p + 1) / 2;
  check_fft_buffers(pl, q);
  const int64_t n = pl->n;
  const std::vector<int>& rad = pl->radices_n;
  cplx *A = pl->ws.fb[0], *Bf = pl->ws.fb[1], *C = pl->ws.fb[2], *D = pl->ws.fb[3];
  hipStream_t s = pl->stream;
  const int g = stream_grid(n * q);
  const double inv = 1.0 / double(n);
  // the first factor pair: spectra applied reversed (transposed factors)
  const cplx* f1 = tr ? pl->ncx.p : pl->nsj.p;
  const cplx* f2 = tr ? pl->ncz.p : pl->nsz.p;
  // the second pair
  const cplx* g1 = tr ? pl->nsj.p : pl->ncx.p;
  const cplx* g2 = tr ? pl->nsz.p : pl->ncz.p;
  // A = V (rows scaled by 1/d in the forward product), twisted by D^{-1}
  // for the skew-circulant S(.)^T that acts first in T^{-1}
  hipLaunchKernelGGL((k_pack_twist<T>), dim3(g), dim3(kThreads), 0, s, n, p, int64_t(p), q, V,
                     A, 1.0, transpose ? nullptr : di, tr ? 0.0 : -1.0);
  fft_len(pl, n, rad, A, Bf, C, q, -1.0);
  hipLaunchKernelGGL(k_spec_mul_rev_to, dim3(g), dim3(kThreads), 0, s, n, q, Bf, f1, C, inv);
  hipLaunchKernelGGL(k_spec_mul_rev_to, dim3(g), dim3(kThreads), 0, s, n, q, Bf, f2, D, inv);
  fft_len(pl, n, rad, C, A, Bf, q, +1.0);
  fft_len(pl, n, rad, D, C, Bf, q, +1.0);
  // D u: closes S(.)^T (forward) or opens S(.) (transposed)
  hipLaunchKernelGGL(k_twist, dim3(g), dim3(kThreads), 0, s, n, q, A, 1.0);
  hipLaunchKernelGGL(k_twist, dim3(g), dim3(kThreads), 0, s, n, q, C, 1.0);
  fft_len(pl, n, rad, A, Bf, D, q, -1.0);
  fft_len(pl, n, rad, C, A, D, q, -1.0);
  hipLaunchKernelGGL(k_spec_mul2, dim3(g), dim3(kThreads), 0, s, n, q, Bf, g1, A, g2, D, inv);
  fft_len(pl, n, rad, D, Bf, C, q, +1.0);
  // D^{-1} closes S(.) (transposed); rows scaled by 1/d after T^{-T}
  hipLaunchKernelGGL((k_unpack_twist<T>), dim3(stream_grid(n * p)), dim3(kThreads), 0, s, n, p,
                     int64_t(p), q, Bf, W, scale / (2.0 * pl->x0), transpose ? di : nullptr,
                     tr ? -1.0 : 0.0);
}

// W = scale * T^{-1} V (or T^{-T} V) by the Gohberg-Semencul formula
//   T^{-1} = (1/x0) (L(x) L(Jy)^T - L(Zy) L(ZJx)^T),
//   T^{-T} = (1/x0) (L(Jy) L(x)^T - L(ZJx) L(Zy)^T),
// x = T^{-1} e_1, y = T^{-1} e_n (symmetric T: y = J x), L(h)^T v =
// rev(L(h) rev(v)); with spectra a1, a2 for the two transposed factors and
// b1, b2 for the lower ones: W = (L(b1) L(a1)^T - L(b2) L(a2)^T) V / x0.
// Six length-L FFTs per block.  With A = -diag(d) T the inverse of K / t is
// T^{-1} diag(1/d) (1/d scales V's rows on packing), transposed
// diag(1/d) T^{-T} (1/d scales W's rows on unpacking).
template <typename T>
void toeplitz_gsf(expmv_plan_s* pl, int transpose, const T* V, T* W, int p, double scale) {
  if (pl->gsf_n) {
    toeplitz_gsf_n<T>(pl, transpose, V, W, p, scale);
    return;
  }
  const bool tr = transpose && !pl->tsym;
  const cplx* gx = pl->xhat.p;                                // x
  const cplx* gzjx = pl->yhat.p;                              // Z J x
  const cplx* gjy = pl->tsym ? pl->xhat.p : pl->jyhat.p;       // J y
  const cplx* gzy = pl->tsym ? pl->yhat.p : pl->zyhat.p;       // Z y
  const double* di = pl->tdinv.p;
  const cplx* a1 = tr ? gx : gjy;
  const cplx* a2 = tr ? gzy : gzjx;
  const cplx* b1 = tr ? gjy : gx;
  const cplx* b2 = tr ? gzjx : gzy;
  const int q = (p + 1) / 2;
  check_fft_buffers(pl, q);
  const int64_t L = pl->L, n = pl->n;
  cplx *A = pl->ws.fb[0], *Bf = pl->ws.fb[1], *C = pl->ws.fb[2], *D = pl->ws.fb[3];
  hipStream_t s = pl->stream;
  const int g = stream_grid(L * q);
  const double inv = 1.0 / double(L);
  hipLaunchKernelGGL((k_pack<T>), dim3(g), dim3(kThreads), 0, s, n, p, int64_t(p), q, L, V, A, 1,
                     1.0, transpose ? nullptr : di);
  fft(pl, A, Bf, C, q, -1.0);                                   // B = F rev(V)
  hipLaunchKernelGGL(k_spec_mul_to, dim3(g), dim3(kThreads), 0, s, L, q, Bf, a1, C, inv);
  hipLaunchKernelGGL(k_spec_mul_to, dim3(g), dim3(kThreads), 0, s, L, q, Bf, a2, D, inv);
  fft(pl, C, A, Bf, q, +1.0);                                   // A = L(a1) rev(V)
  hipLaunchKernelGGL(k_rev_trunc, dim3(g), dim3(kThreads), 0, s, L, n, q, A, C, 1.0);  // C = L(a1)^T V
  fft(pl, D, A, Bf, q, +1.0);                                   // A = L(a2) rev(V)
  hipLaunchKernelGGL(k_rev_trunc, dim3(g), dim3(kThreads), 0, s, L, n, q, A, D, 1.0);  // D = L(a2)^T V
  fft(pl, C, A, Bf, q, -1.0);                                   // A = F C
  fft(pl, D, C, Bf, q, -1.0);                                   // C = F D
  hipLaunchKernelGGL(k_spec_mul2, dim3(g), dim3(kThreads), 0, s, L, q, A, b1, C, b2, Bf, inv);
  fft(pl, Bf, A, C, q, +1.0);
  hipLaunchKernelGGL((k_unpack<T>), dim3(stream_grid(n * p)), dim3(kThreads), 0, s, n, p,
                     int64_t(p), q, A, W, 0, scale / pl->x0, 0, transpose ? di : nullptr);
}

// zero `bytes` bytes (a multiple of 4) of device memory on the plan's stream
void zero_device(expmv_plan_s* pl, void* ptr, size_t bytes) {
  const int64_t words = int64_t(bytes / 4);
  const int grid = int(std::max<int64_t>(1, std::min<int64_t>(2048, (words + kThreads - 1) / kThreads)));
  hipLaunchKernelGGL(k_zero32, dim3(grid), dim3(kThreads), 0, pl->stream, words,
                     reinterpret_cast<uint32_t*>(ptr));
}

double device_dot(expmv_plan_s* pl, int64_t len, const double* x, const double* y) {
  const int grid = 256;
  hipLaunchKernelGGL(k_dot_partial, dim3(grid), dim3(kThreads), 0, pl->stream, len, x, y,
                     pl->ws.partial);
  std::vector<double> part(grid);
  HIPCHK(hipMemcpyAsync(part.data(), pl->ws.partial, sizeof(double) * grid,
                        hipMemcpyDeviceToHost, pl->stream));
  HIPCHK(hipStreamSynchronize(pl->stream));
  double acc = 0.0;
  for (double v : part) acc += v;
  return acc;
}

// -------------------------------------------------------------------------
// block Gram-Schmidt (two passes) + CholQR2

struct OrthLaunch {
  int TR;
  int64_t rows_per_wg;
  int nwg;
  size_t lds;
};

OrthLaunch orth_config(int64_t n, int p, int npan, int O, size_t elem) {
  OrthLaunch L;
  int TR = 32;
  auto lds_for = [&](int tr) {
    return size_t(O) * 8 + size_t(tr) * (size_t(npan) * p + 2 * p) * elem;
  };
  while (TR > 1 && lds_for(TR) > 150 * 1024) TR /= 2;
  L.TR = TR;
  const int64_t tiles = (n + TR - 1) / TR;
  const int64_t nwg = std::min<int64_t>(256, tiles);
  const int64_t tiles_per = (tiles + nwg - 1) / nwg;
  L.rows_per_wg = tiles_per * TR;
  L.nwg = int((n + L.rows_per_wg - 1) / L.rows_per_wg);
  L.lds = lds_for(TR);
  return L;
}

// Workgroups of a matrix-core Gram-Schmidt pass: as many as the CUs hold at
// once by the kernel's LDS, up to three per CU (its registers allow three
// waves per SIMD), and no more than the 64-row steps; a second generation
// of workgroups would only start once the first had finished its rows.
int orth_mma_grid(size_t lds, int64_t steps) {
  const int per_cu = int(std::max<size_t>(1, std::min<size_t>(3, kLdsPerCU / lds)));
  return int(std::max<int64_t>(1, std::min<int64_t>(int64_t(kCUs) * per_cu, steps)));
}

// One streaming pass; returns the number of workgroups whose partials are
// in ws.partial (0 when the mode writes no partials).
template <typename T>
int orth_pass(expmv_plan_s* pl, int mode, int p, const T* V, int npan, const T* Win, T* Wout,
              const double* C, const int* gate = nullptr) {
  const bool proj = (mode == kProj || mode == kUpdProj);
  const bool gram = (mode == kUpdGram || mode == kScaleGram);
  const bool use_v = (mode == kProj || mode == kUpdProj || mode == kUpdGram);
  const int npv = use_v ? npan : 0;
  const int O = proj ? npv * p * p + (mode == kProj ? p : 0) : (gram ? p * p : 0);
  // matrix-core path: up to 32 column blocks of 16 (4 waves x MBW)
  const int nmb = (npv * p + 15) / 16;
  if (p <= 32 && nmb <= 32) {
    const int64_t steps = (pl->n + 63) / 64;
    int grid = 1;
    const int NB = (p + 15) / 16;
    const int MBW = nmb <= 8 ? 2 : (nmb <= 16 ? 4 : (nmb <= 24 ? 6 : 8));
    const bool upd = (mode == kUpdProj || mode == kUpdGram);
    // timed bytes: the panels of V used and W read once, W' written (all
    // modes but the projection); the conditional third pass is not timed
    KtEv ev;
    if (!gate) {
      const double el = double(sizeof(T)) * double(pl->n) * p;
      ev = kt_take(pl, EXPMV_KT_ORTH, el * (mode == kProj ? npv + 1 : (upd ? npv + 2 : 2)));
    }
    hipEvent_t e0 = ev.e0, e1 = ev.e1;
#define ORTH_MMA(NB_, MBW_)                                                                     \
  do {                                                                                          \
    grid = orth_mma_grid(orth_mma_lds<T, NB_, MBW_>(), steps);                                  \
    if (p == 16 * NB_)                                                                          \
      hipExtLaunchKernelGGL((k_orth_mma<T, NB_, MBW_, 16 * NB_>), dim3(grid), dim3(kThreads), 0, \
                            pl->stream, e0, e1, 0, mode, pl->n, p, V, npv, Win, Wout, C,        \
                            pl->ws.partial, gate);                                             \
    else                                                                                        \
      hipExtLaunchKernelGGL((k_orth_mma<T, NB_, MBW_, 0>), dim3(grid), dim3(kThreads), 0,        \
                            pl->stream, e0, e1, 0, mode, pl->n, p, V, npv, Win, Wout, C,        \
                            pl->ws.partial, gate);                                             \
  } while (0)
    if (NB == 1) {
      if (MBW == 2) ORTH_MMA(1, 2);
      else if (MBW == 4) ORTH_MMA(1, 4);
      else if (MBW == 6) ORTH_MMA(1, 6);
      else ORTH_MMA(1, 8);
    } else {
      if (MBW == 2) ORTH_MMA(2, 2);
      else if (MBW == 4) ORTH_MMA(2, 4);
      else if (MBW == 6) ORTH_MMA(2, 6);
      else ORTH_MMA(2, 8);
    }
#undef ORTH_MMA
    return (proj || gram) ? grid : 0;
  }
  OrthLaunch L = orth_config(pl->n, p, npv, O, sizeof(T));
  HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_orth<T>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(L.lds)));
  hipLaunchKernelGGL(k_orth<T>, dim3(L.nwg), dim3(kThreads), L.lds, pl->stream, mode, pl->n, p, V,
                     npv, Win, Wout, C, pl->ws.partial, L.TR, L.rows_per_wg, gate);
  return (proj || gram) ? L.nwg : 0;
}

void reduce_partials(expmv_plan_s* pl, int nwg, int O, double* out, double* H, int ldh, int col0,
                     int p, int O_h) {
  const int grid = (O + kRedOut - 1) / kRedOut;
  hipLaunchKernelGGL(k_reduce_partials, dim3(grid), dim3(kRedOut * kRedLanes), 0, pl->stream,
                     pl->ws.partial, nwg, O, out, H, ldh, col0, p, O_h);
}

// FP64 true residuals R_j = B - (M - tau_j I) X_j of the 7 shifted systems of
// one time block (X block Xq, poles tau_re/tau_im), their coordinates
// S_j = V_last^T R_j on the block that follows the basis (written to S,
// p x p complex each: the refined restart right-hand sides), and the norms
// res[j] = ||R_j||_F, rem[j] = ||R_j - V_last S_j||_F.  Algorithm 2, Step 4
// with the residual of eq. 4.8 recomputed from X_j.
template <typename T>
void shift_residuals(expmv_plan_s* pl, int transpose, const double* B, int p, const double* Xq,
                     int ldx, const double* tau_re, const double* tau_im, const T* Vlast, cplx* S,
                     double* res, double* rem) {
  Workspace& w = pl->ws;
  hipStream_t s = pl->stream;
  const int64_t n = pl->n;
  const int W = 2 * kNShift * p;
  double* R = w.Rres;
  const int PP = pow2_lanes(p);
  const int g1 = grid_for(n, PP, 512);
  double* part1 = w.rpart;                     // g1 x 7
  double* part3 = w.rpart + 512 * kNShift;     // kResGrid x 7
  if (pl->kind == 0) {
    Csr<double> A = csr_of<double>(pl, transpose);
    DISPATCH_PP(PP, hipLaunchKernelGGL((k_shift_residual<P_>), dim3(g1), dim3(kThreads), 0, s, n,
                                       p, A.rowptr, A.colind, A.val, nullptr, B, Xq, ldx, tau_re,
                                       tau_im, R, part1));
  } else {
    // K X_j by the FFT product into R, then R = B + K X + tau X in place
    for (int j = 0; j < kNShift; ++j)
      toeplitz_apply<double>(pl, Xq + 2 * p * j, ldx, R + 2 * p * j, W, 2 * p, pl->t, 0, transpose);
    DISPATCH_PP(PP, hipLaunchKernelGGL((k_shift_residual<P_>), dim3(g1), dim3(kThreads), 0, s, n,
                                       p, nullptr, nullptr, nullptr, R, B, Xq, ldx, tau_re, tau_im,
                                       R, part1));
  }
  const int g2 = int(std::max<int64_t>(1, std::min<int64_t>(kResGrid, n / 64)));
  DISPATCH_PP(PP, hipLaunchKernelGGL((k_project_block<T, P_>), dim3(g2), dim3(kThreads), 0, s, n, p,
                                     Vlast, R, W, w.partial));
  reduce_partials(pl, g2, p * W, w.projC, nullptr, 0, 0, p, 0);
  DISPATCH_PP(PP, hipLaunchKernelGGL((k_remainder_norms<T, P_>), dim3(g2), dim3(kThreads), 0, s, n,
                                     p, Vlast, R, W, w.projC, part3));
  hipLaunchKernelGGL(k_restart_rhs, dim3((kNShift * p * p + kThreads - 1) / kThreads),
                     dim3(kThreads), 0, s, p, w.projC, W, S);
  std::vector<double> h(size_t(512 + kResGrid) * kNShift);
  HIPCHK(hipMemcpyAsync(h.data(), w.rpart, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int j = 0; j < kNShift; ++j) {
    double a = 0.0, b = 0.0;
    for (int g = 0; g < g1; ++g) a += h[size_t(g) * kNShift + j];
    for (int g = 0; g < g2; ++g) b += h[size_t(512 + g) * kNShift + j];
    res[j] = std::sqrt(a);
    rem[j] = std::sqrt(b);
  }
}

// Orthonormalise W (n x p) against panels 0..npan-1 of Vb (two block
// Gram-Schmidt passes), then CholQR2; the result goes to Vout.
//   H != nullptr: H(0:npan*p, col0:col0+p) += coefficients of both passes,
//                 H(npan*p:npan*p+p, col0:col0+p) = R2 R1.
//   H == nullptr: Rhat (p x p) = R2 R1 (initial block, npan = 0).
// Projections, Gram matrices and R are FP64 for either working type.
template <typename T>
void orthonormalize(expmv_plan_s* pl, int p, const T* Vb, int npan, T* W, T* Vout, double* H,
                    int ldh, int col0, double* Rhat) {
  Workspace& w = pl->ws;
  hipStream_t s = pl->stream;
  const int Oc = npan * p * p;
  T* Wt = reinterpret_cast<T*>(w.Wt);
  if (npan > 0) {
    int nwg = orth_pass<T>(pl, kProj, p, Vb, npan, W, nullptr, nullptr);
    // coefficients of pass 1, then ||W(:,b)||^2 in hcoef[Oc..Oc+p)
    reduce_partials(pl, nwg, Oc + p, w.hcoef, H, ldh, col0, p, Oc);
    nwg = orth_pass<T>(pl, kUpdProj, p, Vb, npan, W, Wt, w.hcoef);
    reduce_partials(pl, nwg, Oc, w.w0 + p, H, ldh, col0, p, Oc);
    HIPCHK(hipMemcpyAsync(w.w0, w.hcoef + Oc, sizeof(double) * p, hipMemcpyDeviceToDevice, s));
    nwg = orth_pass<T>(pl, kUpdGram, p, Vb, npan, Wt, Wt, w.w0 + p);
    reduce_partials(pl, nwg, p * p, w.gram, nullptr, 0, 0, p, 0);
  } else {
    int nwg = orth_pass<T>(pl, kUpdGram, p, static_cast<const T*>(nullptr), 0, W, Wt, nullptr);
    reduce_partials(pl, nwg, p * p, w.gram, nullptr, 0, 0, p, 0);
  }
  // shift of the fallback (shifted Cholesky QR): 11 (n p + p (p + 1)) u
  // times trace(G), u = 2^-53 (the Gram matrices are FP64)
  const double shift_rel = 11.0 * (double(pl->n) * p + double(p) * (p + 1)) * 0x1p-53;
  hipLaunchKernelGGL(k_cholqr_factor, dim3(1), dim3(64), 0, s, p, w.gram, w.R1, w.Rinv,
                     npan > 0 ? w.w0 : nullptr, 1, nullptr, nullptr, 0, 0, 0, shift_rel,
                     w.flags);
  int nwg = orth_pass<T>(pl, kScaleGram, p, static_cast<const T*>(nullptr), 0, Wt, Wt, w.Rinv);
  reduce_partials(pl, nwg, p * p, w.gram, nullptr, 0, 0, p, 0);
  double* Hb = H != nullptr ? H : Rhat;
  const int ldb = H != nullptr ? ldh : p;
  const int hr = H != nullptr ? npan * p : 0, hc = H != nullptr ? col0 : 0;
  hipLaunchKernelGGL(k_cholqr_factor, dim3(1), dim3(64), 0, s, p, w.gram, w.R2, w.Rinv,
                     nullptr, 2, w.R1, Hb, ldb, hr, hc, 0.0, w.flags);
  // third pass, only after a shifted first factor (flags[2]; the kernels
  // return at once otherwise)
  const int* gate = w.flags + 2;
  nwg = orth_pass<T>(pl, kScaleGram, p, static_cast<const T*>(nullptr), 0, Wt, Wt, w.Rinv, gate);
  reduce_partials(pl, nwg, p * p, w.gram, nullptr, 0, 0, p, 0);
  hipLaunchKernelGGL(k_cholqr_factor, dim3(1), dim3(64), 0, s, p, w.gram, w.R1, w.Rinv,
                     nullptr, 3, nullptr, Hb, ldb, hr, hc, 0.0, w.flags);
  orth_pass<T>(pl, kScale, p, static_cast<const T*>(nullptr), 0, Wt, Vout, w.Rinv);
}

template <typename T, typename TO>
void panel_gemm(expmv_plan_s* pl, int p, const T* V, int npan, const double* C, int ldc,
                int nchunks, TO* out, int64_t chunk_stride, int64_t ldo, int accumulate) {
  const int np_cols = npan * p;
  // matrix-core path: output columns in 16-wide blocks spread over 4 waves
  const int nout = nchunks * p;
  const int nnb = (nout + 15) / 16;
  if (nnb <= 32) {
    const int NBW = (nnb + 3) / 4;
    const int RB = NBW <= 2 ? 4 : (NBW <= 4 ? 2 : 1);
    const int64_t steps = (pl->n + 16 * RB - 1) / (16 * RB);
    const int grid = int(std::max<int64_t>(1, std::min<int64_t>(2048, steps)));
#define PG_MMA(NBW_, RB_)                                                                         \
  do {                                                                                            \
    if (p == 16)                                                                                  \
      hipLaunchKernelGGL((k_panel_gemm_mma<T, TO, NBW_, RB_, 16>), dim3(grid), dim3(kThreads), 0,  \
                         pl->stream, pl->n, p, V, npan, C, ldc, nout, out, chunk_stride, ldo,     \
                         accumulate);                                                             \
    else                                                                                          \
      hipLaunchKernelGGL((k_panel_gemm_mma<T, TO, NBW_, RB_>), dim3(grid), dim3(kThreads), 0,      \
                         pl->stream, pl->n, p, V, npan, C, ldc, nout, out, chunk_stride, ldo,     \
                         accumulate);                                                             \
  } while (0)
    if (NBW <= 1) PG_MMA(1, 4);
    else if (NBW <= 2) PG_MMA(2, 4);
    else if (NBW <= 4) PG_MMA(4, 2);
    else PG_MMA(8, 1);
#undef PG_MMA
    return;
  }
  int TR = 32;
  auto lds_for = [&](int tr) {
    return size_t(np_cols) * p * 8 + size_t(tr) * np_cols * sizeof(T);
  };
  while (TR > 1 && lds_for(TR) > 150 * 1024) TR /= 2;
  const int64_t n = pl->n;
  const int64_t tiles = (n + TR - 1) / TR;
  const int64_t nwg = std::min<int64_t>(512, tiles);
  const int64_t rows_per_wg = ((tiles + nwg - 1) / nwg) * TR;
  const int grid = int((n + rows_per_wg - 1) / rows_per_wg);
  const size_t lds = lds_for(TR);
  HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_panel_gemm<T, TO>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  hipLaunchKernelGGL((k_panel_gemm<T, TO>), dim3(grid, nchunks), dim3(kThreads), lds, pl->stream, n,
                     p, V, npan, C, ldc, out, chunk_stride, ldo, accumulate, TR, rows_per_wg);
}

double host_now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// -------------------------------------------------------------------------
// restart step on the host (Algorithm 1, Steps 5-8)

// Modified Gram-Schmidt (twice) on the columns of P (d x k row-major).
// Returns the number of independent columns kept (dependent ones dropped).
int host_orthonormalize_columns(int d, int k, std::vector<double>& P) {
  int kept = 0;
  std::vector<double> out(size_t(d) * k, 0.0);
  for (int c = 0; c < k; ++c) {
    std::vector<double> v(d);
    for (int i = 0; i < d; ++i) v[i] = P[size_t(i) * k + c];
    double n0 = 0.0;
    for (double x : v) n0 += x * x;
    n0 = std::sqrt(n0);
    for (int pass = 0; pass < 2; ++pass)
      for (int q = 0; q < kept; ++q) {
        double h = 0.0;
        for (int i = 0; i < d; ++i) h += out[size_t(i) * k + q] * v[i];
        for (int i = 0; i < d; ++i) v[i] -= h * out[size_t(i) * k + q];
      }
    double nv = 0.0;
    for (double x : v) nv += x * x;
    nv = std::sqrt(nv);
    if (!(nv > 1e-10 * n0)) continue;
    for (int i = 0; i < d; ++i) out[size_t(i) * k + kept] = v[i] / nv;
    ++kept;
  }
  P = out;
  return kept;
}

struct RitzBasis {
  std::vector<double> Pk;   // dlive x keff, row-major, orthonormal columns
  int keff = 0;
};

// The k wanted Ritz vectors of Hd (dlive x dlive): largest |theta| for
// Algorithm 2 (Remark 4.1), smallest for Algorithm 1; a complex pair is kept
// whole (real and imaginary parts), so keff may be k + 1.
RitzBasis ritz_basis(bool symmetric, bool precond, int dl, const std::vector<double>& Hd, int k) {
  RitzBasis rb;
  std::vector<int> ord(dl);
  std::iota(ord.begin(), ord.end(), 0);
  if (symmetric) {
    std::vector<double> wv(dl), Q(size_t(dl) * dl);
    // an unconverged eigen-decomposition would give a restart basis that is
    // not the Ritz basis of Step 5: the solve stops with a breakdown
    if (!sym_eig(dl, Hd.data(), wv.data(), Q.data())) throw StatusError{EXPMV_EBREAKDOWN};
    auto key = [&](int a) { return std::fabs(wv[a]); };
    if (precond) std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return key(a) > key(b); });
    else std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return key(a) < key(b); });
    rb.keff = std::min(k, dl);
    rb.Pk.assign(size_t(dl) * rb.keff, 0.0);
    for (int c = 0; c < rb.keff; ++c)
      for (int i = 0; i < dl; ++i) rb.Pk[size_t(i) * rb.keff + c] = Q[size_t(i) * dl + ord[c]];
    return rb;
  }
  std::vector<double> wr(dl), wi(dl), Vr(size_t(dl) * dl), Vi(size_t(dl) * dl);
  HessForm hf;
  if (!general_eigvals(dl, Hd.data(), wr.data(), wi.data(), &hf)) throw StatusError{EXPMV_EBREAKDOWN};
  auto mag = [&](int a) { return std::hypot(wr[a], wi[a]); };
  if (precond) std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return mag(a) > mag(b); });
  else std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return mag(a) < mag(b); });
  {
    // eigenvectors only of the Ritz values kept (one per conjugate pair)
    std::vector<char> want(dl, 0), seen(dl, 0);
    int chosen = 0;
    for (int idx : ord) {
      if (chosen >= k) break;
      if (seen[idx]) continue;
      seen[idx] = 1;
      want[idx] = 1;
      ++chosen;
      if (wi[idx] != 0.0) {
        for (int j = 0; j < dl; ++j)
          if (!seen[j] && wr[j] == wr[idx] && wi[j] == -wi[idx]) {
            seen[j] = 1;
            break;
          }
        ++chosen;
      }
    }
    general_eigvecs(dl, Hd.data(), wr.data(), wi.data(), want.data(), Vr.data(), Vi.data(), &hf);
  }
  std::vector<char> taken(dl, 0);
  std::vector<std::vector<double>> cols;
  int chosen = 0;
  for (int idx : ord) {
    if (chosen >= k) break;
    if (taken[idx]) continue;
    taken[idx] = 1;
    std::vector<double> re(dl), im(dl);
    for (int i = 0; i < dl; ++i) {
      re[i] = Vr[size_t(i) * dl + idx];
      im[i] = Vi[size_t(i) * dl + idx];
    }
    cols.push_back(re);
    ++chosen;
    if (wi[idx] != 0.0) {
      // the conjugate partner: exact pair from general_eig
      for (int j = 0; j < dl; ++j)
        if (!taken[j] && wr[j] == wr[idx] && wi[j] == -wi[idx]) {
          taken[j] = 1;
          break;
        }
      cols.push_back(im);
      ++chosen;
    }
  }
  const int kk = int(cols.size());
  std::vector<double> P(size_t(dl) * kk);
  for (int c = 0; c < kk; ++c)
    for (int i = 0; i < dl; ++i) P[size_t(i) * kk + c] = cols[c][i];
  const int kept = host_orthonormalize_columns(dl, kk, P);
  rb.keff = kept;
  rb.Pk.assign(size_t(dl) * kept, 0.0);
  for (int i = 0; i < dl; ++i)
    for (int c = 0; c < kept; ++c) rb.Pk[size_t(i) * kept + c] = P[size_t(i) * kk + c];
  return rb;
}

// Steps 5-8 in the projected coordinates, on the host: from H~ (ldh x ldh,
// row-major, the first d + p rows live) the Ritz basis P_k of its live part
// (every padded coordinate but those after the kept Ritz vectors, keff..kp),
// then H~ is overwritten by P_{k+p}^T H~ P_k (top kn x kn block and the p
// rows of the last block below it, from row kpn).  Pk comes back as d x kpn
// in padded coordinates (zero rows at the padding, zero columns after kn).
struct RestartCoords {
  std::vector<double> Pk;
  int kn = 0, kpn = 0;
};

RestartCoords restart_coordinates(bool symmetric, bool precond, int d, int p, int k, int ldh,
                                  int keff, int kp, std::vector<double>& Hh) {
  std::vector<int> live;
  for (int i = 0; i < d; ++i)
    if (!(i >= keff && i < kp)) live.push_back(i);
  const int dl = int(live.size());
  std::vector<double> Hd(size_t(dl) * dl);
  for (int i = 0; i < dl; ++i)
    for (int j = 0; j < dl; ++j) Hd[size_t(i) * dl + j] = Hh[size_t(live[i]) * ldh + live[j]];
  RitzBasis rb = ritz_basis(symmetric, precond, dl, Hd, k);
  RestartCoords rc;
  const int kn = rb.keff;
  const int kpn = (kn + p - 1) / p * p;
  rc.kn = kn;
  rc.kpn = kpn;
  if (kn < 1) return rc;
  std::vector<double>& Pk = rc.Pk;
  Pk.assign(size_t(d) * kpn, 0.0);
  for (int i = 0; i < dl; ++i)
    for (int c = 0; c < kn; ++c) Pk[size_t(live[i]) * kpn + c] = rb.Pk[size_t(i) * kn + c];
  // H~_new = P_{k+p}^T H~ P_k (both products row by row, inner loops along rows)
  std::vector<double> HP(size_t(d + p) * kn, 0.0);
  for (int i = 0; i < d + p; ++i) {
    double* hp = &HP[size_t(i) * kn];
    for (int j = 0; j < d; ++j) {
      const double h = Hh[size_t(i) * ldh + j];
      if (h == 0.0) continue;
      const double* pk = &Pk[size_t(j) * kpn];
      for (int c = 0; c < kn; ++c) hp[c] += h * pk[c];
    }
  }
  std::fill(Hh.begin(), Hh.end(), 0.0);
  for (int i = 0; i < d; ++i) {
    const double* pk = &Pk[size_t(i) * kpn];
    const double* hp = &HP[size_t(i) * kn];
    for (int r = 0; r < kn; ++r) {
      const double pr = pk[r];
      if (pr == 0.0) continue;
      double* hr = &Hh[size_t(r) * ldh];
      for (int c = 0; c < kn; ++c) hr[c] += pr * hp[c];
    }
  }
  for (int r = 0; r < p; ++r)
    for (int c = 0; c < kn; ++c) Hh[size_t(kpn + r) * ldh + c] = HP[size_t(d + r) * kn + c];
  return rc;
}

// -------------------------------------------------------------------------
// the method

// Preconditioner application between basis type T and inner-solver type TI.
// In the mixed forms each FP32 solve may be followed by rounds of iterative
// refinement: R = V - M W in FP64 with the exact operator, D = M^{-1} R by
// the FP32 solver, W += D.
template <typename T, typename TI>
InnerResult apply_inverse_mixed(expmv_plan_s* pl, int transpose, const T* V, T* Wout, int p) {
  int rounds = 0;
  if (!std::is_same<TI, double>::value && pl->kind == 0)
    rounds = pl->opts.inner_refine >= 0 ? pl->opts.inner_refine : (pl->symmetric ? 0 : 1);
  const int64_t cnt = pl->n * int64_t(p);
  hipStream_t s = pl->stream;
  InnerResult total{0, 0};
  auto accumulate = [&](InnerResult r) {
    total.iters += r.iters;
    total.hit_cap |= r.hit_cap;
  };
  if constexpr (std::is_same<T, TI>::value) {
    accumulate(apply_inverse<T>(pl, transpose, V, Wout, p));
  } else {
    TI* vi = reinterpret_cast<TI*>(pl->ws.Win);
    TI* wi = reinterpret_cast<TI*>(pl->ws.Wout);
    hipLaunchKernelGGL((k_convert<T, TI>), dim3(512), dim3(kThreads), 0, s, cnt, V, vi, 1.0);
    accumulate(apply_inverse<TI>(pl, transpose, vi, wi, p));
    hipLaunchKernelGGL((k_convert<TI, T>), dim3(512), dim3(kThreads), 0, s, cnt, wi, Wout, 1.0);
  }
  if (rounds > 0) {
    Csr<double> A = csr_of<double>(pl, transpose);
    TI* ri = reinterpret_cast<TI*>(pl->ws.Rin);
    TI* di = reinterpret_cast<TI*>(pl->ws.Din);
    const int PP = pow2_lanes(p);
    const int grid = grid_for(pl->n, PP, 4096);
    for (int r = 0; r < rounds; ++r) {
      DISPATCH_PP(PP, hipLaunchKernelGGL((k_refine_residual<T, TI, P_>), dim3(grid), dim3(kThreads),
                                         0, s, int(pl->n), p, A.rowptr, A.colind, A.val, V, Wout,
                                         ri));
      accumulate(apply_inverse<TI>(pl, transpose, ri, di, p));
      hipLaunchKernelGGL((k_add_to<T, TI>), dim3(512), dim3(kThreads), 0, s, cnt, di, Wout);
    }
  }
  return total;
}

// The projected shifted solves (k_proj_solve), one workgroup per shift
void proj_solve(hipStream_t s, int ns, int d, int p, int precond, const double* H, int ldh,
                const double* tau_re, const double* tau_im, const cplx* G, cplx* Ascr, cplx* Zs,
                double* Cr, int ldc, cplx* S, double* rho, int* singular) {
  hipLaunchKernelGGL(k_proj_solve, dim3(ns), dim3(1024), 0, s, d, p, precond, H, ldh, tau_re,
                     tau_im, G, Ascr, Zs, Cr, ldc, S, rho, singular);
}

// Source-term mode: a single time; Z receives
//   U = r(M) U0 + (r(M) - r(sigma)) t (M - sigma I)^{-1} S
//     = omega_0 U0 + Re sum_j c_j (M - tau_j I)^{-1} (U0 + t / (tau_j - sigma) S),
// the solution at time t of u' = A u + e^{gamma s} S, u(0) = U0, with both
// exponentials in the CF form (sigma = gamma t; partial fractions of r).
// B is the joined n x 2p' block [U0 | S] (p = 2p', Z n x p'), or S alone
// when U0 = 0 (s_only: Z = Re sum_j s_j X_j, no omega_0 term).
struct SourceMode {
  double sigma;
  double t;
  bool s_only;
};

// Z_q = r(s_q M) B for the scale factors s_q > 0 of `scales` (M = tA of the
// plan; Z_q is the q-th n x p block of Z).  Since r(s M) B = omega_0 B +
// Re sum_j (c_j / s)(M - (tau_j / s) I)^{-1} B, every time adds 7 shifted
// systems with poles tau_j / s_q on the one Krylov basis of M^{-1}: the
// basis, the inner solves and the restarts are shared, the projected solves
// and the solution updates run over all 7 nt shifts.
template <typename T, typename TI>
expmv_status execute_impl(expmv_plan_s* pl, int transpose, const double* B, int p, double tol,
                          double* Z, expmv_info* info, const std::vector<double>& scales,
                          const SourceMode* src) {
  hipStream_t s = pl->stream;
  Workspace& w = pl->ws;   // bound by the caller for (p, nt)
  const int64_t n = pl->n;
  const int m = pl->opts.m;
  const int ldh = pl->ldh;
  const int kk_opt = pl->opts.k > 0 ? pl->opts.k : p * (m / 3);
  const int k = std::max(p, std::min(kk_opt, (m - 2) * p) / p * p);
  const bool precond = pl->opts.preconditioned != 0;
  const size_t blk = size_t(n) * p;
  const int nt = int(scales.size());
  const int ns = kNShift * nt;   // shifted systems
  const int ldx = 2 * ns * p;
  // poles tau_j / s_q and coefficients c_j / s_q, shift index q * 7 + j
  std::vector<double> tau_h(2 * size_t(ns)), coef_h(2 * size_t(ns));
  for (int q = 0; q < nt; ++q)
    for (int j = 0; j < kNShift; ++j) {
      tau_h[q * kNShift + j] = CF_TAU_RE[j] / scales[q];
      tau_h[ns + q * kNShift + j] = CF_TAU_IM[j] / scales[q];
      coef_h[q * kNShift + j] = CF_C_RE[j] / scales[q];
      coef_h[ns + q * kNShift + j] = CF_C_IM[j] / scales[q];
    }
  HIPCHK(hipMemcpyAsync(w.taus, tau_h.data(), sizeof(double) * tau_h.size(),
                        hipMemcpyHostToDevice, s));
  // source mode: s_j = c_j t / (tau_j - sigma), the coefficients of the S part
  double s_re[kNShift] = {0}, s_im[kNShift] = {0};
  if (src) {
    coef_h.resize(4 * size_t(ns));
    for (int j = 0; j < kNShift; ++j) {
      const std::complex<double> cj(CF_C_RE[j], CF_C_IM[j]), tj(CF_TAU_RE[j], CF_TAU_IM[j]);
      const std::complex<double> sj = cj * src->t / (tj - src->sigma);
      s_re[j] = coef_h[2 * ns + j] = sj.real();
      s_im[j] = coef_h[3 * ns + j] = sj.imag();
    }
  }
  HIPCHK(hipMemcpyAsync(w.coefs, coef_h.data(), sizeof(double) * coef_h.size(),
                        hipMemcpyHostToDevice, s));
  const double* tau_re_d = w.taus;
  const double* tau_im_d = w.taus + ns;
  const double* c_re_d = w.coefs;
  const double* c_im_d = w.coefs + ns;
  const double* s_re_d = w.coefs + 2 * ns;
  const double* s_im_d = w.coefs + 3 * ns;
  const double t_start = host_now_ms();
  expmv_info inf{};
  double ms_apply = 0, ms_orth = 0, ms_small = 0, ms_update = 0;
  {
    KernelTimer& kt = pl->kt;
    kt.used = 0;
    kt.cur_iter = -1;
    kt.sampling = false;
    for (int c = 0; c < EXPMV_KT_COUNT; ++c) {
      kt.ms[c] = kt.by[c] = 0.0;
      kt.cnt[c] = 0;
    }
  }

  // bound weights: |c_j| (source mode: |(c_j, s_j)|, since the two parts'
  // errors E, E' give |c_j E + s_j E'| <= |(c_j, s_j)| ||(E, E')||_F; S
  // alone: |s_j|)
  double cw[kNShift], delta[kNShift];
  for (int j = 0; j < kNShift; ++j) {
    cw[j] = std::hypot(CF_C_RE[j], CF_C_IM[j]);
    if (src && src->s_only) cw[j] = std::hypot(s_re[j], s_im[j]);
    else if (src) cw[j] = std::hypot(cw[j], std::hypot(s_re[j], s_im[j]));
    delta[j] = CF_TAU_RE[j] >= 0.0 ? std::hypot(CF_TAU_RE[j], CF_TAU_IM[j]) : std::fabs(CF_TAU_IM[j]);
  }

  zero_device(pl, w.X, sizeof(double) * size_t(n) * ldx);
  zero_device(pl, w.H, sizeof(double) * size_t(ldh) * ldh);
  zero_device(pl, w.flags, sizeof(int) * 4);
  zero_device(pl, w.singular, sizeof(int) * ns);
  if (pl->opts.inner_relax) zero_device(pl, w.singular2, sizeof(int) * ns);

  const int cgrid = 512;
  std::vector<double> part(size_t(cgrid) * nt);
  // ||B||_F (k_combine with X = 0 and omega0 = 1 writes B to Z and its norm;
  // in source mode Z is narrower than B)
  if (src) {
    inf.bnorm = std::sqrt(device_dot(pl, int64_t(blk), B, B));
  } else {
    hipLaunchKernelGGL(k_combine, dim3(cgrid), dim3(kThreads), 0, s, n, p, B, w.X, ldx, 1.0,
                       c_re_d, c_im_d, Z, w.partial);
    HIPCHK(hipMemcpyAsync(part.data(), w.partial, sizeof(double) * cgrid, hipMemcpyDeviceToHost,
                          s));
    HIPCHK(hipStreamSynchronize(s));
    double bb = 0.0;
    for (int i = 0; i < cgrid; ++i) bb += part[i];
    inf.bnorm = std::sqrt(bb);
  }
  if (!(inf.bnorm > 0.0) || !std::isfinite(inf.bnorm)) {
    if (info) *info = inf;
    return EXPMV_EINVAL;
  }

  int cur = 0;
  T* Vb = reinterpret_cast<T*>(w.V[cur]);
  T* Wk = reinterpret_cast<T*>(w.W);
  // Steps 1-2: V_1 R^ = B
  hipLaunchKernelGGL((k_convert<double, T>), dim3(512), dim3(kThreads), 0, s, int64_t(blk), B, Wk,
                     1.0);
  orthonormalize<T>(pl, p, nullptr, 0, Wk, Vb, nullptr, 0, 0, w.Rhat);

  int d = m * p;          // projected dimension (padded coordinates)
  int kp = 0;             // columns taken by the Ritz block (k_eff rounded up to p)
  int keff = 0;           // live Ritz vectors
  int first_block = 0;    // first panel to expand in this cycle
  expmv_status status = EXPMV_OK;
  std::vector<double> Hh(size_t(ldh) * ldh);
  std::vector<double> rho(ns);
  // relaxed inner solves (opts.inner_relax = c > 0): the inner tolerance of
  // block j grows like rho_0 / rho_{j-1}, capped at 10^c (10^2 in the mixed
  // forms) times the base value
  const bool relax = pl->opts.inner_relax != 0 && precond && pl->kind == 0;
  const double relax_cap =
      std::min(std::pow(10.0, double(pl->opts.inner_relax)), pl->mixed ? 1e2 : 1e12);
  double rho_prev = 0.0;
  bool rhs_from_S = false;
  // Wk = M^{-1} Vj (Algorithm 2; Algorithm 1: M Vj)
  auto apply_block = [&](const T* Vj) {
    if (precond) {
      // relaxed inner tolerance: factor rho_0 / rho_{j-1} (capped), rho the
      // largest residual estimate over the shifts after the previous block
      pl->relax_scale = 1.0;
      if (relax && rho_prev > 0.0)
        pl->relax_scale = std::min(relax_cap, std::max(1.0, inf.bnorm / rho_prev));
      InnerResult r = apply_inverse_mixed<T, TI>(pl, transpose, Vj, Wk, p);
      pl->relax_scale = 1.0;
      inf.inner_iters += r.iters;
      inf.inner_maxit_hit += r.hit_cap;
    } else {
      apply_K<T>(pl, transpose, Vj, Wk, p);
      // M V = -K V
      hipLaunchKernelGGL((k_convert<T, T>), dim3(512), dim3(kThreads), 0, s, int64_t(blk), Wk, Wk,
                         -1.0);
    }
    inf.block_apps += 1;
  };
  bool first_applied = false;   // Wk already holds the first block's product
  int cycle = 0;
  for (;;) {
    ++cycle;
    // Step 3 / Step 9: block Arnoldi on the operator from panel first_block
    for (int jb = first_block; jb < m; ++jb) {
      double t0 = host_now_ms();
      const T* Vj = Vb + size_t(jb) * blk;
      if (!(first_applied && jb == first_block)) apply_block(Vj);
      first_applied = false;
      double t1 = host_now_ms();
      ms_apply += t1 - t0;
      orthonormalize<T>(pl, p, Vb, jb + 1, Wk, Vb + size_t(jb + 1) * blk, w.H, ldh, jb * p,
                        nullptr);
      ms_orth += host_now_ms() - t1;
      if (relax && jb + 1 < m && (jb - first_block) % 2 == 1) {
        // residual estimates of the projected systems on the first jb + 1
        // blocks, after every second block (each is a latency-bound dense
        // solve per shift); scratch outputs: the cycle's own S and Cr stay
        // intact
        const int dj = (jb + 1) * p;
        dim3 g(std::max(1, (dj * p + kThreads - 1) / kThreads), ns);
        hipLaunchKernelGGL(k_build_rhs, g, dim3(kThreads), 0, s, dj, p, rhs_from_S ? kp : 0,
                           rhs_from_S ? 1 : 0, w.Rhat, w.S, w.G);
        proj_solve(s, ns, dj, p, 1, w.H, ldh, tau_re_d, tau_im_d, w.G, w.Ascr, w.Zs,
                   nullptr, ldx, w.S2, w.rho, w.singular2);
        HIPCHK(hipMemcpyAsync(rho.data(), w.rho, sizeof(double) * ns, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        rho_prev = 0.0;
        for (int q = 0; q < ns; ++q) rho_prev = std::max(rho_prev, rho[q]);
        if (!std::isfinite(rho_prev)) rho_prev = 0.0;
      }
    }
    rho_prev = 0.0;
    double t0 = host_now_ms();
    {
      dim3 g(std::max(1, (d * p + kThreads - 1) / kThreads), ns);
      hipLaunchKernelGGL(k_build_rhs, g, dim3(kThreads), 0, s, d, p, rhs_from_S ? kp : 0,
                         rhs_from_S ? 1 : 0, w.Rhat, w.S, w.G);
    }
    // Step 4: projected shifted systems, residual estimates, update coefficients
    proj_solve(s, ns, d, p, precond ? 1 : 0, w.H, ldh, tau_re_d, tau_im_d, w.G, w.Ascr,
               w.Zs, w.Cr, ldx, w.S, w.rho, w.singular);
    double t1 = host_now_ms();
    // X_j += V_{d+p} (H~ Z_j)  [Algorithm 1: V_d Z_j]
    panel_gemm<T, double>(pl, p, Vb, d / p + 1, w.Cr, ldx, 2 * ns, w.X, p, ldx, 1);
    if (src && src->s_only)
      hipLaunchKernelGGL(k_combine, dim3(cgrid), dim3(kThreads), 0, s, n, p, B, w.X, ldx, 0.0,
                         s_re_d, s_im_d, Z, w.partial);
    else if (src)
      hipLaunchKernelGGL(k_combine_source, dim3(cgrid), dim3(kThreads), 0, s, n, p / 2, B, w.X,
                         ldx, double(CF_OMEGA0), c_re_d, c_im_d, s_re_d, s_im_d, Z, w.partial);
    else
      for (int q = 0; q < nt; ++q)
        hipLaunchKernelGGL(k_combine, dim3(cgrid), dim3(kThreads), 0, s, n, p, B,
                           w.X + size_t(2 * kNShift * p) * q, ldx, double(CF_OMEGA0),
                           c_re_d + kNShift * q, c_im_d + kNShift * q, Z + blk * q,
                           w.partial + size_t(cgrid) * q);
    HIPCHK(hipMemcpyAsync(part.data(), w.partial, sizeof(double) * cgrid * nt,
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(rho.data(), w.rho, sizeof(double) * ns, hipMemcpyDeviceToHost, s));
    int flags_h[4];
    HIPCHK(hipMemcpyAsync(flags_h, w.flags, sizeof(int) * 4, hipMemcpyDeviceToHost, s));
    std::vector<int> sing_h(ns);
    HIPCHK(hipMemcpyAsync(sing_h.data(), w.singular, sizeof(int) * ns, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double t2 = host_now_ms();
    ms_small += t1 - t0;
    ms_update += t2 - t1;
    // Step 4 in FP64: the true residuals of the shifted systems, recomputed
    // from X_j; with opts.restart_refine their coordinates on the block after
    // the basis are the next cycle's right-hand sides (refinement)
    const T* Vlast = Vb + size_t(d / p) * blk;
    cplx* Sdst = pl->opts.restart_refine ? w.S : w.Sref;
    std::vector<double> zn_q(nt);
    for (int q = 0; q < nt; ++q) {
      double zz = 0.0;
      for (int i = 0; i < cgrid; ++i) zz += part[size_t(cgrid) * q + i];
      zn_q[q] = std::sqrt(zz);
    }
    double res_bound = 0.0, rem_bound = 0.0;
    for (int j = 0; j < kNShift; ++j) inf.true_res[j] = inf.noncollinear[j] = 0.0;
    for (int q = 0; q < nt; ++q) {
      double res[kNShift], rem[kNShift];
      shift_residuals<T>(pl, transpose, B, p, w.X + size_t(2 * kNShift * p) * q, ldx,
                         tau_re_d + kNShift * q, tau_im_d + kNShift * q, Vlast,
                         Sdst + size_t(kNShift) * p * p * q, res, rem);
      double rb = 0.0, nb = 0.0;
      for (int j = 0; j < kNShift; ++j) {
        inf.true_res[j] = std::max(inf.true_res[j], res[j]);
        inf.noncollinear[j] = std::max(inf.noncollinear[j], rem[j]);
        rb += cw[j] * res[j] / delta[j];
        nb += cw[j] * rem[j] / delta[j];
      }
      const double zn = zn_q[q] > 0.0 ? zn_q[q] : 1.0;
      res_bound = std::max(res_bound, rb / zn);
      rem_bound = std::max(rem_bound, nb / zn);
    }
    inf.true_bound = res_bound;
    inf.noncollinear_bound = rem_bound;
    ms_update += host_now_ms() - t2;
    // per time: ||Z~_q|| and the bound sum_j |c_j / s| rho / (delta_j / s)
    bool conv_bound = true, finite = true;
    double rmax = 0.0, worst = 0.0;
    for (int q = 0; q < nt; ++q) {
      const double zn = zn_q[q];
      if (!std::isfinite(zn)) finite = false;
      double bound = 0.0;
      for (int j = 0; j < kNShift; ++j) {
        const double r = rho[q * kNShift + j];
        if (!std::isfinite(r)) finite = false;
        bound += cw[j] * r / delta[j];
        rmax = std::max(rmax, r);
      }
      if (!(bound <= tol * zn)) conv_bound = false;
      const double rel_b = zn > 0.0 ? bound / zn : bound;
      if (q == 0) inf.znorm = zn;
      worst = std::max(worst, rel_b);
    }
    for (int j = 0; j < kNShift; ++j) inf.est[j] = rho[j];
    inf.err_bound = worst;
    inf.cycles = cycle;
    inf.breakdown = flags_h[0];
    bool singular = false;
    for (int v : sing_h) singular = singular || v != 0;
    // a rank-deficient block, a singular projected system (eq. 4.7) or a
    // non-finite estimate or norm: the iterate cannot be trusted
    if (flags_h[1] || singular || !finite) {
      status = EXPMV_EBREAKDOWN;
      break;
    }
    // an inner solve that stopped at its cap leaves the Arnoldi relation
    // (eq. 4.5) inexact, whatever the estimates say
    if (inf.inner_maxit_hit) {
      status = EXPMV_EINNER;
      break;
    }
    bool conv;
    if (pl->opts.stop_rule == EXPMV_STOP_PAPER) conv = rmax <= tol * inf.bnorm;
    else conv = conv_bound;
    if (!(rmax > 0.0)) conv = true;   // invariant space or exact
    if (conv) break;
    if (cycle >= pl->opts.max_cycles) {
      status = EXPMV_ENOCONV;
      break;
    }
    if (pl->opts.restart_refine) inf.refined_restarts += 1;
    // Steps 5-8: deflated restart (host eigensolve of the live part of H_d).
    // The restart keeps the basis's last block as the block after the Ritz
    // panels, so the next cycle's first product M^{-1} V_{m+1} needs nothing
    // from the eigensolve: it runs on the GPU while a host thread computes
    // the Ritz basis and the rotated H~.
    double t3 = host_now_ms();
    HIPCHK(hipMemcpyAsync(Hh.data(), w.H, sizeof(double) * size_t(ldh) * ldh,
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    auto coords = std::async(std::launch::async, restart_coordinates, bool(pl->symmetric), precond,
                             d, p, k, ldh, keff, kp, std::ref(Hh));
    const double ta = host_now_ms();
    apply_block(Vb + size_t(d / p) * blk);
    first_applied = true;
    const double tb = host_now_ms();
    ms_apply += tb - ta;
    RestartCoords rcd = coords.get();
    const int kn = rcd.kn;
    const int kpn = rcd.kpn;
    if (kn < 1 || kpn / p + 1 > m) {
      status = EXPMV_EBREAKDOWN;
      break;
    }
    const std::vector<double>& Pk = rcd.Pk;
    HIPCHK(hipMemcpyAsync(w.Crot, Pk.data(), sizeof(double) * Pk.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(w.H, Hh.data(), sizeof(double) * Hh.size(), hipMemcpyHostToDevice, s));
    // V_new = V_{d+p} P_{k+p}: the Ritz panels by a panel GEMM, then the last panel
    T* Vn = reinterpret_cast<T*>(w.V[cur ^ 1]);
    panel_gemm<T, T>(pl, p, Vb, d / p, w.Crot, kpn, kpn / p, Vn, int64_t(blk), p, 0);
    HIPCHK(hipMemcpyAsync(Vn + size_t(kpn / p) * blk, Vb + size_t(d / p) * blk, sizeof(T) * blk,
                          hipMemcpyDeviceToDevice, s));
    // Pk's constant header (host copy) must stay alive until the copies ran
    HIPCHK(hipStreamSynchronize(s));
    cur ^= 1;
    Vb = reinterpret_cast<T*>(w.V[cur]);
    keff = kn;
    kp = kpn;
    d = m * p;   // kp + (m - kp/p) p
    first_block = kp / p;
    rhs_from_S = true;
    ms_small += host_now_ms() - t3 - (tb - ta);
  }
  HIPCHK(hipStreamSynchronize(s));
  inf.ms_total = host_now_ms() - t_start;
  inf.ms_apply = ms_apply;
  inf.ms_orth = ms_orth;
  inf.ms_small = ms_small;
  inf.ms_update = ms_update;
  kt_collect(pl, 0);
  for (int c = 0; c < EXPMV_KT_COUNT; ++c) {
    const int cnt = pl->kt.cnt[c];
    inf.kern_launches[c] = cnt;
    inf.kern_ms[c] = cnt ? pl->kt.ms[c] / cnt : 0.0;
    inf.kern_bytes[c] = cnt ? pl->kt.by[c] / cnt : 0.0;
  }
  inf.amg_levels = pl->amg ? int(pl->amg->lv.size()) : 0;
  if (info) *info = inf;
  return status;
}

void bind_workspace(expmv_plan_s* pl, int p, int nt, bool joined, void* work, size_t bytes) {
  const size_t need = layout_workspace(pl, p, nt, joined, nullptr);
  if (!work || bytes < need || reinterpret_cast<uintptr_t>(work) % 256 != 0) {
    std::snprintf(g_error_detail, sizeof(g_error_detail),
                  "workspace %p of %zu bytes: this call needs %zu bytes, 256-byte aligned",
                  work, bytes, need);
    throw StatusError{EXPMV_EINVAL};
  }
  layout_workspace(pl, p, nt, joined, static_cast<char*>(work));
}

expmv_status dispatch_execute(expmv_plan_s* pl, int transpose, const double* B, int p, double tol,
                              double* Z, expmv_info* info,
                              const std::vector<double>& scales = std::vector<double>{1.0},
                              const SourceMode* src = nullptr) {
  if (pl->basis32)
    return execute_impl<float, float>(pl, transpose, B, p, tol, Z, info, scales, src);
  if (pl->mixed)
    return execute_impl<double, float>(pl, transpose, B, p, tol, Z, info, scales, src);
  return execute_impl<double, double>(pl, transpose, B, p, tol, Z, info, scales, src);
}

}  // namespace
}  // namespace expmv

// ===========================================================================
// C ABI

namespace {

template <typename F>
expmv_status guarded(F&& f) {
  g_error_detail[0] = '\0';
  try {
    return f();
  } catch (const expmv::HipError& e) {
    std::snprintf(g_error_detail, sizeof(g_error_detail), "HIP call at expmv.hip:%d: %s", e.line,
                  hipGetErrorString(e.err));
    return EXPMV_EHIP;
  } catch (const expmv::StatusError& e) {
    return e.st;
  } catch (const std::bad_alloc&) {
    std::snprintf(g_error_detail, sizeof(g_error_detail), "host allocation failed");
    return EXPMV_ENOMEM;
  } catch (const std::exception& e) {
    std::snprintf(g_error_detail, sizeof(g_error_detail), "C++ exception: %s", e.what());
    return EXPMV_EHIP;
  } catch (...) {
    std::snprintf(g_error_detail, sizeof(g_error_detail), "unknown C++ exception");
    return EXPMV_EHIP;
  }
}

bool valid_opts(const expmv_opts& o) {
  if (o.m < 2 || o.m > 64) return false;
  if (o.k < 0) return false;
  if (o.max_cycles < 1) return false;
  if (o.precision != EXPMV_FP64 && o.precision != EXPMV_MIXED && o.precision != EXPMV_MIXED_INNER)
    return false;
  if (o.stop_rule != EXPMV_STOP_PAPER && o.stop_rule != EXPMV_STOP_BOUND) return false;
  if (!(o.inner_tol >= 0.0 && o.inner_tol < 1.0)) return false;
  if (o.inner_maxit < 1) return false;
  if (o.profile < 0) return false;
  if (o.inner_refine < -1 || o.inner_refine > 8) return false;
  if (o.inner_precond < -1 || o.inner_precond > 1) return false;
  if (o.amg_degree < 0 || o.amg_degree > kAmgMaxDeg) return false;
  if (o.inner_relax < 0 || o.inner_relax > 10) return false;
  if (o.amg_fp32 != 0 && o.amg_fp32 != 1) return false;
  if (o.amg_coarse_degree < 0 || o.amg_coarse_degree > kAmgMaxDeg) return false;
  if (o.restart_refine != 0 && o.restart_refine != 1) return false;
  return true;
}

void upload_cf(expmv_plan_s* pl) {
  pl->tau_re.alloc(kNShift);
  pl->tau_im.alloc(kNShift);
  pl->c_re.alloc(kNShift);
  pl->c_im.alloc(kNShift);
  HIPCHK(hipMemcpy(pl->tau_re.p, CF_TAU_RE, sizeof(double) * kNShift, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(pl->tau_im.p, CF_TAU_IM, sizeof(double) * kNShift, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(pl->c_re.p, CF_C_RE, sizeof(double) * kNShift, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(pl->c_im.p, CF_C_IM, sizeof(double) * kNShift, hipMemcpyHostToDevice));
}

void init_plan_common(expmv_plan_s* pl) {
  HIPCHK(hipGetDevice(&pl->device));
  HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&pl->host_flags), sizeof(int) * 8,
                       hipHostMallocDefault));
  std::memset(pl->host_flags, 0, sizeof(int) * 8);
  HIPCHK(hipEventCreateWithFlags(&pl->ev[0], hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&pl->ev[1], hipEventDisableTiming));
  if (pl->opts.profile > 0) {
    KernelTimer& kt = pl->kt;
    kt.ev.assign(2 * size_t(kKtSlots), nullptr);
    kt.cls.assign(kKtSlots, 0);
    kt.iter.assign(kKtSlots, -1);
    kt.bytes.assign(kKtSlots, 0.0);
    for (auto& e : kt.ev) HIPCHK(hipEventCreate(&e));
  }
  upload_cf(pl);
}

// Host-side CSR build of K = -tA (and K^T), with validation.
expmv_status build_csr(expmv_plan_s* pl, const int32_t* rowptr_d, const int32_t* colind_d,
                       const double* val_d) {
  const int64_t n = pl->n, nnz = pl->nnz;
  std::vector<int32_t> rp(n + 1), ci(nnz);
  std::vector<double> v(nnz);
  HIPCHK(hipMemcpy(rp.data(), rowptr_d, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost));
  if (nnz > 0) {
    HIPCHK(hipMemcpy(ci.data(), colind_d, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(v.data(), val_d, sizeof(double) * nnz, hipMemcpyDeviceToHost));
  }
  if (rp[0] != 0 || rp[n] != nnz) return EXPMV_EINVAL;
  for (int64_t i = 0; i < n; ++i)
    if (rp[i + 1] < rp[i]) return EXPMV_EINVAL;
  std::vector<double> diag(n, 0.0);
  std::vector<char> has_diag(n, 0);
  for (int64_t i = 0; i < n; ++i)
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
      if (ci[e] < 0 || ci[e] >= n) return EXPMV_EINVAL;
      if (!std::isfinite(v[e])) return EXPMV_EINVAL;
      v[e] *= -pl->t;   // K = -tA
      if (ci[e] == i) {
        diag[i] += v[e];
        has_diag[i] = 1;
      }
    }
  for (int64_t i = 0; i < n; ++i)
    if (!has_diag[i] || !(diag[i] > 0.0)) return EXPMV_ENOTNEG;
  // symmetry detection: K^T by counting sort, compare entry by entry
  std::vector<int32_t> rpt(n + 1, 0), cit(nnz);
  std::vector<double> vt(nnz);
  for (int64_t e = 0; e < nnz; ++e) rpt[ci[e] + 1]++;
  for (int64_t i = 0; i < n; ++i) rpt[i + 1] += rpt[i];
  {
    std::vector<int32_t> pos(rpt.begin(), rpt.end() - 1);
    for (int64_t i = 0; i < n; ++i)
      for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
        const int32_t dst = pos[ci[e]]++;
        cit[dst] = int32_t(i);
        vt[dst] = v[e];
      }
  }
  bool sym = pl->opts.symmetric == 1;
  if (pl->opts.symmetric == -1) {
    // compare row i of K with row i of K^T as sorted (col, value) lists
    sym = true;
    std::vector<std::pair<int32_t, double>> a, b;
    for (int64_t i = 0; i < n && sym; ++i) {
      a.clear();
      b.clear();
      for (int32_t e = rp[i]; e < rp[i + 1]; ++e) a.emplace_back(ci[e], v[e]);
      for (int32_t e = rpt[i]; e < rpt[i + 1]; ++e) b.emplace_back(cit[e], vt[e]);
      if (a.size() != b.size()) {
        sym = false;
        break;
      }
      std::sort(a.begin(), a.end());
      std::sort(b.begin(), b.end());
      for (size_t q = 0; q < a.size(); ++q)
        if (a[q].first != b[q].first || a[q].second != b[q].second) {
          sym = false;
          break;
        }
    }
  }
  pl->symmetric = sym;
  std::vector<double> dinv(n);
  for (int64_t i = 0; i < n; ++i) dinv[i] = 1.0 / diag[i];
  pl->rowptr.alloc(n + 1);
  pl->colind.alloc(std::max<int64_t>(nnz, 1));
  pl->val.alloc(std::max<int64_t>(nnz, 1));
  pl->dinv.alloc(n);
  HIPCHK(hipMemcpy(pl->rowptr.p, rp.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(pl->colind.p, ci.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(pl->val.p, v.data(), sizeof(double) * nnz, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(pl->dinv.p, dinv.data(), sizeof(double) * n, hipMemcpyHostToDevice));
  {   // FP32 Jacobi scaling (mixed forms, FP32 V-cycles)
    std::vector<float> df(dinv.begin(), dinv.end());
    pl->dinvf.alloc(n);
    HIPCHK(hipMemcpy(pl->dinvf.p, df.data(), sizeof(float) * n, hipMemcpyHostToDevice));
    if (!sym) {
      pl->dinvTf.alloc(n);
      HIPCHK(hipMemcpy(pl->dinvTf.p, df.data(), sizeof(float) * n, hipMemcpyHostToDevice));
    }
  }
  if (!sym) {
    pl->rowptrT.alloc(n + 1);
    pl->colindT.alloc(std::max<int64_t>(nnz, 1));
    pl->valT.alloc(std::max<int64_t>(nnz, 1));
    pl->dinvT.alloc(n);
    HIPCHK(hipMemcpy(pl->rowptrT.p, rpt.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(pl->colindT.p, cit.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(pl->valT.p, vt.data(), sizeof(double) * nnz, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(pl->dinvT.p, dinv.data(), sizeof(double) * n, hipMemcpyHostToDevice));
  }
  return EXPMV_OK;
}

template <typename D, typename S>
void upload_vec(DevBuf<D>& dst, const std::vector<S>& src) {
  std::vector<D> tmp(src.begin(), src.end());
  dst.alloc(std::max<size_t>(tmp.size(), 1));
  if (!tmp.empty())
    HIPCHK(hipMemcpy(dst.p, tmp.data(), sizeof(D) * tmp.size(), hipMemcpyHostToDevice));
}

void upload_csr(const HostCsr& A, DevBuf<int32_t>& rp, DevBuf<int32_t>& ci, DevBuf<double>& v) {
  if (A.nnz() > INT32_MAX) throw StatusError{EXPMV_ENOMEM};
  upload_vec(rp, A.rp);
  upload_vec(ci, A.ci);
  upload_vec(v, A.v);
}

// Chebyshev coefficients of the smoother on [lmax / ratio, lmax]: step 0
// d = (1/theta) D^{-1} r; step k: d = rho_k rho_{k-1} d + (2 rho_k / delta) D^{-1} r.
void chebyshev_coefficients(double lmax, int degree, double* cd, double* ad) {
  const double lmin = lmax / (degree == 1 ? kAmgJacobiRatio : kAmgEigRatio);
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  cd[0] = 0.0;
  ad[0] = 1.0 / theta;
  for (int k = 1; k < degree; ++k) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    cd[k] = rn * rho;
    ad[k] = 2.0 * rn / delta;
    rho = rn;
  }
}

// Build the AMG hierarchy of K (tr = 0) or K^T (tr = 1) on the host and
// upload it.  Default smoothing degree: 2 for symmetric K (Chebyshev), 1 for
// nonsymmetric K (damped Jacobi: higher Chebyshev degrees amplify the
// complex part of a convection operator's spectrum).
expmv_status build_amg(expmv_plan_s* pl, int tr) {
  const int64_t n = pl->n, nnz = pl->nnz;
  const Csr<double> A = csr_of<double>(pl, tr);
  HostCsr K;
  K.nrows = K.ncols = n;
  {
    std::vector<int32_t> rp(n + 1);
    HIPCHK(hipMemcpy(rp.data(), A.rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost));
    K.rp.assign(rp.begin(), rp.end());
    K.ci.resize(nnz);
    K.v.resize(nnz);
    HIPCHK(hipMemcpy(K.ci.data(), A.colind, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(K.v.data(), A.val, sizeof(double) * nnz, hipMemcpyDeviceToHost));
  }
  AmgParams prm;
  prm.symmetric = pl->symmetric;
  AmgHost h;
  if (amg_build(K, prm, h) != 0) return EXPMV_EINVAL;
  if (h.lv.size() < 2) return EXPMV_OK;   // n <= max_coarse: no coarse level, Jacobi
  std::unique_ptr<AmgDev> H(new AmgDev());
  H->degree = pl->opts.amg_degree > 0 ? pl->opts.amg_degree : (pl->symmetric ? 2 : 1);
  for (size_t l = 0; l < h.lv.size(); ++l) {
    const AmgLevelHost& Lh = h.lv[l];
    std::unique_ptr<AmgDevLevel> L(new AmgDevLevel());
    L->n = Lh.A.nrows;
    if (l == 0) {
      const bool t = tr && !pl->symmetric;
      L->arp = A.rowptr;
      L->aci = A.colind;
      L->av = A.val;
      L->dinv64 = t ? pl->dinvT.p : pl->dinv.p;
      L->dinv32 = t ? pl->dinvTf.p : pl->dinvf.p;
    } else {
      upload_csr(Lh.A, L->Arp, L->Aci, L->Av);
      upload_vec(L->dinv, Lh.dinv);
      L->arp = L->Arp.p;
      L->aci = L->Aci.p;
      L->av = L->Av.p;
      L->dinv64 = L->dinv.p;
      upload_vec(L->dinvf, Lh.dinv);
      L->dinv32 = L->dinvf.p;
    }
    upload_vec(L->Av32, Lh.A.v);   // level 0: the values of K (or K^T) as the host copy holds them
    L->avg_a = double(Lh.A.nnz()) / double(std::max<int64_t>(1, Lh.A.nrows));
    L->nnz_a = Lh.A.nnz();
    if (l + 1 < h.lv.size()) {
      upload_csr(Lh.P, L->Prp, L->Pci, L->Pv);
      upload_csr(Lh.R, L->Rrp, L->Rci, L->Rv);
      upload_vec(L->Pv32, Lh.P.v);
      upload_vec(L->Rv32, Lh.R.v);
      L->avg_p = double(Lh.P.nnz()) / double(std::max<int64_t>(1, Lh.P.nrows));
      L->avg_r = double(Lh.R.nnz()) / double(std::max<int64_t>(1, Lh.R.nrows));
      L->nnz_p = Lh.P.nnz();
      L->nnz_r = Lh.R.nnz();
    }
    L->degree = l == 0 ? H->degree
                       : (pl->opts.amg_coarse_degree > 0 ? pl->opts.amg_coarse_degree
                                                         : std::max(1, H->degree - 1));
    chebyshev_coefficients(Lh.lmax, L->degree, L->cd, L->ad);
    H->lv.push_back(std::move(L));
  }
  upload_vec(H->cinv, h.coarse_inv);
  const int nlev = int(h.lv.size());
  const int64_t nc_last = h.lv.back().A.nrows, nl_last = h.lv[nlev - 2].A.nrows;
  const bool dense_last = nc_last * nl_last <= kAmgFusedMax;
  // fused levels: below the finest, above the coarsest, one smoothing step;
  // a level whose fused operators could outgrow kAmgFuseGrowth times its own
  // operator and prolongator (a bound on the product patterns) stays unfused
  for (int l = 1; l + 1 < nlev; ++l) {
    AmgDevLevel& L = *H->lv[l];
    if (L.degree != 1) continue;
    const AmgLevelHost& Lh = h.lv[l];
    const double s0 = L.ad[0];
    const int64_t cap = kAmgFuseGrowth * (Lh.A.nnz() + Lh.P.nnz());
    if (fused_prolongation_nnz_bound(Lh) > cap || fused_restriction_nnz_bound(Lh, 0.0) > cap)
      continue;
    L.fused = true;
    L.alpha = 2.0 * s0;   // of the prolongation-plus-smoothing pass
    L.beta = s0 * s0;
    const HostCsr Pf = fused_prolongation(Lh, s0);
    upload_csr(Pf, L.Pfrp, L.Pfci, L.Pfv);
    upload_vec(L.Pfv32, Pf.v);
    L.avg_pf = double(Pf.nnz()) / double(std::max<int64_t>(1, Pf.nrows));
    L.nnz_pf = Pf.nnz();
    if (l + 2 == nlev && dense_last) continue;   // Inv Rf below
    const HostCsr Rf = fused_restriction(Lh, s0, 0.0);
    upload_csr(Rf, L.Rfrp, L.Rfci, L.Rfv);
    upload_vec(L.Rfv32, Rf.v);
    L.avg_rf = double(Rf.nnz()) / double(std::max<int64_t>(1, Rf.nrows));
    L.nnz_rf = Rf.nnz();
  }
  {
    // the finest level at degree 2, when it restricts to a sparse level:
    // x1 = D^{-1} (alpha b - beta A D^{-1} b), b - A x1 = (I - A D^{-1} S) b
    // with S = alpha I - beta A D^{-1}
    AmgDevLevel& L = *H->lv[0];
    const AmgLevelHost& Lh = h.lv[0];
    if (L.degree == 2 && !(nlev == 2 && dense_last)) {
      const double alpha = (1.0 + L.cd[1]) * L.ad[0] + L.ad[1];
      const double beta = L.ad[1] * L.ad[0];
      const int64_t cap = kAmgFuseGrowth * (Lh.A.nnz() + Lh.P.nnz());
      if (fused_restriction_nnz_bound(Lh, beta) <= cap) {
        const HostCsr Rf = fused_restriction(Lh, alpha, beta);
        upload_csr(Rf, L.Rfrp, L.Rfci, L.Rfv);
        upload_vec(L.Rfv32, Rf.v);
        L.avg_rf = double(Rf.nnz()) / double(std::max<int64_t>(1, Rf.nrows));
        L.nnz_rf = Rf.nnz();
        L.alpha = alpha;
        L.beta = beta;
        L.fused = true;
      }
    } else if (L.degree == 1 && !pl->symmetric && !(nlev == 2 && dense_last)) {
      // the finest level of a nonsymmetric K at one step (BiCGStab, whose
      // V-cycles write no partial sums): fused like the levels below it
      const double s0 = L.ad[0];
      const int64_t cap = kAmgFuseGrowth * (Lh.A.nnz() + Lh.P.nnz());
      if (fused_restriction_nnz_bound(Lh, 0.0) <= cap && fused_prolongation_nnz_bound(Lh) <= cap) {
        const HostCsr Rf = fused_restriction(Lh, s0, 0.0);
        upload_csr(Rf, L.Rfrp, L.Rfci, L.Rfv);
        upload_vec(L.Rfv32, Rf.v);
        L.avg_rf = double(Rf.nnz()) / double(std::max<int64_t>(1, Rf.nrows));
        L.nnz_rf = Rf.nnz();
        const HostCsr Pf = fused_prolongation(Lh, s0);
        upload_csr(Pf, L.Pfrp, L.Pfci, L.Pfv);
        upload_vec(L.Pfv32, Pf.v);
        L.avg_pf = double(Pf.nnz()) / double(std::max<int64_t>(1, Pf.nrows));
        L.nnz_pf = Pf.nnz();
        L.alpha = 2.0 * s0;
        L.beta = s0 * s0;
        L.fused = true;
      }
    }
  }
  for (int l = 0; l + 1 < nlev; ++l) {
    AmgDevLevel& L = *H->lv[l];
    if (!L.fused || L.degree != 1) continue;
    const AmgLevelHost& Lh = h.lv[l];
    std::vector<double> adv(Lh.A.v.size());
    for (int64_t i = 0; i < Lh.A.nrows; ++i)
      for (int64_t e = Lh.A.rp[i]; e < Lh.A.rp[i + 1]; ++e)
        adv[e] = Lh.A.v[e] * Lh.dinv[Lh.A.ci[e]];
    upload_vec(L.ADv, adv);
  }
  if (dense_last) {
    // Inv R for the level above the coarsest: nc x n_l dense, built from the
    // sparse R row by row (same sums as R then Inv, another order); on a
    // fused level Inv Rf = (Inv R)(I - s0 A D^{-1}), built from it the same way
    const AmgLevelHost& Lp = h.lv[nlev - 2];
    const int64_t nc = nc_last, nl = nl_last;
    std::vector<double> IR(size_t(nc) * nl, 0.0);
    for (int64_t i = 0; i < nc; ++i)
      for (int64_t q = 0; q < nc; ++q) {
        const double a = h.coarse_inv[size_t(i) * nc + q];
        for (int64_t e = Lp.R.rp[q]; e < Lp.R.rp[q + 1]; ++e)
          IR[size_t(i) * nl + Lp.R.ci[e]] += a * Lp.R.v[e];
      }
    if (H->lv[nlev - 2]->fused) {
      const HostCsr M = jacobi_step_operator(Lp.A, Lp.dinv, H->lv[nlev - 2]->ad[0], false);
      std::vector<double> IRf(size_t(nc) * nl, 0.0);
      for (int64_t i = 0; i < nc; ++i)
        for (int64_t q = 0; q < nl; ++q) {
          const double a = IR[size_t(i) * nl + q];
          for (int64_t e = M.rp[q]; e < M.rp[q + 1]; ++e)
            IRf[size_t(i) * nl + M.ci[e]] += a * M.v[e];
        }
      IR.swap(IRf);
    }
    upload_vec(H->cinvR, IR);
  }
  (tr && !pl->symmetric ? pl->amgT : pl->amg) = std::move(H);
  return EXPMV_OK;
}

// ---------------------------------------------------------------------------
// Toeplitz plan set-up: spectra of the circulant embeddings of T (and T^T)
// and of the Gohberg-Semencul generators x = T^{-1} e_1 (and y = T^{-1} e_n)

// Host-driven Krylov solve T z = e_k with the FFT product: CG for symmetric
// T; for general T BiCGStab, right-preconditioned by the inverse of T's
// Strang circulant (first column c_0..c_{n/2}, r_{n/2-1}..r_1) when n has no
// prime factor above 5 (a length-n FFT), unpreconditioned otherwise.  Returns the
// true relative residual ||e_k - T z|| (z on the device).
double toeplitz_setup_solve(expmv_plan_s* pl, const std::vector<double>& c,
                            const std::vector<double>& r, int64_t k, double* z) {
  const int64_t n = pl->n;
  hipStream_t s = pl->stream;
  const int g = stream_grid(n);
  std::vector<DevBuf<double>> v(9);
  for (auto& b : v) b.alloc(n);
  double *x = z, *res = v[0].p, *rh = v[1].p, *pv = v[2].p, *vv = v[3].p, *sv = v[4].p,
         *tv = v[5].p, *ph = v[6].p, *sh = v[7].p, *tmp = v[8].p;
  HIPCHK(hipMemsetAsync(x, 0, sizeof(double) * n, s));
  HIPCHK(hipMemsetAsync(res, 0, sizeof(double) * n, s));
  const double one = 1.0;
  HIPCHK(hipMemcpyAsync(res + k, &one, sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  auto Tapply = [&](const double* in, double* outp) {
    toeplitz_apply<double>(pl, in, 1, outp, 1, 1, 1.0, 0, 0, false);
  };
  auto axpby = [&](double a, const double* xx, double b, double* yy) {
    hipLaunchKernelGGL(k_axpby, dim3(g), dim3(kThreads), 0, s, n, a, xx, b, yy);
  };
  auto copy = [&](const double* from, double* to) {
    HIPCHK(hipMemcpyAsync(to, from, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  };
  if (pl->tsym) {
    copy(res, pv);
    double rr = 1.0;
    for (int it = 0; it < 20000; ++it) {
      Tapply(pv, vv);
      const double pq = device_dot(pl, n, pv, vv);
      if (!(pq > 0.0)) throw StatusError{EXPMV_ENOTNEG};   // T not positive definite
      const double alpha = rr / pq;
      axpby(alpha, pv, 1.0, x);
      axpby(-alpha, vv, 1.0, res);
      const double rr2 = device_dot(pl, n, res, res);
      if (std::sqrt(rr2) <= 1e-14) break;
      axpby(1.0, res, rr2 / rr, pv);
      rr = rr2;
    }
  } else {
    // Strang circulant preconditioner (n 2,3,5-smooth)
    std::vector<int> rad_n = fft_radices(n);
    const bool strang = !rad_n.empty() && n >= 4;
    DevBuf<cplx> inv_eig;
    if (strang) {
      std::vector<double> sc(n, 0.0);
      for (int64_t i = 0; i <= n / 2; ++i) sc[i] = c[i];
      for (int64_t i = n / 2 + 1; i < n; ++i) sc[i] = r[n - i];
      DevBuf<double> scd;
      scd.alloc(n);
      HIPCHK(hipMemcpyAsync(scd.p, sc.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL((k_pack<double>), dim3(stream_grid(n)), dim3(kThreads), 0, s, n, 1,
                         int64_t(1), 1, n, scd.p, pl->setup_fb[0].p, 0, 1.0, nullptr);
      fft_len(pl, n, rad_n, pl->setup_fb[0].p, pl->setup_fb[1].p, pl->setup_fb[2].p, 1, -1.0);
      std::vector<cplx> ev(n);
      HIPCHK(hipMemcpyAsync(ev.data(), pl->setup_fb[1].p, sizeof(cplx) * n, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (auto& e : ev) {
        const double d = e.x * e.x + e.y * e.y;
        e = d > 0.0 ? cplx{e.x / d, -e.y / d} : cplx{0.0, 0.0};
      }
      inv_eig.alloc(n);
      HIPCHK(hipMemcpyAsync(inv_eig.p, ev.data(), sizeof(cplx) * n, hipMemcpyHostToDevice, s));
      HIPCHK(hipStreamSynchronize(s));
    }
    auto Papply = [&](const double* in, double* outp) {
      if (!strang) {
        copy(in, outp);
        return;
      }
      hipLaunchKernelGGL((k_pack<double>), dim3(stream_grid(n)), dim3(kThreads), 0, s, n, 1,
                         int64_t(1), 1, n, in, pl->setup_fb[0].p, 0, 1.0, nullptr);
      fft_len(pl, n, rad_n, pl->setup_fb[0].p, pl->setup_fb[1].p, pl->setup_fb[2].p, 1, -1.0);
      hipLaunchKernelGGL(k_spec_mul, dim3(stream_grid(n)), dim3(kThreads), 0, s, n, 1,
                         pl->setup_fb[1].p, inv_eig.p, 1.0 / double(n));
      fft_len(pl, n, rad_n, pl->setup_fb[1].p, pl->setup_fb[0].p, pl->setup_fb[2].p, 1, +1.0);
      hipLaunchKernelGGL((k_unpack<double>), dim3(stream_grid(n)), dim3(kThreads), 0, s, n, 1,
                         int64_t(1), 1, pl->setup_fb[0].p, outp, 0, 1.0, 0, nullptr);
    };
    copy(res, rh);
    HIPCHK(hipMemsetAsync(pv, 0, sizeof(double) * n, s));
    HIPCHK(hipMemsetAsync(vv, 0, sizeof(double) * n, s));
    double rho_prev = 1.0, alpha = 1.0, omega = 1.0;
    for (int it = 0; it < 20000; ++it) {
      const double rho = device_dot(pl, n, rh, res);
      if (rho == 0.0 || omega == 0.0) break;
      const double beta = (rho / rho_prev) * (alpha / omega);
      // p = r + beta (p - omega v)
      axpby(-omega, vv, 1.0, pv);
      axpby(1.0, res, beta, pv);
      Papply(pv, ph);
      Tapply(ph, vv);
      const double rv = device_dot(pl, n, rh, vv);
      if (rv == 0.0) break;
      alpha = rho / rv;
      copy(res, sv);
      axpby(-alpha, vv, 1.0, sv);                      // s = r - alpha v
      Papply(sv, sh);
      Tapply(sh, tv);
      const double tt = device_dot(pl, n, tv, tv);
      omega = tt > 0.0 ? device_dot(pl, n, tv, sv) / tt : 0.0;
      axpby(alpha, ph, 1.0, x);
      axpby(omega, sh, 1.0, x);                        // x += alpha p^ + omega s^
      copy(sv, res);
      axpby(-omega, tv, 1.0, res);                     // r = s - omega t
      rho_prev = rho;
      if (std::sqrt(device_dot(pl, n, res, res)) <= 1e-14) break;
    }
  }
  // true residual e_k - T z
  Tapply(x, tmp);
  HIPCHK(hipMemsetAsync(res, 0, sizeof(double) * n, s));
  HIPCHK(hipMemcpyAsync(res + k, &one, sizeof(double), hipMemcpyHostToDevice, s));
  axpby(-1.0, tmp, 1.0, res);
  const double rn = std::sqrt(device_dot(pl, n, res, res));
  HIPCHK(hipStreamSynchronize(s));
  return rn;
}

expmv_status build_toeplitz(expmv_plan_s* pl, const std::vector<double>& c,
                            const std::vector<double>& r) {
  const int64_t n = pl->n;
  hipStream_t s = pl->stream;
  int64_t L = 1;
  while (L < 2 * n) L <<= 1;
  pl->L = L;
  pl->radices = fft_radices(L);
  // set-up buffers (plan-owned, released below): the FFT work arrays for
  // one complex column and the partial sums of the set-up solves' dots
  for (auto& b : pl->setup_fb) b.alloc(size_t(L));
  DevBuf<double> part;
  part.alloc(4096);
  pl->ws = Workspace();
  for (int i = 0; i < 3; ++i) pl->ws.fb[i] = pl->setup_fb[i].p;
  pl->ws.fq = 1;
  pl->ws.partial = part.p;
  DevBuf<double> tmp;
  tmp.alloc(L);
  auto spectrum = [&](const std::vector<double>& h, DevBuf<cplx>& dst) {
    dst.alloc(L);
    HIPCHK(hipMemcpyAsync(tmp.p, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL((k_pack<double>), dim3(stream_grid(L)), dim3(kThreads), 0, s,
                       int64_t(h.size()), 1, int64_t(1), 1, L, tmp.p, pl->setup_fb[0].p, 0, 1.0,
                       nullptr);
    fft(pl, pl->setup_fb[0].p, dst.p, pl->setup_fb[1].p, 1, -1.0);
    HIPCHK(hipStreamSynchronize(s));
  };
  // circulant embeddings [c_0 .. c_{n-1}, 0 .., r_{n-1} .. r_1] of T and
  // [r_0 .. r_{n-1}, 0 .., c_{n-1} .. c_1] of T^T
  std::vector<double> emb(L, 0.0);
  for (int64_t i = 0; i < n; ++i) emb[i] = c[i];
  for (int64_t i = 1; i < n; ++i) emb[L - i] = r[i];
  spectrum(emb, pl->chat);
  if (!pl->tsym) {
    std::fill(emb.begin(), emb.end(), 0.0);
    for (int64_t i = 0; i < n; ++i) emb[i] = r[i];
    for (int64_t i = 1; i < n; ++i) emb[L - i] = c[i];
    spectrum(emb, pl->chatT);
  }
  // generators (once per plan)
  DevBuf<double> xd, yd;
  xd.alloc(n);
  if (toeplitz_setup_solve(pl, c, r, 0, xd.p) > 1e-10) return EXPMV_ENOCONV;
  std::vector<double> xh(n), yh;
  HIPCHK(hipMemcpy(xh.data(), xd.p, sizeof(double) * n, hipMemcpyDeviceToHost));
  pl->x0 = xh[0];
  if (!(pl->x0 > 0.0)) return EXPMV_ENOTNEG;
  if (pl->tsym) {
    yh.assign(xh.rbegin(), xh.rend());   // y = J x
  } else {
    yd.alloc(n);
    if (toeplitz_setup_solve(pl, c, r, n - 1, yd.p) > 1e-10) return EXPMV_ENOCONV;
    yh.resize(n);
    HIPCHK(hipMemcpy(yh.data(), yd.p, sizeof(double) * n, hipMemcpyDeviceToHost));
  }
  // the length-n form when n has no prime factor above 5 (spectra of x,
  // Z_1 y, D J y and D Z_{-1} J x, D = diag(exp(i pi k / n))), else the
  // triangular factors through the length-L embedding (spectra of the
  // zero-padded x, Z J x, J y, Z y)
  pl->radices_n = fft_radices(n);
  pl->gsf_n = !pl->radices_n.empty() && n >= 2;
  if (!pl->gsf_n) {
    std::vector<double> e(L, 0.0);
    auto gen = [&](auto f, DevBuf<cplx>& dst) {
      std::fill(e.begin(), e.end(), 0.0);
      for (int64_t i = 0; i < n; ++i) e[i] = f(i);
      spectrum(e, dst);
    };
    gen([&](int64_t i) { return xh[i]; }, pl->xhat);                            // x
    gen([&](int64_t i) { return i ? xh[n - i] : 0.0; }, pl->yhat);             // Z J x
    if (!pl->tsym) {
      gen([&](int64_t i) { return yh[n - 1 - i]; }, pl->jyhat);                 // J y
      gen([&](int64_t i) { return i ? yh[i - 1] : 0.0; }, pl->zyhat);          // Z y
    }
  } else {
    auto spectrum_n = [&](auto f, double sign, DevBuf<cplx>& dst) {
      std::vector<double> h(n);
      for (int64_t i = 0; i < n; ++i) h[i] = f(i);
      dst.alloc(n);
      HIPCHK(hipMemcpyAsync(tmp.p, h.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL((k_pack_twist<double>), dim3(stream_grid(n)), dim3(kThreads), 0, s, n, 1,
                         int64_t(1), 1, tmp.p, pl->setup_fb[0].p, 1.0, nullptr, sign);
      fft_len(pl, n, pl->radices_n, pl->setup_fb[0].p, dst.p, pl->setup_fb[1].p, 1, -1.0);
      HIPCHK(hipStreamSynchronize(s));
    };
    spectrum_n([&](int64_t i) { return xh[i]; }, 0.0, pl->ncx);                       // x
    spectrum_n([&](int64_t i) { return yh[(i + n - 1) % n]; }, 0.0, pl->ncz);          // Z_1 y
    spectrum_n([&](int64_t i) { return yh[n - 1 - i]; }, 1.0, pl->nsj);                // J y
    spectrum_n([&](int64_t i) { return i ? xh[n - i] : -xh[0]; }, 1.0, pl->nsz);       // Z_{-1} J x
  }
  HIPCHK(hipStreamSynchronize(s));
  for (auto& b : pl->setup_fb) b.release();
  pl->ws = Workspace();
  return EXPMV_OK;
}

}  // namespace

struct expmv_amg_s {
  expmv::AmgHost h;
};

extern "C" {

expmv_status expmv_default_opts(expmv_opts* o) {
  if (!o) return EXPMV_EINVAL;
  o->m = 10;
  o->k = 0;
  o->max_cycles = 50;
  o->precision = EXPMV_FP64;
  o->stop_rule = EXPMV_STOP_BOUND;
  o->inner_tol = 0.0;
  o->inner_maxit = 50000;
  o->symmetric = -1;
  o->preconditioned = 1;
  o->profile = 0;
  o->inner_refine = -1;
  o->inner_precond = -1;
  o->amg_degree = 0;
  o->inner_relax = 8;
  o->amg_fp32 = 0;
  o->amg_coarse_degree = 0;
  o->restart_refine = 0;
  return EXPMV_OK;
}

expmv_status expmv_plan_csr(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colind,
                            const double* val, double t, const expmv_opts* opts, hipStream_t stream,
                            expmv_plan* out) {
  if (!out) return EXPMV_EINVAL;
  *out = nullptr;
  if (n < 1 || n > INT32_MAX - 1 || nnz < 1 || nnz > INT32_MAX || !rowptr || !colind || !val)
    return EXPMV_EINVAL;
  if (!(t != 0.0) || !std::isfinite(t)) return EXPMV_EINVAL;
  expmv_opts o;
  expmv_default_opts(&o);
  if (opts) o = *opts;
  if (!valid_opts(o)) return EXPMV_EINVAL;
  return guarded([&]() -> expmv_status {
    std::unique_ptr<expmv_plan_s> pl(new expmv_plan_s());
    pl->kind = 0;
    pl->n = n;
    pl->nnz = nnz;
    pl->t = t;
    pl->opts = o;
    pl->stream = stream;
    pl->mixed = (o.precision != EXPMV_FP64);
    pl->basis32 = (o.precision == EXPMV_MIXED);
    init_plan_common(pl.get());
    expmv_status st = build_csr(pl.get(), rowptr, colind, val);
    if (st != EXPMV_OK) return st;
    const int ip = o.inner_precond;
    if (o.preconditioned && (ip == 1 || (ip == -1 && n >= 4096))) {
      st = build_amg(pl.get(), 0);
      if (st == EXPMV_OK && !pl->symmetric && pl->amg) {
        st = build_amg(pl.get(), 1);
        if (st != EXPMV_OK) pl->amg.reset();   // both or neither
      }
      if (st != EXPMV_OK && ip == 1) return st;
    }
    *out = pl.release();
    return EXPMV_OK;
  });
}

expmv_status expmv_plan_toeplitz(int64_t n, const double* col0, double t, const expmv_opts* opts,
                                 hipStream_t stream, expmv_plan* out) {
  return expmv_plan_toeplitz_general(n, col0, nullptr, nullptr, t, opts, stream, out);
}

expmv_status expmv_plan_toeplitz_general(int64_t n, const double* col0, const double* row0,
                                         const double* diag, double t, const expmv_opts* opts,
                                         hipStream_t stream, expmv_plan* out) {
  if (!out) return EXPMV_EINVAL;
  *out = nullptr;
  if (n < 2 || n > (int64_t(1) << 28) || !col0) return EXPMV_EINVAL;
  if (!(t != 0.0) || !std::isfinite(t)) return EXPMV_EINVAL;
  if (t < 0.0) return EXPMV_ENOTNEG;   // tA = -t T needs t > 0
  expmv_opts o;
  expmv_default_opts(&o);
  if (opts) o = *opts;
  if (!valid_opts(o)) return EXPMV_EINVAL;
  return guarded([&]() -> expmv_status {
    std::vector<double> c(n), r(n);
    HIPCHK(hipMemcpy(c.data(), col0, sizeof(double) * n, hipMemcpyDeviceToHost));
    if (row0) HIPCHK(hipMemcpy(r.data(), row0, sizeof(double) * n, hipMemcpyDeviceToHost));
    else r = c;
    r[0] = c[0];
    for (int64_t i = 0; i < n; ++i)
      if (!std::isfinite(c[i]) || !std::isfinite(r[i])) return EXPMV_EINVAL;
    if (!(c[0] > 0.0)) return EXPMV_ENOTNEG;
    std::vector<double> dg;
    if (diag) {
      dg.resize(n);
      HIPCHK(hipMemcpy(dg.data(), diag, sizeof(double) * n, hipMemcpyDeviceToHost));
      for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(dg[i])) return EXPMV_EINVAL;
        if (!(dg[i] > 0.0)) return EXPMV_ENOTNEG;   // diag(tA) = -t d_i c_0 must be < 0
      }
    }
    std::unique_ptr<expmv_plan_s> pl(new expmv_plan_s());
    pl->kind = 1;
    pl->n = n;
    pl->nnz = 0;
    pl->t = t;
    pl->opts = o;
    pl->stream = stream;
    pl->mixed = (o.precision != EXPMV_FP64);
    pl->basis32 = (o.precision == EXPMV_MIXED);
    pl->tsym = (c == r);
    pl->symmetric = pl->tsym && !diag;
    init_plan_common(pl.get());
    expmv_status st = build_toeplitz(pl.get(), c, r);
    if (st != EXPMV_OK) return st;
    if (diag) {
      std::vector<double> di(n);
      for (int64_t i = 0; i < n; ++i) di[i] = 1.0 / dg[i];
      pl->tdiag.alloc(n);
      pl->tdinv.alloc(n);
      HIPCHK(hipMemcpy(pl->tdiag.p, dg.data(), sizeof(double) * n, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(pl->tdinv.p, di.data(), sizeof(double) * n, hipMemcpyHostToDevice));
    }
    *out = pl.release();
    return EXPMV_OK;
  });
}

expmv_status expmv_workspace_size(expmv_plan plan, int64_t p, size_t* bytes) {
  if (!plan || !bytes || p < 1 || p > kMaxP || p > plan->n) return EXPMV_EINVAL;
  return guarded([&]() -> expmv_status {
    *bytes = layout_workspace(plan, int(p), 1, false, nullptr);
    return EXPMV_OK;
  });
}

expmv_status expmv_workspace_size_times(expmv_plan plan, int64_t p, int nt, size_t* bytes) {
  if (!plan || !bytes || p < 1 || p > kMaxP || p > plan->n || nt < 1 || nt > kMaxTimes)
    return EXPMV_EINVAL;
  return guarded([&]() -> expmv_status {
    *bytes = layout_workspace(plan, int(p), nt, false, nullptr);
    return EXPMV_OK;
  });
}

expmv_status expmv_workspace_size_source(expmv_plan plan, int64_t p, size_t* bytes) {
  if (!plan || !bytes || p < 1 || 2 * p > kMaxP || 2 * p > plan->n) return EXPMV_EINVAL;
  return guarded([&]() -> expmv_status {
    // the joined block [U0 | S] (2p columns) or one of its halves alone
    *bytes = std::max(layout_workspace(plan, int(2 * p), 1, true, nullptr),
                      layout_workspace(plan, int(p), 1, false, nullptr));
    return EXPMV_OK;
  });
}

expmv_status expmv_execute(expmv_plan plan, int transpose, const double* B, int64_t p, double tol,
                           void* work, size_t work_bytes, double* Z, expmv_info* info) {
  if (!plan || !B || !Z || p < 1 || p > kMaxP || p > plan->n) return EXPMV_EINVAL;
  if (!(tol > 0.0 && tol < 1.0)) return EXPMV_EINVAL;
  return guarded([&]() {
    bind_workspace(plan, int(p), 1, false, work, work_bytes);
    return dispatch_execute(plan, transpose, B, int(p), tol, Z, info);
  });
}

expmv_status expmv_execute_times(expmv_plan plan, int transpose, const double* times, int nt,
                                 const double* B, int64_t p, double tol, void* work,
                                 size_t work_bytes, double* Z, expmv_info* info) {
  if (!plan || !times || !B || !Z || p < 1 || p > kMaxP || p > plan->n) return EXPMV_EINVAL;
  if (nt < 1 || nt > kMaxTimes) return EXPMV_EINVAL;
  if (!(tol > 0.0 && tol < 1.0)) return EXPMV_EINVAL;
  std::vector<double> scales(nt);
  for (int q = 0; q < nt; ++q) {
    if (!std::isfinite(times[q])) return EXPMV_EINVAL;
    scales[q] = times[q] / plan->t;
    if (!(scales[q] > 0.0)) return EXPMV_ENOTNEG;   // t_q A must stay negative definite
  }
  return guarded([&]() {
    bind_workspace(plan, int(p), nt, false, work, work_bytes);
    return dispatch_execute(plan, transpose, B, int(p), tol, Z, info, scales);
  });
}

expmv_status expmv_execute_source(expmv_plan plan, int transpose, const double* U0,
                                  const double* S, int64_t p, double gamma, double tol, void* work,
                                  size_t work_bytes, double* U, expmv_info* info) {
  if (!plan || !U0 || !S || !U || p < 1 || 2 * p > kMaxP || 2 * p > plan->n) return EXPMV_EINVAL;
  if (!(tol > 0.0 && tol < 1.0) || !std::isfinite(gamma)) return EXPMV_EINVAL;
  return guarded([&]() -> expmv_status {
    const int64_t n = plan->n;
    // an all-zero part would make the joined block rank deficient: S = 0 is
    // the plain exponential, U0 = 0 runs on S alone
    bind_workspace(plan, int(p), 1, false, work, work_bytes);
    const double uu = device_dot(plan, n * p, U0, U0), ss = device_dot(plan, n * p, S, S);
    if (!std::isfinite(uu) || !std::isfinite(ss) || !(uu + ss > 0.0)) return EXPMV_EINVAL;
    if (ss == 0.0) return dispatch_execute(plan, transpose, U0, int(p), tol, U, info);
    const SourceMode sm{gamma * plan->t, plan->t, uu == 0.0};
    if (sm.s_only)
      return dispatch_execute(plan, transpose, S, int(p), tol, U, info, std::vector<double>{1.0},
                              &sm);
    bind_workspace(plan, int(2 * p), 1, true, work, work_bytes);
    double* J = plan->ws.srcB;
    // joined block [U0 | S]: row i holds U0's row i, then S's row i
    HIPCHK(hipMemcpy2DAsync(J, sizeof(double) * 2 * p, U0, sizeof(double) * p,
                            sizeof(double) * p, n, hipMemcpyDeviceToDevice, plan->stream));
    HIPCHK(hipMemcpy2DAsync(J + p, sizeof(double) * 2 * p, S, sizeof(double) * p,
                            sizeof(double) * p, n, hipMemcpyDeviceToDevice, plan->stream));
    return dispatch_execute(plan, transpose, J, int(2 * p), tol, U, info, std::vector<double>{1.0},
                            &sm);
  });
}

expmv_status expmv_adjoint(expmv_plan plan, const double* G, const double* B, int64_t p,
                           double tol, void* work, size_t work_bytes, double* gradB,
                           double* grad_t, expmv_info* info) {
  if (!plan || !G || !B || !gradB || !grad_t || p < 1 || p > kMaxP || p > plan->n)
    return EXPMV_EINVAL;
  if (!(tol > 0.0 && tol < 1.0)) return EXPMV_EINVAL;
  return guarded([&]() -> expmv_status {
    bind_workspace(plan, int(p), 1, false, work, work_bytes);
    expmv_status st = dispatch_execute(plan, 1, G, int(p), tol, gradB, info);
    if (st != EXPMV_OK && st != EXPMV_ENOCONV) return st;
    hipStream_t s = plan->stream;
    Workspace& w = plan->ws;
    // K B (K = -tA = -M), for the omega_0 <G, M B> term
    double* KB = w.Rres;
    const int grid = 512;
    apply_K<double>(plan, 0, B, KB, int(p));
    hipLaunchKernelGGL(k_adjoint_dots, dim3(grid), dim3(kThreads), 0, s, plan->n, int(p), w.X,
                       B, G, KB, w.partial);
    std::vector<double> part(size_t(grid) * 16);
    HIPCHK(hipMemcpyAsync(part.data(), w.partial, sizeof(double) * part.size(),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double d[16] = {0};
    for (int g = 0; g < grid; ++g)
      for (int v = 0; v < 16; ++v) d[v] += part[size_t(g) * 16 + v];
    double sum_c = 0.0, acc = 0.0;
    for (int j = 0; j < kNShift; ++j) {
      sum_c += CF_C_RE[j];
      // Re(c_j tau_j (d_re + i d_im))
      const double ctr = CF_C_RE[j] * CF_TAU_RE[j] - CF_C_IM[j] * CF_TAU_IM[j];
      const double cti = CF_C_RE[j] * CF_TAU_IM[j] + CF_C_IM[j] * CF_TAU_RE[j];
      acc += ctr * d[2 * j] - cti * d[2 * j + 1];
    }
    // <G, M B> = -<G, K B>
    *grad_t = (CF_OMEGA0 * (-d[15]) + sum_c * d[14] + acc) / plan->t;
    return st;
  });
}

expmv_status expmv_grad_t(expmv_plan plan, const double* G, const double* Zm, int64_t p,
                          void* work, size_t work_bytes, double* out) {
  if (!plan || !G || !Zm || !out || p < 1 || p > kMaxP || p > plan->n) return EXPMV_EINVAL;
  return guarded([&]() -> expmv_status {
    bind_workspace(plan, int(p), 1, false, work, work_bytes);
    hipStream_t s = plan->stream;
    if (plan->kind == 1) {
      // <G, A Z> = -<G, T Z>
      double* TZ = plan->ws.Rres;
      toeplitz_apply<double>(plan, Zm, p, TZ, p, int(p), 1.0, 0);
      *out = -device_dot(plan, plan->n * p, G, TZ);
      return EXPMV_OK;
    }
    const int PP = pow2_lanes(int(p));
    const int grid = grid_for(plan->n, PP, 512);
    DISPATCH_PP(PP, hipLaunchKernelGGL((k_dot_spmm<P_>), dim3(grid), dim3(kThreads), 0, s,
                                       plan->n, int(p), plan->rowptr.p, plan->colind.p,
                                       plan->val.p, G, Zm, plan->ws.partial));
    std::vector<double> part(grid);
    HIPCHK(hipMemcpyAsync(part.data(), plan->ws.partial, sizeof(double) * grid,
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double acc = 0.0;
    for (double v : part) acc += v;
    // <G, A Z> = -<G, K Z> / t  (K = -tA)
    *out = -acc / plan->t;
    return EXPMV_OK;
  });
}

expmv_status expmv_apply_operator(expmv_plan plan, int transpose, const double* X, int64_t p,
                                  void* work, size_t work_bytes, double* Y) {
  if (!plan || !X || !Y || p < 1 || p > kMaxP || p > plan->n) return EXPMV_EINVAL;
  return guarded([&]() -> expmv_status {
    bind_workspace(plan, int(p), 1, false, work, work_bytes);
    apply_K<double>(plan, transpose, X, Y, int(p));
    const int64_t cnt = plan->n * p;
    hipLaunchKernelGGL((k_convert<double, double>), dim3(512), dim3(kThreads), 0, plan->stream, cnt,
                       Y, Y, -1.0);
    HIPCHK(hipGetLastError());
    return EXPMV_OK;
  });
}

expmv_status expmv_apply_inverse(expmv_plan plan, int transpose, const double* X, int64_t p,
                                 void* work, size_t work_bytes, double* Y, long long* iters) {
  if (!plan || !X || !Y || p < 1 || p > kMaxP || p > plan->n) return EXPMV_EINVAL;
  return guarded([&]() -> expmv_status {
    bind_workspace(plan, int(p), 1, false, work, work_bytes);
    InnerResult r;
    if (plan->mixed) {
      float* xf = reinterpret_cast<float*>(plan->ws.W);
      float* yf = reinterpret_cast<float*>(plan->ws.Wt);
      const int64_t cnt = plan->n * p;
      hipLaunchKernelGGL((k_convert<double, float>), dim3(512), dim3(kThreads), 0, plan->stream,
                         cnt, X, xf, 1.0);
      r = apply_inverse<float>(plan, transpose, xf, yf, int(p));
      hipLaunchKernelGGL((k_convert<float, double>), dim3(512), dim3(kThreads), 0, plan->stream,
                         cnt, yf, Y, 1.0);
    } else {
      r = apply_inverse<double>(plan, transpose, X, Y, int(p));
    }
    HIPCHK(hipStreamSynchronize(plan->stream));
    if (iters) *iters = r.iters;
    return r.hit_cap ? EXPMV_EINNER : EXPMV_OK;
  });
}

expmv_status expmv_apply_preconditioner(expmv_plan plan, int transpose, const double* X,
                                        int64_t p, void* work, size_t work_bytes, double* Y) {
  if (!plan || !X || !Y || p < 1 || p > kMaxP || p > plan->n || plan->kind != 0)
    return EXPMV_EINVAL;
  return guarded([&]() -> expmv_status {
    bind_workspace(plan, int(p), 1, false, work, work_bytes);
    hipStream_t s = plan->stream;
    const int64_t cnt = plan->n * p;
    auto apply = [&](auto tag, const auto* x, auto* y) {
      using T = decltype(tag);
      if (AmgDev* H = amg_for(plan, transpose)) {
        amg_vcycle<T>(plan, *H, int(p), x, y, 0, nullptr, nullptr);
      } else {
        Csr<T> A = csr_of<T>(plan, transpose);
        hipLaunchKernelGGL((k_scale_rows<T>), dim3(grid_for(plan->n, 1, 4096)), dim3(kThreads), 0,
                           s, plan->n, int(p), A.dinv, x, y);
      }
    };
    // the V-cycle in the precision the inner solver uses
    const bool v32 = plan->mixed || (plan->opts.amg_fp32 && plan->symmetric &&
                                     amg_for(plan, transpose) != nullptr);
    if (v32) {
      float* xf = reinterpret_cast<float*>(plan->ws.W);
      float* yf = reinterpret_cast<float*>(plan->ws.Wt);
      hipLaunchKernelGGL((k_convert<double, float>), dim3(512), dim3(kThreads), 0, s, cnt, X, xf,
                         1.0);
      apply(float(), xf, yf);
      hipLaunchKernelGGL((k_convert<float, double>), dim3(512), dim3(kThreads), 0, s, cnt, yf, Y,
                         1.0);
    } else {
      apply(double(), X, Y);
    }
    HIPCHK(hipStreamSynchronize(s));
    return EXPMV_OK;
  });
}

expmv_status expmv_host_amg_build(int64_t n, const int32_t* rowptr, const int32_t* colind,
                                  const double* val, int symmetric, double theta, int max_coarse,
                                  expmv_amg* out) {
  if (!out) return EXPMV_EINVAL;
  *out = nullptr;
  if (n < 1 || n > INT32_MAX - 1 || !rowptr || !colind || !val || !(theta >= 0.0) ||
      max_coarse < 1 || max_coarse > 4096)
    return EXPMV_EINVAL;
  if (rowptr[0] != 0) return EXPMV_EINVAL;
  for (int64_t i = 0; i < n; ++i)
    if (rowptr[i + 1] < rowptr[i]) return EXPMV_EINVAL;
  const int64_t nnz = rowptr[n];
  for (int64_t e = 0; e < nnz; ++e)
    if (colind[e] < 0 || colind[e] >= n || !std::isfinite(val[e])) return EXPMV_EINVAL;
  try {
    std::unique_ptr<expmv_amg_s> h(new expmv_amg_s());
    HostCsr A;
    A.nrows = A.ncols = n;
    A.rp.assign(rowptr, rowptr + n + 1);
    A.ci.assign(colind, colind + nnz);
    A.v.assign(val, val + nnz);
    AmgParams prm;
    prm.symmetric = symmetric != 0;
    prm.theta = theta;
    prm.max_coarse = max_coarse;
    if (amg_build(A, prm, h->h) != 0) return EXPMV_EINVAL;
    *out = h.release();
    return EXPMV_OK;
  } catch (const std::bad_alloc&) {
    return EXPMV_ENOMEM;
  }
}

int expmv_host_amg_levels(expmv_amg h) { return h ? int(h->h.lv.size()) : 0; }

expmv_status expmv_host_amg_fused(expmv_amg h, int level, int which, double alpha, double beta,
                                  int64_t* dims, int32_t* rowptr, int32_t* colind, double* val) {
  if (!h || level < 0 || level + 1 >= int(h->h.lv.size()) || (which != 0 && which != 1) ||
      !std::isfinite(alpha) || !std::isfinite(beta))
    return EXPMV_EINVAL;
  try {
    const AmgLevelHost& L = h->h.lv[level];
    const HostCsr F = which == 0 ? fused_restriction(L, alpha, beta) : fused_prolongation(L, alpha);
    if (F.nnz() > INT32_MAX) return EXPMV_ENOMEM;
    if (dims) {
      dims[0] = F.nrows;
      dims[1] = F.ncols;
      dims[2] = F.nnz();
    }
    if (rowptr) std::copy(F.rp.begin(), F.rp.end(), rowptr);
    if (colind) std::copy(F.ci.begin(), F.ci.end(), colind);
    if (val) std::copy(F.v.begin(), F.v.end(), val);
    return EXPMV_OK;
  } catch (const std::bad_alloc&) {
    return EXPMV_ENOMEM;
  }
}

expmv_status expmv_host_amg_level(expmv_amg h, int level, int64_t* dims, double* lmax,
                                  int32_t* a_rowptr, int32_t* a_colind, double* a_val,
                                  int32_t* p_rowptr, int32_t* p_colind, double* p_val,
                                  int32_t* agg) {
  if (!h || level < 0 || level >= int(h->h.lv.size())) return EXPMV_EINVAL;
  const AmgLevelHost& L = h->h.lv[level];
  const bool coarsest = level + 1 == int(h->h.lv.size());
  if (dims) {
    dims[0] = L.A.nrows;
    dims[1] = L.A.nnz();
    dims[2] = coarsest ? 0 : L.P.ncols;
    dims[3] = coarsest ? 0 : L.P.nnz();
  }
  if (lmax) *lmax = L.lmax;
  if (a_rowptr) std::copy(L.A.rp.begin(), L.A.rp.end(), a_rowptr);
  if (a_colind) std::copy(L.A.ci.begin(), L.A.ci.end(), a_colind);
  if (a_val) std::copy(L.A.v.begin(), L.A.v.end(), a_val);
  if (!coarsest) {
    if (p_rowptr) std::copy(L.P.rp.begin(), L.P.rp.end(), p_rowptr);
    if (p_colind) std::copy(L.P.ci.begin(), L.P.ci.end(), p_colind);
    if (p_val) std::copy(L.P.v.begin(), L.P.v.end(), p_val);
    if (agg) std::copy(L.agg.begin(), L.agg.end(), agg);
  }
  return EXPMV_OK;
}

expmv_status expmv_host_amg_coarse_inverse(expmv_amg h, double* inv) {
  if (!h || !inv) return EXPMV_EINVAL;
  std::copy(h->h.coarse_inv.begin(), h->h.coarse_inv.end(), inv);
  return EXPMV_OK;
}

void expmv_host_amg_destroy(expmv_amg h) { delete h; }

expmv_status expmv_cf_table(double* tau_re, double* tau_im, double* c_re, double* c_im,
                            double* omega0) {
  for (int j = 0; j < kNShift; ++j) {
    if (tau_re) tau_re[j] = CF_TAU_RE[j];
    if (tau_im) tau_im[j] = CF_TAU_IM[j];
    if (c_re) c_re[j] = CF_C_RE[j];
    if (c_im) c_im[j] = CF_C_IM[j];
  }
  if (omega0) *omega0 = CF_OMEGA0;
  return EXPMV_OK;
}

expmv_status expmv_host_eig_sym(int n, const double* A, double* w, double* Q) {
  if (n < 1 || !A || !w || !Q) return EXPMV_EINVAL;
  return guarded([&]() -> expmv_status {
    return sym_eig(n, A, w, Q) ? EXPMV_OK : EXPMV_ENOCONV;
  });
}

expmv_status expmv_host_eig_general(int n, const double* A, double* wr, double* wi, double* Vr,
                                    double* Vi) {
  if (n < 1 || !A || !wr || !wi || !Vr || !Vi) return EXPMV_EINVAL;
  return guarded([&]() -> expmv_status {
    return general_eig(n, A, wr, wi, Vr, Vi) ? EXPMV_OK : EXPMV_ENOCONV;
  });
}

void expmv_plan_destroy(expmv_plan plan) {
  if (!plan) return;
  if (plan->stream) (void)hipStreamSynchronize(plan->stream);
  else (void)hipDeviceSynchronize();
  if (plan->host_flags) (void)hipHostFree(plan->host_flags);
  if (plan->ev[0]) (void)hipEventDestroy(plan->ev[0]);
  if (plan->ev[1]) (void)hipEventDestroy(plan->ev[1]);
  for (auto& e : plan->kt.ev)
    if (e) (void)hipEventDestroy(e);
  delete plan;
}

const char* expmv_last_error_detail(void) { return g_error_detail; }

const char* expmv_status_string(expmv_status s) {
  switch (s) {
    case EXPMV_OK: return "ok";
    case EXPMV_EINVAL: return "invalid argument";
    case EXPMV_ENOTNEG: return "tA is not negative definite (diagonal entry >= 0)";
    case EXPMV_ENOMEM: return "out of memory";
    case EXPMV_ENOCONV: return "no convergence within max_cycles";
    case EXPMV_EBREAKDOWN: return "rank-deficient Krylov block";
    case EXPMV_EHIP: return "HIP runtime error";
    case EXPMV_EINNER: return "inner solve reached its iteration cap";
  }
  return "unknown status";
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Workspace of expmv_execute_noalloc: a static device array, one copy per GPU
// (the runtime places it when the library's code object is loaded on a
// device), so that call allocates nothing.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in); it asks the
// runtime once per device for that device's address and uses that.

namespace {

constexpr size_t kStaticWorkBytes = EXPMV_STATIC_WORKSPACE_BYTES;
__device__ __align__(256) char scratch[kStaticWorkBytes];

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;                   // one no-allocation call at a time per process
void* g_scratch_ptr[kMaxDevices] = {};    // device address of `scratch` on each device

// address of this device's copy of `scratch`; the device must be current
void* scratch_of_device(int dev) {
  if (dev < 0 || dev >= kMaxDevices) throw StatusError{EXPMV_EINVAL};
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) throw StatusError{EXPMV_EHIP};
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

expmv_status expmv_execute_noalloc(expmv_plan plan, int transpose, const double* B, int64_t p,
                                   double tol, double* Z, expmv_info* info) {
  if (!plan || !B || !Z || p < 1 || p > kMaxP || p > plan->n) return EXPMV_EINVAL;
  if (!(tol > 0.0 && tol < 1.0)) return EXPMV_EINVAL;
  std::lock_guard<std::mutex> lock(g_static_mu);
  return guarded([&]() {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev != plan->device) {
      std::snprintf(g_error_detail, sizeof(g_error_detail),
                    "current device %d is not the plan's device %d", dev, plan->device);
      throw StatusError{EXPMV_EINVAL};
    }
    void* work = scratch_of_device(dev);
    // bind_workspace refuses a call whose workspace exceeds the array (EINVAL)
    bind_workspace(plan, int(p), 1, false, work, kStaticWorkBytes);
    return dispatch_execute(plan, transpose, B, int(p), tol, Z, info);
  });
}

// one-shot forms: plan, a workspace of their own (allocated like the plan's
// set-up buffers), execute, destroy
static expmv_status one_shot(expmv_plan pl, const double* B, int64_t p, double tol, double* Z) {
  size_t bytes = 0;
  expmv_status st = expmv_workspace_size(pl, p, &bytes);
  if (st != EXPMV_OK) return st;
  return guarded([&]() -> expmv_status {
    DevBuf<char> work;
    work.alloc(bytes);
    const expmv_status r = expmv_execute(pl, 0, B, p, tol, work.p, bytes, Z, nullptr);
    HIPCHK(hipStreamSynchronize(pl->stream));
    return r;
  });
}

expmv_status expmv_block_csr(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colind,
                             const double* val, const double* B, int64_t p, double t, double tol,
                             double* Z, hipStream_t stream) {
  expmv_plan pl = nullptr;
  expmv_status st = expmv_plan_csr(n, nnz, rowptr, colind, val, t, nullptr, stream, &pl);
  if (st != EXPMV_OK) return st;
  st = one_shot(pl, B, p, tol, Z);
  expmv_plan_destroy(pl);
  return st;
}

expmv_status expmv_block_toeplitz(int64_t n, const double* col0, const double* B, int64_t p,
                                  double t, double tol, double* Z, hipStream_t stream) {
  expmv_plan pl = nullptr;
  expmv_status st = expmv_plan_toeplitz(n, col0, t, nullptr, stream, &pl);
  if (st != EXPMV_OK) return st;
  st = one_shot(pl, B, p, tol, Z);
  expmv_plan_destroy(pl);
  return st;
}

}  // extern "C"
