// Dense kernels of the expmv library: block Gram-Schmidt passes and CholQR
// on the tall n x p panels, the batched projected shifted solves, the
// panel GEMMs for the solution update and the restart rotation, the final
// pole combination and the true residuals.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "kernels.hpp"

namespace expmv {

enum OrthMode : int {
  kProj = 0,       // partial = V^T W  (+ ||W(:,b)||^2 in the extra p outputs)
  kUpdProj = 1,    // W' = W - V C;  partial = V^T W'
  kUpdGram = 2,    // W' = W - V C;  partial = W'^T W'
  kScaleGram = 3,  // W' = W C (C p x p);  partial = W'^T W'
  kScale = 4       // W' = W C
};

// One streaming pass over the n x p block W against npan basis panels
// (panel i at V + i*n*p), staged through LDS in tiles of TR rows.
// Dynamic LDS: sV[TR][npan*p] (T), sW[TR][p], sW2[TR][p] (T), acc[O] (double).
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_orth(int mode, int64_t n, int p, const T* __restrict__ V, int npan, const T* __restrict__ W,
       T* __restrict__ Wout, const double* __restrict__ C, double* __restrict__ partial,
       int TR, int64_t rows_per_wg, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;   // conditional pass not requested
  extern __shared__ double lds_d[];
  const int tid = threadIdx.x;
  const int np_cols = npan * p;
  const bool use_v = (mode == kProj || mode == kUpdProj || mode == kUpdGram);
  const bool gram = (mode == kUpdGram || mode == kScaleGram);
  const bool proj = (mode == kProj || mode == kUpdProj);
  const int O = proj ? np_cols * p + (mode == kProj ? p : 0) : (gram ? p * p : 0);
  double* acc = lds_d;
  T* sV = reinterpret_cast<T*>(lds_d + O);
  T* sW = sV + (use_v ? size_t(TR) * np_cols : 0);
  T* sW2 = sW + size_t(TR) * p;
  for (int o = tid; o < O; o += kThreads) acc[o] = 0.0;
  const int64_t r_begin = int64_t(blockIdx.x) * rows_per_wg;
  const int64_t r_end = min<int64_t>(n, r_begin + rows_per_wg);
  for (int64_t r0 = r_begin; r0 < r_end; r0 += TR) {
    const int rows = int(min<int64_t>(TR, r_end - r0));
    __syncthreads();
    if (use_v) {
      // panel i holds rows r0..r0+rows-1 as one contiguous run of rows*p values
      const int run = rows * p;
      for (int idx = tid; idx < npan * TR * p; idx += kThreads) {
        const int i = idx / (TR * p), w = idx % (TR * p);
        const int rr = w / p, a = w % p;
        sV[rr * np_cols + i * p + a] =
            (w < run) ? V[int64_t(i) * n * p + r0 * p + w] : T(0);
      }
    }
    for (int idx = tid; idx < TR * p; idx += kThreads)
      sW[idx] = (idx < rows * p) ? W[r0 * p + idx] : T(0);
    __syncthreads();
    if (mode != kProj) {
      for (int idx = tid; idx < TR * p; idx += kThreads) {
        const int rr = idx / p, b = idx % p;
        double s;
        if (mode == kUpdProj || mode == kUpdGram) {
          s = double(sW[idx]);
          const T* vr = sV + rr * np_cols;
          for (int col = 0; col < np_cols; ++col) s -= double(vr[col]) * C[col * p + b];
        } else {
          s = 0.0;
          const T* wr = sW + rr * p;
          for (int a = 0; a < p; ++a) s += double(wr[a]) * C[a * p + b];
        }
        sW2[idx] = T(s);
        if (rr < rows) Wout[r0 * p + idx] = T(s);
      }
      __syncthreads();
    }
    const T* wsrc = (mode == kProj) ? sW : sW2;
    if (proj) {
      for (int o = tid; o < np_cols * p; o += kThreads) {
        const int col = o / p, b = o % p;
        double s = 0.0;
        for (int rr = 0; rr < rows; ++rr) s += double(sV[rr * np_cols + col]) * double(wsrc[rr * p + b]);
        acc[o] += s;
      }
      if (mode == kProj) {
        for (int b = tid; b < p; b += kThreads) {
          double s = 0.0;
          for (int rr = 0; rr < rows; ++rr) s += double(wsrc[rr * p + b]) * double(wsrc[rr * p + b]);
          acc[np_cols * p + b] += s;
        }
      }
    } else if (gram) {
      for (int o = tid; o < p * p; o += kThreads) {
        const int a = o / p, b = o % p;
        double s = 0.0;
        for (int rr = 0; rr < rows; ++rr) s += double(wsrc[rr * p + a]) * double(wsrc[rr * p + b]);
        acc[o] += s;
      }
    }
  }
  __syncthreads();
  for (int o = tid; o < O; o += kThreads) partial[size_t(blockIdx.x) * O + o] = acc[o];
}

// out[o] = sum_w partial[w*O + o], fixed order.  A workgroup takes 16
// adjacent outputs (one 128-byte line of every partial row) with 64 lanes
// each: lane l sums the rows w = l, l + 64, ..., and the 64 sums of an
// output are added in a fixed tree in LDS.  A wavefront reads four whole
// lines per load.
// If H != nullptr the first O_h outputs (rows of C = (npan*p) x p) are also
// added to H[(row) * ldh + col0 + b].
constexpr int kRedOut = 16;     // outputs per workgroup
constexpr int kRedLanes = 64;   // lanes per output
__global__ void __launch_bounds__(kRedOut * kRedLanes)
k_reduce_partials(const double* __restrict__ partial, int nwg, int O, double* __restrict__ out,
                  double* __restrict__ H, int ldh, int col0, int p, int O_h) {
  __shared__ double red[kRedLanes][kRedOut];
  const int oo = threadIdx.x % kRedOut, l = threadIdx.x / kRedOut;
  const int o = blockIdx.x * kRedOut + oo;
  double s = 0.0;
  if (o < O) {
    constexpr int U = 4;
    int w = l;
    for (; w + (U - 1) * kRedLanes < nwg; w += U * kRedLanes) {
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = partial[size_t(w + u * kRedLanes) * O + o];
#pragma unroll
      for (int u = 0; u < U; ++u) s += v[u];
    }
    for (; w < nwg; w += kRedLanes) s += partial[size_t(w) * O + o];
  }
  red[l][oo] = s;
  __syncthreads();
  for (int st = kRedLanes / 2; st >= 1; st >>= 1) {
    if (l < st) red[l][oo] += red[l + st][oo];
    __syncthreads();
  }
  if (l == 0 && o < O) {
    const double v = red[0][oo];
    out[o] = v;
    if (H != nullptr && o < O_h) {
      const int row = o / p, b = o % p;
      H[int64_t(row) * ldh + col0 + b] += v;
    }
  }
}

// Upper Cholesky factor of G + shift I into R (p x p, row-major): 0 = done,
// 1 = done but some pivot is at most 1e-14 of its diagonal entry (a column
// within an angle of about 1e-7 of the span of the earlier ones), 2 = a
// pivot not above 1e-28 trace (or NaN).
__device__ inline int chol_upper(int p, const double* __restrict__ G, double shift, double tr,
                                 double* __restrict__ R) {
  int st = 0;
  for (int j = 0; j < p; ++j) {
    const double gjj = G[j * p + j] + shift;
    double djj = gjj;
    for (int k = 0; k < j; ++k) djj -= R[k * p + j] * R[k * p + j];
    if (!(djj > 1e-28 * tr)) return 2;
    if (djj <= 1e-14 * gjj) st = 1;
    const double rjj = sqrt(djj);
    R[j * p + j] = rjj;
    for (int i = j + 1; i < p; ++i) {
      double s = G[j * p + i];
      for (int k = 0; k < j; ++k) s -= R[k * p + j] * R[k * p + i];
      R[j * p + i] = s / rjj;
    }
    for (int i = 0; i < j; ++i) R[j * p + i] = 0.0;
  }
  return st;
}

// Cholesky of the p x p Gram matrix G = R^T R (R upper) and R^{-1}.
// stage 1 (after Gram-Schmidt): w0norm2 = ||W||_F^2 before projection; a
//   trace(G) <= (1e-12)^2 * w0norm2 is an invariant subspace (happy
//   breakdown): R = R^{-1} = 0 and flags[0] = 1 (w0norm2 = NULL: the
//   initial QR, no such test).  A block that plain
//   Cholesky QR cannot resolve (a nearly collinear column, chol_upper 1 or
//   2) is factored as G + shift trace(G) I instead (shifted Cholesky QR,
//   Fukaya, Kannan, Nakatsukasa, Yamamoto and Yanagisawa, SIAM J. Sci.
//   Comput. 42 (2020)) and flags[2] = 1 requests a third pass; flags[2] = 0
//   otherwise; a failure even then sets flags[1] (rank-deficient block).
// stage 2: H(hrow.., hcol..) = R2 * R1 (R1 from stage 1 in Rprev).
// stage 3 (runs only when flags[2] = 1): the third pass's factor; the H
//   block becomes R3 * (H block).
__global__ void __launch_bounds__(64)
k_cholqr_factor(int p, const double* __restrict__ G, double* __restrict__ R,
                double* __restrict__ Rinv, const double* __restrict__ w0norm2, int stage,
                const double* __restrict__ Rprev, double* __restrict__ H, int ldh, int hrow,
                int hcol, double shift_rel, int* __restrict__ flags) {
  // one wavefront: G, R, R^{-1} and the H block in LDS; the p^3/6 Cholesky on
  // one lane, R^{-1} one column per lane, the products one entry per lane
  __shared__ double sG[kMaxP * kMaxP], sR[kMaxP * kMaxP], sRi[kMaxP * kMaxP],
      sX[kMaxP * kMaxP];
  __shared__ int s_zero;
  const int tid = threadIdx.x;
  if (blockIdx.x != 0) return;
  if (stage == 3 && flags[2] == 0) return;
  const int pp = p * p;
  for (int i = tid; i < pp; i += 64) {
    sG[i] = G[i];
    sR[i] = 0.0;
    sRi[i] = 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    double tr = 0.0;
    for (int i = 0; i < p; ++i) tr += sG[i * p + i];
    // stage 1 of the initial QR (w0norm2 = NULL) has no invariant-subspace test
    double wn = 0.0;
    if (stage == 1 && w0norm2)
      for (int b = 0; b < p; ++b) wn += w0norm2[b];
    bool zero = (stage == 1 && w0norm2) ? (tr <= 1e-24 * wn) : (tr == 0.0);
    if (stage == 1) flags[2] = 0;
    if (!zero) {
      int st = chol_upper(p, sG, 0.0, tr, sR);
      if (stage == 1 && st != 0) {
        st = chol_upper(p, sG, shift_rel * tr, tr, sR);
        if (st != 2) flags[2] = 1;
      } else if (st == 1) {
        st = 0;   // passes 2 and 3 work on blocks already close to orthonormal
      }
      if (st == 2) {   // rank deficient (or NaN)
        flags[1] = 1;
        zero = true;
      }
    } else if (stage == 1 && w0norm2) {
      flags[0] = 1;
    }
    s_zero = zero ? 1 : 0;
  }
  __syncthreads();
  const bool zero = s_zero != 0;
  if (zero) {
    for (int i = tid; i < pp; i += 64) sR[i] = 0.0;
  } else if (tid < p) {
    // column j of R^{-1} (upper triangular) by back substitution
    const int j = tid;
    sRi[j * p + j] = 1.0 / sR[j * p + j];
    for (int i = j - 1; i >= 0; --i) {
      double acc = 0.0;
      for (int k = i + 1; k <= j; ++k) acc += sR[i * p + k] * sRi[k * p + j];
      sRi[i * p + j] = -acc / sR[i * p + i];
    }
  }
  __syncthreads();
  for (int i = tid; i < pp; i += 64) {
    R[i] = sR[i];
    Rinv[i] = sRi[i];
  }
  if (H == nullptr || (stage != 2 && stage != 3)) return;
  // stage 2: H block = R2 * R1 (Rprev); stage 3: H block <- R3 * H block
  for (int i = tid; i < pp; i += 64)
    sX[i] = stage == 2 ? Rprev[i] : H[int64_t(hrow + i / p) * ldh + hcol + i % p];
  __syncthreads();
  for (int o = tid; o < pp; o += 64) {
    const int i = o / p, j = o % p;
    double acc = 0.0;
    for (int k = stage == 2 ? 0 : i; k < p; ++k) acc += sR[i * p + k] * sX[k * p + j];
    H[int64_t(hrow + i) * ldh + hcol + j] = acc;
  }
}

// ---------------------------------------------------------------------------
// complex helpers
struct cplx {
  double x, y;
};
__device__ inline cplx cmul(cplx a, cplx b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ inline cplx csub(cplx a, cplx b) { return {a.x - b.x, a.y - b.y}; }
__device__ inline cplx cdiv(cplx a, cplx b) {
  // Smith's algorithm
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, den = b.x + b.y * r;
    return {(a.x + a.y * r) / den, (a.y - a.x * r) / den};
  }
  const double r = b.x / b.y, den = b.x * r + b.y;
  return {(a.x * r + a.y) / den, (a.y * r - a.x) / den};
}

constexpr int kProjMaxD = 64 * kMaxP;   // m <= 64 block steps of p <= kMaxP columns
constexpr int kProjLdsZ = 4096;   // d * p of the back substitution through LDS
constexpr int kProjLdsRows = 256; // and its largest d
constexpr int kProjUCols = 8;     // columns of U per LDS chunk

// Projected shifted systems, one workgroup per pole j (Section 4.1, eq. 4.7):
//   precond: (I - tau_j H_d) Z_j = G_j,  S_j = tau_j H(d:d+p, 0:d) Z_j,
//            Cr(:, shift j) = H~ Z_j  ((d+p) x p, real and imaginary parts;
//            skipped when Cr is NULL)
//   plain:   (H_d - tau_j I) Z_j = G_j,  S_j = -H(d:d+p, 0:d) Z_j,
//            Cr(:, shift j) = [Z_j; 0]
// LU with partial pivoting on a d x d complex matrix in global scratch
// (in LDS its column accesses, at a stride of d entries, hit one bank: it
// measured slower), limited to the matrix's lower band: L(c), the last row
// that can be nonzero in column c during the elimination, is the running
// maximum over columns c' <= c of the last nonzero row of H in column c'.
// Rows below L(c) are zero in every column up to c, are never chosen as a
// pivot and receive zero updates, so they are skipped: the same arithmetic
// as the dense elimination, with p to 2p - 1 rows per column instead of
// d - c on the block Hessenberg H_d of one cycle (a dense leading block
// after a restart widens the band there).
// rho_j = ||S_j||_F (eq. 4.9 / eq. 3.6).
__global__ void __launch_bounds__(1024)
k_proj_solve(int d, int p, int precond, const double* __restrict__ H, int ldh,
             const double* __restrict__ tau_re, const double* __restrict__ tau_im,
             const cplx* __restrict__ G, cplx* __restrict__ Ascr, cplx* __restrict__ Zs,
             double* __restrict__ Cr, int ldc, cplx* __restrict__ S, double* __restrict__ rho,
             int* __restrict__ singular) {
  const int j = blockIdx.x;
  const int tid = threadIdx.x, nt = blockDim.x;
  const cplx tau{tau_re[j], tau_im[j]};
  cplx* A = Ascr + size_t(j) * d * d;
  cplx* Z = Zs + size_t(j) * d * p;
  const cplx* Gj = G + size_t(j) * d * p;
  __shared__ int s_piv, s_zero;
  __shared__ cplx s_inv;   // 1 / pivot
  __shared__ int s_lim[kProjMaxD];   // L(c)
  for (int c = tid; c < d; c += nt) s_lim[c] = c;
  __syncthreads();
  for (int idx = tid; idx < d * d; idx += nt) {
    const int r = idx / d, c = idx % d;
    const double h = H[int64_t(r) * ldh + c];
    if (r > c && h != 0.0) atomicMax(&s_lim[c], r);
    cplx a;
    if (precond) {
      a = {-tau.x * h, -tau.y * h};
      if (r == c) a.x += 1.0;
    } else {
      a = {h, 0.0};
      if (r == c) {
        a.x -= tau.x;
        a.y -= tau.y;
      }
    }
    A[idx] = a;
  }
  for (int idx = tid; idx < d * p; idx += nt) Z[idx] = Gj[idx];
  __syncthreads();
  if (tid < 64) {   // running maximum, one wavefront, 64 columns per step
    int carry = 0;
    for (int c0 = 0; c0 < d; c0 += 64) {
      int v = c0 + tid < d ? s_lim[c0 + tid] : 0;
      for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(v, off, 64);
        if (tid >= off) v = max(v, o);
      }
      v = max(v, carry);
      if (c0 + tid < d) s_lim[c0 + tid] = v;
      carry = __shfl(v, 63, 64);
    }
  }
  __syncthreads();
  int sing = 0;
  for (int c = 0; c < d; ++c) {
    const int last = s_lim[c];
    // pivot: the first row of largest |a|^2 in column c, by one wavefront,
    // and its reciprocal (one division per column instead of one per entry)
    if (tid < 64) {
      double best = -1.0;
      int bi = c;
      cplx bv{0.0, 0.0};
      for (int r = c + tid; r <= last; r += 64) {
        const cplx a = A[r * d + c];
        const double v = a.x * a.x + a.y * a.y;
        if (v > best) {
          best = v;
          bi = r;
          bv = a;
        }
      }
      for (int off = 32; off >= 1; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        const cplx ov{__shfl_xor(bv.x, off, 64), __shfl_xor(bv.y, off, 64)};
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
          bv = ov;
        }
      }
      if (tid == 0) {
        s_piv = bi;
        s_zero = !(best > 0.0);
        s_inv = best > 0.0 ? cdiv(cplx{1.0, 0.0}, bv) : cplx{0.0, 0.0};
      }
    }
    __syncthreads();
    const int pv = s_piv;
    if (s_zero) {   // zero column: singular, nothing to eliminate
      sing = 1;
      __syncthreads();   // every thread has read s_piv, s_zero before the next pivot
      continue;
    }
    if (pv != c) {
      for (int cc = c + tid; cc < d; cc += nt) {
        const cplx t0 = A[c * d + cc];
        A[c * d + cc] = A[pv * d + cc];
        A[pv * d + cc] = t0;
      }
      for (int b = tid; b < p; b += nt) {
        const cplx t0 = Z[c * p + b];
        Z[c * p + b] = Z[pv * p + b];
        Z[pv * p + b] = t0;
      }
    }
    __syncthreads();
    // rows c+1..L(c): multiplier l_r = a_rc * (1 / a_cc) formed where it is used
    const cplx inv = s_inv;
    const int m1 = d - c - 1;
    const int wide = m1 + p;
    const int rows = last - c;
    for (int idx = tid; idx < rows * wide; idx += nt) {
      const int r = c + 1 + idx / wide;
      const int cc = idx % wide;
      const cplx l = cmul(A[r * d + c], inv);
      if (cc < m1) {
        const int col = c + 1 + cc;
        A[r * d + col] = csub(A[r * d + col], cmul(l, A[c * d + col]));
      } else {
        const int b = cc - m1;
        Z[r * p + b] = csub(Z[r * p + b], cmul(l, Z[c * p + b]));
      }
    }
    __syncthreads();
  }
  if (d * p <= kProjLdsZ && d <= kProjLdsRows) {
    // back substitution through LDS: Z, the reciprocals of the diagonal of
    // U (formed once, in parallel) and U in chunks of kProjUCols columns
    // (one global load pass and one extra barrier per chunk), so that a
    // step costs two complex products and one barrier; x_c = z_c * (1/u_cc)
    // rounds differently from z_c / u_cc by an ulp
    __shared__ cplx sZ[kProjLdsZ];
    __shared__ cplx sU[kProjUCols][kProjLdsRows];   // column c in slot c % kProjUCols
    __shared__ cplx sInv[kProjLdsRows];
    for (int idx = tid; idx < d * p; idx += nt) sZ[idx] = Z[idx];
    for (int c = tid; c < d; c += nt) {
      const cplx dg = A[c * d + c];
      sInv[c] = (dg.x == 0.0 && dg.y == 0.0) ? cplx{0.0, 0.0} : cdiv(cplx{1.0, 0.0}, dg);
    }
    auto xval = [&](int c, int b) -> cplx { return cmul(sZ[c * p + b], sInv[c]); };
    for (int c = d - 1; c >= 0; --c) {
      if (c == d - 1 || c % kProjUCols == kProjUCols - 1) {
        // columns lo..c, rows above the diagonal; readers of the previous
        // chunk finished before the last barrier
        const int lo = c - c % kProjUCols, nc = c - lo + 1;
        for (int idx = tid; idx < c * nc; idx += nt) {
          const int r = idx / nc, col = lo + idx % nc;
          if (r < col) sU[col % kProjUCols][r] = A[r * d + col];
        }
        __syncthreads();
      }
      cplx xn{0.0, 0.0};
      const bool wr = c + 1 < d && tid < p;
      if (wr) xn = xval(c + 1, tid);
      const cplx* u = sU[c % kProjUCols];
      for (int idx = tid; idx < c * p; idx += nt) {
        const int r = idx / p, b = idx % p;
        sZ[r * p + b] = csub(sZ[r * p + b], cmul(u[r], xval(c, b)));
      }
      if (wr) sZ[(c + 1) * p + tid] = xn;
      __syncthreads();
    }
    if (tid < p) sZ[tid] = xval(0, tid);
    __syncthreads();
    for (int idx = tid; idx < d * p; idx += nt) Z[idx] = sZ[idx];
    __syncthreads();
  } else {
    // back substitution, one barrier per column: every thread forms
    // x_c = z_c / u_cc itself; row c of Z is overwritten by x_c one step
    // later, when no thread reads it any more
    auto xval = [&](int c, int b) -> cplx {
      const cplx dg = A[c * d + c];
      return (dg.x == 0.0 && dg.y == 0.0) ? cplx{0.0, 0.0} : cdiv(Z[c * p + b], dg);
    };
    for (int c = d - 1; c >= 0; --c) {
      cplx xn{0.0, 0.0};
      const bool wr = c + 1 < d && tid < p;
      if (wr) xn = xval(c + 1, tid);
      for (int idx = tid; idx < c * p; idx += nt) {
        const int r = idx / p, b = idx % p;
        Z[r * p + b] = csub(Z[r * p + b], cmul(A[r * d + c], xval(c, b)));
      }
      if (wr) Z[(c + 1) * p + tid] = xn;
      __syncthreads();
    }
    if (tid < p) Z[tid] = xval(0, tid);   // row 0: each thread its own entry
    __syncthreads();
  }
  if (tid == 0 && sing) singular[j] = 1;
  // update coefficients Cr (rows d+p, ld ldc = 2 p x shifts): real part then
  // imaginary part (Cr = NULL: only the residual estimates are wanted)
  for (int idx = tid; Cr && idx < (d + p) * p; idx += nt) {
    const int r = idx / p, b = idx % p;
    cplx s{0.0, 0.0};
    if (precond) {
      for (int c = 0; c < d; ++c) {
        const double h = H[int64_t(r) * ldh + c];
        const cplx z = Z[c * p + b];
        s.x += h * z.x;
        s.y += h * z.y;
      }
    } else if (r < d) {
      s = Z[r * p + b];
    }
    Cr[int64_t(r) * ldc + 2 * p * j + b] = s.x;
    Cr[int64_t(r) * ldc + 2 * p * j + p + b] = s.y;
  }
  // S_j and rho_j
  for (int idx = tid; idx < p * p; idx += nt) {
    const int a = idx / p, b = idx % p;
    cplx s{0.0, 0.0};
    for (int c = 0; c < d; ++c) {
      const double h = H[int64_t(d + a) * ldh + c];
      const cplx z = Z[c * p + b];
      s.x += h * z.x;
      s.y += h * z.y;
    }
    S[size_t(j) * p * p + idx] = precond ? cmul(tau, s) : cplx{-s.x, -s.y};
  }
  __syncthreads();
  if (tid == 0) {
    double ss = 0.0;
    for (int idx = 0; idx < p * p; ++idx) {
      const cplx v = S[size_t(j) * p * p + idx];
      ss += v.x * v.x + v.y * v.y;
    }
    rho[j] = sqrt(ss);
  }
}

// Right-hand sides of the projected systems: G_j = 0 except rows
// row0..row0+p-1 = src (cycle 1: src = R^ real p x p, same for all j;
// after a restart: src = S_j complex).
__global__ void k_build_rhs(int d, int p, int row0, int complex_src, const double* __restrict__ Rhat,
                            const cplx* __restrict__ S, cplx* __restrict__ G) {
  const int j = blockIdx.y;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < d * p; idx += gridDim.x * blockDim.x) {
    const int r = idx / p, b = idx % p;
    cplx v{0.0, 0.0};
    if (r >= row0 && r < row0 + p) {
      const int a = r - row0;
      if (complex_src) v = S[size_t(j) * p * p + a * p + b];
      else v = {Rhat[a * p + b], 0.0};
    }
    G[size_t(j) * d * p + idx] = v;
  }
}

// out chunk q (p columns) (+)= sum_c V(:, c) C(c, q*p + b), V = npan panels.
// Output chunk q starts at out + q * chunk_stride with row stride ldo.
// Dynamic LDS: sV[TR][npan*p] (T), sC[npan*p][p] (double).
template <typename T, typename TO>
__global__ void __launch_bounds__(kThreads)
k_panel_gemm(int64_t n, int p, const T* __restrict__ V, int npan, const double* __restrict__ C,
             int ldc, TO* __restrict__ out, int64_t chunk_stride, int64_t ldo, int accumulate,
             int TR, int64_t rows_per_wg) {
  extern __shared__ double lds_d[];
  const int q = blockIdx.y;
  const int np_cols = npan * p;
  double* sC = lds_d;
  T* sV = reinterpret_cast<T*>(lds_d + size_t(np_cols) * p);
  const int tid = threadIdx.x;
  for (int idx = tid; idx < np_cols * p; idx += kThreads) {
    const int c = idx / p, b = idx % p;
    sC[idx] = C[int64_t(c) * ldc + q * p + b];
  }
  TO* o = out + q * chunk_stride;
  const int64_t r_begin = int64_t(blockIdx.x) * rows_per_wg;
  const int64_t r_end = min<int64_t>(n, r_begin + rows_per_wg);
  for (int64_t r0 = r_begin; r0 < r_end; r0 += TR) {
    const int rows = int(min<int64_t>(TR, r_end - r0));
    __syncthreads();
    const int run = rows * p;
    for (int idx = tid; idx < npan * TR * p; idx += kThreads) {
      const int i = idx / (TR * p), w = idx % (TR * p);
      const int rr = w / p, a = w % p;
      sV[rr * np_cols + i * p + a] = (w < run) ? V[int64_t(i) * n * p + r0 * p + w] : T(0);
    }
    __syncthreads();
    for (int idx = tid; idx < rows * p; idx += kThreads) {
      const int rr = idx / p, b = idx % p;
      const T* vr = sV + rr * np_cols;
      double s = 0.0;
      for (int c = 0; c < np_cols; ++c) s += double(vr[c]) * sC[c * p + b];
      TO* dst = o + (r0 + rr) * ldo + b;
      *dst = accumulate ? TO(double(*dst) + s) : TO(s);
    }
  }
}

// Z = omega0 B + sum_j Re(c_j X_j), X row-major n x 14p (shift j: real part
// in columns 2pj..2pj+p-1, imaginary part in 2pj+p..2pj+2p-1); partial ||Z||^2.
__global__ void __launch_bounds__(kThreads)
k_combine(int64_t n, int p, const double* __restrict__ B, const double* __restrict__ X, int ldx,
          double omega0, const double* __restrict__ c_re, const double* __restrict__ c_im,
          double* __restrict__ Z, double* __restrict__ partial) {
  __shared__ double red[kThreads];
  double zz = 0.0;
  for (int64_t idx = int64_t(blockIdx.x) * kThreads + threadIdx.x; idx < n * p;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t r = idx / p;
    const int b = int(idx % p);
    double s = omega0 * B[idx];
    const double* xr = X + r * ldx;
    for (int j = 0; j < kNShift; ++j) s += c_re[j] * xr[2 * p * j + b] - c_im[j] * xr[2 * p * j + p + b];
    Z[idx] = s;
    zz += s * s;
  }
  red[threadIdx.x] = zz;
  __syncthreads();
  for (int st = kThreads / 2; st >= 1; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Source-term combination over the joined block [U0 | S] (width 2 pu):
// U = omega0 U0 + sum_j Re(c_j X_j[U0 part]) + Re(s_j X_j[S part]), X_j's real
// part in columns 4 pu j .. 4 pu j + 2 pu - 1 (the U0 part first, then the S
// part), its imaginary part in the next 2 pu columns; partial ||U||^2.
__global__ void __launch_bounds__(kThreads)
k_combine_source(int64_t n, int pu, const double* __restrict__ B, const double* __restrict__ X,
                 int ldx, double omega0, const double* __restrict__ c_re,
                 const double* __restrict__ c_im, const double* __restrict__ s_re,
                 const double* __restrict__ s_im, double* __restrict__ U,
                 double* __restrict__ partial) {
  __shared__ double red[kThreads];
  double uu = 0.0;
  for (int64_t idx = int64_t(blockIdx.x) * kThreads + threadIdx.x; idx < n * pu;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t r = idx / pu;
    const int b = int(idx % pu);
    double u = omega0 * B[r * 2 * pu + b];
    const double* xr = X + r * ldx;
    for (int j = 0; j < kNShift; ++j) {
      const double* xj = xr + 4 * pu * j;
      u += c_re[j] * xj[b] - c_im[j] * xj[2 * pu + b] + s_re[j] * xj[pu + b] -
           s_im[j] * xj[3 * pu + b];
    }
    U[idx] = u;
    uu += u * u;
  }
  red[threadIdx.x] = uu;
  __syncthreads();
  for (int st = kThreads / 2; st >= 1; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// words 32-bit words of p set to zero (a kernel rather than a memset, so the
// clearing is an ordinary launch on the stream)
__global__ void __launch_bounds__(kThreads) k_zero32(int64_t words, uint32_t* __restrict__ p) {
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < words;
       i += int64_t(gridDim.x) * kThreads)
    p[i] = 0u;
}

// partial dot <G, K Z> per workgroup (K in CSR)
template <int PP>
__global__ void __launch_bounds__(kThreads)
k_dot_spmm(int64_t n, int p, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
           const double* __restrict__ val, const double* __restrict__ Gm,
           const double* __restrict__ Zm, double* __restrict__ partial) {
  __shared__ double red[kThreads];
  const int c = threadIdx.x % PP;
  double s = 0.0;
  const int64_t rows_per_grid = int64_t(gridDim.x) * (kThreads / PP);
  for (int64_t row = int64_t(blockIdx.x) * (kThreads / PP) + threadIdx.x / PP; row < n;
       row += rows_per_grid) {
    if (c < p) {
      double acc = 0.0;
      for (int e = rowptr[row]; e < rowptr[row + 1]; ++e) acc += val[e] * Zm[int64_t(colind[e]) * p + c];
      s += Gm[row * p + c] * acc;
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = kThreads / 2; st >= 1; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// partial[wg * 16 + v]: v = 2j, 2j+1: sum Re(X_j) . B and Im(X_j) . B
// (j < 7); v = 14: G . B; v = 15: G . KB (KB given, may be null)
__global__ void __launch_bounds__(kThreads)
k_adjoint_dots(int64_t n, int p, const double* __restrict__ X, const double* __restrict__ B,
               const double* __restrict__ G, const double* __restrict__ KB,
               double* __restrict__ partial) {
  __shared__ double red[kThreads];
  const int ldx = 2 * kNShift * p;
  double acc[16];
  for (int v = 0; v < 16; ++v) acc[v] = 0.0;
  for (int64_t idx = int64_t(blockIdx.x) * kThreads + threadIdx.x; idx < n * p;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t r = idx / p;
    const int b = int(idx % p);
    const double bv = B[idx];
    for (int j = 0; j < kNShift; ++j) {
      acc[2 * j] += X[r * ldx + 2 * p * j + b] * bv;
      acc[2 * j + 1] += X[r * ldx + 2 * p * j + p + b] * bv;
    }
    acc[14] += G[idx] * bv;
    if (KB) acc[15] += G[idx] * KB[idx];
  }
  for (int v = 0; v < 16; ++v) {
    red[threadIdx.x] = acc[v];
    __syncthreads();
    for (int st = kThreads / 2; st >= 1; st >>= 1) {
      if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[size_t(blockIdx.x) * 16 + v] = red[0];
    __syncthreads();
  }
}

// small helpers
template <typename TI, typename TO>
__global__ void k_convert(int64_t count, const TI* __restrict__ in, TO* __restrict__ out, double scale) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * blockDim.x)
    out[i] = TO(scale * double(in[i]));
}

__global__ void k_fill_zero_d(int64_t count, double* __restrict__ out) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * blockDim.x)
    out[i] = 0.0;
}

}  // namespace expmv
