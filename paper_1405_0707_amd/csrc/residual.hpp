// True residuals of the shifted systems after a cycle, in FP64, and their
// split into the part along the last basis block and the rest.
//
// After a cycle of Algorithm 2 (and of Algorithm 1) every shifted system's
// residual is, in exact arithmetic, R_j = B - (M - tau_j I) X_j =
// V_{d+1} S_j: a combination of the one block that follows the basis (the
// collinearity of Section 3, eq. 4.8), which the restart keeps as its
// right-hand side.  Inexact inner solves and an FP32 basis add a defect to
// each R_j.  Here R_j is recomputed from X_j with the FP64 operator, its
// coordinates S_j = V_{d+1}^T R_j replace the restart right-hand side
// (iterative refinement: the next cycle solves for the defect's projection
// too), and ||R_j - V_{d+1} S_j||_F measures what the shared block cannot
// carry.
//
// Layout: R is row-major n x 14p for the 7 shifts of one time (shift j:
// real part in columns 2pj..2pj+p-1, imaginary part in the next p), like X.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "kernels.hpp"
#include "kernels_dense.hpp"

namespace expmv {

constexpr int kResGrid = 512;   // workgroups of the projection and remainder passes

// R = B + K X_j + tau_j X_j (K = -M) for the 7 shifts of one time block and
// partial[wg * 7 + j] = sum of |R_j|^2 over the workgroup's rows.  K is CSR
// (rowptr != NULL) or given as the product KX (n x 14p, ld 14p, rowptr ==
// NULL; KX may be R itself: each entry is read by the thread that
// overwrites it).  PP lanes per row, lane c < p owns column c of every shift.
template <int PP>
__global__ void __launch_bounds__(kThreads)
k_shift_residual(int64_t n, int p, const int32_t* __restrict__ rowptr,
                 const int32_t* __restrict__ colind, const double* __restrict__ val,
                 const double* KX, const double* __restrict__ B, const double* __restrict__ X,
                 int ldx, const double* __restrict__ tau_re, const double* __restrict__ tau_im,
                 double* R, double* __restrict__ partial) {
  __shared__ double red[kThreads];
  const int c = threadIdx.x % PP;
  const int W = 2 * kNShift * p;
  double nr[kNShift];
#pragma unroll
  for (int j = 0; j < kNShift; ++j) nr[j] = 0.0;
  const int64_t rows_per_grid = int64_t(gridDim.x) * (kThreads / PP);
  for (int64_t row = int64_t(blockIdx.x) * (kThreads / PP) + threadIdx.x / PP; row < n;
       row += rows_per_grid) {
    if (c < p) {
      const double bv = B[row * p + c];
      int e0 = 0, e1 = 0;
      // the row's first kRU entries, loaded once for all seven poles
      constexpr int kRU = 8;
      int32_t jj[kRU];
      double vv[kRU];
      if (rowptr) {
        e0 = rowptr[row];
        e1 = rowptr[row + 1];
#pragma unroll
        for (int u = 0; u < kRU; ++u) {
          const bool ok = e0 + u < e1;
          jj[u] = ok ? colind[e0 + u] : -1;
          vv[u] = ok ? val[e0 + u] : 0.0;
        }
      }
#pragma unroll 1
      for (int j = 0; j < kNShift; ++j) {
        double kr = 0.0, ki = 0.0;
        if (rowptr) {
          // the gathers of one pole all in flight, in the row's order
          double xr[kRU], xi[kRU];
#pragma unroll
          for (int u = 0; u < kRU; ++u) {
            if (jj[u] >= 0) {
              const double* xc = X + int64_t(jj[u]) * ldx + 2 * p * j;
              xr[u] = xc[c];
              xi[u] = xc[p + c];
            } else {
              xr[u] = xi[u] = 0.0;
            }
          }
#pragma unroll
          for (int u = 0; u < kRU; ++u) {
            kr += vv[u] * xr[u];
            ki += vv[u] * xi[u];
          }
          for (int e = e0 + kRU; e < e1; ++e) {
            const double* xc = X + int64_t(colind[e]) * ldx + 2 * p * j;
            kr += val[e] * xc[c];
            ki += val[e] * xc[p + c];
          }
        } else {
          kr = KX[row * W + 2 * p * j + c];
          ki = KX[row * W + 2 * p * j + p + c];
        }
        const double* xs = X + row * ldx + 2 * p * j;
        const double xr = xs[c], xi = xs[p + c];
        const double rr = bv + kr + tau_re[j] * xr - tau_im[j] * xi;
        const double ri = ki + tau_re[j] * xi + tau_im[j] * xr;
        R[row * W + 2 * p * j + c] = rr;
        R[row * W + 2 * p * j + p + c] = ri;
        nr[j] += rr * rr + ri * ri;
      }
    }
  }
  for (int j = 0; j < kNShift; ++j) {
    red[threadIdx.x] = nr[j];
    __syncthreads();
    for (int st = kThreads / 2; st >= 1; st >>= 1) {
      if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[size_t(blockIdx.x) * kNShift + j] = red[0];
    __syncthreads();
  }
}

// Contiguous rows of workgroup b out of G.
__device__ inline void res_rows(int64_t n, int64_t& r0, int64_t& r1) {
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  r0 = min<int64_t>(n, int64_t(blockIdx.x) * per);
  r1 = min<int64_t>(n, r0 + per);
}

// partial[wg][a * W + col] = sum over the workgroup's rows of V(i, a) R(i, col)
// (V: the last basis block, n x p in the basis type; R: n x W FP64, W = 14p
// <= 2 kThreads).  Thread t owns columns t and t + kThreads; every thread of
// a row reads the same p entries of V.
// The workgroup's rows go in chunks of kResChunk: the chunk's rows of V are
// staged in LDS (one coalesced load), then every thread walks them kResU
// rows at a time with all of those rows' R loads issued together.
constexpr int kResChunk = 64, kResU = 8;

template <typename T, int PP>
__device__ inline void stage_v_chunk(const T* __restrict__ V, int p, int64_t i0, int rows,
                                     double (*sv)[PP]) {
  for (int e = threadIdx.x; e < rows * PP; e += kThreads) {
    const int r = e / PP, a = e % PP;
    sv[r][a] = a < p ? double(V[(i0 + r) * p + a]) : 0.0;
  }
}

template <typename T, int PP>
__global__ void __launch_bounds__(kThreads)
k_project_block(int64_t n, int p, const T* __restrict__ V, const double* __restrict__ R, int W,
                double* __restrict__ partial) {
  __shared__ double sv[kResChunk][PP];
  const int col0 = threadIdx.x, col1 = threadIdx.x + kThreads;
  const bool has0 = col0 < W, has1 = col1 < W;
  double a0[PP], a1[PP];
#pragma unroll
  for (int a = 0; a < PP; ++a) a0[a] = a1[a] = 0.0;
  int64_t r0, r1;
  res_rows(n, r0, r1);
  for (int64_t i0 = r0; i0 < r1; i0 += kResChunk) {
    const int rows = int(min<int64_t>(kResChunk, r1 - i0));
    __syncthreads();   // the previous chunk is consumed
    stage_v_chunk<T, PP>(V, p, i0, rows, sv);
    __syncthreads();
    for (int r = 0; r < rows; r += kResU) {
      double x0[kResU], x1[kResU];
#pragma unroll
      for (int u = 0; u < kResU; ++u) {
        const bool ok = r + u < rows;
        const int64_t i = i0 + r + u;
        x0[u] = (ok && has0) ? R[i * W + col0] : 0.0;
        x1[u] = (ok && has1) ? R[i * W + col1] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kResU; ++u) {
        if (r + u >= rows) continue;   // past the chunk (sv there is stale)
#pragma unroll
        for (int a = 0; a < PP; ++a) {
          const double v = sv[r + u][a];
          a0[a] += v * x0[u];
          a1[a] += v * x1[u];
        }
      }
    }
  }
  double* out = partial + size_t(blockIdx.x) * size_t(p) * W;
#pragma unroll
  for (int a = 0; a < PP; ++a) {
    if (a < p) {
      if (has0) out[a * W + col0] = a0[a];
      if (has1) out[a * W + col1] = a1[a];
    }
  }
}

// partial[wg * 7 + j] = sum over the workgroup's rows of |R_j - V S_j|^2,
// C = [S_j] as the p x W real matrix (C(a, 2pj + b) = Re S_j(a, b),
// C(a, 2pj + p + b) = Im S_j(a, b)).
template <typename T, int PP>
__global__ void __launch_bounds__(kThreads)
k_remainder_norms(int64_t n, int p, const T* __restrict__ V, const double* __restrict__ R, int W,
                  const double* __restrict__ C, double* __restrict__ partial) {
  __shared__ double scol[2 * kThreads];
  const int col0 = threadIdx.x, col1 = threadIdx.x + kThreads;
  const bool has0 = col0 < W, has1 = col1 < W;
  double c0[PP], c1[PP];
#pragma unroll
  for (int a = 0; a < PP; ++a) {
    c0[a] = (a < p && has0) ? C[a * W + col0] : 0.0;
    c1[a] = (a < p && has1) ? C[a * W + col1] : 0.0;
  }
  __shared__ double sv[kResChunk][PP];
  double s0 = 0.0, s1 = 0.0;
  int64_t r0, r1;
  res_rows(n, r0, r1);
  for (int64_t i0 = r0; i0 < r1; i0 += kResChunk) {
    const int rows = int(min<int64_t>(kResChunk, r1 - i0));
    __syncthreads();
    stage_v_chunk<T, PP>(V, p, i0, rows, sv);
    __syncthreads();
    for (int r = 0; r < rows; r += kResU) {
      double e0[kResU], e1[kResU];
#pragma unroll
      for (int u = 0; u < kResU; ++u) {
        const bool ok = r + u < rows;
        const int64_t i = i0 + r + u;
        e0[u] = (ok && has0) ? R[i * W + col0] : 0.0;
        e1[u] = (ok && has1) ? R[i * W + col1] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kResU; ++u) {
        if (r + u >= rows) continue;
#pragma unroll
        for (int a = 0; a < PP; ++a) {
          const double v = sv[r + u][a];
          e0[u] -= v * c0[a];
          e1[u] -= v * c1[a];
        }
        s0 += e0[u] * e0[u];
        s1 += e1[u] * e1[u];
      }
    }
  }
  scol[col0] = s0;
  scol[col1] = s1;
  __syncthreads();
  if (threadIdx.x < kNShift) {
    const int j = threadIdx.x;
    double s = 0.0;
    for (int q = 2 * p * j; q < 2 * p * (j + 1); ++q) s += scol[q];
    partial[size_t(blockIdx.x) * kNShift + j] = s;
  }
}

// S_j (complex p x p, S[j][a][b]) from the real p x W coordinates C.
__global__ void __launch_bounds__(kThreads)
k_restart_rhs(int p, const double* __restrict__ C, int W, cplx* __restrict__ S) {
  const int total = kNShift * p * p;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += gridDim.x * blockDim.x) {
    const int j = idx / (p * p), a = (idx / p) % p, b = idx % p;
    S[idx] = cplx{C[a * W + 2 * p * j + b], C[a * W + 2 * p * j + p + b]};
  }
}

}  // namespace expmv
