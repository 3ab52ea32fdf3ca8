// Device kernels of the smoothed-aggregation AMG V-cycle that preconditions
// the inner solver of (tA)^{-1} V (the hierarchy is built on the host, see
// amg_host.hpp).  Every kernel works on n x p row-major blocks with PP lanes
// per row, like the inner solver, and returns at once when the inner solve
// it belongs to has finished (ctl, iteration k; ctl = NULL: never).
//
// Smoother: Chebyshev iteration on D^{-1} A over [lmax / ratio, lmax]
// (three-term recurrence, Saad, Iterative Methods for Sparse Linear
// Systems, Algorithm 12.1):
//   step 0:  d = a_0 D^{-1} (b - A x),            x <- x + d
//   step k:  d = c_k d + a_k D^{-1} (b - A x),    x <- x + d
// From x = 0 the first step is x = a_0 D^{-1} b = d; that iterate is never
// stored (mode kAmgX0 recomputes it from b wherever it is read).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "kernels.hpp"

namespace expmv {

enum : int {
  kAmgX0 = 1,      // x (and the previous d) = s0 D^{-1} b, not stored
  kAmgResid = 2,   // out = b - A x instead of a smoothing step
  kAmgWriteD = 4,  // store the new direction d
  kAmgHasD = 8,    // the step continues a recurrence: uses c * (previous d)
  kAmgRz = 16,     // partial sums (b, out) per column into part[wg][0][c]
                   // (finest level, inner-solver launch shape only)
};

// A row is handled by a group of PP * G lanes: lane (c, g) = c + PP g takes
// column c and the nonzeros e0 + g, e0 + g + G, ... of the row, and the G
// partial sums of a column are added with shuffles inside the group (G > 1
// for the long rows of Galerkin operators and restrictions, whose serial
// sums would otherwise set the kernel's latency).  PP * G <= 64, so a group
// never straddles a wavefront.
//
// Rows of a group: SEG = one contiguous XCD-aware segment per workgroup (the
// inner solver's layout), else a grid-stride loop.  Every lane of a group
// runs the same rows, so the shuffles always see a whole group.
template <int NT, int PP, bool SEG>
struct RowRange {
  int64_t r, end, step;
  __device__ RowRange(int64_t n, int G) {
    const int lanes = PP * G;
    if (SEG) {
      int64_t s0, s1;
      xcd_rows(n, s0, s1);
      r = s0 + threadIdx.x / lanes;
      end = s1;
      step = NT / lanes;
    } else {
      r = int64_t(blockIdx.x) * (NT / lanes) + threadIdx.x / lanes;
      end = n;
      step = int64_t(gridDim.x) * (NT / lanes);
    }
  }
};

// sum over the row's nonzeros of val[e] * w(j) with w(j) = x[j * ld + c] (or
// s0 * dinv[j] * x[j * ld + c] when scaled), split over the G sub-lanes and
// summed across them; every lane of the group receives the row's sum.  The
// operator values have the vectors' type (an FP32 V-cycle reads FP32 values);
// the sums are FP64.
template <typename T, int PP, bool SCALED>
__device__ inline double row_dot_split(const int32_t* __restrict__ colind,
                                       const T* __restrict__ val, const T* __restrict__ x,
                                       const T* __restrict__ dinv, int e0, int e1, int ld, int c,
                                       bool active, int g, int G) {
  constexpr int U = 8;   // nonzeros per sub-lane step, all loads issued first
  double acc = 0.0;
  if (active) {
    for (int e = e0 + g; e < e1; e += U * G) {
      int32_t j[U];
      double v[U], w[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool ok = e + u * G < e1;
        j[u] = ok ? colind[e + u * G] : -1;
        v[u] = ok ? double(val[e + u * G]) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t jj = j[u];
        w[u] = jj < 0 ? 0.0
                      : (SCALED ? double(dinv[jj]) * double(x[jj * ld + c]) : double(x[jj * ld + c]));
      }
#pragma unroll
      for (int u = 0; u < U; ++u) acc += v[u] * w[u];
    }
  }
  for (int off = PP; off < PP * G; off <<= 1) acc += __shfl_xor(acc, off, 64);
  return acc;
}

// One smoothing step or a residual on one level (see the mode bits).
template <typename T, int PP, int NT, bool SEG>
__global__ void __launch_bounds__(NT)
k_amg_step(int k, const KrylovCtl* ctl, int n, int p, int G, const int32_t* __restrict__ rowptr,
           const int32_t* __restrict__ colind, const T* __restrict__ val,
           const T* __restrict__ dinv, const T* __restrict__ b, const T* __restrict__ x,
           T* __restrict__ d, T* __restrict__ out, double s0, double cd, double ad, int mode,
           double* __restrict__ part) {
  if (ctl && finished_by(ctl, k)) return;
  const int c = threadIdx.x % PP;
  const int g = (threadIdx.x / PP) % G;
  const bool x0 = (mode & kAmgX0) != 0;
  double rz = 0.0;
  for (RowRange<NT, PP, SEG> rr(n, G); rr.r < rr.end; rr.r += rr.step) {
    const int64_t row = rr.r;
    const int e0 = rowptr[row], e1 = rowptr[row + 1];
    double acc;
    if (x0)
      acc = s0 * row_dot_split<T, PP, true>(colind, val, b, dinv, e0, e1, p, c, c < p, g, G);
    else
      acc = row_dot_split<T, PP, false>(colind, val, x, dinv, e0, e1, p, c, c < p, g, G);
    if (c >= p || g != 0) continue;
    const int64_t i = row * p + c;
    const double bi = double(b[i]);
    const double ri = bi - acc;
    if (mode & kAmgResid) {
      out[i] = T(ri);
      continue;
    }
    const double xi = x0 ? s0 * double(dinv[row]) * bi : double(x[i]);
    double di = ad * double(dinv[row]) * ri;
    if (mode & kAmgHasD) di += cd * (x0 ? xi : double(d[i]));
    const T o = T(xi + di);
    out[i] = o;
    if (mode & kAmgWriteD) d[i] = T(di);
    rz += bi * double(o);
  }
  if constexpr (NT == kCgThreads) {
    if (mode & kAmgRz) {
      __shared__ double red[kCgThreads];
      write_col_partial<PP>(rz, red, part, 2 * PP, 0);
    }
  }
}

// bc = R r (restriction to the next level; R = P^T in CSR)
template <typename T, int PP, int NT, bool SEG>
__global__ void __launch_bounds__(NT)
k_amg_restrict(int k, const KrylovCtl* ctl, int nc, int p, int G,
               const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
               const T* __restrict__ val, const T* __restrict__ r, T* __restrict__ bc) {
  if (ctl && finished_by(ctl, k)) return;
  const int c = threadIdx.x % PP;
  const int g = (threadIdx.x / PP) % G;
  for (RowRange<NT, PP, SEG> rr(nc, G); rr.r < rr.end; rr.r += rr.step) {
    const int64_t row = rr.r;
    const double acc = row_dot_split<T, PP, false>(colind, val, r, r, rowptr[row],
                                                   rowptr[row + 1], p, c, c < p, g, G);
    if (c < p && g == 0) bc[row * p + c] = T(acc);
  }
}

// x = x_base + P xc with x_base = x, or s0 D^{-1} b (mode kAmgX0)
template <typename T, int PP, int NT, bool SEG>
__global__ void __launch_bounds__(NT)
k_amg_prolong(int k, const KrylovCtl* ctl, int n, int p, int G,
              const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
              const T* __restrict__ val, const T* __restrict__ xc,
              const T* __restrict__ dinv, const T* __restrict__ b, double s0, int mode,
              T* __restrict__ x) {
  if (ctl && finished_by(ctl, k)) return;
  const int c = threadIdx.x % PP;
  const int g = (threadIdx.x / PP) % G;
  for (RowRange<NT, PP, SEG> rr(n, G); rr.r < rr.end; rr.r += rr.step) {
    const int64_t row = rr.r;
    const double corr = row_dot_split<T, PP, false>(colind, val, xc, xc, rowptr[row],
                                                    rowptr[row + 1], p, c, c < p, g, G);
    if (c >= p || g != 0) continue;
    const int64_t i = row * p + c;
    const double base = (mode & kAmgX0) ? s0 * double(dinv[row]) * double(b[i]) : double(x[i]);
    x[i] = T(base + corr);
  }
}

// x = M b with M dense nr x ncols (row-major, FP64): the coarsest solve
// (M = the inverse of the coarsest operator, ncols = nr), or the restriction
// and coarsest solve in one (M = Inv R, b the finer level's residual).  One
// row per workgroup step; its ncols products are split over the 1024 / PP
// lane groups, four loads issued before their products, then summed per
// column with wavefront shuffles.
template <typename T, int PP>
__global__ void __launch_bounds__(1024)
k_amg_dense(int k, const KrylovCtl* ctl, int nr, int ncols, int p, const double* __restrict__ M,
            const T* __restrict__ b, T* __restrict__ x) {
  if (ctl && finished_by(ctl, k)) return;
  constexpr int NT = 1024, groups = NT / PP, U = 4;
  __shared__ double red[NT / 64 * PP + PP];
  const int c = threadIdx.x % PP;
  const int g = threadIdx.x / PP;
  for (int row = blockIdx.x; row < nr; row += gridDim.x) {
    double acc = 0.0;
    if (c < p) {
      const double* mr = M + int64_t(row) * ncols;
      int q = g;
      for (; q + (U - 1) * groups < ncols; q += U * groups) {
        double a[U], v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          a[u] = mr[q + u * groups];
          v[u] = double(b[int64_t(q + u * groups) * p + c]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc += a[u] * v[u];
      }
      for (; q < ncols; q += groups) acc += mr[q] * double(b[int64_t(q) * p + c]);
    }
    wave_col_reduce<PP, NT>(acc, red);
    if (threadIdx.x < p) x[int64_t(row) * p + threadIdx.x] = T(red[threadIdx.x]);
    __syncthreads();
  }
}

// Y = D^{-1} X (Jacobi preconditioner), one thread per element
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_scale_rows(int64_t n, int p, const T* __restrict__ dinv, const T* __restrict__ x,
             T* __restrict__ y) {
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n * p;
       i += int64_t(gridDim.x) * kThreads)
    y[i] = dinv[i / p] * x[i];
}

}  // namespace expmv
