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
#include <type_traits>

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

// A row is handled by a group of PPL * G lanes: lane (l, g) = l + PPL g takes
// the VW columns c = VW l .. VW l + VW - 1 (VW = 2 for even p: two adjacent
// columns in one 8- or 16-byte access, half the lanes and index loads of one
// column per lane; VW = 4 for p a multiple of 4 in FP32, or in FP64 from 16
// columns, and VW = 8 for FP32 from 16 columns: 16 or 32 bytes per lane, with
// 16 / VW nonzeros per sub-lane step so that the registers stay those of
// VW = 2) and the nonzeros e0 + g, e0 + g + G, ... of the row, and
// the G partial sums of a column are added with shuffles inside the group
// (G > 1 for the long rows of Galerkin operators and restrictions, whose
// serial sums would otherwise set the kernel's latency).  PPL * G <= 64, so a
// group never straddles a wavefront.
//
// Rows of a group: SEG = one contiguous XCD-aware segment per workgroup (the
// inner solver's layout), else a grid-stride loop that stays inside one XCD:
// the workgroups are handed to the 8 XCDs round-robin, so XCD b % 8 takes
// the (b % 8)-th contiguous eighth of the rows and its workgroups b / 8
// stride through it together.  A gather by a restriction or prolongation
// then reads the fine (or coarse) rows near its own from its own XCD's L2;
// striding over the whole range instead made every XCD fetch every source
// row (the 128^3 restriction read 4.5x its algorithmic bytes).  Every lane
// of a group runs the same rows, so the shuffles always see a whole group.
template <int NT, int PPL, bool SEG>
struct RowRange {
  int64_t r, end, step;
  __device__ RowRange(int64_t n, int G) {
    const int lanes = PPL * G;
    if (SEG) {
      int64_t s0, s1;
      xcd_rows(n, s0, s1);
      r = s0 + threadIdx.x / lanes;
      end = s1;
      step = NT / lanes;
    } else if (gridDim.x % 8 == 0) {
      const int64_t per = (n + 7) / 8;
      const int64_t s0 = min<int64_t>(n, int64_t(blockIdx.x % 8) * per);
      r = s0 + int64_t(blockIdx.x / 8) * (NT / lanes) + threadIdx.x / lanes;
      end = min<int64_t>(n, s0 + per);
      step = int64_t(gridDim.x / 8) * (NT / lanes);
    } else {
      r = int64_t(blockIdx.x) * (NT / lanes) + threadIdx.x / lanes;
      end = n;
      step = int64_t(gridDim.x) * (NT / lanes);
    }
  }
};

// VW consecutive entries of a row-major block (VW = 2: one 2-element access;
// the offset is even, so it is aligned)
template <int VW, typename T>
__device__ inline void load_vw(const T* __restrict__ src, double (&o)[VW]) {
  if constexpr (VW == 1) {
    o[0] = double(src[0]);
  } else if constexpr (VW >= 4) {
    T v[VW];
    ld_vw<VW>(src, v);
#pragma unroll
    for (int q = 0; q < VW; ++q) o[q] = double(v[q]);
  } else if constexpr (std::is_same<T, double>::value) {
    const double2 v = *reinterpret_cast<const double2*>(src);
    o[0] = v.x;
    o[1] = v.y;
  } else {
    const float2 v = *reinterpret_cast<const float2*>(src);
    o[0] = double(v.x);
    o[1] = double(v.y);
  }
}
template <int VW, typename T>
__device__ inline void store_vw(T* __restrict__ dst, const double (&o)[VW]) {
  if constexpr (VW == 1) {
    dst[0] = T(o[0]);
  } else if constexpr (VW >= 4) {
    T v[VW];
#pragma unroll
    for (int q = 0; q < VW; ++q) v[q] = T(o[q]);
    st_vw<VW>(dst, v);
  } else if constexpr (std::is_same<T, double>::value) {
    *reinterpret_cast<double2*>(dst) = double2{o[0], o[1]};
  } else {
    *reinterpret_cast<float2*>(dst) = float2{float(o[0]), float(o[1])};
  }
}

// acc[k] = sum over the row's nonzeros of val[e] * w_k(j) with w_k(j) =
// x[j * ld + c0 + k] (or s0 * dinv[j] * x[j * ld + c0 + k] when scaled),
// split over the G sub-lanes and summed across them; every lane of the
// group receives the row's sums.  The operator values have the vectors'
// type (an FP32 V-cycle reads FP32 values); the sums are FP64.
// UOV overrides the nonzeros per sub-lane step (0: 16 / max(VW, 2)).
template <typename T, int PPL, int VW, bool SCALED, int UOV = 0>
__device__ inline void row_dot_split(const int32_t* __restrict__ colind,
                                     const T* __restrict__ val, const T* __restrict__ x,
                                     const T* __restrict__ dinv, int e0, int e1, int ld, int c0,
                                     bool active, int g, int G, double (&acc)[VW]) {
  constexpr int U = UOV ? UOV : 16 / (VW > 2 ? VW : 2);   // nonzeros per sub-lane step, all loads issued first
#pragma unroll
  for (int k = 0; k < VW; ++k) acc[k] = 0.0;
  if (active) {
    for (int e = e0 + g; e < e1; e += U * G) {
      int32_t j[U];
      double v[U], w[U][VW];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool ok = e + u * G < e1;
        j[u] = ok ? colind[e + u * G] : -1;
        v[u] = ok ? double(val[e + u * G]) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t jj = j[u];
        if (jj < 0) {
#pragma unroll
          for (int k = 0; k < VW; ++k) w[u][k] = 0.0;
        } else {
          load_vw<VW>(x + jj * ld + c0, w[u]);
          if (SCALED) {
            const double dj = double(dinv[jj]);
#pragma unroll
            for (int k = 0; k < VW; ++k) w[u][k] *= dj;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int k = 0; k < VW; ++k) acc[k] += v[u] * w[u][k];
    }
  }
#pragma unroll
  for (int k = 0; k < VW; ++k)
    for (int off = PPL; off < PPL * G; off <<= 1) acc[k] += __shfl_xor(acc[k], off, 64);
}

// Both sums of k_amg_affine_pair in one loop, so that their loads are in flight
// together: accA over row ea0..ea1 of the operator with the scaled vector
// s_j = dinv[j] * b[j], accP over row ep0..ep1 of Pf with xc.  Same split
// over the G sub-lanes and the same order within each sum as row_dot_split.
// SA: the operator values already hold a_ij dinv[j] (no dinv gather).
template <typename T, int PPL, int VW, bool SA = false>
__device__ inline void row_dot_pair(const int32_t* __restrict__ aci, const T* __restrict__ av,
                                    const T* __restrict__ b, const T* __restrict__ dinv, int ea0,
                                    int ea1, const int32_t* __restrict__ pci,
                                    const T* __restrict__ pv, const T* __restrict__ xc, int ep0,
                                    int ep1, int ld, int c0, bool active, int g, int G,
                                    double (&accA)[VW], double (&accP)[VW]) {
  constexpr int U = 16 / (VW > 2 ? VW : 2);
#pragma unroll
  for (int k = 0; k < VW; ++k) accA[k] = accP[k] = 0.0;
  if (active) {
    for (int ea = ea0 + g, ep = ep0 + g; ea < ea1 || ep < ep1; ea += U * G, ep += U * G) {
      int32_t ja[U], jp[U];
      double va[U], vp[U], wa[U][VW], wp[U][VW];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool oa = ea + u * G < ea1, op = ep + u * G < ep1;
        ja[u] = oa ? aci[ea + u * G] : -1;
        va[u] = oa ? double(av[ea + u * G]) : 0.0;
        jp[u] = op ? pci[ep + u * G] : -1;
        vp[u] = op ? double(pv[ep + u * G]) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (ja[u] < 0) {
#pragma unroll
          for (int k = 0; k < VW; ++k) wa[u][k] = 0.0;
        } else {
          load_vw<VW>(b + int64_t(ja[u]) * ld + c0, wa[u]);
          if constexpr (!SA) {
            const double dj = double(dinv[ja[u]]);
#pragma unroll
            for (int k = 0; k < VW; ++k) wa[u][k] *= dj;
          }
        }
        if (jp[u] < 0) {
#pragma unroll
          for (int k = 0; k < VW; ++k) wp[u][k] = 0.0;
        } else {
          load_vw<VW>(xc + int64_t(jp[u]) * ld + c0, wp[u]);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int k = 0; k < VW; ++k) {
          accA[k] += va[u] * wa[u][k];
          accP[k] += vp[u] * wp[u][k];
        }
    }
  }
#pragma unroll
  for (int k = 0; k < VW; ++k)
    for (int off = PPL; off < PPL * G; off <<= 1) {
      accA[k] += __shfl_xor(accA[k], off, 64);
      accP[k] += __shfl_xor(accP[k], off, 64);
    }
}

// One smoothing step or a residual on one level (see the mode bits).
template <typename T, int PPL, int VW, int NT, bool SEG>
__global__ void __launch_bounds__(NT)
k_amg_step(int k, const KrylovCtl* ctl, int n, int p, int G, const int32_t* __restrict__ rowptr,
           const int32_t* __restrict__ colind, const T* __restrict__ val,
           const T* __restrict__ dinv, const T* __restrict__ b, const T* __restrict__ x,
           T* __restrict__ d, T* __restrict__ out, double s0, double cd, double ad, int mode,
           double* __restrict__ part) {
  if (ctl && finished_by(ctl, k)) return;
  const int c0 = VW * (threadIdx.x % PPL);
  const int g = (threadIdx.x / PPL) % G;
  const bool x0 = (mode & kAmgX0) != 0;
  double rz[VW];
#pragma unroll
  for (int q = 0; q < VW; ++q) rz[q] = 0.0;
  for (RowRange<NT, PPL, SEG> rr(n, G); rr.r < rr.end; rr.r += rr.step) {
    const int64_t row = rr.r;
    const int e0 = rowptr[row], e1 = rowptr[row + 1];
    double acc[VW];
    if (x0) {
      row_dot_split<T, PPL, VW, true>(colind, val, b, dinv, e0, e1, p, c0, c0 < p, g, G, acc);
#pragma unroll
      for (int q = 0; q < VW; ++q) acc[q] *= s0;
    } else {
      row_dot_split<T, PPL, VW, false>(colind, val, x, dinv, e0, e1, p, c0, c0 < p, g, G, acc);
    }
    if (c0 >= p || g != 0) continue;
    const int64_t i = row * p + c0;
    double bi[VW], o[VW];
    load_vw<VW>(b + i, bi);
    if (mode & kAmgResid) {
#pragma unroll
      for (int q = 0; q < VW; ++q) o[q] = bi[q] - acc[q];
      store_vw<VW>(out + i, o);
      continue;
    }
    const double dr = double(dinv[row]);
    double xi[VW], di[VW], dold[VW];
    if (x0) {
#pragma unroll
      for (int q = 0; q < VW; ++q) xi[q] = s0 * dr * bi[q];
    } else {
      load_vw<VW>(x + i, xi);
    }
    const bool hasd = (mode & kAmgHasD) != 0;
    if (hasd && !x0) load_vw<VW>(d + i, dold);
#pragma unroll
    for (int q = 0; q < VW; ++q) {
      di[q] = ad * dr * (bi[q] - acc[q]);
      if (hasd) di[q] += cd * (x0 ? xi[q] : dold[q]);
      o[q] = double(T(xi[q] + di[q]));   // the value stored (and summed) in type T
    }
    store_vw<VW>(out + i, o);
    if (mode & kAmgWriteD) store_vw<VW>(d + i, di);
#pragma unroll
    for (int q = 0; q < VW; ++q) rz[q] += bi[q] * o[q];
  }
  if constexpr (NT == kCgThreads) {
    if (mode & kAmgRz) {
      __shared__ double red[kCgThreads];
      // column c0 + q of this lane into part[wg][0][c0 + q] (layout of PP = PPL VW)
#pragma unroll
      for (int q = 0; q < VW; ++q) {
        wave_col_reduce<PPL, kCgThreads>(rz[q], red);
        if (threadIdx.x < PPL)
          part[size_t(blockIdx.x) * (2 * PPL * VW) + VW * threadIdx.x + q] = red[threadIdx.x];
        __syncthreads();
      }
    }
  }
}

// bc = R r (restriction to the next level; R = P^T in CSR)
template <typename T, int PPL, int VW, int NT, bool SEG>
__global__ void __launch_bounds__(NT)
k_amg_restrict(int k, const KrylovCtl* ctl, int nc, int p, int G,
               const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
               const T* __restrict__ val, const T* __restrict__ r, T* __restrict__ bc) {
  if (ctl && finished_by(ctl, k)) return;
  const int c0 = VW * (threadIdx.x % PPL);
  const int g = (threadIdx.x / PPL) % G;
  for (RowRange<NT, PPL, SEG> rr(nc, G); rr.r < rr.end; rr.r += rr.step) {
    const int64_t row = rr.r;
    double acc[VW];
    // five nonzeros per sub-lane step at four columns per lane: a 72-entry
    // row of the finest fused restriction in one step of a wave's 16
    // sub-lanes (the same order per sub-lane as four per step): 0.270 ->
    // 0.264 ms on the 128^3 workload
    row_dot_split<T, PPL, VW, false, (VW == 4 ? 5 : 0)>(colind, val, r, r, rowptr[row],
                                                         rowptr[row + 1], p, c0, c0 < p, g, G,
                                                         acc);
    if (c0 < p && g == 0) store_vw<VW>(bc + row * p + c0, acc);
  }
}

// x = x_base + P xc with x_base = x, or s0 D^{-1} b (mode kAmgX0)
template <typename T, int PPL, int VW, int NT, bool SEG>
__global__ void __launch_bounds__(NT)
k_amg_prolong(int k, const KrylovCtl* ctl, int n, int p, int G,
              const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
              const T* __restrict__ val, const T* __restrict__ xc,
              const T* __restrict__ dinv, const T* __restrict__ b, double s0, int mode,
              T* __restrict__ x) {
  if (ctl && finished_by(ctl, k)) return;
  const int c0 = VW * (threadIdx.x % PPL);
  const int g = (threadIdx.x / PPL) % G;
  for (RowRange<NT, PPL, SEG> rr(n, G); rr.r < rr.end; rr.r += rr.step) {
    const int64_t row = rr.r;
    double corr[VW];
    row_dot_split<T, PPL, VW, false>(colind, val, xc, xc, rowptr[row], rowptr[row + 1], p, c0,
                                     c0 < p, g, G, corr);
    if (c0 >= p || g != 0) continue;
    const int64_t i = row * p + c0;
    double base[VW];
    if (mode & kAmgX0) {
      load_vw<VW>(b + i, base);
      const double sd = s0 * double(dinv[row]);
#pragma unroll
      for (int q = 0; q < VW; ++q) base[q] *= sd;
    } else {
      load_vw<VW>(x + i, base);
    }
#pragma unroll
    for (int q = 0; q < VW; ++q) base[q] += corr[q];
    store_vw<VW>(x + i, base);
  }
}

// x = D^{-1} (alpha b - beta A D^{-1} b) + P' xc in one pass (G sub-lanes
// per row serve both sums):
//  * a level below the finest smoothed by one step from x0 = s0 D^{-1} b,
//    prolongation and post-smoothing step together:
//      x1 = x0 + P xc,  out = x1 + s0 D^{-1} (b - A x1)
//         = D^{-1} (2 s0 b - s0^2 A D^{-1} b) + Pf xc,  Pf = (I - s0 D^{-1} A) P
//  * the finest level at degree 2, whose pre-smoothed iterate
//      x1 = (1 + c1) x0 + a1 D^{-1} (b - A x0) = D^{-1} ((s0 + c1 s0 + a1) b - a1 s0 A D^{-1} b)
//    is not stored: the prolongation x1 + P xc recomputes it.
// Quad broadcast: the value of lane I of each group of four consecutive
// lanes to all four (DPP quad_perm [I, I, I, I]).  Every lane of the quad
// must be active.
template <int I>
__device__ __forceinline__ int quad_bcast(int v) {
  return __builtin_amdgcn_update_dpp(0, v, I * 0x55, 0xf, 0xf, false);
}
template <int I>
__device__ __forceinline__ double quad_bcast(double v) {
  const int lo = quad_bcast<I>(__double2loint(v));
  const int hi = quad_bcast<I>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

// row_dot_pair for four lanes per row (one quad) and av = A D^{-1}: each
// lane of the quad loads one of four consecutive nonzeros of a row and the
// quad exchanges them by broadcasts, so one index load serves four
// nonzeros.  Sub-lane g owns the groups starting at e0 + 4 (g + G u).  A
// column outside [0, nb) of A or [0, nx) of Pf is skipped.
template <typename T, int VW>
__device__ inline void row_dot_pair_q(const int32_t* __restrict__ aci, const T* __restrict__ av,
                                      const T* __restrict__ b, int nb, int ea0, int ea1,
                                      const int32_t* __restrict__ pci, const T* __restrict__ pv,
                                      const T* __restrict__ xc, int nx, int ep0, int ep1, int ld,
                                      int c0, bool active, int g, int G, double (&accA)[VW],
                                      double (&accP)[VW]) {
  const int q = threadIdx.x & 3;
#pragma unroll
  for (int k = 0; k < VW; ++k) accA[k] = accP[k] = 0.0;
  for (int ea = ea0 + 4 * g, ep = ep0 + 4 * g; ea < ea1 || ep < ep1; ea += 4 * G, ep += 4 * G) {
    const bool oa = ea + q < ea1, op = ep + q < ep1;
    const int mja = oa ? aci[ea + q] : -1;
    const double mva = oa ? double(av[ea + q]) : 0.0;
    const int mjp = op ? pci[ep + q] : -1;
    const double mvp = op ? double(pv[ep + q]) : 0.0;
    int ja[4], jp[4];
    double va[4], vp[4];
    ja[0] = quad_bcast<0>(mja); ja[1] = quad_bcast<1>(mja);
    ja[2] = quad_bcast<2>(mja); ja[3] = quad_bcast<3>(mja);
    va[0] = quad_bcast<0>(mva); va[1] = quad_bcast<1>(mva);
    va[2] = quad_bcast<2>(mva); va[3] = quad_bcast<3>(mva);
    jp[0] = quad_bcast<0>(mjp); jp[1] = quad_bcast<1>(mjp);
    jp[2] = quad_bcast<2>(mjp); jp[3] = quad_bcast<3>(mjp);
    vp[0] = quad_bcast<0>(mvp); vp[1] = quad_bcast<1>(mvp);
    vp[2] = quad_bcast<2>(mvp); vp[3] = quad_bcast<3>(mvp);
    double wa[4][VW], wp[4][VW];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (active && ja[u] >= 0 && ja[u] < nb) {
        load_vw<VW>(b + int64_t(ja[u]) * ld + c0, wa[u]);
      } else {
#pragma unroll
        for (int k = 0; k < VW; ++k) wa[u][k] = 0.0;
      }
      if (active && jp[u] >= 0 && jp[u] < nx) {
        load_vw<VW>(xc + int64_t(jp[u]) * ld + c0, wp[u]);
      } else {
#pragma unroll
        for (int k = 0; k < VW; ++k) wp[u][k] = 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int k = 0; k < VW; ++k) {
        accA[k] += va[u] * wa[u][k];
        accP[k] += vp[u] * wp[u][k];
      }
  }
#pragma unroll
  for (int k = 0; k < VW; ++k)
    for (int off = 4; off < 4 * G; off <<= 1) {
      accA[k] += __shfl_xor(accA[k], off, 64);
      accP[k] += __shfl_xor(accP[k], off, 64);
    }
}

// The prolongation-plus-smoothing pass of one row range.  SA: av holds the
// values of A D^{-1} (a_ij dinv[j]); dinv still scales the row's own term.
template <typename T, int PPL, int VW, int NT, bool SEG, bool SA>
__device__ __forceinline__ void affine_pair_rows(int k, const KrylovCtl* ctl, int n, int p, int G,
                                                 const int32_t* __restrict__ arp,
                                                 const int32_t* __restrict__ aci,
                                                 const T* __restrict__ av,
                                                 const T* __restrict__ dinv,
                                                 const T* __restrict__ b,
                                                 const int32_t* __restrict__ prp,
                                                 const int32_t* __restrict__ pci,
                                                 const T* __restrict__ pv,
                                                 const T* __restrict__ xc, double alpha,
                                                 double beta, T* __restrict__ out) {
  if (ctl && finished_by(ctl, k)) return;
  const int c0 = VW * (threadIdx.x % PPL);
  const int g = (threadIdx.x / PPL) % G;
  for (RowRange<NT, PPL, SEG> rr(n, G); rr.r < rr.end; rr.r += rr.step) {
    const int64_t row = rr.r;
    double ab[VW], corr[VW];
    row_dot_pair<T, PPL, VW, SA>(aci, av, b, dinv, arp[row], arp[row + 1], pci, pv, xc,
                                 prp[row], prp[row + 1], p, c0, c0 < p, g, G, ab, corr);
    if (c0 >= p || g != 0) continue;
    const int64_t i = row * p + c0;
    double bi[VW], o[VW];
    load_vw<VW>(b + i, bi);
    const double dr = double(dinv[row]);
#pragma unroll
    for (int q = 0; q < VW; ++q) o[q] = dr * (alpha * bi[q] - beta * ab[q]) + corr[q];
    store_vw<VW>(out + i, o);
  }
}

template <typename T, int PPL, int VW, int NT, bool SEG>
__global__ void __launch_bounds__(NT)
k_amg_affine_pair(int k, const KrylovCtl* ctl, int n, int p, int G,
                  const int32_t* __restrict__ arp, const int32_t* __restrict__ aci,
                  const T* __restrict__ av, const T* __restrict__ dinv, const T* __restrict__ b,
                  const int32_t* __restrict__ prp, const int32_t* __restrict__ pci,
                  const T* __restrict__ pv, const T* __restrict__ xc, double alpha, double beta,
                  T* __restrict__ out) {
  affine_pair_rows<T, PPL, VW, NT, SEG, false>(k, ctl, n, p, G, arp, aci, av, dinv, b, prp, pci,
                                               pv, xc, alpha, beta, out);
}

// The same pass with av = A D^{-1}: one gather per nonzero of A instead of
// two; held to 128 VGPRs (4 waves per SIMD, as the kernel above runs at four
// columns per lane)
template <typename T, int PPL, int VW, int NT, bool SEG>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4)))
k_amg_affine_pair_ad(int k, const KrylovCtl* ctl, int n, int p, int G,
                     const int32_t* __restrict__ arp, const int32_t* __restrict__ aci,
                     const T* __restrict__ adv, const T* __restrict__ dinv,
                     const T* __restrict__ b, const int32_t* __restrict__ prp,
                     const int32_t* __restrict__ pci, const T* __restrict__ pv,
                     const T* __restrict__ xc, double alpha, double beta, T* __restrict__ out) {
  affine_pair_rows<T, PPL, VW, NT, SEG, true>(k, ctl, n, p, G, arp, aci, adv, dinv, b, prp, pci,
                                              pv, xc, alpha, beta, out);
}

// k_amg_affine_pair_ad with four lanes per row sharing their index loads
// (row_dot_pair_q); nx = rows of xc
template <typename T, int VW, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4)))
k_amg_affine_pair_q(int k, const KrylovCtl* ctl, int n, int p, int G,
                    const int32_t* __restrict__ arp, const int32_t* __restrict__ aci,
                    const T* __restrict__ adv, const T* __restrict__ dinv,
                    const T* __restrict__ b, const int32_t* __restrict__ prp,
                    const int32_t* __restrict__ pci, const T* __restrict__ pv,
                    const T* __restrict__ xc, int nx, double alpha, double beta,
                    T* __restrict__ out) {
  if (ctl && finished_by(ctl, k)) return;
  const int c0 = VW * (threadIdx.x % 4);
  const int g = (threadIdx.x / 4) % G;
  for (RowRange<NT, 4, false> rr(n, G); rr.r < rr.end; rr.r += rr.step) {
    const int64_t row = rr.r;
    double ab[VW], corr[VW];
    row_dot_pair_q<T, VW>(aci, adv, b, n, arp[row], arp[row + 1], pci, pv, xc, nx, prp[row],
                          prp[row + 1], p, c0, c0 < p, g, G, ab, corr);
    if (c0 >= p || g != 0) continue;
    const int64_t i = row * p + c0;
    double bi[VW], o[VW];
    load_vw<VW>(b + i, bi);
    const double dr = double(dinv[row]);
#pragma unroll
    for (int q = 0; q < VW; ++q) o[q] = dr * (alpha * bi[q] - beta * ab[q]) + corr[q];
    store_vw<VW>(out + i, o);
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
