// Device kernels of the expmv library (gfx950 / CDNA4).
//
// Blocks are n x p row-major (ld = p).  Streaming kernels use 256-thread
// workgroups and a grid-stride loop over rows; a group of PP lanes (PP = p
// rounded up to a power of two, PP | 64) owns one row, so every row's p
// values are one contiguous, coalesced segment.  The inner-solver kernels
// (1024-thread workgroups) give each lane VW = 2 adjacent columns when p is
// even, so PPL = PP / 2 lanes own a row and loads are 16 bytes wide; for odd
// p, VW = 1 and PPL = PP.  Reductions are
// deterministic: per-workgroup partial sums in a fixed tree order, then a
// fixed-order sum over workgroups (no floating-point atomics).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <type_traits>

namespace expmv {

constexpr int kThreads = 256;
constexpr int kCgThreads = 1024;   // workgroup size of the inner-solver kernels
constexpr int kNShift = 7;   // conjugate-pair poles of the degree-14 CF form
constexpr int kMaxP = 32;    // widest supported block

struct KrylovScalars {
  double rho;         // CG: (r, D^{-1} r)            BiCGStab: (r0~, r)
  double alpha;       // step of the current iteration
  double alpha_prev;  // step still owed to x (CG)
  double beta;
  double omega;       // BiCGStab
  double rnorm2;      // ||r||^2
  double bnorm2;      // ||b||^2
  double tmp;         // BiCGStab (r0~, v)
  int active;         // 1 until the column meets its tolerance or the cap
  int iters;          // iterations taken while active
  int hit_cap;        // stopped by the iteration cap
  int pad;
};

struct KrylovCtl {
  unsigned int counter;  // unused
  int done;              // -1 while running; else the iteration whose first kernel
                         // found every column inactive
  int iters_max;
  int hit_cap;
};

// A kernel of iteration k returns at once if the solve finished at an
// earlier iteration (first kernel of an iteration: strictly earlier; the
// later kernels: at this iteration or earlier).  `done` is one 32-bit word
// written once per solve, so every workgroup sees either -1 or its final
// value.
__device__ inline bool finished_before(const KrylovCtl* ctl, int k) {
  const int d = ctl->done;
  return d >= 0 && d < k;
}
__device__ inline bool finished_by(const KrylovCtl* ctl, int k) {
  const int d = ctl->done;
  return d >= 0 && d <= k;
}

// ---------------------------------------------------------------------------
// block reduction helpers

// Sum v over the lanes of a workgroup that share (tid % PP); result for
// column c ends in red[c].  red has kThreads doubles.
template <int PP, int NT = kThreads>
__device__ inline void block_col_reduce(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
#pragma unroll
  for (int s = NT / 2; s >= PP; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
}

// Column sums over a workgroup of NT threads (column = tid % PP) using
// wavefront shuffles and one LDS exchange; the result for column c is left
// in red[c] (red holds at least NT / 64 * PP doubles).  Fixed order.
template <int PP, int NT>
__device__ inline void wave_col_reduce(double v, double* red) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int off = 32; off >= PP; off >>= 1) v += __shfl_xor(v, off, 64);
  const int wave = tid / 64, lane = tid % 64;
  if (lane < PP) red[wave * PP + lane] = v;
  __syncthreads();
  if (tid < PP) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += red[w * PP + tid];
    red[NT / 64 * PP + tid] = s;
  }
  __syncthreads();
  if (tid < PP) red[tid] = red[NT / 64 * PP + tid];
  __syncthreads();
}

// Rows of workgroup blockIdx.x: one contiguous segment per workgroup, with
// the segments of the workgroups that run on one XCD adjacent.  Workgroups
// are handed to the 8 XCDs round-robin, so logical segment
// (b % 8) * (G / 8) + b / 8 puts each XCD on one contiguous eighth of the
// rows and keeps stencil neighbours in that XCD's L2.
__device__ inline void xcd_rows(int64_t n, int64_t& r0, int64_t& r1) {
  const int G = gridDim.x, b = blockIdx.x;
  const int L = (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
  const int64_t per = (n + G - 1) / G;
  r0 = min<int64_t>(n, int64_t(L) * per);
  r1 = min<int64_t>(n, r0 + per);
}

// acc (+)= sum_e val[e] * x[colind[e] * ld + c] over one CSR row, in order,
// eight nonzeros per step with every load of a step issued before the first
// product (predicated, no serial tail): a stencil row costs one round trip
// for its indices and one for its gathers.
// The operator's values are FP64 for every working type T: in the mixed
// form the FP32 inner solver thus works with the exact operator (rounding
// its entries to FP32 would move the eigenvalues of a non-normal operator
// by the eigenvector condition number times 6e-8).
template <typename T>
__device__ inline T csr_row_dot(const int32_t* __restrict__ colind, const double* __restrict__ val,
                                const T* __restrict__ x, int e0, int e1, int ld, int c) {
  constexpr int U = 8;
  double acc = 0.0;
  for (int e = e0; e < e1; e += U) {
    int32_t j[U];
    double v[U], w[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool ok = e + u < e1;
      j[u] = ok ? colind[e + u] : -1;
      v[u] = ok ? val[e + u] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) w[u] = j[u] >= 0 ? double(x[int64_t(j[u]) * ld + c]) : 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) acc += v[u] * w[u];
  }
  return T(acc);
}

// ---------------------------------------------------------------------------
// CSR SpMM  y = K x  (n x p blocks, PP lanes per row)

template <typename T, int PP>
__global__ void __launch_bounds__(kThreads)
k_spmm(int n, int p, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
       const double* __restrict__ val, const T* __restrict__ x, T* __restrict__ y) {
  const int c = threadIdx.x % PP;
  const int64_t rows_per_grid = int64_t(gridDim.x) * (kThreads / PP);
  for (int64_t row = int64_t(blockIdx.x) * (kThreads / PP) + threadIdx.x / PP; row < n;
       row += rows_per_grid) {
    if (c < p) {
      y[row * p + c] = csr_row_dot(colind, val, x, rowptr[row], rowptr[row + 1], p, c);
    }
  }
}

// ---------------------------------------------------------------------------
// Batched Jacobi-preconditioned CG on K x = b (K SPD), column-wise, the p
// columns in lock step, b = sign * src.  No kernel synchronises its own
// workgroups: every workgroup of a kernel sums the previous kernel's
// per-workgroup partials itself, in one fixed order, so all of them obtain
// bitwise the same scalars (visibility across kernels is the stream's).
// Workgroup 0 records the scalars later kernels need in a two-slot table
// indexed by the iteration's parity.
//
// Iteration k (z = D^{-1} r, or z = the AMG V-cycle applied to r, computed
// between B_{k-1} and C_k together with the (r, z) partials), three
// streaming kernels:
//   C_k: rho_k = (r_k, z_k), |r_k|^2 from B_{k-1}'s partials (init's for k=0);
//        beta = rho_k / rho_{k-1}; convergence test;
//        x += alpha_{k-1} p_{k-1};  p_k = z_k + beta p_{k-1}.
//   A_k: q = K p_k (the CSR SpMM), partial sigma_k = (p_k, q).
//   B_k: alpha_k = rho_k / sigma_k; r_{k+1} = r_k - alpha_k q;
//        partials (r_{k+1}, z_{k+1}) and |r_{k+1}|^2.
// A column whose |r_k| <= tol |b| (or that reached maxit) stops: its last
// step alpha_{k-1} p_{k-1} is added by C_k and every later step is zero.
// When no column is active C_k sets ctl->done; later kernels return at once.

struct CgSlot {
  double rho[kMaxP];
  double alpha[kMaxP];
  int active[kMaxP];
  int iters[kMaxP];
};

struct CgState {
  CgSlot slot[2];
  double bnorm2[kMaxP];
};

// Sum NV x PP per-workgroup partials (layout [wg][v][c]) in a fixed order;
// every thread of the workgroup ends with out[v * PP + c] in LDS.
template <int PP, int NV>
__device__ inline void reduce_parts(const double* __restrict__ part, int nwg, double* red,
                                    double* out) {
  constexpr int slots = PP * NV;
  constexpr int lanes = (kCgThreads / slots) > 64 ? 64 : kCgThreads / slots;
  const int tid = threadIdx.x;
  const int sidx = tid / lanes, l = tid % lanes;
  double v = 0.0;
  if (sidx < slots) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int w = l;
    for (; w + 3 * lanes < nwg; w += 4 * lanes) {
      a0 += part[size_t(w) * slots + sidx];
      a1 += part[size_t(w + lanes) * slots + sidx];
      a2 += part[size_t(w + 2 * lanes) * slots + sidx];
      a3 += part[size_t(w + 3 * lanes) * slots + sidx];
    }
    for (; w < nwg; w += lanes) a0 += part[size_t(w) * slots + sidx];
    v = (a0 + a1) + (a2 + a3);
  }
  // the `lanes` threads of one slot are consecutive and aligned inside one
  // wavefront: reduce them with shuffles
#pragma unroll
  for (int st = lanes / 2; st >= 1; st >>= 1) v += __shfl_xor(v, st, 64);
  if (l == 0 && sidx < slots) out[sidx] = v;
  __syncthreads();
  (void)red;
}

// per-workgroup column sums of v (PP columns) -> part[wg * stride + off + c]
template <int PP>
__device__ inline void write_col_partial(double v, double* red, double* part, int stride, int off) {
  wave_col_reduce<PP, kCgThreads>(v, red);
  if (threadIdx.x < PP) part[size_t(blockIdx.x) * stride + off + threadIdx.x] = red[threadIdx.x];
  __syncthreads();
}

// The same layout when each lane holds VW adjacent columns: lane l's value q
// is column VW l + q of the PPL VW columns.
template <int PPL, int VW>
__device__ inline void write_col_partial_vw(const double (&v)[VW], double* red, double* part,
                                            int stride, int off) {
#pragma unroll
  for (int q = 0; q < VW; ++q) {
    wave_col_reduce<PPL, kCgThreads>(v[q], red);
    if (threadIdx.x < PPL)
      part[size_t(blockIdx.x) * stride + off + VW * threadIdx.x + q] = red[threadIdx.x];
    __syncthreads();
  }
}

// VW adjacent entries of a row-major block in the block's own type: VW = 2
// (the offset is even, so it is aligned: one access) or VW = 4 (the offset
// and the row length are multiples of 4: one 16-byte FP32 access, or two
// 16-byte FP64 ones)
template <int VW, typename T>
__device__ inline void ld_vw(const T* __restrict__ src, T (&o)[VW]) {
  static_assert(VW == 1 || VW == 2 || VW == 4 || (VW == 8 && sizeof(T) == 4), "lane width");
  if constexpr (VW == 1) {
    o[0] = src[0];
  } else if constexpr (VW == 8) {
    const float4 v0 = *reinterpret_cast<const float4*>(src);
    const float4 v1 = *reinterpret_cast<const float4*>(src + 4);
    o[0] = v0.x;
    o[1] = v0.y;
    o[2] = v0.z;
    o[3] = v0.w;
    o[4] = v1.x;
    o[5] = v1.y;
    o[6] = v1.z;
    o[7] = v1.w;
  } else if constexpr (VW == 4 && sizeof(T) == 8) {
    const double2 v0 = *reinterpret_cast<const double2*>(src);
    const double2 v1 = *reinterpret_cast<const double2*>(src + 2);
    o[0] = v0.x;
    o[1] = v0.y;
    o[2] = v1.x;
    o[3] = v1.y;
  } else if constexpr (VW == 4) {
    const float4 v = *reinterpret_cast<const float4*>(src);
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
  } else if constexpr (std::is_same<T, double>::value) {
    const double2 v = *reinterpret_cast<const double2*>(src);
    o[0] = v.x;
    o[1] = v.y;
  } else {
    const float2 v = *reinterpret_cast<const float2*>(src);
    o[0] = v.x;
    o[1] = v.y;
  }
}
template <int VW, typename T>
__device__ inline void st_vw(T* __restrict__ dst, const T (&o)[VW]) {
  static_assert(VW == 1 || VW == 2 || VW == 4 || (VW == 8 && sizeof(T) == 4), "lane width");
  if constexpr (VW == 1) {
    dst[0] = o[0];
  } else if constexpr (VW == 8) {
    *reinterpret_cast<float4*>(dst) = float4{o[0], o[1], o[2], o[3]};
    *reinterpret_cast<float4*>(dst + 4) = float4{o[4], o[5], o[6], o[7]};
  } else if constexpr (VW == 4 && sizeof(T) == 8) {
    *reinterpret_cast<double2*>(dst) = double2{o[0], o[1]};
    *reinterpret_cast<double2*>(dst + 2) = double2{o[2], o[3]};
  } else if constexpr (VW == 4) {
    *reinterpret_cast<float4*>(dst) = float4{o[0], o[1], o[2], o[3]};
  } else if constexpr (std::is_same<T, double>::value) {
    *reinterpret_cast<double2*>(dst) = double2{o[0], o[1]};
  } else {
    *reinterpret_cast<float2*>(dst) = float2{o[0], o[1]};
  }
}

// csr_row_dot for the VW columns c0 .. c0 + VW - 1 (sums in FP64)
template <int VW, typename T>
__device__ inline void csr_row_dot_vw(const int32_t* __restrict__ colind,
                                      const double* __restrict__ val, const T* __restrict__ x,
                                      int e0, int e1, int ld, int c0, double (&acc)[VW]) {
  constexpr int U = 16 / (VW > 2 ? VW : 2);   // VW = 4, 8: same registers as VW = 2
#pragma unroll
  for (int q = 0; q < VW; ++q) acc[q] = 0.0;
  for (int e = e0; e < e1; e += U) {
    int32_t j[U];
    double v[U];
    T w[U][VW];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool ok = e + u < e1;
      j[u] = ok ? colind[e + u] : -1;
      v[u] = ok ? val[e + u] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (j[u] >= 0) {
        ld_vw<VW>(x + int64_t(j[u]) * ld + c0, w[u]);
      } else {
#pragma unroll
        for (int q = 0; q < VW; ++q) w[u][q] = T(0);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int q = 0; q < VW; ++q) acc[q] += v[u] * double(w[u][q]);
  }
}

// Entries a0 .. a0 + U - 1 of a CSR row ending at a1 (j = -1, v = 0 past it).
template <int U>
__device__ inline void csr_entries(const int32_t* __restrict__ colind,
                                   const double* __restrict__ val, int a0, int a1,
                                   int32_t (&j)[U], double (&v)[U]) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const bool ok = a0 + u < a1;
    j[u] = ok ? colind[a0 + u] : -1;
    v[u] = ok ? val[a0 + u] : 0.0;
  }
}

// For the rows row, row + st, ... < end of a CSR operator K:
//   acc = K[row, :] y[:, c0 .. c0 + VW),  y = x (dinv NULL) or D^{-1} x,
// then body(row, acc).  The loop is software-pipelined so that one row costs
// one memory round trip instead of three: while the gathers of a row are in
// flight, the first U entries of the next row and the extents of the row
// after it are already being loaded.  Entries past the first U of a row
// (rows longer than U) follow without prefetch.  The sum runs over the row's
// entries in order, as csr_row_dot_vw does; inactive lanes (masked columns)
// issue no gathers and get zero sums.
template <int U, int VW, typename T, typename Body>
__device__ inline void csr_rows_pipelined(const int32_t* __restrict__ rowptr,
                                          const int32_t* __restrict__ colind,
                                          const double* __restrict__ val, const T* __restrict__ x,
                                          const T* __restrict__ dinv, int ld, int c0, bool active,
                                          int64_t row, int64_t st, int64_t end, Body&& body) {
  int e0 = 0, e1 = 0, ne0 = 0, ne1 = 0;
  if (row < end) {
    e0 = rowptr[row];
    e1 = rowptr[row + 1];
  }
  if (row + st < end) {
    ne0 = rowptr[row + st];
    ne1 = rowptr[row + st + 1];
  }
  int32_t j[U];
  double v[U];
  csr_entries<U>(colind, val, e0, e1, j, v);
  for (; row < end; row += st) {
    T w[U][VW];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (active && j[u] >= 0) {
        ld_vw<VW>(x + int64_t(j[u]) * ld + c0, w[u]);
        if (dinv) {
          const T dj = dinv[j[u]];
#pragma unroll
          for (int q = 0; q < VW; ++q) w[u][q] = dj * w[u][q];
        }
      } else {
#pragma unroll
        for (int q = 0; q < VW; ++q) w[u][q] = T(0);
      }
    }
    int32_t nj[U];
    double nv[U];
    csr_entries<U>(colind, val, ne0, ne1, nj, nv);
    int n2e0 = 0, n2e1 = 0;
    if (row + 2 * st < end) {
      n2e0 = rowptr[row + 2 * st];
      n2e1 = rowptr[row + 2 * st + 1];
    }
    double acc[VW];
#pragma unroll
    for (int q = 0; q < VW; ++q) acc[q] = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int q = 0; q < VW; ++q) acc[q] += v[u] * double(w[u][q]);
    for (int e = e0 + U; e < e1; e += U) {
      int32_t tj[U];
      double tv[U];
      csr_entries<U>(colind, val, e, e1, tj, tv);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (active && tj[u] >= 0) {
          ld_vw<VW>(x + int64_t(tj[u]) * ld + c0, w[u]);
          if (dinv) {
            const T dj = dinv[tj[u]];
#pragma unroll
            for (int q = 0; q < VW; ++q) w[u][q] = dj * w[u][q];
          }
        } else {
#pragma unroll
          for (int q = 0; q < VW; ++q) w[u][q] = T(0);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int q = 0; q < VW; ++q) acc[q] += tv[u] * double(w[u][q]);
    }
    body(row, acc);
    e0 = ne0;
    e1 = ne1;
    ne0 = n2e0;
    ne1 = n2e1;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      j[u] = nj[u];
      v[u] = nv[u];
    }
  }
}

// Entries per pipelined row step of the inner solver's SpMM: 8 (a 7-point
// stencil row in one step) for up to 16 bytes of columns per lane; wider
// lanes take 4, as 8 would spill past the 128 VGPRs a wave of a 1024-thread
// workgroup may hold.
template <typename T, int VW>
constexpr int spmm_unroll() {
  return (VW * sizeof(T) <= 16) ? 8 : 4;
}

// The CG kernels take VW adjacent columns per lane (VW = 2 for even p) and
// PPL = PP / VW lanes per row; per-column scalars and partials keep the layout
// of PP columns.
template <typename T, typename TS, int PPL, int VW>
__global__ void __launch_bounds__(kCgThreads)
k_cg_init(int n, int p, double sign, const TS* __restrict__ src, const T* __restrict__ dinv,
          T* __restrict__ x, T* __restrict__ r, T* __restrict__ pold,
          KrylovCtl* ctl, double* __restrict__ part_rr, float* __restrict__ r32) {
  constexpr int PP = PPL * VW;
  __shared__ double red[kCgThreads];
  const int c0 = VW * (threadIdx.x % PPL);
  double rz[VW], bb[VW];
#pragma unroll
  for (int q = 0; q < VW; ++q) rz[q] = bb[q] = 0.0;
  int64_t seg0, seg1;
  xcd_rows(n, seg0, seg1);
  for (int64_t row = seg0 + threadIdx.x / PPL; row < seg1; row += kCgThreads / PPL) {
    if (c0 < p) {
      const int64_t i = row * p + c0;
      TS sv[VW];
      ld_vw<VW>(src + i, sv);
      T b[VW], zero[VW];
      float b32[VW];
      const double dr = double(dinv[row]);
#pragma unroll
      for (int q = 0; q < VW; ++q) {
        b[q] = T(sign * double(sv[q]));
        zero[q] = T(0);
        b32[q] = float(b[q]);
        const double bd = double(b[q]);
        rz[q] += bd * dr * bd;
        bb[q] += bd * bd;
      }
      st_vw<VW>(r + i, b);
      if (r32) st_vw<VW>(r32 + i, b32);   // input of an FP32 preconditioner
      st_vw<VW>(x + i, zero);
      st_vw<VW>(pold + i, zero);
    }
  }
  write_col_partial_vw<PPL, VW>(rz, red, part_rr, 2 * PP, 0);
  write_col_partial_vw<PPL, VW>(bb, red, part_rr, 2 * PP, PP);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->done = -1;
    ctl->iters_max = 0;
    ctl->hit_cap = 0;
    ctl->counter = 0u;
  }
}

// z: the preconditioned residual (TZ = float for an FP32 V-cycle), or NULL
// for Jacobi (D^{-1} r formed here)
template <typename T, typename TZ, int PPL, int VW>
__global__ void __launch_bounds__(kCgThreads)
k_cg_c(int k, int n, int p, const T* __restrict__ dinv, const T* __restrict__ r,
       const TZ* __restrict__ z, const T* __restrict__ pold, T* __restrict__ pnew,
       T* __restrict__ x, CgState* st, KrylovCtl* ctl, const double* __restrict__ part_rr,
       double tol2, int maxit) {
  constexpr int PP = PPL * VW;
  if (finished_before(ctl, k)) return;
  __shared__ double red[kCgThreads];
  __shared__ double tot[2 * PP];
  __shared__ double s_beta[PP], s_aprev[PP];
  __shared__ int s_any;
  // the operands of this thread's first row are loaded before the scalar
  // reduction, so their latency overlaps it (they are final at kernel start)
  const int c0 = VW * (threadIdx.x % PPL);
  int64_t seg0, seg1;
  xcd_rows(n, seg0, seg1);
  const int64_t row0 = seg0 + threadIdx.x / PPL;
  const bool pre = row0 < seg1 && c0 < p;
  T po0[VW], xv0[VW], zr0[VW];
  if (pre) {
    const int64_t i = row0 * p + c0;
    ld_vw<VW>(pold + i, po0);
    ld_vw<VW>(x + i, xv0);
    if (z) {
      TZ zz[VW];
      ld_vw<VW>(z + i, zz);
#pragma unroll
      for (int q = 0; q < VW; ++q) zr0[q] = T(zz[q]);
    } else {
      ld_vw<VW>(r + i, zr0);
    }
  }
  reduce_parts<PP, 2>(part_rr, gridDim.x, red, tot);   // tot[c] = rho_k, tot[PP + c] = |r_k|^2
  if (threadIdx.x < 64) {
    // one lane per column (PP <= 64), the control word from the wavefront's
    // reductions: the scalar loads of all columns are in flight together
    const int cc = threadIdx.x;
    const CgSlot& prev = st->slot[(k + 1) & 1];
    double beta = 0.0, aprev = 0.0;
    int act = 0, it = 0, hit = 0;
    if (cc < p) {
      const double rho = tot[cc], rn = tot[PP + cc];
      double bn;
      int act_prev;
      if (k == 0) {
        bn = rn;
        act_prev = bn > 0.0;
      } else {
        bn = st->bnorm2[cc];
        act_prev = prev.active[cc];
        it = prev.iters[cc];
        aprev = prev.alpha[cc];
        beta = (act_prev && prev.rho[cc] != 0.0) ? rho / prev.rho[cc] : 0.0;
      }
      act = act_prev && !(rn <= tol2 * bn);
      if (act && it >= maxit) {
        act = 0;
        hit = 1;
      }
      if (!act) beta = 0.0;
      if (blockIdx.x == 0) {
        CgSlot& cur = st->slot[k & 1];
        cur.rho[cc] = rho;
        cur.active[cc] = act;
        cur.iters[cc] = it + act;
        if (k == 0) st->bnorm2[cc] = bn;
      }
    }
    if (cc < PP) {
      s_beta[cc] = beta;
      s_aprev[cc] = aprev;
    }
    int any = act, itmax = it;
    for (int off = 32; off >= 1; off >>= 1) {
      any |= __shfl_xor(any, off, 64);
      hit |= __shfl_xor(hit, off, 64);
      itmax = max(itmax, __shfl_xor(itmax, off, 64));
    }
    if (cc == 0) {
      s_any = any;
      if (blockIdx.x == 0 && !any) {
        ctl->iters_max = itmax;
        ctl->hit_cap = hit;
        __threadfence();
        ctl->done = k;
      }
    }
  }
  __syncthreads();
  T beta[VW], aprev[VW];
#pragma unroll
  for (int q = 0; q < VW; ++q) {
    beta[q] = T(s_beta[(c0 + q) % PP]);
    aprev[q] = T(s_aprev[(c0 + q) % PP]);
  }
  const bool any = s_any != 0;
  for (int64_t row = row0; row < seg1; row += kCgThreads / PPL) {
    if (c0 < p) {
      const int64_t i = row * p + c0;
      const bool first = row == row0;
      T po[VW], xv[VW];
      if (first) {
#pragma unroll
        for (int q = 0; q < VW; ++q) po[q] = po0[q], xv[q] = xv0[q];
      } else {
        ld_vw<VW>(pold + i, po);
        ld_vw<VW>(x + i, xv);
      }
#pragma unroll
      for (int q = 0; q < VW; ++q) xv[q] += aprev[q] * po[q];
      st_vw<VW>(x + i, xv);
      if (any) {
        T zv[VW];
        if (z) {
          if (first) {
#pragma unroll
            for (int q = 0; q < VW; ++q) zv[q] = zr0[q];
          } else {
            TZ zz[VW];
            ld_vw<VW>(z + i, zz);
#pragma unroll
            for (int q = 0; q < VW; ++q) zv[q] = T(zz[q]);
          }
        } else {
          T rv[VW];
          if (first) {
#pragma unroll
            for (int q = 0; q < VW; ++q) rv[q] = zr0[q];
          } else {
            ld_vw<VW>(r + i, rv);
          }
          const T dr = dinv[row];
#pragma unroll
          for (int q = 0; q < VW; ++q) zv[q] = dr * rv[q];
        }
#pragma unroll
        for (int q = 0; q < VW; ++q) zv[q] = zv[q] + beta[q] * po[q];
        st_vw<VW>(pnew + i, zv);
      }
    }
  }
}

template <typename T, int PPL, int VW>
__global__ void __launch_bounds__(kCgThreads)
k_cg_a(int k, int n, int p, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
       const double* __restrict__ val, const T* __restrict__ pk, T* __restrict__ q,
       const KrylovCtl* ctl, double* __restrict__ part_sig) {
  constexpr int PP = PPL * VW;
  if (finished_by(ctl, k)) return;
  __shared__ double red[kCgThreads];
  const int c0 = VW * (threadIdx.x % PPL);
  double sig[VW];
#pragma unroll
  for (int u = 0; u < VW; ++u) sig[u] = 0.0;
  int64_t seg0, seg1;
  xcd_rows(n, seg0, seg1);
  const bool active = c0 < p;
  csr_rows_pipelined<spmm_unroll<T, VW>(), VW>(
      rowptr, colind, val, pk, static_cast<const T*>(nullptr), p, c0, active,
      seg0 + threadIdx.x / PPL, kCgThreads / PPL, seg1, [&](int64_t row, const double(&acc)[VW]) {
        if (!active) return;
        const int64_t i = row * p + c0;
        T qv[VW], pv[VW];
#pragma unroll
        for (int u = 0; u < VW; ++u) qv[u] = T(acc[u]);
        st_vw<VW>(q + i, qv);
        ld_vw<VW>(pk + i, pv);
#pragma unroll
        for (int u = 0; u < VW; ++u) sig[u] += double(pv[u]) * double(qv[u]);
      });
  write_col_partial_vw<PPL, VW>(sig, red, part_sig, PP, 0);
}

template <typename T, int PPL, int VW>
__global__ void __launch_bounds__(kCgThreads)
k_cg_b(int k, int n, int p, const T* __restrict__ dinv, T* __restrict__ r, const T* __restrict__ q,
       CgState* st, const KrylovCtl* ctl, const double* __restrict__ part_sig,
       double* __restrict__ part_rr, int jacobi, float* __restrict__ r32) {
  constexpr int PP = PPL * VW;
  if (finished_by(ctl, k)) return;
  __shared__ double red[kCgThreads];
  __shared__ double tot[PP];
  __shared__ double s_alpha[PP];
  // the first row's r and q are loaded before the scalar reduction
  const int c0 = VW * (threadIdx.x % PPL);
  int64_t seg0, seg1;
  xcd_rows(n, seg0, seg1);
  const int64_t row0 = seg0 + threadIdx.x / PPL;
  const bool pre = row0 < seg1 && c0 < p;
  T rv0[VW], qv0[VW];
  if (pre) {
    ld_vw<VW>(r + row0 * p + c0, rv0);
    ld_vw<VW>(q + row0 * p + c0, qv0);
  }
  reduce_parts<PP, 1>(part_sig, gridDim.x, red, tot);
  if (threadIdx.x < PP) {
    const int cc = threadIdx.x;
    double a = 0.0;
    if (cc < p) {
      const CgSlot& cur = st->slot[k & 1];
      a = (cur.active[cc] && tot[cc] != 0.0) ? cur.rho[cc] / tot[cc] : 0.0;
      if (blockIdx.x == 0) st->slot[k & 1].alpha[cc] = a;
    }
    s_alpha[cc] = a;
  }
  __syncthreads();
  T alpha[VW];
#pragma unroll
  for (int u = 0; u < VW; ++u) alpha[u] = T(s_alpha[(c0 + u) % PP]);
  double rz[VW], rr[VW];
#pragma unroll
  for (int u = 0; u < VW; ++u) rz[u] = rr[u] = 0.0;
  for (int64_t row = row0; row < seg1; row += kCgThreads / PPL) {
    if (c0 < p) {
      const int64_t i = row * p + c0;
      T rv[VW], qv[VW];
      float r32v[VW];
      if (row == row0) {
#pragma unroll
        for (int u = 0; u < VW; ++u) rv[u] = rv0[u], qv[u] = qv0[u];
      } else {
        ld_vw<VW>(r + i, rv);
        ld_vw<VW>(q + i, qv);
      }
      const double dr = jacobi ? double(dinv[row]) : 0.0;
#pragma unroll
      for (int u = 0; u < VW; ++u) {
        rv[u] = rv[u] - alpha[u] * qv[u];
        r32v[u] = float(rv[u]);
        const double rd = double(rv[u]);
        if (jacobi) rz[u] += rd * dr * rd;
        rr[u] += rd * rd;
      }
      st_vw<VW>(r + i, rv);
      if (r32) st_vw<VW>(r32 + i, r32v);   // input of an FP32 preconditioner
    }
  }
  if (jacobi) write_col_partial_vw<PPL, VW>(rz, red, part_rr, 2 * PP, 0);
  write_col_partial_vw<PPL, VW>(rr, red, part_rr, 2 * PP, PP);
}

// ---------------------------------------------------------------------------
// Batched BiCGStab (right preconditioning, y = M^{-1} p, z = M^{-1} s, with
// M^{-1} = D^{-1} fused into the kernels below, or one AMG V-cycle whose
// results y, z the kernels read) on K x = b for nonsymmetric K, column-wise,
// b = sign * src, r^ = b.  Same scheme as the CG: every kernel re-sums the
// previous kernel's partials.
// Iteration i:
//   U1: rho_i = (r^, r), |r|^2 (partials of U3_{i-1} or init); convergence;
//       beta = (rho_i / rho_{i-1}) (alpha / omega); p = r + beta (p - omega v),
//       p = r at i = 0 (p and v start at zero, so they are neither stored by
//       the init nor read here)
//   S1: v = K D^{-1} p, partial (r^, v)
//   U2: alpha = rho_i / (r^, v); s = r - alpha v
//   S2: t = K D^{-1} s, partials (t, s), (t, t)
//   U3: omega = (t, s) / (t, t); x += alpha D^{-1} p + omega D^{-1} s;
//       r = s - omega t; partials (r^, r), |r|^2
// A column stops at |r| <= tol |b|, at the cap, or at a breakdown
// (rho, (r^, v) or (t, t) zero); its later steps are zero.

// Scalars of iteration i live in slot i & 1: U1_i reads slot (i-1) & 1 and
// writes slot i & 1 while every workgroup still reads the previous one.
struct BcgSlot {
  double rho[kMaxP], alpha[kMaxP], omega[kMaxP];
  int active[kMaxP], iters[kMaxP];
};

struct BcgState {
  BcgSlot slot[2];
  double bnorm2[kMaxP];
};

template <typename T, typename TS, int PP>
__global__ void __launch_bounds__(kCgThreads)
k_bcg_init(int n, int p, double sign, const TS* __restrict__ src, T* __restrict__ x,
           T* __restrict__ r, T* __restrict__ rhat, KrylovCtl* ctl, double* __restrict__ part_rr) {
  __shared__ double red[kCgThreads];
  const int c = threadIdx.x % PP;
  double bb = 0.0;
  int64_t seg0, seg1;
  xcd_rows(n, seg0, seg1);
  for (int64_t row = seg0 + threadIdx.x / PP; row < seg1; row += kCgThreads / PP) {
    if (c < p) {
      const int64_t i = row * p + c;
      const T b = T(sign * double(src[i]));
      r[i] = b;
      rhat[i] = b;
      x[i] = T(0);
      bb += double(b) * double(b);
    }
  }
  write_col_partial<PP>(bb, red, part_rr, 2 * PP, 0);   // (r^, r) = |b|^2 at start
  write_col_partial<PP>(bb, red, part_rr, 2 * PP, PP);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->done = -1;
    ctl->iters_max = 0;
    ctl->hit_cap = 0;
    ctl->counter = 0u;
  }
}

// The three BiCGStab updates take VW adjacent columns per lane (PPL = PP / VW
// lanes per row; VW = 2 for even p: 16-byte FP64 accesses) like the SpMM.
template <typename T, int PPL, int VW>
__global__ void __launch_bounds__(kCgThreads)
k_bcg_u1(int i, int n, int p, const T* __restrict__ r, T* __restrict__ pv, const T* __restrict__ v,
         BcgState* st, KrylovCtl* ctl, const double* __restrict__ part_rr, double tol2, int maxit) {
  constexpr int PP = PPL * VW;
  if (finished_before(ctl, i)) return;
  __shared__ double red[kCgThreads];
  __shared__ double tot[2 * PP];
  __shared__ double s_beta[PP], s_om[PP];
  __shared__ int s_any;
  reduce_parts<PP, 2>(part_rr, gridDim.x, red, tot);
  if (threadIdx.x < 64) {
    // one lane per column, as in k_cg_c
    const int cc = threadIdx.x;
    double beta = 0.0, om = 0.0;
    int act = 0, it = 0, hit = 0;
    if (cc < p) {
      const double rho = tot[cc], rn = tot[PP + cc];
      double bn, rho_prev, a_prev, om_prev;
      int act_prev;
      const BcgSlot& prev = st->slot[(i + 1) & 1];
      if (i == 0) {
        bn = rn;
        act_prev = bn > 0.0;
        rho_prev = a_prev = om_prev = 1.0;
      } else {
        bn = st->bnorm2[cc];
        act_prev = prev.active[cc];
        it = prev.iters[cc];
        rho_prev = prev.rho[cc];
        a_prev = prev.alpha[cc];
        om_prev = prev.omega[cc];
      }
      act = act_prev && !(rn <= tol2 * bn);
      if (act && (it >= maxit || rho == 0.0 || om_prev == 0.0 || rho_prev == 0.0)) {
        act = 0;
        hit = 1;
      }
      if (act) {
        beta = (rho / rho_prev) * (a_prev / om_prev);
        om = om_prev;
      }
      if (blockIdx.x == 0) {
        BcgSlot& cur = st->slot[i & 1];
        cur.rho[cc] = rho;
        cur.active[cc] = act;
        cur.iters[cc] = it + act;
        if (i == 0) st->bnorm2[cc] = bn;
      }
    }
    if (cc < PP) {
      s_beta[cc] = beta;
      s_om[cc] = om;
    }
    int any = act, itmax = it;
    for (int off = 32; off >= 1; off >>= 1) {
      any |= __shfl_xor(any, off, 64);
      hit |= __shfl_xor(hit, off, 64);
      itmax = max(itmax, __shfl_xor(itmax, off, 64));
    }
    if (cc == 0) {
      s_any = any;
      if (blockIdx.x == 0 && !any) {
        ctl->iters_max = itmax;
        ctl->hit_cap = hit;
        __threadfence();
        ctl->done = i;
      }
    }
  }
  __syncthreads();
  if (!s_any) return;
  const int c0 = VW * (threadIdx.x % PPL);
  T beta[VW], om[VW];
#pragma unroll
  for (int q = 0; q < VW; ++q) {
    beta[q] = T(s_beta[(c0 + q) % PP]);
    om[q] = T(s_om[(c0 + q) % PP]);
  }
  int64_t seg0, seg1;
  xcd_rows(n, seg0, seg1);
  for (int64_t row = seg0 + threadIdx.x / PPL; row < seg1; row += kCgThreads / PPL) {
    if (c0 < p) {
      const int64_t idx = row * p + c0;
      T rv[VW];
      ld_vw<VW>(r + idx, rv);
      if (i == 0) {
        st_vw<VW>(pv + idx, rv);
        continue;
      }
      T pw[VW], vv[VW];
      ld_vw<VW>(pv + idx, pw);
      ld_vw<VW>(v + idx, vv);
#pragma unroll
      for (int q = 0; q < VW; ++q) pw[q] = rv[q] + beta[q] * (pw[q] - om[q] * vv[q]);
      st_vw<VW>(pv + idx, pw);
    }
  }
}

// out = K D^{-1} in (out = K in when dinv is NULL: the input is already
// preconditioned), partials (a, out) [NV = 1] or (out, a), (out, out) [NV = 2]
template <typename T, int PPL, int VW, int NV>
__global__ void __launch_bounds__(kCgThreads)
k_bcg_s(int i, int n, int p, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
        const double* __restrict__ val, const T* __restrict__ dinv, const T* __restrict__ in,
        const T* __restrict__ a, T* __restrict__ out, const KrylovCtl* ctl,
        double* __restrict__ part) {
  constexpr int PP = PPL * VW;
  if (finished_by(ctl, i)) return;
  __shared__ double red[kCgThreads];
  const int c0 = VW * (threadIdx.x % PPL);
  double d0[VW], d1[VW];
#pragma unroll
  for (int q = 0; q < VW; ++q) d0[q] = d1[q] = 0.0;
  int64_t seg0, seg1;
  xcd_rows(n, seg0, seg1);
  const bool active = c0 < p;
  csr_rows_pipelined<spmm_unroll<T, VW>(), VW>(
      rowptr, colind, val, in, dinv, p, c0, active, seg0 + threadIdx.x / PPL, kCgThreads / PPL,
      seg1, [&](int64_t row, const double(&accd)[VW]) {
        if (!active) return;
        const int64_t idx = row * p + c0;
        T acc[VW], av[VW];
#pragma unroll
        for (int q = 0; q < VW; ++q) acc[q] = T(accd[q]);
        st_vw<VW>(out + idx, acc);
        ld_vw<VW>(a + idx, av);
#pragma unroll
        for (int q = 0; q < VW; ++q) {
          const double o = double(acc[q]);
          d0[q] += double(av[q]) * o;
          if (NV == 2) d1[q] += o * o;
        }
      });
  write_col_partial_vw<PPL, VW>(d0, red, part, NV * PP, 0);
  if (NV == 2) write_col_partial_vw<PPL, VW>(d1, red, part, NV * PP, PP);
}

template <typename T, int PPL, int VW>
__global__ void __launch_bounds__(kCgThreads)
k_bcg_u2(int i, int n, int p, const T* __restrict__ r, const T* __restrict__ v, T* __restrict__ sv,
         BcgState* st, const KrylovCtl* ctl, const double* __restrict__ part) {
  constexpr int PP = PPL * VW;
  if (finished_by(ctl, i)) return;
  __shared__ double red[kCgThreads];
  __shared__ double tot[PP];
  __shared__ double s_a[PP];
  reduce_parts<PP, 1>(part, gridDim.x, red, tot);
  if (threadIdx.x < PP) {
    const int cc = threadIdx.x;
    BcgSlot& cur = st->slot[i & 1];
    double a = 0.0;
    if (cc < p && cur.active[cc] && tot[cc] != 0.0) a = cur.rho[cc] / tot[cc];
    if (cc < p && blockIdx.x == 0) cur.alpha[cc] = a;
    s_a[cc] = a;
  }
  __syncthreads();
  const int c0 = VW * (threadIdx.x % PPL);
  T a[VW];
#pragma unroll
  for (int q = 0; q < VW; ++q) a[q] = T(s_a[(c0 + q) % PP]);
  int64_t seg0, seg1;
  xcd_rows(n, seg0, seg1);
  for (int64_t row = seg0 + threadIdx.x / PPL; row < seg1; row += kCgThreads / PPL) {
    if (c0 < p) {
      const int64_t idx = row * p + c0;
      T rv[VW], vv[VW];
      ld_vw<VW>(r + idx, rv);
      ld_vw<VW>(v + idx, vv);
#pragma unroll
      for (int q = 0; q < VW; ++q) rv[q] = rv[q] - a[q] * vv[q];
      st_vw<VW>(sv + idx, rv);
    }
  }
}

template <typename T, int PPL, int VW>
__global__ void __launch_bounds__(kCgThreads)
k_bcg_u3(int i, int n, int p, const T* __restrict__ dinv, const T* __restrict__ pv,
         const T* __restrict__ sv, const T* __restrict__ tv, const T* __restrict__ rhat,
         const T* __restrict__ ph, const T* __restrict__ sh, T* __restrict__ x,
         T* __restrict__ r, BcgState* st, const KrylovCtl* ctl, const double* __restrict__ part,
         double* __restrict__ part_rr) {
  constexpr int PP = PPL * VW;
  if (finished_by(ctl, i)) return;
  __shared__ double red[kCgThreads];
  __shared__ double tot[2 * PP];
  __shared__ double s_a[PP], s_om[PP];
  reduce_parts<PP, 2>(part, gridDim.x, red, tot);   // tot[c] = (t, s), tot[PP + c] = (t, t)
  if (threadIdx.x < PP) {
    const int cc = threadIdx.x;
    BcgSlot& cur = st->slot[i & 1];
    double a = 0.0, om = 0.0;
    if (cc < p && cur.active[cc]) {
      a = cur.alpha[cc];
      om = tot[PP + cc] != 0.0 ? tot[cc] / tot[PP + cc] : 0.0;
    }
    if (cc < p && blockIdx.x == 0) cur.omega[cc] = om;
    s_a[cc] = a;
    s_om[cc] = om;
  }
  __syncthreads();
  const int c0 = VW * (threadIdx.x % PPL);
  T a[VW], om[VW];
#pragma unroll
  for (int q = 0; q < VW; ++q) {
    a[q] = T(s_a[(c0 + q) % PP]);
    om[q] = T(s_om[(c0 + q) % PP]);
  }
  double rr_hat[VW], rr[VW];
#pragma unroll
  for (int q = 0; q < VW; ++q) rr_hat[q] = rr[q] = 0.0;
  int64_t seg0, seg1;
  xcd_rows(n, seg0, seg1);
  for (int64_t row = seg0 + threadIdx.x / PPL; row < seg1; row += kCgThreads / PPL) {
    if (c0 < p) {
      const int64_t idx = row * p + c0;
      T sval[VW], xv[VW], tw[VW], rh[VW], u[VW], w[VW];
      ld_vw<VW>(sv + idx, sval);
      ld_vw<VW>(x + idx, xv);
      ld_vw<VW>(tv + idx, tw);
      ld_vw<VW>(rhat + idx, rh);
      if (ph) {
        ld_vw<VW>(ph + idx, u);
        ld_vw<VW>(sh + idx, w);
#pragma unroll
        for (int q = 0; q < VW; ++q) xv[q] += a[q] * u[q] + om[q] * w[q];
      } else {
        const T dv = dinv[row];
        ld_vw<VW>(pv + idx, u);
#pragma unroll
        for (int q = 0; q < VW; ++q) xv[q] += a[q] * (dv * u[q]) + om[q] * (dv * sval[q]);
      }
      st_vw<VW>(x + idx, xv);
      T rn[VW];
#pragma unroll
      for (int q = 0; q < VW; ++q) {
        rn[q] = sval[q] - om[q] * tw[q];
        rr_hat[q] += double(rh[q]) * double(rn[q]);
        rr[q] += double(rn[q]) * double(rn[q]);
      }
      st_vw<VW>(r + idx, rn);
    }
  }
  write_col_partial_vw<PPL, VW>(rr_hat, red, part_rr, 2 * PP, 0);
  write_col_partial_vw<PPL, VW>(rr, red, part_rr, 2 * PP, PP);
}

// R = V + K W (the residual of M W = V, M = -K) in FP64 from blocks of type
// T, stored as TI: the right-hand side of a refinement step.
template <typename T, typename TI, int PP>
__global__ void __launch_bounds__(kThreads)
k_refine_residual(int n, int p, const int32_t* __restrict__ rowptr,
                  const int32_t* __restrict__ colind, const double* __restrict__ val,
                  const T* __restrict__ V, const T* __restrict__ W, TI* __restrict__ R) {
  const int c = threadIdx.x % PP;
  const int64_t rows_per_grid = int64_t(gridDim.x) * (kThreads / PP);
  for (int64_t row = int64_t(blockIdx.x) * (kThreads / PP) + threadIdx.x / PP; row < n;
       row += rows_per_grid) {
    if (c < p) {
      double acc = double(V[row * p + c]);
      for (int e = rowptr[row]; e < rowptr[row + 1]; ++e)
        acc += val[e] * double(W[int64_t(colind[e]) * p + c]);
      R[row * p + c] = TI(acc);
    }
  }
}

// W += D (types may differ)
template <typename T, typename TI>
__global__ void __launch_bounds__(kThreads)
k_add_to(int64_t count, const TI* __restrict__ D, T* __restrict__ W) {
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * kThreads)
    W[i] = T(double(W[i]) + double(D[i]));
}

// out = (double) x
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_to_f64(int64_t count, const T* __restrict__ x, double* __restrict__ out) {
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * kThreads)
    out[i] = double(x[i]);
}

}  // namespace expmv
