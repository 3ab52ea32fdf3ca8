// Block Gram-Schmidt and CholQR passes on matrix cores (MFMA 16x16x4, FP64
// or FP32): the same five modes as k_orth (kernels_dense.hpp), as tall-skinny
// contractions over the n rows.
//
// One workgroup = 4 wavefronts handles 64 rows per step; wave w owns the
// 16-row block w of the step:
//   1. the block's updated rows W' (in the MFMA result layout):
//        kProj                 W' = W
//        kUpdProj / kUpdGram   W' = W - V C     (C: (npan p) x p, K = npan p)
//        kScaleGram / kScale   W' = W C         (C: p x p, K = p)
//      written to Wout (all modes but kProj) and to LDS;
//   2. after a barrier the contractions over the step's 64 rows, the B
//      operands read from LDS:
//        projection V^T W' (kProj, kUpdProj): wave w owns the 16-column
//        blocks mb = w, w + 4, ...; the A operand is read from V;
//        Gram W'^T W' (kUpdGram, kScaleGram): wave w owns block pair w.
// Every K-step of 4 rows is exact in the MFMA's own precision; each 16-row
// block's sums are added to FP64 accumulators, so an FP32 basis accumulates
// in FP32 only within 16 rows.  Partial sums per workgroup, layout as k_orth.
// W and Wout may be the same array (each row is read by the wave that
// rewrites it, before it does).
//
// Lane layout of the 16x16x4 builtins (checked on gfx950): lane l supplies
// A(l % 16, l / 16) and B(l / 16, l % 16); D(i, j) comes back in lane
// j + 16 (i / 4) (FP32) or j + 16 (i % 4) (FP64), register i % 4 (FP32) or
// i / 4 (FP64).  So lane l's register s holds row drow(l, s) of the result,
// and register s of all lanes is exactly the B operand of the K-step whose
// 4 rows are {drow(16 k, s)}.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "kernels_dense.hpp"

namespace expmv {

template <typename T>
struct Mma;

template <>
struct Mma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int drow(int l, int r) { return (l >> 4) + 4 * r; }
};

template <>
struct Mma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int drow(int l, int r) { return 4 * (l >> 4) + r; }
};

// element (row, col) of the basis: column col = panel * p + a
template <typename T>
__device__ inline T basis_at(const T* __restrict__ V, int64_t n, int p, int64_t row, int col) {
  const int pan = col / p;
  return V[int64_t(pan) * n * p + row * p + (col - pan * p)];
}

// Projection column blocks per wave whose sums k_orth_mma keeps in registers
// rather than LDS (at most three), chosen so that one more workgroup fits a
// CU's 160 KB: FP64 with one column block of W and six blocks per wave
// (56.5 -> 48.5 KB, three per CU), and with two column blocks of W, FP64 at
// four (81 -> 65 KB) or six (113 -> 65 KB) and FP32 at six (105 -> 73 KB):
// two per CU.
template <typename T, int NB, int MBW>
constexpr int orth_reg_blocks() {
  return sizeof(T) == 8 ? (NB == 1 ? (MBW == 6 ? 1 : 0) : (MBW == 4 ? 1 : (MBW == 6 ? 3 : 0)))
                        : (NB == 2 && MBW == 6 ? 2 : 0);
}

// LDS bytes of k_orth_mma<T, NB, MBW, *>: sW, sN and sP
template <typename T, int NB, int MBW>
constexpr size_t orth_mma_lds() {
  return sizeof(T) * 64 * 16 * NB + sizeof(double) * 4 * 16 * NB +
         sizeof(double) * 4 * (MBW - orth_reg_blocks<T, NB, MBW>()) * 256 * NB;
}

// NB = 16-column blocks of W (p <= 16 NB); MBW = projection column blocks
// per wave (npan p <= 64 MBW); PC = p when it is known at compile time (16 NB:
// panel and column offsets by shifts), else 0.  Basis and W loads clamp
// their row and column to the array and zero what lies outside, so that
// they need no branch and the compiler can issue a whole batch at once.
template <typename T, int NB, int MBW, int PC>
__global__ void __launch_bounds__(kThreads)
k_orth_mma(int mode, int64_t n, int p_arg, const T* __restrict__ V, int npan, const T* W,
           T* Wout, const double* __restrict__ C, double* __restrict__ partial,
           const int* __restrict__ gate) {
  if (gate && *gate == 0) return;   // conditional pass not requested
  const int p = PC ? PC : p_arg;
  using M = Mma<T>;
  using v4 = typename M::v4;
  __shared__ T sW[64 * 16 * NB];        // W' of the step, row-major, ld 16 NB
  __shared__ double sN[4][16 * NB];     // per-wave column norms (kProj)
  // the projection sums of column block mb live in LDS (sP[mb], NB blocks of
  // 16 x 16, row = basis column within the block), so that the loop over a
  // wave's blocks need not be unrolled to keep them in registers; the first
  // RB blocks (u < RB) keep their sums in registers (racc0 .. racc2)
  // instead, so that one more workgroup fits a CU
  constexpr int RB = orth_reg_blocks<T, NB, MBW>();
  static_assert(RB <= 3 && RB < MBW, "at most three projection blocks in registers");
  __shared__ double sP[4 * (MBW - RB)][256 * NB];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ldw = 16 * NB;
  const int np_cols = npan * p;
  const int nmb = (np_cols + 15) / 16;
  const bool upd = (mode == kUpdProj || mode == kUpdGram);
  const bool scl = (mode == kScaleGram || mode == kScale);
  const bool proj = (mode == kProj || mode == kUpdProj);
  const bool gram = (mode == kUpdGram || mode == kScaleGram);

  double gacc[4] = {0.0, 0.0, 0.0, 0.0};   // Gram block of this wave
  if (proj)
    for (int u = 0; u < MBW - RB; ++u)
      for (int e = lane; e < 256 * NB; e += 64) sP[wave + 4 * u][e] = 0.0;
  double racc0[NB][4], racc1[NB][4], racc2[NB][4];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) racc0[b][r] = racc1[b][r] = racc2[b][r] = 0.0;
  double nrm[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) nrm[b] = 0.0;
  // Gram block pair of this wave (pairs (b1, b2) with b1, b2 < NB)
  const int g1 = wave / NB, g2 = wave % NB;
  const bool gram_owner = gram && wave < NB * NB;

  const int64_t steps = (n + 63) / 64;
  for (int64_t st = blockIdx.x; st < steps; st += gridDim.x) {
    const int64_t r0 = st * 64 + 16 * wave;   // this wave's 16-row block
    // ---- 1. updated rows of the wave's block
    v4 d[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) d[b] = v4{0, 0, 0, 0};
    if (upd || scl) {
      const int K = upd ? np_cols : p;
      const int64_t row = r0 + li;   // A operand row of this lane
      const int64_t rowc = row < n ? row : n - 1;
      // KB K-steps per iteration (8 with one column block, 4 with two),
      // every load issued before the products
      constexpr int KB = NB == 1 ? 8 : 4;
      for (int k0 = 0; k0 < K; k0 += 4 * KB) {
        T a[KB], bv[KB][NB];
#pragma unroll
        for (int u = 0; u < KB; ++u) {
          const int kc = k0 + 4 * u + lk;
          const int kcc = kc < K ? kc : K - 1;
          const T av = upd ? basis_at(V, n, p, rowc, kcc) : W[rowc * p + kcc];
          a[u] = (kc < K && row < n) ? av : T(0);
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const int j = 16 * b + li;
            const double cv = C[int64_t(kcc) * p + (j < p ? j : p - 1)];
            bv[u][b] = (kc < K && j < p) ? T(cv) : T(0);
          }
        }
#pragma unroll
        for (int u = 0; u < KB; ++u)
#pragma unroll
          for (int b = 0; b < NB; ++b) d[b] = M::mma(a[u], bv[u][b], d[b]);
      }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = 16 * b + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = M::drow(lane, r);
        const int64_t row = r0 + i;
        T w = T(0);
        if (row < n && j < p) {
          if (upd) w = T(double(W[row * p + j]) - double(d[b][r]));
          else if (scl) w = d[b][r];
          else w = W[row * p + j];
          if (mode != kProj) Wout[row * p + j] = w;
        }
        sW[(16 * wave + i) * ldw + j] = w;
        if (mode == kProj) nrm[b] += double(w) * double(w);
      }
    }
    __syncthreads();
    // ---- 2. contractions over the step's 64 rows
    if (proj) {
#pragma unroll 1
      for (int u = 0; u < MBW; ++u) {
        const int mb = wave + 4 * u;
        if (mb >= nmb) break;
        const int col = 16 * mb + li;
        v4 t[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) t[b] = v4{0, 0, 0, 0};
        // the 16 K-steps of the step's 64 rows: all 16 loads first
        const int colc = col < np_cols ? col : np_cols - 1;
        T a[16];
#pragma unroll
        for (int qs = 0; qs < 16; ++qs) {
          const int64_t row = st * 64 + 16 * (qs >> 2) + M::drow(lane, qs & 3);
          const T av = basis_at(V, n, p, row < n ? row : n - 1, colc);
          a[qs] = (col < np_cols && row < n) ? av : T(0);
        }
#pragma unroll
        for (int qs = 0; qs < 16; ++qs) {
          const int i = 16 * (qs >> 2) + M::drow(lane, qs & 3);
#pragma unroll
          for (int b = 0; b < NB; ++b) t[b] = M::mma(a[qs], sW[i * ldw + 16 * b + li], t[b]);
        }
        if (RB > 0 && u == 0) {
#pragma unroll
          for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) racc0[b][r] += double(t[b][r]);
        } else if (RB > 1 && u == 1) {
#pragma unroll
          for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) racc1[b][r] += double(t[b][r]);
        } else if (RB > 2 && u == 2) {
#pragma unroll
          for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) racc2[b][r] += double(t[b][r]);
        } else {
#pragma unroll
          for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              sP[mb - 4 * RB][256 * b + M::drow(lane, r) * 16 + li] += double(t[b][r]);
        }
      }
    }
    if (gram_owner) {
      v4 t = v4{0, 0, 0, 0};
      for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int i = M::drow(lane, s);
          const T* rw = sW + (16 * q + i) * ldw;
          t = M::mma(rw[16 * g1 + li], rw[16 * g2 + li], t);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) gacc[r] += double(t[r]);
    }
    __syncthreads();
  }

  // ---- partial sums of this workgroup
  const int O = proj ? np_cols * p + (mode == kProj ? p : 0) : (gram ? p * p : 0);
  double* out = partial + size_t(blockIdx.x) * O;
  if (proj) {
#pragma unroll
    for (int u = 0; u < MBW; ++u) {
      const int mb = wave + 4 * u;
      if (mb >= nmb) break;
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int col = 16 * mb + M::drow(lane, r), j = 16 * b + li;
          if (col < np_cols && j < p)
            out[col * p + j] =
                u < RB ? (u == 0 ? racc0[b][r] : (u == 1 ? racc1[b][r] : racc2[b][r]))
                       : sP[mb - 4 * RB][256 * b + M::drow(lane, r) * 16 + li];
        }
    }
  }
  if (mode == kProj) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      double v = nrm[b];
      v += __shfl_xor(v, 16, 64);
      v += __shfl_xor(v, 32, 64);
      if (lk == 0) sN[wave][16 * b + li] = v;
    }
    __syncthreads();
    if (threadIdx.x < p)
      out[np_cols * p + threadIdx.x] = ((sN[0][threadIdx.x] + sN[1][threadIdx.x]) +
                                        sN[2][threadIdx.x]) + sN[3][threadIdx.x];
  }
  if (gram_owner) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int a = 16 * g1 + M::drow(lane, r), j = 16 * g2 + li;
      if (a < p && j < p) out[a * p + j] = gacc[r];
    }
  }
}

// out (+)= V C on matrix cores in FP64 (an FP32 basis is widened on load):
// V = npan basis panels (n x p each, columns k < npan p), C FP64
// (npan p) x nout with leading dimension ldc; output column oc = q p + b goes
// to out[q chunk_stride + row ldo + b].  The X update (out = X, chunk_stride
// = p, ldo = 14 p) and the restart rotation (out = new panels, chunk_stride =
// n p, ldo = p).  A workgroup handles 16 RB rows per step; wave w computes
// the 16-column output blocks w, w + 4, ... (NBW of them) for all RB row
// blocks, so V is read from memory once and C once per step.
template <typename T, typename TO, int NBW, int RB, int PC = 0>
__global__ void __launch_bounds__(kThreads)
k_panel_gemm_mma(int64_t n, int p_arg, const T* __restrict__ V, int npan,
                 const double* __restrict__ C, int ldc, int nout, TO* __restrict__ out,
                 int64_t chunk_stride, int64_t ldo, int accumulate) {
  const int p = PC ? PC : p_arg;   // PC: p known at compile time
  using M = Mma<double>;
  using v4 = M::v4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int np_cols = npan * p;
  const int nnb = (nout + 15) / 16;
  const int64_t steps = (n + 16 * RB - 1) / (16 * RB);
  for (int64_t st = blockIdx.x; st < steps; st += gridDim.x) {
    const int64_t r0 = st * 16 * RB;
    v4 acc[RB][NBW];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int u = 0; u < NBW; ++u) acc[rb][u] = v4{0, 0, 0, 0};
    // KH K-steps per iteration, every load issued before the products: four
    // with up to two row blocks (the X update: 10.7 against 11.4 ms at
    // m = 24, p = 16), two with four (the restart rotation, where four
    // measured slower)
    constexpr int KH = RB <= 2 ? 4 : 2;
    for (int k0 = 0; k0 < np_cols; k0 += 4 * KH) {
      double a[KH][RB], bv[KH][NBW];
#pragma unroll
      for (int h = 0; h < KH; ++h) {
        const int kc = k0 + 4 * h + lk;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          const int64_t row = r0 + 16 * rb + li;
          a[h][rb] = (kc < np_cols && row < n) ? double(basis_at(V, n, p, row, kc)) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < NBW; ++u) {
          const int oc = 16 * (wave + 4 * u) + li;
          bv[h][u] = (kc < np_cols && oc < nout) ? C[int64_t(kc) * ldc + oc] : 0.0;
        }
      }
#pragma unroll
      for (int h = 0; h < KH; ++h)
#pragma unroll
        for (int u = 0; u < NBW; ++u) {
          if (wave + 4 * u >= nnb) break;
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) acc[rb][u] = M::mma(a[h][rb], bv[h][u], acc[rb][u]);
        }
    }
#pragma unroll
    for (int u = 0; u < NBW; ++u) {
      const int nb = wave + 4 * u;
      if (nb >= nnb) break;
      const int oc = 16 * nb + li;
      if (oc >= nout) continue;
      const int q = oc / p, b = oc - q * p;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = r0 + 16 * rb + M::drow(lane, r);
          if (row >= n) continue;
          TO* dst = out + q * chunk_stride + row * ldo + b;
          *dst = accumulate ? TO(double(*dst) + acc[rb][u][r]) : TO(acc[rb][u][r]);
        }
    }
  }
}

}  // namespace expmv
