// Toeplitz operator kernels: a batched complex FFT (Stockham autosort,
// mixed radix 8/4/2/5/3, q interleaved columns), real <-> complex packing of
// two real columns per complex column, and the pointwise spectral products
// of the circulant-embedding product T v and of the Gohberg-Semencul
// formula for T^{-1} v (paper, Section 4.1 and the fast Toeplitz products of
// Section 2).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "kernels_dense.hpp"

namespace expmv {

// V = DFT_R(v): V_m = sum_r v_r exp(sign 2 pi i r m / R)
template <int R>
__device__ inline void dft_small(const cplx (&v)[R], cplx (&V)[R], double sign) {
  if constexpr (R == 2) {
    V[0] = {v[0].x + v[1].x, v[0].y + v[1].y};
    V[1] = {v[0].x - v[1].x, v[0].y - v[1].y};
  } else if constexpr (R == 4) {
    const cplx a{v[0].x + v[2].x, v[0].y + v[2].y}, b{v[0].x - v[2].x, v[0].y - v[2].y};
    const cplx c2{v[1].x + v[3].x, v[1].y + v[3].y}, d{v[1].x - v[3].x, v[1].y - v[3].y};
    // d * (sign i)
    const cplx di{-sign * d.y, sign * d.x};
    V[0] = {a.x + c2.x, a.y + c2.y};
    V[2] = {a.x - c2.x, a.y - c2.y};
    V[1] = {b.x + di.x, b.y + di.y};
    V[3] = {b.x - di.x, b.y - di.y};
  } else {
    // R = 8, 5, 3: V_m = sum_r v_r exp(sign 2 pi i r m / R), with the
    // cosines and sines of 2 pi e / R, e = 0 .. R-1
    static_assert(R == 8 || R == 5 || R == 3, "radix");
    constexpr double h = 0.70710678118654752440;
    constexpr double c1 = 0.30901699437494742410, c2 = -0.80901699437494742410;
    constexpr double s1 = 0.95105651629515357212, s2 = 0.58778525229247312917;
    constexpr double s3 = 0.86602540378443864676;
    double cs[R], sn[R];
    if constexpr (R == 8) {
      const double c8[8] = {1.0, h, 0.0, -h, -1.0, -h, 0.0, h};
      const double s8[8] = {0.0, h, 1.0, h, 0.0, -h, -1.0, -h};
#pragma unroll
      for (int e = 0; e < 8; ++e) cs[e] = c8[e], sn[e] = s8[e];
    } else if constexpr (R == 5) {
      const double c5[5] = {1.0, c1, c2, c2, c1};
      const double s5[5] = {0.0, s1, s2, -s2, -s1};
#pragma unroll
      for (int e = 0; e < 5; ++e) cs[e] = c5[e], sn[e] = s5[e];
    } else {
      const double c3[3] = {1.0, -0.5, -0.5};
      const double s3v[3] = {0.0, s3, -s3};
#pragma unroll
      for (int e = 0; e < 3; ++e) cs[e] = c3[e], sn[e] = s3v[e];
    }
#pragma unroll
    for (int m = 0; m < R; ++m) {
      double xr = 0.0, xi = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e = (r * m) % R;
        const double wr = cs[e], wi = sign * sn[e];
        xr += v[r].x * wr - v[r].y * wi;
        xi += v[r].x * wi + v[r].y * wr;
      }
      V[m] = {xr, xi};
    }
  }
}

// One Stockham pass of radix R over a length-L transform, q columns
// interleaved (element i of column c at [i * q + c]).  Ns = product of the
// radices of the earlier passes.  Thread (j, c), j < L / R:
//   v_r = in[j + r L/R] * w^{r (j mod Ns)},  w = exp(sign 2 pi i / (Ns R))
//   V = DFT_R(v) (sign),  out[(j / Ns) Ns R + (j mod Ns) + r Ns] = V_r
template <int R>
__global__ void __launch_bounds__(kThreads)
k_fft_pass(int64_t L, int q, int64_t Ns, const cplx* __restrict__ in, cplx* __restrict__ out,
           double sign) {
  const int64_t total = (L / R) * q;
  for (int64_t gid = int64_t(blockIdx.x) * kThreads + threadIdx.x; gid < total;
       gid += int64_t(gridDim.x) * kThreads) {
    const int64_t j = gid / q;
    const int c = int(gid % q);
    const int64_t k = j % Ns;
    cplx v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = in[(j + r * (L / R)) * q + c];
    if (Ns > 1) {
      double sw, cw;
      sincospi(sign * 2.0 * double(k) / double(Ns * R), &sw, &cw);
      cplx w{cw, sw}, wr = w;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        v[r] = cmul(v[r], wr);
        wr = cmul(wr, w);
      }
    }
    cplx V[R];
    dft_small<R>(v, V, sign);
    const int64_t idxD = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) out[(idxD + r * Ns) * q + c] = V[r];
  }
}

// One Stockham pass of radix 64 (same index map as k_fft_pass<64>), the
// 64-point DFT as 8 x 8 in LDS: with r = r1 + 8 r2 and m = m2 + 8 m1,
//   X_m = sum_r1 w8^(r1 m1) w64^(r1 m2) Y_r1(m2),  Y_r1(m2) = sum_r2 v_(r1+8 r2) w8^(r2 m2)
// (w_N = exp(sign 2 pi i / N)).  A workgroup of 512 threads takes 64 (j, c)
// pairs, eight threads t per pair: thread t loads v_(t + 8 s), s < 8, forms
// Y_t, scales it by w64^(t m2) and writes it to LDS; after a barrier thread t
// reads Y_r1(t) of its pair and writes X_(t + 8 m1), m1 < 8.  One pass over
// the data instead of two radix-8 passes.
constexpr int kFft64Threads = 512;
__global__ void __launch_bounds__(kFft64Threads)
k_fft_pass64(int64_t L, int q, int64_t Ns, const cplx* __restrict__ in, cplx* __restrict__ out,
             double sign) {
  __shared__ cplx sY[8][8][64];   // [r1][m2][pair]
  const int pc = threadIdx.x % 64, t = threadIdx.x / 64;
  const int64_t pairs = (L / 64) * q;
  const int64_t stride = L / 64;
  for (int64_t base = int64_t(blockIdx.x) * 64; base < pairs; base += int64_t(gridDim.x) * 64) {
    const int64_t gp = base + pc;
    const bool ok = gp < pairs;
    const int64_t j = ok ? gp / q : 0;
    const int c = ok ? int(gp % q) : 0;
    const int64_t k = j % Ns;
    cplx v[8];
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2)
      v[s2] = ok ? in[(j + (t + 8 * s2) * stride) * q + c] : cplx{0.0, 0.0};
    if (Ns > 1) {
      // v_r *= w^(r k), w = exp(sign 2 pi i / (Ns 64)), r = t + 8 s2
      double sb, cb, ss, cs;
      sincospi(sign * 2.0 * double(t * k) / double(Ns * 64), &sb, &cb);
      sincospi(sign * 2.0 * double(8 * k) / double(Ns * 64), &ss, &cs);
      cplx wr{cb, sb};
      const cplx w8{cs, ss};
#pragma unroll
      for (int s2 = 0; s2 < 8; ++s2) {
        v[s2] = cmul(v[s2], wr);
        wr = cmul(wr, w8);
      }
    }
    cplx Y[8];
    dft_small<8>(v, Y, sign);
#pragma unroll
    for (int m2 = 0; m2 < 8; ++m2) {
      double si, co;
      sincospi(sign * 2.0 * double(t * m2) / 64.0, &si, &co);
      sY[t][m2][pc] = cmul(Y[m2], cplx{co, si});
    }
    __syncthreads();
    cplx Z[8], X[8];
#pragma unroll
    for (int r1 = 0; r1 < 8; ++r1) Z[r1] = sY[r1][t][pc];
    __syncthreads();   // sY is rewritten by the next group of pairs
    dft_small<8>(Z, X, sign);
    if (ok) {
      const int64_t idxD = (j / Ns) * Ns * 64 + k;
#pragma unroll
      for (int m1 = 0; m1 < 8; ++m1) out[(idxD + (t + 8 * m1) * Ns) * q + c] = X[m1];
    }
  }
}

// One Stockham pass of radix 512 (same index map), the 512-point DFT as
// 8 x 64 with the 64-point DFTs as 8 x 8, all in LDS: with r = a + 8 b,
// b = b0 + 8 b1, m = c + 64 d, c = c2 + 8 c1 (w_N = exp(sign 2 pi i / N)),
//   Y_a(c)  = sum_b0 w8^(b0 c1) w64^(b0 c2) sum_b1 v_(a + 8 b0 + 64 b1) w8^(b1 c2)
//   X_m     = sum_a w8^(a d) w512^(a c) Y_a(c).
// A workgroup of 512 threads takes 8 (j, c) pairs, 64 threads t per pair:
// stage 1, t = a + 8 b0: loads v_(t + 64 s), s < 8, the inner 8-point DFT
// over b1; stage 2, t = a + 8 c2: the 8-point DFT over b0; stage 3, t = c:
// the 8-point DFT over a, writing X_(c + 64 d).  One pass over the data
// instead of three radix-8 passes.
constexpr int kFft512Threads = 512;
__global__ void __launch_bounds__(kFft512Threads)
k_fft_pass512(int64_t L, int q, int64_t Ns, const cplx* __restrict__ in, cplx* __restrict__ out,
              double sign) {
  __shared__ cplx sb[8][64][8];   // stage 1: [a][b0 + 8 c2][pair]; stage 2: [a][c][pair]
  // the fixed twiddles of the two inner transposes, exp(sign 2 pi i e / 512)
  // for e = 0..511 (stage 1 uses e = 8 b0 c2), formed once per workgroup
  // rather than by sincospi per element
  __shared__ cplx tw[512];
  for (int e = threadIdx.x; e < 512; e += kFft512Threads) {
    double si, co;
    sincospi(sign * 2.0 * double(e) / 512.0, &si, &co);
    tw[e] = {co, si};
  }
  __syncthreads();
  const int pc = threadIdx.x % 8, t = threadIdx.x / 8;
  const int64_t pairs = (L / 512) * q;
  const int64_t stride = L / 512;
  for (int64_t base = int64_t(blockIdx.x) * 8; base < pairs; base += int64_t(gridDim.x) * 8) {
    const int64_t gp = base + pc;
    const bool ok = gp < pairs;
    const int64_t j = ok ? gp / q : 0;
    const int c = ok ? int(gp % q) : 0;
    const int64_t k = j % Ns;
    // stage 1: thread t = a + 8 b0
    cplx v[8];
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2)
      v[s2] = ok ? in[(j + (t + 64 * s2) * stride) * q + c] : cplx{0.0, 0.0};
    if (Ns > 1) {
      // v_r *= w^(r k), w = exp(sign 2 pi i / (Ns 512)), r = t + 64 s2
      double sbv, cbv, ss, cs;
      sincospi(sign * 2.0 * double(t * k) / double(Ns * 512), &sbv, &cbv);
      sincospi(sign * 2.0 * double(64 * k) / double(Ns * 512), &ss, &cs);
      cplx wr{cbv, sbv};
      const cplx w64{cs, ss};
#pragma unroll
      for (int s2 = 0; s2 < 8; ++s2) {
        v[s2] = cmul(v[s2], wr);
        wr = cmul(wr, w64);
      }
    }
    {
      const int a = t % 8, b0 = t / 8;
      cplx Z[8];
      dft_small<8>(v, Z, sign);
#pragma unroll
      for (int c2 = 0; c2 < 8; ++c2) sb[a][b0 + 8 * c2][pc] = cmul(Z[c2], tw[8 * b0 * c2]);
    }
    __syncthreads();
    // stage 2: thread t = a + 8 c2
    {
      const int a = t % 8, c2 = t / 8;
      cplx u[8], W[8];
#pragma unroll
      for (int b0 = 0; b0 < 8; ++b0) u[b0] = sb[a][b0 + 8 * c2][pc];
      __syncthreads();   // every stage-1 value is read before stage 2 overwrites
      dft_small<8>(u, W, sign);
#pragma unroll
      for (int c1 = 0; c1 < 8; ++c1) {
        const int cc = c2 + 8 * c1;
        sb[a][cc][pc] = cmul(W[c1], tw[a * cc]);
      }
    }
    __syncthreads();
    // stage 3: thread t = c
    cplx y[8], X[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) y[a] = sb[a][t][pc];
    __syncthreads();   // sb is rewritten by the next group of pairs
    dft_small<8>(y, X, sign);
    if (ok) {
      const int64_t idxD = (j / Ns) * Ns * 512 + k;
#pragma unroll
      for (int d = 0; d < 8; ++d) out[(idxD + (t + 64 * d) * Ns) * q + c] = X[d];
    }
  }
}

// out (L x q complex) = rows of src (n x p real, row-major), two real
// columns per complex column (2c -> real part, 2c+1 -> imaginary part),
// rows reversed if `reverse`, zero for rows >= n, times scale and, when rs
// is not null, times rs[source row] (a diagonal applied before the product).
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_pack(int64_t n, int p, int64_t ld, int q, int64_t L, const T* __restrict__ src,
       cplx* __restrict__ out, int reverse, double scale, const double* __restrict__ rs) {
  for (int64_t gid = int64_t(blockIdx.x) * kThreads + threadIdx.x; gid < L * q;
       gid += int64_t(gridDim.x) * kThreads) {
    const int64_t i = gid / q;
    const int c = int(gid % q);
    cplx v{0.0, 0.0};
    if (i < n) {
      const int64_t row = reverse ? (n - 1 - i) : i;
      const double sc = rs ? scale * rs[row] : scale;
      v.x = sc * double(src[row * ld + 2 * c]);
      if (2 * c + 1 < p) v.y = sc * double(src[row * ld + 2 * c + 1]);
    }
    out[gid] = v;
  }
}

// dst (n x p real) (+)= scale * the first n rows of in (reversed if
// `reverse`), unpacking the two real columns of each complex column; when
// rs is not null each destination row i is also scaled by rs[i] (a diagonal
// applied after the product).
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_unpack(int64_t n, int p, int64_t ld, int q, const cplx* __restrict__ in, T* __restrict__ dst,
         int reverse, double scale, int accumulate, const double* __restrict__ rs) {
  for (int64_t gid = int64_t(blockIdx.x) * kThreads + threadIdx.x; gid < n * p;
       gid += int64_t(gridDim.x) * kThreads) {
    const int64_t i = gid / p;
    const int col = int(gid % p);
    const int64_t src_row = reverse ? (n - 1 - i) : i;
    const cplx v = in[src_row * q + col / 2];
    const double x = (rs ? scale * rs[i] : scale) * ((col & 1) ? v.y : v.x);
    T* d = dst + i * ld + col;
    *d = accumulate ? T(double(*d) + x) : T(x);
  }
}

// data[i, c] *= h[i] * scale
__global__ void __launch_bounds__(kThreads)
k_spec_mul(int64_t L, int q, cplx* __restrict__ data, const cplx* __restrict__ h, double scale) {
  for (int64_t gid = int64_t(blockIdx.x) * kThreads + threadIdx.x; gid < L * q;
       gid += int64_t(gridDim.x) * kThreads) {
    const cplx w = h[gid / q];
    const cplx v = cmul(data[gid], w);
    data[gid] = {scale * v.x, scale * v.y};
  }
}

// out[i, c] = in[i, c] * h[i] * scale
__global__ void __launch_bounds__(kThreads)
k_spec_mul_to(int64_t L, int q, const cplx* __restrict__ in, const cplx* __restrict__ h,
              cplx* __restrict__ out, double scale) {
  for (int64_t gid = int64_t(blockIdx.x) * kThreads + threadIdx.x; gid < L * q;
       gid += int64_t(gridDim.x) * kThreads) {
    const cplx v = cmul(in[gid], h[gid / q]);
    out[gid] = {scale * v.x, scale * v.y};
  }
}

// out[i, c] = (ha[i] a[i, c] - hb[i] b[i, c]) * scale
__global__ void __launch_bounds__(kThreads)
k_spec_mul2(int64_t L, int q, const cplx* __restrict__ a, const cplx* __restrict__ ha,
            const cplx* __restrict__ b, const cplx* __restrict__ hb, cplx* __restrict__ out,
            double scale) {
  for (int64_t gid = int64_t(blockIdx.x) * kThreads + threadIdx.x; gid < L * q;
       gid += int64_t(gridDim.x) * kThreads) {
    const int64_t i = gid / q;
    const cplx u = cmul(a[gid], ha[i]), v = cmul(b[gid], hb[i]);
    out[gid] = {scale * (u.x - v.x), scale * (u.y - v.y)};
  }
}

// out[i, c] = in[n - 1 - i, c] * scale for i < n, 0 for n <= i < L
// (the reversal between the two triangular products of Gohberg-Semencul)
__global__ void __launch_bounds__(kThreads)
k_rev_trunc(int64_t L, int64_t n, int q, const cplx* __restrict__ in, cplx* __restrict__ out,
            double scale) {
  for (int64_t gid = int64_t(blockIdx.x) * kThreads + threadIdx.x; gid < L * q;
       gid += int64_t(gridDim.x) * kThreads) {
    const int64_t i = gid / q;
    const int c = int(gid % q);
    cplx v{0.0, 0.0};
    if (i < n) {
      const cplx s = in[(n - 1 - i) * q + c];
      v = {scale * s.x, scale * s.y};
    }
    out[gid] = v;
  }
}

// ---------------------------------------------------------------------------
// Length-n form of the Gohberg-Semencul inverse: products with n x n
// circulants C(g) = F^{-1} diag(F g) F and skew-circulants
// S(h) = D^{-1} C(D h) D, D = diag(exp(i pi k / n)), so every transform has
// length n (no embedding).  exp(sign i pi k / n) is the "twist" below.

__device__ inline cplx twist_factor(int64_t k, int64_t n, double sign) {
  double si, co;
  sincospi(sign * double(k) / double(n), &si, &co);
  return {co, si};
}

// out (n x q complex) = rows of src (n x p real) two real columns per complex
// column (2c -> real, 2c+1 -> imaginary), times scale (and rs[row] when rs is
// not null), then times exp(sign i pi row / n) (sign 0: no twist)
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_pack_twist(int64_t n, int p, int64_t ld, int q, const T* __restrict__ src,
             cplx* __restrict__ out, double scale, const double* __restrict__ rs, double sign) {
  for (int64_t gid = int64_t(blockIdx.x) * kThreads + threadIdx.x; gid < n * q;
       gid += int64_t(gridDim.x) * kThreads) {
    const int64_t i = gid / q;
    const int c = int(gid % q);
    const double sc = rs ? scale * rs[i] : scale;
    cplx v{sc * double(src[i * ld + 2 * c]), 0.0};
    if (2 * c + 1 < p) v.y = sc * double(src[i * ld + 2 * c + 1]);
    out[gid] = sign != 0.0 ? cmul(v, twist_factor(i, n, sign)) : v;
  }
}

// dst (n x p real) = scale (times rs[i] when rs is not null) times the two
// real columns of exp(sign i pi i / n) in[i, c] (sign 0: no twist)
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_unpack_twist(int64_t n, int p, int64_t ld, int q, const cplx* __restrict__ in,
               T* __restrict__ dst, double scale, const double* __restrict__ rs, double sign) {
  for (int64_t gid = int64_t(blockIdx.x) * kThreads + threadIdx.x; gid < n * p;
       gid += int64_t(gridDim.x) * kThreads) {
    const int64_t i = gid / p;
    const int col = int(gid % p);
    cplx v = in[i * q + col / 2];
    if (sign != 0.0) v = cmul(v, twist_factor(i, n, sign));
    dst[i * ld + col] = T((rs ? scale * rs[i] : scale) * ((col & 1) ? v.y : v.x));
  }
}

// data[i, c] *= exp(sign i pi i / n)
__global__ void __launch_bounds__(kThreads)
k_twist(int64_t n, int q, cplx* __restrict__ data, double sign) {
  for (int64_t gid = int64_t(blockIdx.x) * kThreads + threadIdx.x; gid < n * q;
       gid += int64_t(gridDim.x) * kThreads)
    data[gid] = cmul(data[gid], twist_factor(gid / q, n, sign));
}

// out[i, c] = in[i, c] * h[(n - i) mod n] * scale: the spectrum of the
// transposed circulant (index reversal of the spectrum)
__global__ void __launch_bounds__(kThreads)
k_spec_mul_rev_to(int64_t n, int q, const cplx* __restrict__ in, const cplx* __restrict__ h,
                  cplx* __restrict__ out, double scale) {
  for (int64_t gid = int64_t(blockIdx.x) * kThreads + threadIdx.x; gid < n * q;
       gid += int64_t(gridDim.x) * kThreads) {
    const int64_t i = gid / q;
    const cplx v = cmul(in[gid], h[i == 0 ? 0 : n - i]);
    out[gid] = {scale * v.x, scale * v.y};
  }
}

// partial sums of x . y (FP64 vectors of length len) per workgroup
__global__ void __launch_bounds__(kThreads)
k_dot_partial(int64_t len, const double* __restrict__ x, const double* __restrict__ y,
              double* __restrict__ partial) {
  __shared__ double red[kThreads];
  double s = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < len;
       i += int64_t(gridDim.x) * kThreads)
    s += x[i] * y[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = kThreads / 2; st >= 1; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// y = a x + b y  (length len)
__global__ void __launch_bounds__(kThreads)
k_axpby(int64_t len, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < len;
       i += int64_t(gridDim.x) * kThreads)
    y[i] = a * x[i] + b * y[i];
}

}  // namespace expmv
