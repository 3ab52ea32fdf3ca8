// Host eigensolvers for the small projected matrix H_d of the restart step
// (Algorithm 1/2, Step 5: all eigenpairs of H_d, d <= (m+1) p).
//
// Symmetric: Householder reduction to tridiagonal form with the orthogonal
// factor accumulated, then the implicit symmetric QR iteration with the
// Wilkinson shift (Golub & Van Loan, Matrix Computations, Section 8.3).
// General: reduction to upper Hessenberg form H = Q^T A Q, Francis's
// double-shift QR iteration on H for the eigenvalues (real arithmetic), and
// two steps of inverse iteration on H per wanted eigenvalue (complex
// arithmetic, O(n^2) each) for the eigenvectors, mapped back by Q.
#include "eig_host.hpp"

#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

namespace expmv {

bool sym_eig(int n, const double* Ain, double* w, double* Q) {
  std::vector<double> A(Ain, Ain + size_t(n) * n);
  auto at = [&](int i, int j) -> double& { return A[size_t(i) * n + j]; };
  auto q = [&](int i, int j) -> double& { return Q[size_t(i) * n + j]; };
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) q(i, j) = (i == j) ? 1.0 : 0.0;
  // symmetrise
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const double s = 0.5 * (at(i, j) + at(j, i));
      at(i, j) = s;
      at(j, i) = s;
    }
  std::vector<double> v(n), pv(n), wv(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // length of the column part below the diagonal
    double xn = 0.0;
    for (int i = 0; i < m; ++i) xn += at(k + 1 + i, k) * at(k + 1 + i, k);
    xn = std::sqrt(xn);
    if (xn == 0.0) continue;
    const double x0 = at(k + 1, k);
    const double alpha = (x0 >= 0.0) ? -xn : xn;
    for (int i = 0; i < m; ++i) v[i] = at(k + 1 + i, k);
    v[0] -= alpha;
    double vn2 = 0.0;
    for (int i = 0; i < m; ++i) vn2 += v[i] * v[i];
    if (vn2 == 0.0) continue;
    const double beta = 2.0 / vn2;
    // p = beta * A22 v
    for (int i = 0; i < m; ++i) {
      double s = 0.0;
      for (int j = 0; j < m; ++j) s += at(k + 1 + i, k + 1 + j) * v[j];
      pv[i] = beta * s;
    }
    double ptv = 0.0;
    for (int i = 0; i < m; ++i) ptv += pv[i] * v[i];
    for (int i = 0; i < m; ++i) wv[i] = pv[i] - 0.5 * beta * ptv * v[i];
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) at(k + 1 + i, k + 1 + j) -= v[i] * wv[j] + wv[i] * v[j];
    at(k + 1, k) = alpha;
    at(k, k + 1) = alpha;
    for (int i = 1; i < m; ++i) {
      at(k + 1 + i, k) = 0.0;
      at(k, k + 1 + i) = 0.0;
    }
    // Q(:, k+1:) -= beta (Q(:, k+1:) v) v^T
    for (int r = 0; r < n; ++r) {
      double s = 0.0;
      for (int j = 0; j < m; ++j) s += q(r, k + 1 + j) * v[j];
      s *= beta;
      for (int j = 0; j < m; ++j) q(r, k + 1 + j) -= s * v[j];
    }
  }
  std::vector<double> a(n), b(std::max(n - 1, 1));
  for (int i = 0; i < n; ++i) a[i] = at(i, i);
  for (int i = 0; i + 1 < n; ++i) b[i] = at(i + 1, i);
  const double eps = 2.220446049250313e-16;
  int hi = n - 1;
  int guard = 0;
  while (hi > 0 && guard < 60 * n) {
    if (std::fabs(b[hi - 1]) <= eps * (std::fabs(a[hi - 1]) + std::fabs(a[hi]))) {
      b[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && std::fabs(b[lo - 1]) > eps * (std::fabs(a[lo - 1]) + std::fabs(a[lo]))) --lo;
    ++guard;
    // Wilkinson shift from the trailing 2 x 2 block
    const double dd = 0.5 * (a[hi - 1] - a[hi]);
    const double bb = b[hi - 1];
    const double den = dd + std::copysign(std::hypot(dd, bb), dd == 0.0 ? 1.0 : dd);
    const double mu = a[hi] - bb * bb / den;
    double x = a[lo] - mu, z = b[lo];
    for (int k = lo; k < hi; ++k) {
      const double r = std::hypot(x, z);
      const double c = (r == 0.0) ? 1.0 : x / r;
      const double s = (r == 0.0) ? 0.0 : z / r;
      if (k > lo) b[k - 1] = r;
      const double ak = a[k], ak1 = a[k + 1], bk = b[k];
      a[k] = c * c * ak + 2.0 * c * s * bk + s * s * ak1;
      a[k + 1] = s * s * ak - 2.0 * c * s * bk + c * c * ak1;
      b[k] = c * s * (ak1 - ak) + (c * c - s * s) * bk;
      if (k + 1 < hi) {
        z = s * b[k + 1];
        b[k + 1] *= c;
        x = b[k];
      }
      for (int r2 = 0; r2 < n; ++r2) {
        const double qk = q(r2, k), qk1 = q(r2, k + 1);
        q(r2, k) = c * qk + s * qk1;
        q(r2, k + 1) = -s * qk + c * qk1;
      }
    }
  }
  bool finite = true;
  for (int i = 0; i < n; ++i) {
    w[i] = a[i];
    finite = finite && std::isfinite(a[i]);
  }
  for (size_t i = 0; i < size_t(n) * n; ++i) finite = finite && std::isfinite(Q[i]);
  return hi == 0 && finite;
}

// ---------------------------------------------------------------------------
// general real matrix

namespace {
using cd = std::complex<double>;

// Hessenberg reduction A <- Q^T A Q by Householder reflections, row by row
// so that every inner loop runs along a row.  With Q non-null the orthogonal
// factor is formed (row-major) by accumulating the reflectors backwards.
void hessenberg(int n, std::vector<double>& A, std::vector<double>* Q) {
  auto at = [&](int i, int j) -> double& { return A[size_t(i) * n + j]; };
  std::vector<double> v(n), s(n);
  std::vector<double> refl, betas;
  if (Q) {
    refl.assign(size_t(n) * n, 0.0);   // reflector k in row k, columns k+1..n-1
    betas.assign(n, 0.0);
  }
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    double xn = 0.0;
    for (int i = 0; i < m; ++i) xn += at(k + 1 + i, k) * at(k + 1 + i, k);
    xn = std::sqrt(xn);
    if (xn == 0.0) continue;
    const double alpha = (at(k + 1, k) >= 0.0) ? -xn : xn;
    for (int i = 0; i < m; ++i) v[i] = at(k + 1 + i, k);
    v[0] -= alpha;
    double vn2 = 0.0;
    for (int i = 0; i < m; ++i) vn2 += v[i] * v[i];
    if (vn2 == 0.0) continue;
    const double beta = 2.0 / vn2;
    // left: rows k+1.. of columns k..n-1, s = beta v^T A(k+1:, k:)
    for (int j = k; j < n; ++j) s[j] = 0.0;
    for (int i = 0; i < m; ++i) {
      const double vi = v[i];
      const double* row = &A[size_t(k + 1 + i) * n];
      for (int j = k; j < n; ++j) s[j] += vi * row[j];
    }
    for (int j = k; j < n; ++j) s[j] *= beta;
    for (int i = 0; i < m; ++i) {
      const double vi = v[i];
      double* row = &A[size_t(k + 1 + i) * n];
      for (int j = k; j < n; ++j) row[j] -= s[j] * vi;
    }
    // right: columns k+1.. of all rows
    for (int r = 0; r < n; ++r) {
      double sr = 0.0;
      double* row = &A[size_t(r) * n + k + 1];
      for (int j = 0; j < m; ++j) sr += row[j] * v[j];
      sr *= beta;
      for (int j = 0; j < m; ++j) row[j] -= sr * v[j];
    }
    for (int i = 1; i < m; ++i) at(k + 1 + i, k) = 0.0;
    if (Q) {
      for (int i = 0; i < m; ++i) refl[size_t(k) * n + k + 1 + i] = v[i];
      betas[k] = beta;
    }
  }
  if (!Q) return;
  // Q = P_0 P_1 ... P_{n-3}: backwards, P_k touches rows and columns k+1..
  Q->assign(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) (*Q)[size_t(i) * n + i] = 1.0;
  for (int k = n - 3; k >= 0; --k) {
    const double beta = betas[k];
    if (beta == 0.0) continue;
    const int m = n - k - 1;
    const double* vk = &refl[size_t(k) * n + k + 1];
    for (int j = k + 1; j < n; ++j) s[j] = 0.0;
    for (int i = 0; i < m; ++i) {
      const double vi = vk[i];
      const double* row = &(*Q)[size_t(k + 1 + i) * n];
      for (int j = k + 1; j < n; ++j) s[j] += vi * row[j];
    }
    for (int j = k + 1; j < n; ++j) s[j] *= beta;
    for (int i = 0; i < m; ++i) {
      const double vi = vk[i];
      double* row = &(*Q)[size_t(k + 1 + i) * n];
      for (int j = k + 1; j < n; ++j) row[j] -= s[j] * vi;
    }
  }
}

// Eigenvalues of a real 2 x 2 block [a b; c d]: a real pair, or a complex
// conjugate pair (re +- i im, im > 0).  With p = (a - d)/2 and q = p^2 + bc
// the eigenvalues are d + p +- sqrt(q); for q >= 0 the larger one in
// magnitude is formed without cancellation, the other from the product
// of the two (the determinant).
void eig2x2(double a, double b, double c, double d, cd& e1, cd& e2) {
  const double p = 0.5 * (a - d);
  const double q = p * p + b * c;
  if (q >= 0.0) {
    const double z = p + std::copysign(std::sqrt(q), p);
    e1 = cd(d + z, 0.0);
    e2 = (z != 0.0) ? cd(d - b * c / z, 0.0) : cd(d, 0.0);
  } else {
    const double im = std::sqrt(-q);
    e1 = cd(d + p, im);
    e2 = cd(d + p, -im);
  }
}

// Eigenvalues of an upper Hessenberg matrix by the implicit double-shift QR
// iteration of Francis (Golub & Van Loan, Matrix Computations, Section 7.5):
// each step takes the two eigenvalues of the trailing 2 x 2 block of the
// active block as shifts, in real arithmetic through their sum s and
// product t, and chases the bulge that the first column of
// H^2 - s H + t I starts down the block with 3 x 3 Householder reflections.
// A subdiagonal entry below eps (|h_{k-1,k-1}| + |h_kk|) is set to zero,
// and 1 x 1 and 2 x 2 blocks split off give their eigenvalues.  Only the
// eigenvalues are wanted, so each step updates the active block l..hi
// alone.  Every tenth step without a deflation uses two ad hoc shifts
// (h_hi,hi + w and h_hi,hi - w/2, w the last two subdiagonal magnitudes)
// to leave a cycle.
bool hess_eigenvalues(int n, const std::vector<double>& Hin, std::vector<cd>& ev) {
  std::vector<double> H(Hin);
  auto at = [&](int i, int j) -> double& { return H[size_t(i) * n + j]; };
  const double eps = 2.220446049250313e-16;
  ev.assign(n, cd(0.0));
  int hi = n - 1;
  int iter = 0;
  while (hi >= 0) {
    if (hi == 0) {
      ev[0] = at(0, 0);
      break;
    }
    int l = hi;
    while (l > 0) {
      const double s = std::fabs(at(l - 1, l - 1)) + std::fabs(at(l, l));
      if (std::fabs(at(l, l - 1)) <= eps * (s == 0.0 ? 1.0 : s)) {
        at(l, l - 1) = 0.0;
        break;
      }
      --l;
    }
    if (l == hi) {
      ev[hi] = at(hi, hi);
      --hi;
      iter = 0;
      continue;
    }
    if (l == hi - 1) {
      eig2x2(at(hi - 1, hi - 1), at(hi - 1, hi), at(hi, hi - 1), at(hi, hi), ev[hi - 1], ev[hi]);
      hi -= 2;
      iter = 0;
      continue;
    }
    if (++iter > 60 * n) return false;
    double s, t;
    if (iter % 10 == 0) {
      const double w = std::fabs(at(hi, hi - 1)) + std::fabs(at(hi - 1, hi - 2));
      const double m1 = at(hi, hi) + w, m2 = at(hi, hi) - 0.5 * w;
      s = m1 + m2;
      t = m1 * m2;
    } else {
      s = at(hi - 1, hi - 1) + at(hi, hi);
      t = at(hi - 1, hi - 1) * at(hi, hi) - at(hi - 1, hi) * at(hi, hi - 1);
    }
    // first column of (H - mu1 I)(H - mu2 I) on the active block
    double x = at(l, l) * at(l, l) + at(l, l + 1) * at(l + 1, l) - s * at(l, l) + t;
    double y = at(l + 1, l) * (at(l, l) + at(l + 1, l + 1) - s);
    double z = at(l + 1, l) * at(l + 2, l + 1);
    for (int k = l; k <= hi - 2; ++k) {
      // reflection I - beta v v^T taking (x, y, z) to a multiple of e_1
      const double nx = std::sqrt(x * x + y * y + z * z);
      if (nx != 0.0) {
        const double alpha = (x >= 0.0) ? -nx : nx;
        const double v0 = x - alpha, v1 = y, v2 = z;
        const double beta = 2.0 / (v0 * v0 + v1 * v1 + v2 * v2);
        // rows k..k+2, columns max(l, k-1)..hi
        const int c0 = std::max(l, k - 1);
        double* r0 = &H[size_t(k) * n];
        double* r1 = r0 + n;
        double* r2 = r1 + n;
        for (int j = c0; j <= hi; ++j) {
          const double g = beta * (v0 * r0[j] + v1 * r1[j] + v2 * r2[j]);
          r0[j] -= g * v0;
          r1[j] -= g * v1;
          r2[j] -= g * v2;
        }
        // columns k..k+2, rows l..min(k+3, hi)
        const int r_end = std::min(k + 3, hi);
        for (int i = l; i <= r_end; ++i) {
          double* row = &H[size_t(i) * n + k];
          const double g = beta * (row[0] * v0 + row[1] * v1 + row[2] * v2);
          row[0] -= g * v0;
          row[1] -= g * v1;
          row[2] -= g * v2;
        }
        if (k > l) {
          // the reflection zeroed the bulge below the subdiagonal
          at(k + 1, k - 1) = 0.0;
          at(k + 2, k - 1) = 0.0;
        }
      }
      x = at(k + 1, k);
      y = at(k + 2, k);
      if (k + 3 <= hi) z = at(k + 3, k);
    }
    // last step: a 2 x 2 reflection on rows and columns hi-1, hi
    {
      const int k = hi - 1;
      const double nx = std::hypot(x, y);
      if (nx != 0.0) {
        const double alpha = (x >= 0.0) ? -nx : nx;
        const double v0 = x - alpha, v1 = y;
        const double beta = 2.0 / (v0 * v0 + v1 * v1);
        double* r0 = &H[size_t(k) * n];
        double* r1 = r0 + n;
        for (int j = std::max(l, k - 1); j <= hi; ++j) {
          const double g = beta * (v0 * r0[j] + v1 * r1[j]);
          r0[j] -= g * v0;
          r1[j] -= g * v1;
        }
        for (int i = l; i <= hi; ++i) {
          double* row = &H[size_t(i) * n + k];
          const double g = beta * (row[0] * v0 + row[1] * v1);
          row[0] -= g * v0;
          row[1] -= g * v1;
        }
        if (k > l) at(k + 1, k - 1) = 0.0;
      }
    }
  }
  // a NaN or infinite entry passes every deflation test as "not small" or
  // ends in a block split off with non-finite eigenvalues
  for (const cd& e : ev)
    if (!std::isfinite(e.real()) || !std::isfinite(e.imag())) return false;
  return true;
}

// M = H - mu I for an upper Hessenberg H, factorised in place by Gaussian
// elimination with partial pivoting: each column has one entry below the
// diagonal, so row c is swapped (sw[c]) with row c + 1 at most and L keeps
// one multiplier per column (lm[c]); U overwrites the upper triangle.  A
// zero pivot is replaced by 1e-300 (the solve is inverse iteration, where
// an exactly singular shift is the ideal case).  O(n^2).
void hess_shifted_lu(int n, const std::vector<double>& H, cd mu, std::vector<cd>& M,
                     std::vector<cd>& lm, std::vector<char>& sw) {
  M.assign(size_t(n) * n, cd(0.0));
  for (int i = 0; i < n; ++i)
    for (int j = std::max(0, i - 1); j < n; ++j)
      M[size_t(i) * n + j] = H[size_t(i) * n + j] - (i == j ? mu : cd(0.0));
  lm.assign(n, cd(0.0));
  sw.assign(n, 0);
  for (int c = 0; c + 1 < n; ++c) {
    cd* rc = &M[size_t(c) * n];
    cd* rn = &M[size_t(c + 1) * n];
    if (std::abs(rn[c]) > std::abs(rc[c])) {
      for (int j = c; j < n; ++j) std::swap(rc[j], rn[j]);
      sw[c] = 1;
    }
    if (rc[c] == cd(0.0)) rc[c] = cd(1e-300);
    const cd l = rn[c] / rc[c];
    lm[c] = l;
    if (l != cd(0.0))
      for (int j = c + 1; j < n; ++j) rn[j] -= l * rc[j];
  }
  if (M[size_t(n) * n - 1] == cd(0.0)) M[size_t(n) * n - 1] = cd(1e-300);
}

void hess_lu_solve(int n, const std::vector<cd>& M, const std::vector<cd>& lm,
                   const std::vector<char>& sw, std::vector<cd>& x) {
  for (int c = 0; c + 1 < n; ++c) {
    if (sw[c]) std::swap(x[c], x[c + 1]);
    x[c + 1] -= lm[c] * x[c];
  }
  for (int c = n - 1; c >= 0; --c) {
    const cd* row = &M[size_t(c) * n];
    cd s = x[c];
    for (int j = c + 1; j < n; ++j) s -= row[j] * x[j];
    x[c] = s / row[c];
  }
}
}  // namespace

bool general_eigvals(int n, const double* Ain, double* wr, double* wi, HessForm* hf) {
  HessForm local;
  HessForm& f = hf ? *hf : local;
  f.n = n;
  f.H.assign(Ain, Ain + size_t(n) * n);
  hessenberg(n, f.H, hf ? &f.Q : nullptr);
  std::vector<cd> ev;
  if (!hess_eigenvalues(n, f.H, ev)) return false;
  // make conjugate pairs exact: pair each eigenvalue with Im > tol with the
  // closest conjugate candidate
  double scale = 0.0;
  for (auto& e : ev) scale = std::max(scale, std::abs(e));
  const double tol = 1e-10 * (scale == 0.0 ? 1.0 : scale);
  std::vector<int> used(n, 0);
  std::vector<cd> ev2(n);
  for (int i = 0; i < n; ++i) {
    if (used[i]) continue;
    if (std::fabs(ev[i].imag()) <= tol) {
      ev2[i] = cd(ev[i].real(), 0.0);
      used[i] = 1;
      continue;
    }
    int best = -1;
    double bd = 1e300;
    for (int j = 0; j < n; ++j) {
      if (used[j] || j == i) continue;
      const double dj = std::abs(ev[j] - std::conj(ev[i]));
      if (dj < bd) {
        bd = dj;
        best = j;
      }
    }
    const cd avg = (best >= 0) ? 0.5 * (ev[i] + std::conj(ev[best])) : ev[i];
    const cd up = (avg.imag() >= 0.0) ? avg : std::conj(avg);
    ev2[i] = up;
    used[i] = 1;
    if (best >= 0) {
      ev2[best] = std::conj(up);
      used[best] = 1;
    }
  }
  for (int i = 0; i < n; ++i) {
    wr[i] = ev2[i].real();
    wi[i] = ev2[i].imag();
  }
  return true;
}

void general_eigvecs(int n, const double* A, const double* wr, const double* wi,
                     const char* want, double* Vr, double* Vi, const HessForm* hf) {
  HessForm local;
  if (!hf || hf->n != n || hf->Q.size() != size_t(n) * n) {
    local.n = n;
    local.H.assign(A, A + size_t(n) * n);
    hessenberg(n, local.H, &local.Q);
    hf = &local;
  }
  const std::vector<double>& H = hf->H;
  const std::vector<double>& Q = hf->Q;
  double scale = 0.0;
  for (int i = 0; i < n; ++i) scale = std::max(scale, std::hypot(wr[i], wi[i]));
  const double pert = 1e-13 * (scale == 0.0 ? 1.0 : scale);
  // eigenvectors by inverse iteration on the Hessenberg form H = Q^T A Q
  // (one O(n^2) LU of H - (lambda + pert) I, two solves), mapped back by Q;
  // the start vector is the same in A's coordinates for every eigenvalue
  std::vector<cd> y0(n, cd(0.0));
  for (int r = 0; r < n; ++r) {
    const cd xr(1.0 / std::sqrt(double(n)), 0.37 / (r + 1.0));
    const double* qr = &Q[size_t(r) * n];
    for (int c = 0; c < n; ++c) y0[c] += qr[c] * xr;   // y0 = Q^T x0
  }
  std::vector<cd> M, lm, y(n), x(n);
  std::vector<char> sw;
  for (int i = 0; i < n; ++i) {
    if (want && !want[i]) {
      for (int r = 0; r < n; ++r) Vr[size_t(r) * n + i] = Vi[size_t(r) * n + i] = 0.0;
      continue;
    }
    const cd lam(wr[i], wi[i]);
    hess_shifted_lu(n, H, lam + pert, M, lm, sw);
    y = y0;
    for (int it = 0; it < 2; ++it) {
      hess_lu_solve(n, M, lm, sw, y);
      double nr = 0.0;
      for (auto& e : y) nr += std::norm(e);
      nr = std::sqrt(nr);
      for (auto& e : y) e /= nr;
    }
    for (int r = 0; r < n; ++r) {
      const double* qr = &Q[size_t(r) * n];
      cd acc(0.0);
      for (int c = 0; c < n; ++c) acc += qr[c] * y[c];
      x[r] = acc;
    }
    // normalise the phase: largest component real positive
    int im = 0;
    for (int r = 1; r < n; ++r)
      if (std::abs(x[r]) > std::abs(x[im])) im = r;
    const cd ph = std::abs(x[im]) > 0 ? std::conj(x[im]) / std::abs(x[im]) : cd(1.0);
    for (int r = 0; r < n; ++r) {
      const cd e = x[r] * ph;
      Vr[size_t(r) * n + i] = e.real();
      Vi[size_t(r) * n + i] = e.imag();
    }
  }
}

bool general_eig(int n, const double* A, double* wr, double* wi, double* Vr, double* Vi) {
  HessForm hf;
  if (!general_eigvals(n, A, wr, wi, &hf)) return false;
  general_eigvecs(n, A, wr, wi, nullptr, Vr, Vi, &hf);
  return true;
}

}  // namespace expmv
