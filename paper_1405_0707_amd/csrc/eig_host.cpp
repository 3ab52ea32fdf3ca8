// Host eigensolvers for the small projected matrix H_d of the restart step
// (Algorithm 1/2, Step 5: all eigenpairs of H_d, d <= (m+1) p).
//
// Symmetric: Householder reduction to tridiagonal form with the orthogonal
// factor accumulated, then the implicit symmetric QR iteration with the
// Wilkinson shift (Golub & Van Loan, Matrix Computations, Section 8.3).
// General: reduction to upper Hessenberg form, the shifted QR iteration on
// the Hessenberg matrix for the eigenvalues, and one step of inverse
// iteration per eigenvalue (complex arithmetic) for the eigenvectors.
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

// Hessenberg reduction by Householder reflections (no accumulation needed:
// only the eigenvalues are taken from the Hessenberg form).
void hessenberg(int n, std::vector<double>& A) {
  auto at = [&](int i, int j) -> double& { return A[size_t(i) * n + j]; };
  std::vector<double> v(n);
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
    // left: rows k+1.. of columns k..n-1
    for (int j = k; j < n; ++j) {
      double s = 0.0;
      for (int i = 0; i < m; ++i) s += v[i] * at(k + 1 + i, j);
      s *= beta;
      for (int i = 0; i < m; ++i) at(k + 1 + i, j) -= s * v[i];
    }
    // right: columns k+1.. of all rows
    for (int r = 0; r < n; ++r) {
      double s = 0.0;
      for (int j = 0; j < m; ++j) s += at(r, k + 1 + j) * v[j];
      s *= beta;
      for (int j = 0; j < m; ++j) at(r, k + 1 + j) -= s * v[j];
    }
    for (int i = 1; i < m; ++i) at(k + 1 + i, k) = 0.0;
  }
}

// Eigenvalues of an upper Hessenberg matrix: single-shift QR in complex
// arithmetic with Wilkinson shifts and deflation (the shift of the trailing
// 2 x 2 block closest to its last diagonal entry).
bool hess_eigenvalues(int n, const std::vector<double>& Hr, std::vector<cd>& ev) {
  std::vector<cd> H(size_t(n) * n);
  for (size_t i = 0; i < H.size(); ++i) H[i] = Hr[i];
  auto at = [&](int i, int j) -> cd& { return H[size_t(i) * n + j]; };
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
      const double s = std::abs(at(l - 1, l - 1)) + std::abs(at(l, l));
      if (std::abs(at(l, l - 1)) <= eps * (s == 0.0 ? 1.0 : s)) {
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
    if (++iter > 60 * n) return false;
    // Wilkinson shift
    const cd a = at(hi - 1, hi - 1), b = at(hi - 1, hi), c = at(hi, hi - 1), d = at(hi, hi);
    const cd tr = a + d, det = a * d - b * c;
    const cd disc = std::sqrt(tr * tr - 4.0 * det);
    cd mu1 = 0.5 * (tr + disc), mu2 = 0.5 * (tr - disc);
    cd mu = (std::abs(mu1 - d) < std::abs(mu2 - d)) ? mu1 : mu2;
    if (iter % 11 == 10) mu = d + cd(std::abs(at(hi, hi - 1)), 0.0);  // exceptional shift
    // QR step on the active block l..hi with Givens rotations
    for (int k = l; k <= hi; ++k) at(k, k) -= mu;
    std::vector<cd> cs(hi - l), sn(hi - l);
    for (int k = l; k < hi; ++k) {
      const cd x = at(k, k), y = at(k + 1, k);
      const double r = std::hypot(std::abs(x), std::abs(y));
      cd cc = (r == 0.0) ? cd(1.0) : x / r;
      cd ss = (r == 0.0) ? cd(0.0) : y / r;
      cs[k - l] = cc;
      sn[k - l] = ss;
      // rows k, k+1:  [conj(c) conj(s); -s c]
      for (int j = k; j < n; ++j) {
        const cd t1 = at(k, j), t2 = at(k + 1, j);
        at(k, j) = std::conj(cc) * t1 + std::conj(ss) * t2;
        at(k + 1, j) = -ss * t1 + cc * t2;
      }
    }
    for (int k = l; k < hi; ++k) {
      const cd cc = cs[k - l], ss = sn[k - l];
      // columns k, k+1: multiply by the adjoint of the row rotation
      for (int i = 0; i <= std::min(hi, k + 2); ++i) {
        const cd t1 = at(i, k), t2 = at(i, k + 1);
        at(i, k) = t1 * cc + t2 * ss;
        at(i, k + 1) = -t1 * std::conj(ss) + t2 * std::conj(cc);
      }
    }
    for (int k = l; k <= hi; ++k) at(k, k) += mu;
  }
  return true;
}

// LU factorisation with partial pivoting of a dense complex matrix, in
// place: M = P^T L U, L unit lower (below the diagonal), U upper; piv[c] is
// the row swapped into position c.
void complex_lu(int n, std::vector<cd>& M, std::vector<int>& piv) {
  auto at = [&](int i, int j) -> cd& { return M[size_t(i) * n + j]; };
  piv.resize(n);
  for (int c = 0; c < n; ++c) {
    int pv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::abs(at(r, c)) > std::abs(at(pv, c))) pv = r;
    piv[c] = pv;
    if (pv != c)
      for (int j = 0; j < n; ++j) std::swap(at(c, j), at(pv, j));
    if (at(c, c) == cd(0.0)) at(c, c) = cd(1e-300);
    for (int r = c + 1; r < n; ++r) {
      const cd l = at(r, c) / at(c, c);
      at(r, c) = l;
      if (l == cd(0.0)) continue;
      for (int j = c + 1; j < n; ++j) at(r, j) -= l * at(c, j);
    }
  }
}

void complex_lu_solve(int n, const std::vector<cd>& M, const std::vector<int>& piv,
                      std::vector<cd>& x) {
  auto at = [&](int i, int j) { return M[size_t(i) * n + j]; };
  for (int c = 0; c < n; ++c) {
    if (piv[c] != c) std::swap(x[c], x[piv[c]]);
    for (int r = c + 1; r < n; ++r) x[r] -= at(r, c) * x[c];
  }
  for (int c = n - 1; c >= 0; --c) {
    cd s = x[c];
    for (int j = c + 1; j < n; ++j) s -= at(c, j) * x[j];
    x[c] = s / at(c, c);
  }
}
}  // namespace

bool general_eigvals(int n, const double* Ain, double* wr, double* wi) {
  std::vector<double> Hh(Ain, Ain + size_t(n) * n);
  hessenberg(n, Hh);
  std::vector<cd> ev;
  if (!hess_eigenvalues(n, Hh, ev)) return false;
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
                     const char* want, double* Vr, double* Vi) {
  double scale = 0.0;
  for (int i = 0; i < n; ++i) scale = std::max(scale, std::hypot(wr[i], wi[i]));
  // eigenvectors by inverse iteration on the original matrix: one LU of
  // A - (lambda + pert) I, two solves
  std::vector<cd> M(size_t(n) * n);
  std::vector<int> piv;
  for (int i = 0; i < n; ++i) {
    if (want && !want[i]) {
      for (int r = 0; r < n; ++r) Vr[size_t(r) * n + i] = Vi[size_t(r) * n + i] = 0.0;
      continue;
    }
    const cd lam(wr[i], wi[i]);
    const double pert = 1e-13 * (scale == 0.0 ? 1.0 : scale);
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < n; ++c) M[size_t(r) * n + c] = A[size_t(r) * n + c] - ((r == c) ? lam + pert : 0.0);
    complex_lu(n, M, piv);
    std::vector<cd> x(n);
    for (int r = 0; r < n; ++r) x[r] = cd(1.0 / std::sqrt(double(n)), 0.37 / (r + 1.0));
    for (int it = 0; it < 2; ++it) {
      complex_lu_solve(n, M, piv, x);
      double nr = 0.0;
      for (auto& e : x) nr += std::norm(e);
      nr = std::sqrt(nr);
      for (auto& e : x) e /= nr;
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
  if (!general_eigvals(n, A, wr, wi)) return false;
  general_eigvecs(n, A, wr, wi, nullptr, Vr, Vi);
  return true;
}

}  // namespace expmv
