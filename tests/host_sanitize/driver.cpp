// Exercises the exported host code (AMG set-up and the small eigensolvers)
// under AddressSanitizer and UndefinedBehaviorSanitizer, built with g++ on the
// CPU by tests/test_host_sanitize.py.  Each check prints a line; the program
// returns non-zero on the first failed check (the sanitizers abort on their
// own findings).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <random>
#include <vector>

#include "amg_host.hpp"
#include "eig_host.hpp"

using namespace expmv;

static int fails = 0;
static void check(bool ok, const char* what) {
  std::printf("%s %s\n", ok ? "ok  " : "FAIL", what);
  if (!ok) ++fails;
}

// -K for K the upwind convection-diffusion operator on an N^d grid (d = 2, 3),
// stored as K (positive diagonal), unknowns x fastest
static HostCsr convdiff(int N, int d, double pe, bool variable, unsigned seed) {
  const double h = 1.0 / (N + 1);
  const int64_t n = (d == 2) ? int64_t(N) * N : int64_t(N) * N * N;
  std::mt19937_64 rng(seed);
  std::uniform_real_distribution<double> U(0.5, 2.0);
  HostCsr A;
  A.nrows = A.ncols = n;
  A.rp.assign(1, 0);
  const double vel[3] = {1.0, 0.5, 0.25};
  for (int64_t i = 0; i < n; ++i) {
    int64_t c[3] = {i % N, (i / N) % N, (d == 3) ? i / (int64_t(N) * N) : 0};
    const double kap = variable ? U(rng) : 1.0;
    double diag = 0.0;
    std::vector<std::pair<int32_t, double>> row;
    int64_t stride = 1;
    for (int a = 0; a < d; ++a) {
      const double lo = -kap / (h * h) - pe * vel[a] / h, hi = -kap / (h * h);
      diag += 2.0 * kap / (h * h) + pe * vel[a] / h;
      if (c[a] > 0) row.push_back({int32_t(i - stride), lo});
      if (c[a] + 1 < N) row.push_back({int32_t(i + stride), hi});
      stride *= N;
    }
    row.push_back({int32_t(i), diag});
    std::sort(row.begin(), row.end());
    for (auto& e : row) {
      A.ci.push_back(e.first);
      A.v.push_back(e.second);
    }
    A.rp.push_back(int64_t(A.ci.size()));
  }
  return A;
}

// largest |A - B| entry, comparing each row's entries sorted by column
static double max_abs_diff(const HostCsr& A, const HostCsr& B) {
  if (A.nrows != B.nrows || A.rp != B.rp) return 1e300;
  double m = 0.0;
  for (int64_t i = 0; i < A.nrows; ++i) {
    std::vector<std::pair<int32_t, double>> a, b;
    for (int64_t e = A.rp[i]; e < A.rp[i + 1]; ++e) a.push_back({A.ci[e], A.v[e]});
    for (int64_t e = B.rp[i]; e < B.rp[i + 1]; ++e) b.push_back({B.ci[e], B.v[e]});
    std::sort(a.begin(), a.end());
    std::sort(b.begin(), b.end());
    for (size_t k = 0; k < a.size(); ++k) {
      if (a[k].first != b[k].first) return 1e300;
      m = std::max(m, std::fabs(a[k].second - b[k].second));
    }
  }
  return m;
}

static void amg_case(const char* name, const HostCsr& A, bool symmetric) {
  AmgParams prm;
  prm.symmetric = symmetric;
  prm.max_coarse = 40;
  AmgHost H;
  const int st = amg_build(A, prm, H);
  char buf[160];
  std::snprintf(buf, sizeof buf, "%s: amg_build status %d, %zu levels", name, st, H.lv.size());
  check(st == 0 && H.lv.size() >= 2, buf);
  if (st != 0) return;
  for (size_t l = 0; l + 1 < H.lv.size(); ++l) {
    const AmgLevelHost& L = H.lv[l];
    check(max_abs_diff(csr_transpose(csr_transpose(L.P)), L.P) == 0.0, "P^T^T = P");
    const HostCsr Rf = fused_restriction(L, 0.7 / L.lmax, 0.1 / (L.lmax * L.lmax));
    const HostCsr Pf = fused_prolongation(L, 0.7 / L.lmax);
    check(Rf.nnz() <= fused_restriction_nnz_bound(L, 0.1), "nnz(Rf) within its bound");
    check(Pf.nnz() <= fused_prolongation_nnz_bound(L), "nnz(Pf) within its bound");
    check(csr_matmul(L.R, L.A).nnz() <= csr_product_nnz_bound(L.R, L.A), "nnz(RA) within its bound");
  }
  check(H.coarse_inv.size() == size_t(H.lv.back().A.nrows) * H.lv.back().A.nrows,
        "coarse inverse is nc x nc");
}

static void sym_case(int n, unsigned seed) {
  std::mt19937_64 rng(seed);
  std::normal_distribution<double> N01;
  std::vector<double> A(size_t(n) * n), w(n), Q(size_t(n) * n);
  for (auto& x : A) x = N01(rng);
  const bool ok = sym_eig(n, A.data(), w.data(), Q.data());
  double res = 0.0, orth = 0.0, scale = 1e-300;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) scale = std::max(scale, std::fabs(A[size_t(i) * n + j]));
  for (int k = 0; k < n; ++k)
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int j = 0; j < n; ++j)
        s += 0.5 * (A[size_t(i) * n + j] + A[size_t(j) * n + i]) * Q[size_t(j) * n + k];
      res = std::max(res, std::fabs(s - w[k] * Q[size_t(i) * n + k]));
      for (int k2 = 0; k2 < n; ++k2) {
        double d = 0.0;
        for (int r = 0; r < n; ++r) d += Q[size_t(r) * n + k] * Q[size_t(r) * n + k2];
        orth = std::max(orth, std::fabs(d - (k == k2 ? 1.0 : 0.0)));
      }
    }
  char buf[160];
  std::snprintf(buf, sizeof buf, "sym_eig n=%d: converged %d, residual %.1e, orthogonality %.1e", n,
                int(ok), res / scale, orth);
  check(ok && res <= 1e-12 * n * scale && orth <= 1e-12 * n, buf);
}

static void general_case(int n, unsigned seed) {
  std::mt19937_64 rng(seed);
  std::normal_distribution<double> N01;
  std::vector<double> A(size_t(n) * n), wr(n), wi(n), Vr(size_t(n) * n), Vi(size_t(n) * n);
  for (auto& x : A) x = N01(rng);
  const bool ok = general_eig(n, A.data(), wr.data(), wi.data(), Vr.data(), Vi.data());
  double res = 0.0, scale = 1e-300;
  for (auto x : A) scale = std::max(scale, std::fabs(x));
  for (int k = 0; k < n; ++k)
    for (int i = 0; i < n; ++i) {
      double sr = 0.0, si = 0.0;
      for (int j = 0; j < n; ++j) {
        sr += A[size_t(i) * n + j] * Vr[size_t(j) * n + k];
        si += A[size_t(i) * n + j] * Vi[size_t(j) * n + k];
      }
      const double vr = Vr[size_t(i) * n + k], vi = Vi[size_t(i) * n + k];
      sr -= wr[k] * vr - wi[k] * vi;
      si -= wr[k] * vi + wi[k] * vr;
      res = std::max(res, std::hypot(sr, si));
    }
  char buf[160];
  std::snprintf(buf, sizeof buf, "general_eig n=%d: converged %d, residual %.1e", n, int(ok),
                res / scale);
  check(ok && res <= 1e-10 * n * scale, buf);
}

int main() {
  amg_case("2D Laplacian 30^2", convdiff(30, 2, 0.0, false, 1), true);
  amg_case("2D variable diffusion 33^2", convdiff(33, 2, 0.0, true, 2), true);
  amg_case("3D convection-diffusion 12^3", convdiff(12, 3, 50.0, false, 3), false);
  {
    HostCsr Z = convdiff(6, 2, 0.0, false, 4);
    for (int64_t i = 0; i < Z.nrows; ++i)
      for (int64_t e = Z.rp[i]; e < Z.rp[i + 1]; ++e)
        if (Z.ci[e] == i && i == 17) Z.v[e] = 0.0;
    AmgHost H;
    check(amg_build(Z, AmgParams{}, H) == 1, "zero diagonal entry refused (status 1)");
  }
  for (int n : {1, 2, 5, 40, 97}) sym_case(n, 100 + n);
  for (int n : {1, 2, 7, 30, 61}) general_case(n, 200 + n);
  {
    std::vector<double> A = {1.0, std::numeric_limits<double>::quiet_NaN(), 2.0, 3.0}, w(2), Q(4);
    check(!sym_eig(2, A.data(), w.data(), Q.data()), "sym_eig reports a NaN input");
    std::vector<double> wr(2), wi(2), Vr(4), Vi(4);
    check(!general_eig(2, A.data(), wr.data(), wi.data(), Vr.data(), Vi.data()),
          "general_eig reports a NaN input");
  }
  std::printf("%s\n", fails ? "FAILED" : "ALL OK");
  return fails ? 1 : 0;
}
