// Host-side set-up of the smoothed-aggregation algebraic multigrid (SA-AMG)
// hierarchy that preconditions the inner solver of (tA)^{-1} V.
//
// The paper applies its preconditioner A^{-1} through a sparse LU
// factorisation and, for matrices too large to factor, through an iterative
// inner solver (Section 4.1).  On the GPU A^{-1} V is an inner Krylov solve;
// this hierarchy is that solve's preconditioner, so the result is still
// A^{-1} V to the inner tolerance.  Construction follows the
// standard smoothed-aggregation recipe:
//   strength   |a_ij| >= theta_l sqrt(a_ii a_jj), symmetrised, theta_l = theta / 2^l
//   aggregates greedy three-phase aggregation of the strength graph
//   T          piecewise-constant tentative prolongator, unit-norm columns
//   P          (I - omega D^{-1} A) T, omega = (4/3) / lambda_max(D^{-1} A)
//   A_{l+1}    P^T A_l P (Galerkin), R = P^T
// down to at most max_coarse unknowns, whose operator is inverted densely.
#pragma once

#include <cstdint>
#include <vector>

namespace expmv {

struct HostCsr {
  int64_t nrows = 0, ncols = 0;
  std::vector<int64_t> rp;   // nrows + 1
  std::vector<int32_t> ci;
  std::vector<double> v;
  int64_t nnz() const { return rp.empty() ? 0 : rp.back(); }
};

struct AmgParams {
  double theta = 0.08;         // strength threshold of the finest level
  int max_coarse = 500;        // coarsest level size (dense inverse)
  int max_levels = 12;
  bool symmetric = true;       // A symmetric: Lanczos eigenvalue estimate
};

struct AmgLevelHost {
  HostCsr A;                   // operator of the level (level 0: the input)
  HostCsr P, R;                // prolongator to this level from the next, R = P^T
  std::vector<int32_t> agg;    // aggregate of each unknown (empty on the coarsest)
  std::vector<double> dinv;    // 1 / diag(A)
  double lmax = 0.0;           // upper estimate of lambda_max(D^{-1} A)
};

struct AmgHost {
  std::vector<AmgLevelHost> lv;      // lv.back() is the coarsest level
  std::vector<double> coarse_inv;    // nc x nc row-major inverse of lv.back().A
};

// 0 on success; 1 for a zero or non-positive diagonal; 2 for a singular
// coarsest operator.
int amg_build(const HostCsr& A, const AmgParams& prm, AmgHost& out);

HostCsr csr_transpose(const HostCsr& A);
HostCsr csr_matmul(const HostCsr& A, const HostCsr& B);

// I - s A D^{-1} (left = false) or I - s D^{-1} A (left = true) with
// D^{-1} = diag(dinv), on A's pattern plus the diagonal: the residual map
// b - A x and the error map of one Jacobi step x = s D^{-1} b.
// sum over the entries a_ik of A of the length of row k of B: an upper
// bound of nnz(A B) that costs one pass over A
int64_t csr_product_nnz_bound(const HostCsr& A, const HostCsr& B);

// a A + b B (union of the patterns)
HostCsr csr_add(const HostCsr& A, const HostCsr& B, double a, double b);

HostCsr jacobi_step_operator(const HostCsr& A, const std::vector<double>& dinv, double s,
                             bool left);

// Fused transfer operators of a V-cycle level whose pre-smoothed iterate is
// x1 = D^{-1} (alpha b - beta A D^{-1} b) (one Jacobi/Chebyshev step from zero:
// alpha = s0, beta = 0; two Chebyshev steps: see the device V-cycle):
//   restriction of the residual b - A x1:  Rf = R (I - A D^{-1} S),
//                                           S = alpha I - beta A D^{-1};
//   prolongation followed by one step x += s0 D^{-1} (b - A x):
//                                           Pf = (I - s0 D^{-1} A) P.
HostCsr fused_restriction(const AmgLevelHost& L, double alpha, double beta);
HostCsr fused_prolongation(const AmgLevelHost& L, double s0);
// upper bounds of nnz(Rf) and nnz(Pf) from the product patterns (one pass)
int64_t fused_restriction_nnz_bound(const AmgLevelHost& L, double beta);
int64_t fused_prolongation_nnz_bound(const AmgLevelHost& L);

}  // namespace expmv
